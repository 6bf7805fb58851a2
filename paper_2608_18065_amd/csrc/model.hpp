// Internal state of a model handle and the launchers each translation unit
// provides.  Not part of the ABI.
#pragma once
#include "common.hpp"

struct minsr_model {
  minsr_model_desc d;
  int N, H, dim, cplx, ds;
  int f64;                 // compute precision: 1 double, 0 float
  int linear = 0;          // the linear recurrent test model (MINSR_OPT_LINEAR)
  double* adapt = nullptr;  // adaptive step: [rows] tau, [8] report, [4] trial stats,
                            //   [4] spare, [256] norm partials
  double* theta_bak = nullptr;  // [Np] parameters held while the trial step is evaluated
  minsr::Layout L;
  int device;

  double* theta = nullptr;  // [Np] master parameters
  void* work = nullptr;     // packed working copy (compute precision)
  size_t work_elems = 0;
  minsr::Work<float> wf{};
  minsr::Work<double> wd{};

  int* nbr = nullptr;       // [N][2] path positions of the horizontal and
                            // vertical predecessors (-1 outside the lattice)
  uint8_t* subA = nullptr;  // [N] 1 if the site is on the Marshall sublattice
  int* bonds = nullptr;     // [nb][2] J1-J2 bonds (path positions, a < b):
  int n_nn = 0, n_nnn = 0;  //   n_nn nearest neighbours first, then n_nnn

  // ---- workspace sized for d.max_Ns
  int max_terms = 0;        // off-diagonal terms per sample (upper bound)
  void* states = nullptr;   // [max_Ns][N][H] hidden states
  void* gates = nullptr;    // [max_Ns][N][4][H] gate tape (FP32 1D models, d_h <= 64)
  void* jdp = nullptr;      // [seeds][max_Ns][N][3][H] gate adjoints of the Jacobian (same models)
  void* jtape = nullptr;    // FP32 1D d_h = 128: [seeds][max_Ns][N][4][H] gate adjoints, then
                            //   [seeds][max_Ns][N][2] head adjoints (matrix-core Jacobian)
  double* site = nullptr;   // [max_Ns][N][4]: log p(0), log p(1), phi(0), phi(1)
  double* contrib = nullptr;// [max_terms][max_Ns][2]
  int* elist = nullptr;     // [max_terms][max_Ns] samples with a nonzero matrix element
  int* ecount = nullptr;    // [max_terms + 1] their counts, then the item count
  int* eitems = nullptr;    // [max_terms * ceil(max_Ns / 32)][2] (term, chunk)
  uint32_t* eloc_q = nullptr;  // local-energy work queue: next item, finished waves (zero between launches)
  double* diag = nullptr;   // [max_Ns]
  void* ring = nullptr;     // 2D local-energy recompute windows
  int ring_blocks = 0;
  uint8_t* sigma = nullptr; // [max_Ns][N]
  double* logpsi = nullptr; // [max_Ns][2]
  double* eloc = nullptr;   // [max_Ns][2]
  double* stats = nullptr;  // [4]
  void* O = nullptr;        // [2 max_Ns][Np] raw log-derivatives (compute precision)
  void* R = nullptr;        // [2 max_Ns][Np] centred real form (step precision)
  double* colpart = nullptr;// column-sum partials
  double* colmean = nullptr;// [2][Np]
  double* T = nullptr;      // [n][n] Gram (FP64, or FP32 in the plain form)
  double* Lf = nullptr;     // [n][n] Cholesky factor of T + lambda I
  double* Dinv = nullptr;   // [n/64][64][64] inverses of its diagonal blocks
  float* gpart = nullptr;   // split-K Gram partials
  size_t gpart_elems = 0;
  double* epsp = nullptr;   // [n] eps'
  double* x = nullptr;      // [n] solution
  double* vwork = nullptr;  // solver scratch: forward-substitution vector, tile contributions
  uint32_t* csync = nullptr;// Cholesky tickets and flags
  double* dpart = nullptr;  // update partials
  double* dtheta = nullptr; // [Np]
  uint32_t* status = nullptr;
  double* eig = nullptr;    // eigen solver workspace
  size_t eig_elems = 0;
  int eig_nmax = 0;         // largest n the eigen workspace serves
  int last_n = 0;
  int last_form = 0;
  int force_vector = 0;     // testing: route FP32 local energies to the vector kernel
  // launch parameters (0 = built-in choice), set by the autotuner
  int tune_gram_split = 0;
  int tune_eloc_grid = 0;
  int tune_sample_r = 0;
  int tune_jac_parts = 0;
  int tune_spin_limit = 0;   // polls before a solver wait gives up (0: built in)

  // per-phase event timing of minsr_step (profiling only)
  std::vector<hipEvent_t> ev;   // [t_max][NPHASE + 1]
  int t_max = 0, t_slot = 0;
};

namespace minsr {

// gru.hip
// parameter blocks of theta: Glorot-uniform a (2u - 1) with half-width a,
// u the Philox4x64-10 uniform of (init seed, parameter index); zero where
// a = 0 or outside every block
struct InitBlocks {
  int n;
  long long off[16], size[16];
  double a[16];  // Glorot half-width, 0 for biases
};
int launch_init_blocks(double* theta, long long Np, const InitBlocks& b, uint64_t seed,
                       hipStream_t s);
int launch_init_theta(minsr_model* m, hipStream_t s);
int launch_pack(minsr_model* m, hipStream_t s);
// mode 0: sample, 1: evaluate.  states/site may be null.
// gates (1D, store_every == 1, may be null): [Ns][N][4][H] gate values u, r,
// candidate pre-activation and candidate of every site, for the Jacobian.
// sample_mfma.hip: sampling of 1D FP32 models with d_h = 64 or 128 (N <= 256)
// on the matrix cores; launch_forward takes it for mode 0 where it applies
bool sample_mfma_supported(const minsr_model* m);
int launch_sample_mfma(minsr_model* m, int Ns, const double* uniforms, uint64_t key,
                       uint64_t counter, const uint64_t* counter_ptr, uint8_t* sigma,
                       double* logpsi, void* states, int store_every, double* site, void* gates,
                       uint32_t* zero_word, hipStream_t s);
int launch_forward(minsr_model* m, int mode, int Ns, const double* uniforms, uint64_t key,
                   uint64_t counter, uint8_t* sigma, double* logpsi, void* states,
                   int store_every, double* site, hipStream_t s,
                   const uint64_t* counter_ptr = nullptr, void* gates = nullptr,
                   uint32_t* zero_word = nullptr);
// which: 1 = off-diagonal terms (the recurrence), 2 = diagonal + sum, 3 = both
int launch_eloc(minsr_model* m, const minsr_hamiltonian* H, int Ns, const uint8_t* sigma,
                const double* logpsi, const void* states, const double* site, double* eloc,
                hipStream_t s, int which = 3);
int launch_stats(minsr_model* m, int Ns, const double* eloc, double* stats, double* epsp,
                 uint32_t* status, hipStream_t s);
// gru_mfma.hip: local-energy recurrence of FP32 models on MFMA
bool eloc_mfma_supported(minsr_model* m);
int launch_eloc_mfma(minsr_model* m, const minsr_hamiltonian* H, int Ns, const uint8_t* sigma,
                     const void* states, const double* site, int M, hipStream_t s);
// jacobian.hip: raw rows (scaled by 1/sqrt(Ns)) into O (compute precision)
// gates: the tape written by launch_forward for the same configurations
// (used with ckpt_every == 1 only; may be null)
int launch_jacobian(minsr_model* m, int Ns, const uint8_t* sigma, const void* states,
                    int ckpt_every, void* O, const double* g, double* vjp_part,
                    hipStream_t s, const void* gates = nullptr,
                    const double* site = nullptr);
// jac_mfma.hip: the Jacobian of FP32 1D models with d_h = 128 (N <= 128) on
// the matrix cores; the tape it needs (elements of jtape, 0 if the path
// does not apply) and whether checkpoint stride C fits its shared memory
size_t jac_mfma_tape_elems(int dim, int f64, int H, int N, int cplx, size_t max_Ns);
bool jac_mfma_supported(const minsr_model* m, int C);
int launch_jacobian_mfma(minsr_model* m, int Ns, const uint8_t* sigma, int C, void* O,
                         const double* site, hipStream_t s);
// linalg.hip
// centred (colmean != null) or plain copy of O into R with row stride ldo
// (ldo >= Np; columns Np..ldo-1 are written as zeros)
int launch_center(int rows_per_block, int nblocks, size_t Np, const void* O, int in_f64,
                  void* R, int out_dtype, double* colpart, double* colmean, size_t ldo,
                  hipStream_t s, void* Rlo = nullptr);
// the step keeps O' with rows padded to a multiple of 64 columns
inline size_t padded_ld(size_t Np) { return (Np + 63) / 64 * 64; }
// one instance's Gram in a grouped launch (BF16 split form): its work items
// are [item0, item0 + npairs S) of the tile kernel's grid and
// [ritem0, ritem0 + 16 npairs) of the reduction's
// 32 x 32 sub-tiles of one 128 x 128 Gram tile: the reduction's work items per pair
constexpr int GRAM_SUBTILES = 16;
struct GramJob {
  const void* R;      // BF16 hi rows, stride ld
  const void* Rlo;    // BF16 lo rows
  double* part;       // FP64 partial tiles [S][npairs][128][128]
  double* T;          // [n][n]
  size_t ld, kchunk;
  int n, npairs, S, item0, ritem0, pad;
};
// fills the split, K range and item counts of a job (the same choice as
// launch_gram for the instance); returns an error if its workspace is short
int gram_job(int n, size_t Np, const void* R, const void* Rlo, double* T, float* gpart,
             size_t gpart_elems, int want_split, GramJob* job);
// one launch of tile products and one of reductions over all jobs (a device
// copy of the job table, item0 / ritem0 prefix sums filled in)
int launch_gram_grouped(const GramJob* dev_jobs, int njobs, int items, int ritems,
                        hipStream_t s);
// which: 1 = tile products, 2 = split-K reduction and mirror, 3 = both
// Rlo (BF16 only, may be null): low parts of a hi/lo split of R
// split: split-K factor (0 = heuristic)
int launch_gram(int n, size_t Np, const void* R, int dtype, double* T, float* gpart,
                size_t gpart_elems, hipStream_t s, int which = 3, const void* Rlo = nullptr,
                int split = 0);
// factors T + lambda I into Lf (T is left unchanged) and solves for x
// (yv: chol_vec_elems(n) elements of scratch; sync: chol_sync_words(n) words)
// lam_floor_rel > 0 (FP64 solve of a low-precision Gram): the shift used is
// max(lambda, lam_floor_rel * tr T), with MINSR_ST_SHIFT_FLOOR set in *status
// when the floor is the larger; rep_tn / rep_lam (may be null) receive tr T
// and the shift used
// lam_in (FP64 only, may be null): the shift is read from the device
// instead of `lambda` (the floor still applies).  spin_limit: polls before
// a wait between workgroups gives up (0: the built-in limit of about a
// second or more)
int launch_cholesky_solve(int n, const double* T, double* Lf, double* Dinv, int f32,
                          double lambda, const double* b, double* x, double* yv, uint32_t* sync,
                          uint32_t* status, hipStream_t s, double lam_floor_rel = 0.0,
                          double* rep_tn = nullptr, double* rep_lam = nullptr,
                          const double* lam_in = nullptr, uint32_t spin_limit = 0);
// tr T into rep_tn and 0 into rep_lam (the report of a pseudo-inverse step)
int launch_report_trace(int n, const double* T, double* rep_tn, double* rep_lam, hipStream_t s);
size_t chol_dinv_elems(int n);
size_t chol_sync_words(int n);
size_t chol_vec_elems(int n);
// x = T^+ b with eigenvalues <= cutoff * lambda_max dropped (n <= 4096);
// eig: pinv_workspace_doubles(nmax) doubles, nmax >= n
int launch_pinv_solve(int n, double* T, double cutoff, const double* b, double* x,
                      double* eig, size_t eig_elems, int nmax, uint32_t* status, hipStream_t s);
size_t pinv_workspace_doubles(int nmax);
// qgt.hip: S = R^T R over `rows` rows of R (row stride ld), N_p x N_p FP64
int launch_param_gram(const void* R, int r_f64, int rows, int Np, size_t ld, double* S,
                      hipStream_t s);
// the eigenvalues of the symmetric T in ascending order into w_out (n <= 4096,
// the pseudo-inverse workspace), and if cond is set (w_min, w_max,
// kappa_2(T + lambda I), -log10(kappa_2 eps)) into cond[0..3]
int launch_spectrum(int n, const double* T, double lambda, double eps, double* w_out,
                    double* cond, double* eig, size_t eig_elems, int nmax, uint32_t* status,
                    hipStream_t s);
int launch_update(int n, size_t Np, const void* R, int dtype, const double* x, double eta,
                  double mu, double* dpart, double* dtheta, double* momentum, double* theta,
                  uint32_t* status, int apply, hipStream_t s, const void* Rlo = nullptr,
                  uint64_t* bump = nullptr);
// adaptive.hip: report layout [0] ||T||_F [1] shift [2] ||tau|| [3] rate
// [4] e'^T tau [5] E_trial [6] rho [7] next shift
constexpr int ADAPT_FROB_PARTS = 256;
// ||T||_F and the shift of lambda mode `mode` into report[0..1]; part:
// ADAPT_FROB_PARTS doubles of scratch
int launch_adapt_lambda(int n, const void* T, int t_f32, int mode, double lambda,
                        const double* carried, double* part, double* report, hipStream_t s);
// tau, ||tau||, e'^T tau, the rate into report[2..4]; x scaled by rate / eta
int launch_tau(int n, const double* T, const double* ep, double* x, double* tau, int pinv,
               double eta, int trust, double* report, hipStream_t s);
int launch_trial_theta(double* theta, double* bak, const double* dth, size_t Np, int restore,
                       hipStream_t s);
int launch_lm(const double* E0, const double* E1, double omega, double* carried, double* report,
              hipStream_t s);
// linear.hip: the linear recurrent test model (model option MINSR_OPT_LINEAR)
size_t linear_num_params(int H);
int launch_linear_init(minsr_model* m, hipStream_t s);
// mode 0: sample (uniforms, or Philox(key, counter) if null), 1: evaluate;
// stores the states h_{i-1} and log p_i(0), log p_i(1) into the model's
// workspace for the Jacobian
int launch_linear_forward(minsr_model* m, int mode, int Ns, const double* uniforms,
                          uint64_t key, uint64_t counter, uint8_t* sigma, double* logpsi,
                          hipStream_t s);
// raw rows d log Psi / d theta / sqrt(Ns) (FP64) of the configurations the
// last forward pass evaluated
int launch_linear_jacobian(minsr_model* m, int Ns, const uint8_t* sigma, double* O,
                           hipStream_t s);

}  // namespace minsr
