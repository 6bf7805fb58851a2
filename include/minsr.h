/*
 * minsr.h -- C ABI of the MI355X minimum-step stochastic reconfiguration
 * (minSR) hot path for recurrent (GRU) neural quantum states.
 *
 * The method is the one of "Quantum Geometric Tensor Preconditioning for
 * Stable Training of Recurrent Neural Quantum States": one iteration of its
 * Algorithm 1 draws N_s configurations exactly from an autoregressive GRU
 * wave function, evaluates local energies, forms the per-sample
 * log-derivatives O, centres them, builds the sample-space Gram matrix
 * T = O'^T O' and applies the regularised update
 *     dtheta = eta * O' (T + lambda I)^{-1} eps'          (Eq. minsrR)
 * followed by the momentum step of App. B.
 *
 * Conventions shared by every call
 *   - Every function returns an int status: MINSR_OK (0) or a negative
 *     MINSR_E_* code.  minsr_last_error() returns a thread-local message
 *     describing the last failure of the calling thread.
 *   - Array arguments named dev_* are device pointers owned by the caller,
 *     contiguous and row-major, with their lengths given by the other
 *     arguments.  The library never frees or retains them.
 *   - The library owns only what a model or batch handle holds: the FP64
 *     master parameters, working copies of them in the compute precision,
 *     and workspace sized at creation for max_Ns samples.
 *   - Every call takes a hipStream_t, only enqueues work on it and never
 *     synchronises the host, so calls can be captured in a hip graph.
 *     Numerical failures found on the device are reported through a status
 *     word the caller reads after its own synchronisation.
 *   - Spins are uint8 0/1 in lattice-path order; 0 is z = +1 (spin up).
 *   - Complex numbers are interleaved (re, im) doubles.
 *   - log Psi is complex: re = 0.5 log P(sigma), im = phase (Eqs. 2, 6, 8).
 *   - Identical inputs give bitwise identical outputs (no floating-point
 *     atomics anywhere).
 *   - A handle must not be used from two host threads at once, and the
 *     device work of its calls must not overlap (one stream, or streams
 *     ordered by events): the calls share the handle's workspace.
 */
#ifndef MINSR_H
#define MINSR_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MINSR_OK              0
#define MINSR_E_INVALID_ARG  -1   /* NULL pointer or out-of-range scalar  */
#define MINSR_E_SHAPE        -2   /* size outside what the handle supports */
#define MINSR_E_DEVICE       -3   /* a HIP runtime call failed             */
#define MINSR_E_NUMERIC      -4   /* reserved: host-visible numeric error  */
#define MINSR_E_NOMEM        -5   /* device allocation failed              */
#define MINSR_E_UNSUPPORTED  -6   /* option not available in this library  */

/* floating-point formats */
#define MINSR_F64   0
#define MINSR_F32   1
#define MINSR_BF16  2

/* Hamiltonians (Sec. 3): transverse-field Ising chain, periodic cluster
 * chain -sum Z X Z, and the open square-lattice J1-J2 model (J2 = 0 is the
 * Heisenberg model). */
#define MINSR_HAM_TFIM     0
#define MINSR_HAM_CLUSTER  1
#define MINSR_HAM_J1J2     2

/* numerical precision of one minSR step */
#define MINSR_FORM_FP64_REF   0  /* everything in FP64                       */
#define MINSR_FORM_BF16_FP64  1  /* O' rounded to BF16 as a hi/lo pair, Gram
                                    (hi + lo)(hi + lo)^T on BF16 MFMA (four
                                    products, FP32 accumulation flushed to
                                    FP64); FP64 reductions, solve, update   */
#define MINSR_FORM_FP32_PLAIN 2  /* FP32 O', Gram, solve and update          */
#define MINSR_FORM_BF16_1PASS 3  /* as BF16_FP64 with O' a single BF16 array
                                    (one MFMA pass; larger Gram error)       */

/* device status-word bits (minsr_step_out.dev_status).  The bits in
 * MINSR_ST_ERRORS are failures: a step that sets any of them leaves theta
 * and the momentum unchanged.  MINSR_ST_SHIFT_FLOOR only reports that a
 * BF16 form raised the shift to its floor (see minsr_step).              */
#define MINSR_ST_NONFINITE_ELOC  0x1u
#define MINSR_ST_NOT_PD          0x2u   /* Cholesky met a pivot <= 0 / NaN */
#define MINSR_ST_NONFINITE_DTH   0x4u
#define MINSR_ST_EIG_NOCONV      0x8u   /* pseudo-inverse met a non-finite
                                           tridiagonal entry                 */
#define MINSR_ST_SHIFT_FLOOR     0x10u  /* informational, not a failure      */
#define MINSR_ST_SOLVE_TIMEOUT   0x20u  /* a wait between workgroups of the
                                           Cholesky solve gave up (see the
                                           tunable "solve_spin_limit")      */
#define MINSR_ST_ERRORS          0x2Fu

/* Architecture of one wave function (Sec. 2, Sec. 2.1 and App. A).
 *   Lx, Ly        lattice extent; a chain has Ly = 1 and dim = 1
 *   dim           1: the 1D GRU; 2: the 2D GRU on the zigzag path
 *   hidden        d_h; supported: 8, 16, 32, 64, 128
 *   complex_head  1 adds the softsign phase head (cRNN), 0 is a pRNN
 *   marshall      multiply Psi by (-1)^{sigma_A}, A = {(x, y): x + y even}
 *   zero_mag      restrict the autoregressive conditionals to S^z = 0
 *   compute_dtype MINSR_F64 or MINSR_F32: precision of every GRU evaluation
 *   init_seed     Philox key of the Glorot-uniform initialisation
 *   max_Ns        largest N_s any call on this handle will use
 *   options       bit MINSR_OPT_PINV reserves the pseudo-inverse workspace
 *                 at creation (about 2.2 n^2 doubles for n = max_Ns, or
 *                 2 max_Ns for a cRNN; n <= 4096); without it the workspace
 *                 is allocated by the first pseudo-inverse call, which
 *                 therefore must not be captured into a graph.
 *                 Bit MINSR_OPT_LINEAR makes the handle the linear
 *                 recurrent test model of App. C instead of a GRU (see
 *                 below)                                                  */
typedef struct {
  int32_t Lx, Ly, dim, hidden;
  int32_t complex_head, marshall, zero_mag;
  int32_t compute_dtype;
  uint64_t init_seed;
  int32_t max_Ns;
  int32_t options;
} minsr_model_desc;
#define MINSR_OPT_PINV    0x1
/* The linear recurrent test model of App. C (Eq. linear_rnn): a real,
 * positive wave function over N = Lx sites with h_0 = 0,
 *   z_i = U h_{i-1} + c,  p_i = softmax(z_i),
 *   h_i = W h_{i-1} + V onehot(sigma_i) + b,
 *   log Psi = (1/2) sum_i log p_i[sigma_i]   (re part; im part 0),
 * theta = (W [H x H], V [H x 2], b [H], U [2 x H], c [2]) row-major in that
 * order, N_p = H^2 + 5H + 2.  It needs dim = 1, Ly = 1, no complex head,
 * Marshall sign or S^z mask, compute_dtype MINSR_F64 and hidden 8, 16, 32
 * or 64; W, V and U start Glorot-uniform as above, b and c at zero.  Its
 * exact gauge zero modes (Prop. 1) and closed-form bias element (Prop. 2)
 * make it a check of the log-derivative, centring and Gram kernels that
 * does not depend on the GRU.  Supported calls: minsr_num_params,
 * minsr_num_sites, minsr_get/set_params, minsr_sample, minsr_logpsi,
 * minsr_jacobian, minsr_param_gram, minsr_gram, minsr_solve and
 * minsr_spectrum; the others return MINSR_E_UNSUPPORTED.                  */
#define MINSR_OPT_LINEAR  0x2

typedef struct {
  int32_t kind;      /* MINSR_HAM_*                                      */
  int32_t pbc;       /* TFIM only: 1 adds the bond (N-1, 0)             */
  double J;          /* TFIM ZZ coupling; J1-J2 nearest-neighbour J1     */
  double h;          /* TFIM transverse field                            */
  double J2;         /* J1-J2 next-nearest-neighbour coupling            */
} minsr_hamiltonian;

typedef struct minsr_model minsr_model;
typedef struct minsr_batch minsr_batch;

const char* minsr_last_error(void);

/* ---- model -------------------------------------------------------------
 * Creates a wave function and initialises theta_0: every weight matrix
 * Glorot-uniform a (2u - 1), a = sqrt(6 / (fan_in + fan_out)), with u the
 * Philox4x64-10 uniform of (key = init_seed, counter = parameter index),
 * every bias zero (Sec. 2 and App. A define the cell; the paper leaves the
 * initialisation open).  The flat parameter order is, each block
 * row-major: [U1, U2 (2D only)], Wu [H x (H+ds)], bu, Wr [H x (H+ds)], br,
 * Wh [H x H], bh, Win [H x ds], bin, U [2 x H], c [2], [Uphi [2 x H],
 * cphi [2] (complex head only)], with ds = 2 (1D) or 4 (2D).
 * Allocates device memory on the current device; returns MINSR_E_NOMEM if
 * that fails.  All later calls must run with the same device current.   */
int minsr_create_model(const minsr_model_desc* desc, minsr_model** out);
int minsr_destroy_model(minsr_model* m);
int minsr_num_params(const minsr_model* m, size_t* np);
int minsr_num_sites(const minsr_model* m, int* n);
/* copy the FP64 master parameters out / in (np doubles, device)          */
int minsr_get_params(minsr_model* m, double* dev_theta, hipStream_t s);
int minsr_set_params(minsr_model* m, const double* dev_theta, hipStream_t s);

/* ---- sampling (Sec. 2, exact autoregressive sampling; Alg. 1 step 3) ---
 * Draws Ns configurations.  At path position i the conditional
 * p_i = softmax(U h_i + c) (masked to S^z = 0 if requested) gives
 * sigma_i = 0 if u < p_i(0), else 1.  u[s, i] is dev_uniforms[s * N + i]
 * (doubles in [0, 1)) or, if dev_uniforms is NULL, the uniform
 * (w >> 11) * 2^-53 of word (i mod 4) of Philox4x64-10 with
 * counter (counter, s, i / 4, 0) and key (key, 0).
 * Outputs: dev_sigma [Ns x N] uint8, dev_logpsi [Ns] complex.            */
int minsr_sample(minsr_model* m, int Ns, const double* dev_uniforms,
                 uint64_t key, uint64_t counter, uint8_t* dev_sigma,
                 double* dev_logpsi, hipStream_t s);

/* ---- evaluation: log Psi(sigma) for given configurations (Eqs. 2, 6, 8) */
int minsr_logpsi(minsr_model* m, int Ns, const uint8_t* dev_sigma,
                 double* dev_logpsi, hipStream_t s);

/* ---- local energies (Sec. 2.3) -------------------------------------------
 * eps(sigma) = sum_{sigma'} H_{sigma sigma'} Psi(sigma') / Psi(sigma) for
 * the Hamiltonian H.  dev_logpsi must hold log Psi(dev_sigma) (as returned
 * by minsr_sample / minsr_logpsi).  Outputs dev_eloc [Ns] complex and
 * dev_stats [3] = (Re E, Im E, Var eps) with E the sample mean of eps
 * (Eq. energy), all FP64.  Supported Hamiltonians: TFIM and cluster on
 * 1D models, J1-J2 on 2D models.                                         */
int minsr_local_energy(minsr_model* m, const minsr_hamiltonian* H, int Ns,
                       const uint8_t* dev_sigma, const double* dev_logpsi,
                       double* dev_eloc, double* dev_stats, hipStream_t s);

/* ---- per-sample log-derivatives (Sec. 2.3, Alg. 1 step 5) ---------------
 * Writes O[r, k] = d log Psi(sigma^(s)) / d theta_k / sqrt(Ns), computed
 * by a reverse pass through the recurrence that recomputes hidden states
 * between checkpoints taken every ckpt_every sites (1D models; 2D models
 * keep every hidden state).  Rows: a pRNN has Ns rows (r = s); a cRNN has
 * 2 Ns rows, r = s for Re (0.5 d log P) and r = Ns + s for Im (d phase).
 * centered != 0 subtracts, per block of Ns rows, the column mean, which is
 * also written to dev_colmean (rows/Ns x Np doubles, may be NULL when
 * centered == 0).  out_dtype: MINSR_F64, MINSR_F32 or MINSR_BF16 (BF16
 * only with centered != 0; centring happens in FP32/FP64 before rounding).
 * ckpt_every in [1, 16].                                                  */
int minsr_jacobian(minsr_model* m, int Ns, const uint8_t* dev_sigma,
                   int out_dtype, int centered, int ckpt_every, void* dev_O,
                   double* dev_colmean, hipStream_t s);

/* ---- vector-Jacobian product of log Psi ---------------------------------
 * dev_grad_theta[k] = sum_s (g_re[s] * d Re log Psi_s / d theta_k
 *                            + g_im[s] * d Im log Psi_s / d theta_k)
 * with dev_g [Ns] complex (g_re, g_im) interleaved.  Used as the backward
 * of a log Psi autograd function.                                         */
int minsr_logpsi_vjp(minsr_model* m, int Ns, const uint8_t* dev_sigma,
                     const double* dev_g, double* dev_grad_theta,
                     hipStream_t s);

/* ---- one minSR iteration (Alg. 1 loop body; App. B momentum) -------------
 * Samples, evaluates eps, forms O, E, eps' = 2 (Re ebar; -Im ebar) with
 * ebar_s = (eps_s - E)^* / sqrt(Ns) (Eq. real-valued), T = O'^T O', solves
 * (T + lambda I) x = eps' by Cholesky (pinv_cutoff == 0) or, at
 * lambda = 0, with the Moore-Penrose pseudo-inverse that drops eigenvalues
 * <= pinv_cutoff * lambda_max(T) (App. F), and sets
 *     dtheta = eta O' x;  m = mu m + (1 - mu) dtheta;  theta -= m.
 * theta and m change only if apply_update != 0 and no MINSR_ST_ERRORS bit
 * is set.  The uniforms are Philox (key, counter) as in minsr_sample; the
 * caller advances counter between steps.
 * The shift: the FP64 and FP32 forms factor T + lambda I with lambda as
 * given.  The BF16 forms use max(lambda, 2^-24 tr T): every entry of their
 * Gram carries FP32 accumulation error of about 2^-24 sqrt(T_ii T_jj), whose
 * spectral norm is below 2^-24 tr T, and a smaller shift can leave the
 * computed T + lambda I indefinite; MINSR_ST_SHIFT_FLOOR is set when the
 * floor is the larger.  The step reports the shift it used and the trace
 * norm of T (tr T, the nuclear norm of the positive semidefinite T) through
 * dev_lambda_used and dev_tnorm (the pseudo-inverse step reports shift 0).  */
typedef struct {
  int32_t Ns;
  int32_t form;          /* MINSR_FORM_*                                    */
  double eta, lambda, mu;
  double pinv_cutoff;    /* 0: Cholesky of T + lambda I                     */
  int32_t ckpt_every;    /* Jacobian checkpoint stride (1D models)          */
  int32_t apply_update;
} minsr_step_cfg;

typedef struct {
  double* dev_momentum;  /* [Np] FP64, caller-owned, updated in place       */
  uint64_t key, counter; /* Philox stream of the sampling uniforms          */
  uint64_t* dev_counter; /* optional [1]: if not NULL the counter is read
                            from here and incremented by one at the end of
                            the step, so a captured graph of the step can be
                            replayed with fresh uniforms each time          */
} minsr_step_state;

typedef struct {
  double* dev_energy;    /* [3]: Re E, Im E, Var eps                        */
  double* dev_dtheta;    /* [Np] FP64, may be NULL                          */
  uint32_t* dev_status;  /* [1] MINSR_ST_* bits, written every step         */
  double* dev_eloc;      /* [Ns] complex, may be NULL                       */
  uint8_t* dev_sigma;    /* [Ns x N], may be NULL                           */
  double* dev_tnorm;     /* [1] tr T (trace norm of T), may be NULL         */
  double* dev_lambda_used; /* [1] the shift the solve used, may be NULL     */
} minsr_step_out;

int minsr_step(minsr_model* m, const minsr_hamiltonian* H,
               const minsr_step_cfg* cfg, const minsr_step_state* st,
               const minsr_step_out* out, hipStream_t s);

/* ---- the regularised solve alone (Eq. minsrR; App. F) --------------------
 * Solves with the symmetric positive semi-definite FP64 matrix dev_T
 * (n x n, row-major, caller-owned, left unchanged):
 *   pinv_cutoff == 0: (T + lambda I) x = b by tiled Cholesky (lambda >= 0;
 *     only the lower triangle of T is read);
 *   pinv_cutoff > 0: x = T^+ b, the pseudo-inverse that keeps the
 *     eigenvalues > pinv_cutoff * lambda_max(T) (lambda must be 0; the full
 *     matrix is read and assumed symmetric).
 * This is the solve minsr_step runs, exposed for direct use and tests; it
 * uses the model's workspace, so n <= max_Ns (2 max_Ns for a cRNN) and the
 * call must not overlap a minsr_step on the same handle.  A pivot <= 0
 * sets MINSR_ST_NOT_PD in *dev_status (OR-ed in; the caller clears it), and
 * x is then not meaningful.                                                */
int minsr_solve(minsr_model* m, int n, const double* dev_T, double lambda,
                double pinv_cutoff, const double* dev_b, double* dev_x,
                uint32_t* dev_status, hipStream_t s);

/* ---- the parameter-space metric (Eq. SR; Prop. 3) -------------------------
 * dev_S [Np x Np] FP64, row-major, exactly symmetric: S = O' O'^T with O'
 * the centred real form of the log-derivatives of the Ns configurations
 * dev_sigma (as minsr_jacobian with centred rows: Re rows then Im rows for
 * a cRNN), i.e. S_ij = Re sum_s (O_si - mean_i)(O_sj - mean_j)^* / Ns, the
 * subsampled SR metric of the samples.  Uses the handle's workspace.        */
int minsr_param_gram(minsr_model* m, int Ns, const uint8_t* dev_sigma, double* dev_S,
                     hipStream_t s);

/* ---- the sample-space Gram matrix of one form (Alg. 1; Eq. real-valued) ---
 * dev_T [n x n] FP64, n = Ns (2 Ns for a cRNN): T = O' O'^T of the centred
 * real form O' of the log-derivatives of the configurations dev_sigma (as
 * minsr_jacobian with centred rows, scaled by 1/sqrt(Ns)), formed with the
 * arithmetic of `form` (MINSR_FORM_*): FP64 throughout; BF16 hi/lo split
 * operands on BF16 MFMA (four products, or one for MINSR_FORM_BF16_1PASS)
 * with FP32 accumulation flushed to FP64; or FP32 (MINSR_FORM_FP32_PLAIN,
 * widened to FP64 on output) -- the T a minSR step of that form solves
 * with.  FP64_REF needs an FP64 model.  Uses the handle's workspace.      */
int minsr_gram(minsr_model* m, int Ns, const uint8_t* dev_sigma, int form, double* dev_T,
               hipStream_t s);

/* ---- spectrum and conditioning of T (App. E) ------------------------------
 * The eigenvalues of the symmetric FP64 dev_T (n x n, row-major, read in
 * full and left unchanged) in ascending order into dev_w [n], from the
 * Householder tridiagonalisation and divide-and-conquer of the
 * pseudo-inverse solve.  If dev_cond [4] is not NULL it receives
 * (w_min, w_max, kappa_2(T + lambda I), d) with, for a positive
 * semidefinite T, kappa_2 = (w_max + lambda) / (max(w_min, 0) + lambda) and
 * the digit estimate d = -log10(kappa_2 eps) of App. E (eps: the machine
 * epsilon of interest, e.g. 2^-52 for FP64, 2^-23 for FP32; an infinite
 * kappa_2 gives d = -inf).  Uses the model's pseudo-inverse workspace
 * (reserved with MINSR_OPT_PINV or by the first uncaptured call), so
 * n <= min(max_Ns (2 max_Ns for a cRNN), 4096) and the call must not
 * overlap other calls on the handle.  A non-finite entry of the
 * tridiagonal form sets MINSR_ST_EIG_NOCONV in *dev_status.               */
int minsr_spectrum(minsr_model* m, int n, const double* dev_T, double lambda, double eps,
                   double* dev_w, double* dev_cond, uint32_t* dev_status, hipStream_t s);

/* ---- one minSR iteration with adaptive regularisation ---------------------
 * (Sec. 3.3; Apps. F and G.)  The iteration of minsr_step with three
 * optional changes, chosen by ad:
 *   lambda_mode  MINSR_LAMBDA_CONST: the shift is cfg->lambda, as in
 *                minsr_step.
 *                MINSR_LAMBDA_POW23: the shift is cfg->lambda * ||T||_F^(2/3)
 *                (Sec. 3.3 schedule; the paper's 2D runs take the
 *                coefficient 3e-4), ||T||_F the Frobenius norm of the
 *                step's T.
 *                MINSR_LAMBDA_LM: the shift is *ad->dev_lambda, a damping
 *                carried from step to step (cfg->lambda is not used).
 *                After the update direction dtheta is formed, Ns fresh
 *                samples of the trial parameters theta - dtheta (Philox key
 *                st->key, counter st->counter XOR 2^63) give the trial
 *                energy E_t, and App. G's ratio
 *                  rho = (E - E_t) / (eta_u e'^T tau - eta_u^2 ||tau||^2 / 2)
 *                sets *ad->dev_lambda to omega * lambda when rho < 1/4 or is
 *                not a number, lambda / omega when rho > 3/4, and leaves it
 *                otherwise.  The update itself is applied whatever rho is.
 *   trust_region 1: the rate is eta_u = cfg->eta / ||tau||_2 (App. F),
 *                tau = e' - lambda x for the Cholesky solve (lambda the
 *                shift actually used, floor included) and tau = T x for
 *                the pseudo-inverse; 0: eta_u = cfg->eta.
 * The BF16 forms keep minsr_step's shift floor.  POW23 and LM need the
 * Cholesky solve (pinv_cutoff = 0) of an FP64 form (not
 * MINSR_FORM_FP32_PLAIN), and LM a host-side counter (st->dev_counter NULL)
 * and omega > 1.  For CONST and LM, cfg->lambda must be > 0 with the
 * Cholesky solve, as in minsr_step.
 * ad->dev_report (device, 8 doubles, may be NULL): ||T||_F, the shift used,
 * ||tau||_2, eta_u, e'^T tau, E_t, rho, the next damping (the last three
 * are 0 outside LM mode).  out is filled as by minsr_step.  The call also
 * uses the handle's workspace; it is not meant for graph capture.        */
#define MINSR_LAMBDA_CONST  0
#define MINSR_LAMBDA_POW23  1
#define MINSR_LAMBDA_LM     2
typedef struct {
  int32_t lambda_mode;   /* MINSR_LAMBDA_*                                  */
  int32_t trust_region;  /* 0 or 1                                          */
  double omega;          /* LM damping factor (App. G: 3/2)                 */
  double* dev_lambda;    /* LM: [1] the carried damping, updated in place   */
  double* dev_report;    /* [8] FP64, may be NULL                           */
} minsr_adaptive_cfg;

int minsr_step_adaptive(minsr_model* m, const minsr_hamiltonian* H,
                        const minsr_step_cfg* cfg, const minsr_adaptive_cfg* ad,
                        const minsr_step_state* st, const minsr_step_out* out,
                        hipStream_t s);

/* ---- the Cholesky solve without device allocation --------------------------
 * For callers that cannot allocate device memory (code under hip graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * solve as minsr_solve with pinv_cutoff == 0, (T + lambda I) x = b with
 * lambda > 0 by tiled Cholesky (lower triangle of dev_T read, dev_T left
 * unchanged; MINSR_ST_NOT_PD OR-ed into *dev_status on a pivot <= 0), with
 * no model handle.  Its factor and solver workspace live in one static
 * device array of 9 MiB per device, which the library holds until
 * the process ends; it serves n <= 1024 (MINSR_E_SHAPE beyond).  The call
 * allocates nothing.  Its first call on a device resolves that device's
 * array address (a host-side lookup, no enqueued work): make it outside any
 * stream capture, with n == 0 if nothing is to be solved yet.  Every call on
 * one device uses the same array, so calls whose device work overlaps
 * (different streams without ordering, or host threads) race; the array
 * keeps the last call's contents and each call re-initialises what it
 * reads.  dev_T [n x n], dev_b [n], dev_x [n], dev_status [1]: device,
 * caller-owned.                                                            */
int minsr_solve_noalloc(int n, const double* dev_T, double lambda, const double* dev_b,
                        double* dev_x, uint32_t* dev_status, hipStream_t s);

/* ---- many independent instances in one graph ------------------------------
 * A batch steps `count` independent minSR instances (each its own model,
 * Hamiltonian, step configuration, state and outputs; models may differ in
 * lattice, N_s and architecture).  The first minsr_batch_step captures one
 * step of every instance into a single hip graph, each instance on its own
 * stream forked from and joined back into a library-owned origin stream, so
 * the instances' kernels run concurrently.  The Grams of the instances in
 * MINSR_FORM_BF16_FP64 run as one grouped launch between their sampling and
 * their solve (each with the split-K of its own step, so T and every output
 * equal those of single-instance steps bitwise); the first minsr_batch_step
 * copies that launch's job table to device memory the batch owns (one
 * synchronous copy, before the capture).  That call and every later one
 * launch the graph on `s` (which may be the null stream).  Every state must
 * carry a dev_counter (the Philox counter advances on the device at each
 * replay); all pointers in the descriptors must stay valid for the batch's
 * life.  The graph bakes in the launch parameters each model holds (see
 * minsr_set_tunable) at the first minsr_batch_step; later changes to them
 * do not affect the batch.  minsr_batch_step enqueues on `s` only.         */
int minsr_batch_create(minsr_model* const* models, const minsr_hamiltonian* hams,
                       const minsr_step_cfg* cfgs, const minsr_step_state* states,
                       const minsr_step_out* outs, int count, minsr_batch** out);
int minsr_batch_step(minsr_batch* b, hipStream_t s);
int minsr_batch_destroy(minsr_batch* b);

/* ---- launch parameters chosen by the autotuner ---------------------------
 * key "gram_split": split-K factor of the Gram (0 = built-in heuristic);
 * key "eloc_grid": workgroups of the persistent local-energy launch
 * (0 = one per work item up to the window limit);
 * key "sample_r": sequences per thread of the vector sampling recurrence
 * (1 or 4; FP32 1D chains with d_h = 64 or 128 and N <= 256 sample on the
 * matrix cores, which this key does not affect);
 * key "jac_parts": threads per hidden unit of the Jacobian's reverse pass
 * (1, 2 or 4; d_h = 64 and 128 only; 0 = built-in choice);
 * key "solve_spin_limit": polls after which a wait of one workgroup of the
 * Cholesky solve on another gives up (0 = built in, 2^22 polls, of the
 * order of seconds).  A wait that gives up ends every wait of the launch,
 * so the kernels exit, and sets MINSR_ST_SOLVE_TIMEOUT; the step then
 * leaves theta unchanged.  Small values exist to test that path.
 * Values are validated; MINSR_E_INVALID_ARG for an unknown key.           */
int minsr_set_tunable(minsr_model* m, const char* key, int value);
int minsr_get_tunable(const minsr_model* m, const char* key, int* value);

/* Device pointers to the step's intermediates after the last minsr_step
 * on this handle (valid until the next call on it): T (n x n FP64, or
 * FP32 in the FP32_PLAIN form), x (n), eps' (n), with n = Ns (pRNN) or
 * 2 Ns (cRNN); O' (n rows, centred; dtype per form) whose row stride is
 * returned in *Np (the parameter count rounded up to a multiple of 64,
 * zero padded).  For tests.                                              */
int minsr_step_intermediates(minsr_model* m, const void** T, const double** x,
                             const double** eps_prime, const void** Oprime,
                             int* n, int* Np);

/* ---- per-phase timing of minsr_step (profiling) -------------------------
 * minsr_timing_begin arms HIP-event recording on the step's stream for the
 * next max_steps calls of minsr_step on this handle (events are created
 * once, outside the step; do not arm it while capturing a graph).
 * minsr_timing_read waits for the recorded events and returns in ms[] the
 * milliseconds summed over the recorded steps for each phase, and in
 * *nsteps the number of steps recorded; it disarms recording.  Phases:
 *   0 sampling recurrence          5 Gram tile products (MFMA for BF16)
 *   1 local-energy recurrence      6 Gram split-K reduction and mirror
 *   2 eps sums, E, Var, eps'       7 regularised solve
 *   3 BPTT Jacobian                8 dtheta, momentum, parameter update
 *   4 centring and real form       9 working-copy repack                */
#define MINSR_NPHASES 10
int minsr_timing_begin(minsr_model* m, int max_steps);
int minsr_timing_read(minsr_model* m, double* ms, int* nsteps);

#ifdef __cplusplus
}
#endif
#endif /* MINSR_H */
