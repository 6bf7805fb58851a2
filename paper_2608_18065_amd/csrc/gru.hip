// GRU wave-function kernels: parameter initialisation and packing, the
// autoregressive recurrence in its three uses (exact sampling, evaluation
// of given configurations, and re-evaluation of Hamiltonian-connected
// configurations for local energies), and the energy reductions.
//
// The recurrence (Sec. 2, Eqs. 3-7; App. A) walks the lattice path site by
// site.  A workgroup owns B sequences; thread (g, j) owns hidden unit j of
// the R sequences of group g and computes that unit's gate
// pre-activations as a register-blocked product of the packed weights
// (streamed from L2, reused across the R sequences) with the group's
// previous hidden states (broadcast from LDS).  The output head is a
// butterfly reduction over the H units of a group.
#include "model.hpp"
#include <cmath>

namespace minsr {

template <typename T> struct VecT;
template <> struct VecT<float> { typedef float4 type; static constexpr int V = 4; };
template <> struct VecT<double> { typedef double2 type; static constexpr int V = 2; };

__device__ inline float d_exp(float x) { return expf(x); }
__device__ inline double d_exp(double x) { return exp(x); }
__device__ inline float d_tanh(float x) { return tanhf(x); }
__device__ inline double d_tanh(double x) { return tanh(x); }
__device__ inline float d_log1p(float x) { return log1pf(x); }
__device__ inline double d_log1p(double x) { return log1p(x); }
template <typename T> __device__ inline T d_sigmoid(T x) { return T(1) / (T(1) + d_exp(-x)); }

// ------------------------------------------------------------------ init
__global__ void k_init_theta(double* theta, long long Np, InitBlocks b, uint64_t seed) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Np) return;
  double a = 0.0;
  for (int i = 0; i < b.n; ++i)
    if (k >= b.off[i] && k < b.off[i] + b.size[i]) a = b.a[i];
  double v = 0.0;
  if (a != 0.0) {
    U64x4 w = philox4x64_10((uint64_t)(k >> 2), 0, 0, 1, seed, 0);
    double u = u01(w.w[k & 3]);
    double t = 2.0 * u - 1.0;  // exact: u is on the 2^-53 grid
    v = a * t;
  }
  theta[k] = v;
}

int launch_init_theta(minsr_model* m, hipStream_t s) {
  const Layout& L = m->L;
  InitBlocks b{};
  auto add = [&](size_t off, size_t rows, size_t cols, bool weight) {
    b.off[b.n] = (long long)off;
    b.size[b.n] = (long long)(rows * cols);
    b.a[b.n] = weight ? std::sqrt(6.0 / (double)(rows + cols)) : 0.0;
    b.n++;
  };
  int H = L.H, ds = L.ds;
  if (L.dim == 2) { add(L.U1, H, H, true); add(L.U2, H, H, true); }
  add(L.Wu, H, H + ds, true); add(L.Wr, H, H + ds, true); add(L.Wh, H, H, true);
  add(L.Win, H, ds, true); add(L.U, 2, H, true);
  if (L.cplx) add(L.Uphi, 2, H, true);
  return launch_init_blocks(m->theta, (long long)L.Np, b, m->d.init_seed, s);
}

int launch_init_blocks(double* theta, long long Np, const InitBlocks& b, uint64_t seed,
                       hipStream_t s) {
  k_init_theta<<<(unsigned)((Np + 255) / 256), 256, 0, s>>>(theta, Np, b, seed);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

// ------------------------------------------------------------------ pack
struct PackArgs {
  const double* th;
  int H, ds, dim, cplx, V;
  long long Wu, bu, Wr, br, Wh, bh, Win, bin, U, c, Uphi, cphi, U1, U2;
  long long o_fw, o_bw, o_f2, o_b2, o_xc, o_bias, o_head, o_headb, o_mw, o_m2, total;
  int ks, kx, nstep;   // MFMA fragments: h steps, one-hot steps, steps per wave
};

template <typename T>
__global__ void k_pack(T* out, PackArgs p) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p.total) return;
  const int H = p.H, V = p.V, ds = p.ds;
  const double* th = p.th;
  double v = 0.0;
  auto gate = [&](int q, int row, int col) -> double {  // W_q[row][col], col < H
    if (q == 0) return th[p.Wu + (long long)row * (H + ds) + col];
    if (q == 1) return th[p.Wr + (long long)row * (H + ds) + col];
    return th[p.Wh + (long long)row * H + col];
  };
  auto u12 = [&](int q, int row, int col) -> double {
    return th[(q == 0 ? p.U1 : p.U2) + (long long)row * H + col];
  };
  if (e < p.o_bw) {                       // fw [k/V][j][3][V] = W_q[j][k]
    long long r = e - p.o_fw;
    int vv = (int)(r % V); r /= V;
    int q = (int)(r % 3); r /= 3;
    int j = (int)(r % H); int k4 = (int)(r / H);
    v = gate(q, j, k4 * V + vv);
  } else if (e < p.o_f2) {                // bw [i/V][j][3][V] = W_q[i][j]
    long long r = e - p.o_bw;
    int vv = (int)(r % V); r /= V;
    int q = (int)(r % 3); r /= 3;
    int j = (int)(r % H); int i4 = (int)(r / H);
    v = gate(q, i4 * V + vv, j);
  } else if (e < p.o_b2) {                // f2 [k/V][j][2][V] = U_q[j][k]
    long long r = e - p.o_f2;
    int vv = (int)(r % V); r /= V;
    int q = (int)(r % 2); r /= 2;
    int j = (int)(r % H); int k4 = (int)(r / H);
    v = u12(q, j, k4 * V + vv);
  } else if (e < p.o_xc) {                // b2 [i/V][j][2][V] = U_q[i][j]
    long long r = e - p.o_b2;
    int vv = (int)(r % V); r /= V;
    int q = (int)(r % 2); r /= 2;
    int j = (int)(r % H); int i4 = (int)(r / H);
    v = u12(q, i4 * V + vv, j);
  } else if (e < p.o_bias) {              // xc [3][ds][H]
    long long r = e - p.o_xc;
    int j = (int)(r % H); r /= H;
    int c = (int)(r % ds); int q = (int)(r / ds);
    if (q == 0) v = th[p.Wu + (long long)j * (H + ds) + H + c];
    else if (q == 1) v = th[p.Wr + (long long)j * (H + ds) + H + c];
    else v = th[p.Win + (long long)j * ds + c];
  } else if (e < p.o_head) {              // bias [4][H]
    long long r = e - p.o_bias;
    int j = (int)(r % H); int q = (int)(r / H);
    long long base = q == 0 ? p.bu : q == 1 ? p.br : q == 2 ? p.bh : p.bin;
    v = th[base + j];
  } else if (e < p.o_headb) {             // head [4][H]: U rows, Uphi rows
    long long r = e - p.o_head;
    int j = (int)(r % H); int q = (int)(r / H);
    if (q < 2) v = th[p.U + (long long)q * H + j];
    else v = p.cplx ? th[p.Uphi + (long long)(q - 2) * H + j] : 0.0;
  } else if (e < p.o_mw) {                // headb [4]
    int q = (int)(e - p.o_headb);
    if (q < 2) v = th[p.c + q];
    else v = p.cplx ? th[p.cphi + q - 2] : 0.0;
  } else if (e < p.o_m2) {                // mw [wave][step][lane]
    long long r = e - p.o_mw;
    const int lane = (int)(r % 64); r /= 64;
    const int step = (int)(r % p.nstep); const int w = (int)(r / p.nstep);
    const int unit = 32 * w + (lane & 31), half = lane >> 5;
    const int KS = p.ks, KX = p.kx;
    // steps: u (KS + KX), r (KS + KX), g (KS), i (KX); the h part pairs
    // input k = s + half * KS, the one-hot part column c = 2 x + half
    int q, st;
    if (step < KS + KX) { q = 0; st = step; }
    else if (step < 2 * (KS + KX)) { q = 1; st = step - (KS + KX); }
    else if (step < 2 * (KS + KX) + KS) { q = 2; st = step - 2 * (KS + KX); }
    else { q = 3; st = step - 2 * (KS + KX); }
    if (q < 3 && st < KS) {
      v = gate(q, unit, st + half * KS);
    } else {
      const int c = 2 * (st - KS) + half;
      if (q == 0) v = th[p.Wu + (long long)unit * (H + ds) + H + c];
      else if (q == 1) v = th[p.Wr + (long long)unit * (H + ds) + H + c];
      else v = th[p.Win + (long long)unit * ds + c];
      // 1D: exactly one one-hot column is set at every re-evaluated site,
      // so the biases of u, r and the input term ride on these columns
      if (p.dim == 1) v += th[(q == 0 ? p.bu : q == 1 ? p.br : p.bin) + unit];
    }
    // 1D: the local-energy kernel takes exp2 of the pre-activations, so
    // u, r are scaled by -log2(e) and the candidate terms by 2 log2(e)
    if (p.dim == 1) v *= q < 2 ? -1.4426950408889634 : 2.8853900817779268;
  } else {                                // m2 [wave][s][lane]: U1 (half 0), U2 (half 1)
    long long r = e - p.o_m2;
    const int lane = (int)(r % 64); r /= 64;
    const int st = (int)(r % H); const int w = (int)(r / H);
    const int unit = 32 * w + (lane & 31), half = lane >> 5;
    v = u12(half, unit, st);
  }
  out[e] = (T)v;
}

static PackArgs pack_args(minsr_model* m) {
  const Layout& L = m->L;
  PackArgs p{};
  p.th = m->theta;
  p.H = L.H; p.ds = L.ds; p.dim = L.dim; p.cplx = L.cplx;
  p.V = m->f64 ? 2 : 4;
  p.Wu = L.Wu; p.bu = L.bu; p.Wr = L.Wr; p.br = L.br; p.Wh = L.Wh; p.bh = L.bh;
  p.Win = L.Win; p.bin = L.bin; p.U = L.U; p.c = L.c; p.Uphi = L.Uphi; p.cphi = L.cphi;
  p.U1 = L.U1; p.U2 = L.U2;
  long long H = L.H;
  p.o_fw = 0;
  p.o_bw = p.o_fw + 3 * H * H;
  p.o_f2 = p.o_bw + 3 * H * H;
  p.o_b2 = p.o_f2 + (L.dim == 2 ? 2 * H * H : 0);
  p.o_xc = p.o_b2 + (L.dim == 2 ? 2 * H * H : 0);
  p.o_bias = p.o_xc + 3 * L.ds * H;
  p.o_head = p.o_bias + 4 * H;
  p.o_headb = p.o_head + 4 * H;
  p.o_mw = p.o_headb + 4;
  const bool mf = !m->f64 && H >= 32;
  p.ks = (int)H / 2;
  p.kx = L.dim == 1 ? 1 : 2;
  p.nstep = 3 * p.ks + 3 * p.kx;
  p.o_m2 = p.o_mw + (mf ? (H / 32) * p.nstep * 64 : 0);
  p.total = p.o_m2 + (mf && L.dim == 2 ? (H / 32) * H * 64 : 0);
  return p;
}

size_t packed_elems(minsr_model* m) { return (size_t)pack_args(m).total; }

template <typename T>
static void set_work(Work<T>& w, T* base, const PackArgs& p) {
  w.fw = base + p.o_fw; w.bw = base + p.o_bw; w.f2 = base + p.o_f2; w.b2 = base + p.o_b2;
  w.xc = base + p.o_xc; w.bias = base + p.o_bias; w.head = base + p.o_head;
  w.headb = base + p.o_headb;
  w.mw = base + p.o_mw;
  w.m2 = base + p.o_m2;
}

void bind_work(minsr_model* m) {
  PackArgs p = pack_args(m);
  if (m->f64) set_work(m->wd, (double*)m->work, p);
  else set_work(m->wf, (float*)m->work, p);
}

int launch_pack(minsr_model* m, hipStream_t s) {
  PackArgs p = pack_args(m);
  unsigned grid = (unsigned)((p.total + 255) / 256);
  if (m->f64) k_pack<double><<<grid, 256, 0, s>>>((double*)m->work, p);
  else k_pack<float><<<grid, 256, 0, s>>>((float*)m->work, p);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

// --------------------------------------------------------- the recurrence
template <typename T> struct FwdArgs {
  Work<T> w;
  int N, Lx, Ns, mode, zero_mag, cplx, marshall;
  int nchunks, n_items;
  const int* nbr;
  const uint8_t* subA;
  // sampling
  const double* uniforms;
  uint64_t key, counter;
  const uint64_t* counter_ptr;   // if set, the counter is read from here
  uint32_t* zero_word;           // if set, cleared by the first thread (a step's status word)
  // configurations and outputs
  uint8_t* sigma_out;        // mode 0
  const uint8_t* sigma_in;   // modes 1, 2
  double* logpsi;            // modes 0, 1: [Ns][2]
  T* states;                 // modes 0, 1: optional [Ns][N][H]
  T* gates;                  // modes 0, 1 (1D): optional [Ns][N][4][H] u, r, g, ht
  int store_every;
  double* site;              // modes 0, 1: optional [Ns][N][4]
  // local energies (mode 2)
  const T* states_in;
  const double* site_in;
  const int* bonds;
  int n_nn, ham_kind, M;
  double hx, J1, J2;
  double* contrib;           // [M][Ns][2]
  T* ring;                   // 2D: [slots][W][H]
  int W;
};

enum { MODE_SAMPLE = 0, MODE_EVAL = 1, MODE_ELOC = 2 };

// value of the lane picked by DPP control C (quad permutations, row mirrors)
template <int C> __device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), C, 0xF, 0xF, false));
}
template <int C> __device__ inline double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), C, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), C, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int L> __device__ inline float lane_val(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), L));
}
template <int L> __device__ inline double lane_val(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), L);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), L);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int H> struct GroupReduce {
  // sum over the min(H, 64) lanes of a group inside one wavefront, every
  // lane ending with the total: inside rows of 16 lanes by DPP (neighbours,
  // pairs of neighbours, then the mirrored halves and rows, whose lanes by
  // then hold equal values), across rows from one lane of each; no step
  // goes through the LDS crossbar
  template <typename T> __device__ static T run(T v) {
    constexpr int W = H < 64 ? H : 64;
    v += dpp_mov<0xB1>(v);                      // quad_perm [1, 0, 3, 2]
    v += dpp_mov<0x4E>(v);                      // quad_perm [2, 3, 0, 1]
    if constexpr (W > 4) v += dpp_mov<0x141>(v);   // row_half_mirror
    if constexpr (W > 8) v += dpp_mov<0x140>(v);   // row_mirror
    if constexpr (W == 32) {
      const T lo = lane_val<0>(v) + lane_val<16>(v), hi = lane_val<32>(v) + lane_val<48>(v);
      v = (threadIdx.x & 32) ? hi : lo;
    } else if constexpr (W == 64) {
      v = (lane_val<0>(v) + lane_val<16>(v)) + (lane_val<32>(v) + lane_val<48>(v));
    }
    return v;
  }
};

template <typename T, int H, int DIM, int R>
__global__ __launch_bounds__(256) void k_forward(FwdArgs<T> a) {
  using VT = typename VecT<T>::type;
  constexpr int V = VecT<T>::V;
  constexpr int NT = 256;
  constexpr int NG = NT / H;
  constexpr int B = NG * R;
  constexpr int HP = H + V;          // padded row
  constexpr int NW = H > 64 ? H / 64 : 1;   // waves per group
  __shared__ __align__(16) T xin[2][B][HP];
  __shared__ __align__(16) T hh_s[DIM == 2 ? B : 1][HP];
  __shared__ __align__(16) T hv_s[DIM == 2 ? B : 1][HP];
  __shared__ T red[NT / 64][R][4];

  const int tid = threadIdx.x;
  const int g = tid / H, j = tid % H;
  const int wave = tid / 64;
  const int N = a.N;
  const Work<T> w = a.w;
  const VT* fw = reinterpret_cast<const VT*>(w.fw);
  const VT* f2 = reinterpret_cast<const VT*>(w.f2);
  const int ds = DIM == 1 ? 2 : 4;
  // FP32 1D, d_h <= 64: the thread's gate weights (3 H values of its unit)
  // stay in registers for the whole kernel, so a site costs no weight loads
  constexpr bool WR = sizeof(T) == 4 && DIM == 1 && H <= 64 && R == 1;
  VT wreg[WR ? (H / V) * 3 : 1];
  if constexpr (WR) {
#pragma unroll
    for (int i = 0; i < (H / V) * 3; ++i) wreg[i] = fw[((i / 3) * H + j) * 3 + i % 3];
  }

  // per-unit constants
  const T bu = w.bias[j], br = w.bias[H + j], bh = w.bias[2 * H + j], bi = w.bias[3 * H + j];
  // 1D: the input columns of unit j for both spin values, so the spin just
  // drawn selects a register instead of starting a load
  T xc1[3][2];
  if (DIM == 1) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int c = 0; c < 2; ++c) xc1[q][c] = w.xc[(q * 2 + c) * H + j];
  }
  const T U0 = w.head[j], U1v = w.head[H + j];
  const T P0 = w.head[2 * H + j], P1 = w.head[3 * H + j];
  const T c0 = w.headb[0], c1 = w.headb[1], cp0 = w.headb[2], cp1 = w.headb[3];
  const T PI = (T)3.14159265358979323846;
  const uint64_t ctr = a.counter_ptr ? *a.counter_ptr : a.counter;
  if (a.zero_word && blockIdx.x == 0 && threadIdx.x == 0) a.zero_word[0] = 0u;

  for (int item = blockIdx.x; item < a.n_items; item += gridDim.x) {
    const int t = a.mode == MODE_ELOC ? item / a.nchunks : 0;
    const int chunk = a.mode == MODE_ELOC ? item % a.nchunks : item;
    // term of this item (local energies): flip positions f1 < f2 (or -1)
    int f1 = -1, f2p = -1;
    double Jt = 0.0;
    if (a.mode == MODE_ELOC) {
      if (a.ham_kind == MINSR_HAM_J1J2) {
        f1 = a.bonds[2 * t]; f2p = a.bonds[2 * t + 1];
        Jt = t < a.n_nn ? a.J1 : a.J2;
      } else {
        f1 = t;
      }
    }
    const int k0 = f1;
    const int kstart = a.mode == MODE_ELOC ? k0 + 1 : 0;

    int sidx[R];
    bool act[R];
    double lp[R], ph[R], oldlp[R], oldph[R], mel[R];
    int nup[R], ndn[R], nA[R], sprev[R], dA[R];
    U64x4 rw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int b = g * R + r;
      const int s = chunk * B + b;
      act[r] = s < a.Ns;
      sidx[r] = act[r] ? s : 0;
      lp[r] = 0.0; ph[r] = 0.0; oldlp[r] = 0.0; oldph[r] = 0.0; mel[r] = 0.0;
      nup[r] = 0; ndn[r] = 0; nA[r] = 0; sprev[r] = -1; dA[r] = 0;
      rw[r].w[0] = rw[r].w[1] = rw[r].w[2] = rw[r].w[3] = 0;
    }
    // d_h >= 64, one sequence per group: lane c draws Philox block c of the
    // sequence (sites 4c .. 4c + 3) before the site loop, and site k takes
    // its word from lane k / 4, off the sequential path
    constexpr bool PRE_OK = H >= 64 && R == 1;
    const bool pre = PRE_OK && a.mode == MODE_SAMPLE && !a.uniforms && N <= 4 * 64;
    U64x4 rpre;
    rpre.w[0] = rpre.w[1] = rpre.w[2] = rpre.w[3] = 0;
    if (pre) rpre = philox4x64_10(ctr, (uint64_t)sidx[0], (uint64_t)(tid & 63), 0, a.key, 0);

    if (a.mode == MODE_ELOC) {
      // prefix statistics of the flipped configuration and the old suffix
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int s = sidx[r];
        const uint8_t* sg = a.sigma_in + (size_t)s * N;
        const double* st = a.site_in + (size_t)s * N * 4;
        for (int k = 0; k <= k0; ++k) {
          int v = sg[k];
          if (k == f1) v ^= 1;
          nup[r] += v == 0; ndn[r] += v == 1;
        }
        for (int k = k0; k < N; ++k) {
          int v = sg[k];
          oldlp[r] += st[4 * k + v];
          oldph[r] += st[4 * k + 2 + v];
        }
        const int vflip = sg[k0] ^ 1;
        lp[r] = st[4 * k0 + vflip];
        ph[r] = st[4 * k0 + 2 + vflip];
        sprev[r] = vflip;
        // matrix element of the term
        if (a.ham_kind == MINSR_HAM_TFIM) {
          mel[r] = -a.hx;
        } else if (a.ham_kind == MINSR_HAM_CLUSTER) {
          double zl = 1.0 - 2.0 * sg[(f1 - 1 + N) % N];
          double zr = 1.0 - 2.0 * sg[(f1 + 1) % N];
          mel[r] = -zl * zr;
        } else {
          mel[r] = sg[f1] != sg[f2p] ? 0.5 * Jt : 0.0;
        }
        if (a.marshall) {
          if (a.subA[f1]) dA[r] += 1 - 2 * sg[f1];
          if (f2p >= 0 && a.subA[f2p]) dA[r] += 1 - 2 * sg[f2p];
        }
      }
      if (DIM == 1 && kstart < N) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          xin[kstart & 1][g * R + r][j] = a.states_in[((size_t)sidx[r] * N + k0) * H + j];
      }
    } else if (DIM == 1) {
#pragma unroll
      for (int r = 0; r < R; ++r) xin[0][g * R + r][j] = (T)0;
    }
    __syncthreads();

    for (int k = kstart; k < N; ++k) {
      const int cb = k & 1, nb = cb ^ 1;
      T hin_own[R];
      int kh = -1, kv = -1;
      int sh[R], sv[R];
      if (DIM == 2) {
        kh = a.nbr[2 * k]; kv = a.nbr[2 * k + 1];
        // neighbour states (zero outside the lattice) and spins
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int b = g * R + r;
          const int s = sidx[r];
          const size_t slot = a.mode == MODE_ELOC ? (size_t)blockIdx.x * B + b : (size_t)s;
          auto load_state = [&](int q) -> T {
            if (q < 0) return (T)0;
            if (a.mode == MODE_ELOC && q <= k0) return a.states_in[((size_t)s * N + q) * H + j];
            return a.ring[(slot * a.W + (q % a.W)) * H + j];
          };
          // an inactive sequence (sample index clamped to 0) takes no spin
          // input: while sampling, row 0 of sigma_out may not be written yet,
          // and a byte that is not 0 or 1 must never index the input columns
          auto spin = [&](int q) -> int {
            if (q < 0 || !act[r]) return -1;
            int v = a.mode == MODE_SAMPLE ? a.sigma_out[(size_t)s * N + q]
                                          : a.sigma_in[(size_t)s * N + q];
            if (a.mode == MODE_ELOC && (q == f1 || q == f2p)) v ^= 1;
            return v;
          };
          hh_s[b][j] = load_state(kh);
          hv_s[b][j] = load_state(kv);
          sh[r] = spin(kh);
          sv[r] = spin(kv);
        }
        __syncthreads();
        // h' = U1 h_horizontal + U2 h_vertical
        T acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = (T)0;
#pragma unroll 2
        for (int k4 = 0; k4 < H / V; ++k4) {
          const VT w1 = f2[(k4 * H + j) * 2 + 0];
          const VT w2 = f2[(k4 * H + j) * 2 + 1];
          const T* w1s = reinterpret_cast<const T*>(&w1);
          const T* w2s = reinterpret_cast<const T*>(&w2);
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const VT x1 = *reinterpret_cast<const VT*>(&hh_s[g * R + r][k4 * V]);
            const VT x2 = *reinterpret_cast<const VT*>(&hv_s[g * R + r][k4 * V]);
            const T* x1s = reinterpret_cast<const T*>(&x1);
            const T* x2s = reinterpret_cast<const T*>(&x2);
#pragma unroll
            for (int v = 0; v < V; ++v) acc[r] = fma(w1s[v], x1s[v], acc[r]);
#pragma unroll
            for (int v = 0; v < V; ++v) acc[r] = fma(w2s[v], x2s[v], acc[r]);
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          hin_own[r] = acc[r];
          xin[cb][g * R + r][j] = acc[r];
        }
        __syncthreads();
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) hin_own[r] = xin[cb][g * R + r][j];
      }

      // gate pre-activations: bias and spin-input columns first
      T au[R], ar[R], ag[R], ai[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        au[r] = bu; ar[r] = br; ag[r] = bh; ai[r] = bi;
        if (DIM == 1) {
          if (sprev[r] >= 0) {
            au[r] += sprev[r] ? xc1[0][1] : xc1[0][0];
            ar[r] += sprev[r] ? xc1[1][1] : xc1[1][0];
            ai[r] += sprev[r] ? xc1[2][1] : xc1[2][0];
          }
        } else {
          if (sh[r] >= 0) {
            au[r] += w.xc[(0 * ds + sh[r]) * H + j];
            ar[r] += w.xc[(1 * ds + sh[r]) * H + j];
            ai[r] += w.xc[(2 * ds + sh[r]) * H + j];
          }
          if (sv[r] >= 0) {
            au[r] += w.xc[(0 * ds + 2 + sv[r]) * H + j];
            ar[r] += w.xc[(1 * ds + 2 + sv[r]) * H + j];
            ai[r] += w.xc[(2 * ds + 2 + sv[r]) * H + j];
          }
        }
      }
      auto gate_step = [&](int k4, const VT& wu, const VT& wr, const VT& wg) {
        const T* wus = reinterpret_cast<const T*>(&wu);
        const T* wrs = reinterpret_cast<const T*>(&wr);
        const T* wgs = reinterpret_cast<const T*>(&wg);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const VT xv = *reinterpret_cast<const VT*>(&xin[cb][g * R + r][k4 * V]);
          const T* xs = reinterpret_cast<const T*>(&xv);
#pragma unroll
          for (int v = 0; v < V; ++v) {
            au[r] = fma(wus[v], xs[v], au[r]);
            ar[r] = fma(wrs[v], xs[v], ar[r]);
            ag[r] = fma(wgs[v], xs[v], ag[r]);
          }
        }
      };
      if constexpr (WR) {
#pragma unroll
        for (int k4 = 0; k4 < H / V; ++k4)
          gate_step(k4, wreg[k4 * 3 + 0], wreg[k4 * 3 + 1], wreg[k4 * 3 + 2]);
      } else {
#pragma unroll 2
        for (int k4 = 0; k4 < H / V; ++k4)
          gate_step(k4, fw[(k4 * H + j) * 3 + 0], fw[(k4 * H + j) * 3 + 1],
                    fw[(k4 * H + j) * 3 + 2]);
      }
      T hn[R], gu[R], gr[R], gt[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        gu[r] = d_sigmoid(au[r]);
        gr[r] = d_sigmoid(ar[r]);
        gt[r] = d_tanh(gr[r] * ag[r] + ai[r]);
        hn[r] = ((T)1 - gu[r]) * hin_own[r] + gu[r] * gt[r];
      }
      // publish the new state
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int b = g * R + r;
        const int s = sidx[r];
        if (DIM == 1) xin[nb][b][j] = hn[r];
        else if (a.mode == MODE_ELOC || act[r]) {
          // sample/evaluate windows are indexed by sample: inactive lanes
          // (sample index clamped to 0) must not write
          const size_t slot = a.mode == MODE_ELOC ? (size_t)blockIdx.x * B + b : (size_t)s;
          a.ring[(slot * a.W + (k % a.W)) * H + j] = hn[r];
        }
        if (a.mode != MODE_ELOC && a.states && act[r] &&
            ((k + 1) % a.store_every == 0 || DIM == 2))
          a.states[((size_t)s * N + k) * H + j] = hn[r];
        if (DIM == 1 && a.mode != MODE_ELOC && a.gates && act[r]) {
          T* gk = a.gates + ((size_t)s * N + k) * 4 * H;
          gk[j] = gu[r]; gk[H + j] = gr[r]; gk[2 * H + j] = ag[r]; gk[3 * H + j] = gt[r];
        }
      }
      // output head: logits (and phase pre-activations) of every sequence
      T z0[R], z1[R], q0[R], q1[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        z0[r] = GroupReduce<H>::run(U0 * hn[r]);
        z1[r] = GroupReduce<H>::run(U1v * hn[r]);
        if (a.cplx) {
          q0[r] = GroupReduce<H>::run(P0 * hn[r]);
          q1[r] = GroupReduce<H>::run(P1 * hn[r]);
        } else {
          q0[r] = q1[r] = (T)0;
        }
      }
      if (NW > 1) {
        if ((tid & 63) == 0) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            red[wave][r][0] = z0[r]; red[wave][r][1] = z1[r];
            red[wave][r][2] = q0[r]; red[wave][r][3] = q1[r];
          }
        }
      }
      if constexpr (DIM == 1 && NW == 1) {
        // a group's lanes lie in one wavefront: its new state in xin only has
        // to be visible to that wavefront's next site
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else {
        __syncthreads();
      }
      if (NW > 1) {
        const int w0 = g * NW;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          T s0 = red[w0][r][0], s1 = red[w0][r][1], s2 = red[w0][r][2], s3 = red[w0][r][3];
          for (int i = 1; i < NW; ++i) {
            s0 += red[w0 + i][r][0]; s1 += red[w0 + i][r][1];
            s2 += red[w0 + i][r][2]; s3 += red[w0 + i][r][3];
          }
          z0[r] = s0; z1[r] = s1; q0[r] = s2; q1[r] = s3;
        }
        __syncthreads();   // red is rewritten at the next site
      }
      // conditional, sampling decision and accumulation
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int s = sidx[r];
        const T zz0 = z0[r] + c0, zz1 = z1[r] + c1;
        const T mx = zz0 > zz1 ? zz0 : zz1;
        const T d = zz0 > zz1 ? zz1 - zz0 : zz0 - zz1;   // -|z0 - z1|
        const T lse = mx + d_log1p(d_exp(d));
        T lp0 = zz0 - lse, lp1 = zz1 - lse;
        if (a.zero_mag) {
          const int half = N / 2;
          if (nup[r] >= half) { lp0 = -INFINITY; lp1 = (T)0; }
          else if (ndn[r] >= half) { lp0 = (T)0; lp1 = -INFINITY; }
        }
        T ph0 = (T)0, ph1 = (T)0;
        if (a.cplx) {
          const T aa0 = q0[r] + cp0, aa1 = q1[r] + cp1;
          ph0 = PI * aa0 / ((T)1 + fabs(aa0));
          ph1 = PI * aa1 / ((T)1 + fabs(aa1));
        }
        int v;
        if (a.mode == MODE_SAMPLE) {
          double u;
          if (a.uniforms) {
            u = a.uniforms[(size_t)s * N + k];
          } else if (pre) {
            const int q = k & 3;
            const uint64_t wq = q == 0 ? rpre.w[0] : q == 1 ? rpre.w[1] : q == 2 ? rpre.w[2] : rpre.w[3];
            const int lo = __builtin_amdgcn_readlane((int)(uint32_t)wq, k >> 2);
            const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(wq >> 32), k >> 2);
            u = u01(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
          } else {
            if ((k & 3) == 0)
              rw[r] = philox4x64_10(ctr, (uint64_t)s, (uint64_t)(k >> 2), 0, a.key, 0);
            u = u01(rw[r].w[k & 3]);
          }
          const double p0 = (double)d_exp(lp0);
          v = u < p0 ? 0 : 1;
          if (j == 0 && act[r]) a.sigma_out[(size_t)s * N + k] = (uint8_t)v;
        } else {
          v = a.sigma_in[(size_t)s * N + k];
          if (a.mode == MODE_ELOC && k == f2p) v ^= 1;
        }
        lp[r] += (double)(v == 0 ? lp0 : lp1);
        ph[r] += (double)(v == 0 ? ph0 : ph1);
        nup[r] += v == 0; ndn[r] += v == 1;
        if (a.marshall && a.mode != MODE_ELOC) nA[r] += a.subA[k] ? v : 0;
        sprev[r] = v;
        if (a.site && j == 0 && act[r]) {
          double* st = a.site + ((size_t)s * N + k) * 4;
          st[0] = (double)lp0; st[1] = (double)lp1; st[2] = (double)ph0; st[3] = (double)ph1;
        }
      }
      if (DIM == 2) __syncthreads();   // ring writes visible to the next site
    }

    // outputs
    if (j == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!act[r]) continue;
        const int s = sidx[r];
        if (a.mode == MODE_ELOC) {
          double dre = 0.5 * (lp[r] - oldlp[r]);
          double dim_ = (ph[r] - oldph[r]) + 3.14159265358979323846 * (double)dA[r];
          double e = mel[r] == 0.0 ? 0.0 : exp(dre);
          double* o = a.contrib + ((size_t)t * a.Ns + s) * 2;
          o[0] = mel[r] * e * cos(dim_);
          o[1] = mel[r] * e * sin(dim_);
        } else {
          a.logpsi[2 * s] = 0.5 * lp[r];
          a.logpsi[2 * s + 1] = ph[r] + 3.14159265358979323846 * (double)nA[r];
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int H, int DIM, int R>
static int launch_fwd_t(const FwdArgs<T>& a, unsigned grid, hipStream_t s) {
  k_forward<T, H, DIM, R><<<grid, 256, 0, s>>>(a);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

template <typename T, int DIM, int R>
static int dispatch_h(int H, const FwdArgs<T>& a, unsigned grid, hipStream_t s) {
  switch (H) {
    case 8: return launch_fwd_t<T, 8, DIM, R>(a, grid, s);
    case 16: return launch_fwd_t<T, 16, DIM, R>(a, grid, s);
    case 32: return launch_fwd_t<T, 32, DIM, R>(a, grid, s);
    case 64: return launch_fwd_t<T, 64, DIM, R>(a, grid, s);
    case 128: return launch_fwd_t<T, 128, DIM, R>(a, grid, s);
  }
  return fail(MINSR_E_UNSUPPORTED, "hidden width must be 8, 16, 32, 64 or 128");
}

template <typename T, int R>
static int dispatch_dim(minsr_model* m, const FwdArgs<T>& a, unsigned grid, hipStream_t s) {
  if (m->dim == 1) return dispatch_h<T, 1, R>(m->H, a, grid, s);
  return dispatch_h<T, 2, R>(m->H, a, grid, s);
}

template <typename T>
static FwdArgs<T> base_args(minsr_model* m, const Work<T>& w) {
  FwdArgs<T> a{};
  a.w = w;
  a.N = m->N; a.Lx = m->d.Lx;
  a.zero_mag = m->d.zero_mag; a.cplx = m->cplx; a.marshall = m->d.marshall;
  a.nbr = m->nbr; a.subA = m->subA;
  a.ring = (T*)m->ring; a.W = 2 * m->d.Lx;
  a.store_every = 1;
  return a;
}

static int seqs_per_block(int H, int R) { return (256 / H) * R; }

template <typename T>
static int forward_t(minsr_model* m, const Work<T>& w, int mode, int Ns, const double* uniforms,
                     uint64_t key, uint64_t counter, const uint64_t* counter_ptr, uint8_t* sigma,
                     double* logpsi, void* states, int store_every, double* site, void* gates,
                     hipStream_t s, uint32_t* zero_word) {
  FwdArgs<T> a = base_args<T>(m, w);
  a.zero_word = zero_word;
  a.Ns = Ns; a.mode = mode;
  a.uniforms = uniforms; a.key = key; a.counter = counter; a.counter_ptr = counter_ptr;
  if (mode == MODE_SAMPLE) a.sigma_out = sigma; else a.sigma_in = sigma;
  a.logpsi = logpsi;
  a.states = (T*)states; a.store_every = store_every; a.site = site;
  a.gates = (m->dim == 1 && store_every == 1 && mode != MODE_ELOC) ? (T*)gates : nullptr;
  // few sequences per block by default: the site loop is latency-bound
  const int R = m->tune_sample_r == 4 ? 4 : 1;
  const int B = seqs_per_block(m->H, R);
  a.nchunks = (Ns + B - 1) / B;
  a.n_items = a.nchunks;
  if (R == 4) return dispatch_dim<T, 4>(m, a, (unsigned)a.n_items, s);
  return dispatch_dim<T, 1>(m, a, (unsigned)a.n_items, s);
}

int launch_forward(minsr_model* m, int mode, int Ns, const double* uniforms, uint64_t key,
                   uint64_t counter, uint8_t* sigma, double* logpsi, void* states,
                   int store_every, double* site, hipStream_t s, const uint64_t* counter_ptr,
                   void* gates, uint32_t* zero_word) {
  if (Ns == 0) return MINSR_OK;
  // FP32 chains of 64 or 128 units sample on the matrix cores; evaluation
  // keeps the vector recurrence, whose arithmetic the Jacobian's checkpoint
  // recomputation repeats exactly
  if (mode == MODE_SAMPLE && sample_mfma_supported(m))
    return launch_sample_mfma(m, Ns, uniforms, key, counter, counter_ptr, sigma, logpsi, states,
                              store_every, site, m->dim == 1 ? gates : nullptr, zero_word, s);
  if (m->f64)
    return forward_t<double>(m, m->wd, mode, Ns, uniforms, key, counter, counter_ptr, sigma,
                             logpsi, states, store_every, site, gates, s, zero_word);
  return forward_t<float>(m, m->wf, mode, Ns, uniforms, key, counter, counter_ptr, sigma, logpsi,
                          states, store_every, site, gates, s, zero_word);
}

// ------------------------------------------------------ local energies
// diagonal part and the sum over off-diagonal terms (fixed term order)
struct DiagArgs {
  const uint8_t* sigma;
  const double* contrib;
  double* eloc;
  const int* bonds;
  int n_nn, n_nnn, N, Ns, M, kind, pbc;
  double J, J2;
};

// one wavefront per sample: lanes take bonds and terms in strides of 64,
// then a fixed butterfly sums them
__global__ __launch_bounds__(256) void k_eloc_sum(DiagArgs a) {
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (s >= a.Ns) return;   // uniform per wavefront
  const uint8_t* sg = a.sigma + (size_t)s * a.N;
  double d = 0.0;
  if (a.kind == MINSR_HAM_TFIM) {
    const int nbond = (a.pbc && a.N > 2) ? a.N : a.N - 1;
    for (int i = lane; i < nbond; i += 64) {
      const int j = i + 1 < a.N ? i + 1 : 0;
      d += -a.J * ((1.0 - 2.0 * sg[i]) * (1.0 - 2.0 * sg[j]));
    }
  } else if (a.kind == MINSR_HAM_J1J2) {
    for (int b = lane; b < a.n_nn + a.n_nnn; b += 64) {
      const double Jb = b < a.n_nn ? a.J : a.J2;
      const int p = a.bonds[2 * b], q = a.bonds[2 * b + 1];
      d += 0.25 * Jb * (1.0 - 2.0 * sg[p]) * (1.0 - 2.0 * sg[q]);
    }
  }
  double re = d, im = 0.0;
  for (int t = lane; t < a.M; t += 64) {
    const double* c = a.contrib + ((size_t)t * a.Ns + s) * 2;
    re += c[0];
    im += c[1];
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    re += __shfl_xor(re, m, 64);
    im += __shfl_xor(im, m, 64);
  }
  if (lane == 0) {
    a.eloc[2 * s] = re;
    a.eloc[2 * s + 1] = im;
  }
}

template <typename T>
static int eloc_t(minsr_model* m, const Work<T>& w, const minsr_hamiltonian* H, int Ns,
                  const uint8_t* sigma, const void* states, const double* site, double* eloc,
                  hipStream_t s, int which) {
  FwdArgs<T> a = base_args<T>(m, w);
  a.Ns = Ns; a.mode = MODE_ELOC;
  a.sigma_in = sigma;
  a.states_in = (const T*)states; a.site_in = site;
  a.bonds = m->bonds; a.n_nn = m->n_nn;
  a.ham_kind = H->kind;
  a.hx = H->h; a.J1 = H->J; a.J2 = H->J2;
  int M = 0;
  if (H->kind == MINSR_HAM_J1J2) M = m->n_nn + (H->J2 != 0.0 ? m->n_nnn : 0);
  else M = m->N;
  a.M = M;
  a.contrib = m->contrib;
  const int R = 4;
  const int B = seqs_per_block(m->H, R);
  a.nchunks = (Ns + B - 1) / B;
  a.n_items = a.nchunks * M;
  unsigned grid = (unsigned)a.n_items;
  if (m->tune_eloc_grid > 0) grid = std::min<unsigned>(grid, (unsigned)m->tune_eloc_grid);
  if (m->dim == 2) {
    // the recompute windows are indexed by block: a persistent grid
    int cap = m->ring_blocks / B;
    if (cap < 1) return fail(MINSR_E_SHAPE, "recompute window too small");
    if ((int)grid > cap) grid = (unsigned)cap;
  }
  if (a.n_items > 0 && (which & 1)) {
    int rc;
    if (!m->f64 && !m->force_vector && eloc_mfma_supported(m))
      rc = launch_eloc_mfma(m, H, Ns, sigma, states, site, M, s);
    else
      rc = dispatch_dim<T, 4>(m, a, grid, s);
    if (rc) return rc;
  }
  if (!(which & 2)) return MINSR_OK;
  DiagArgs d{};
  d.sigma = sigma; d.contrib = m->contrib; d.eloc = eloc; d.bonds = m->bonds;
  d.n_nn = m->n_nn; d.n_nnn = m->n_nnn; d.N = m->N; d.Ns = Ns; d.M = M; d.kind = H->kind;
  d.pbc = H->pbc; d.J = H->J; d.J2 = H->J2;
  k_eloc_sum<<<(Ns + 3) / 4, 256, 0, s>>>(d);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int launch_eloc(minsr_model* m, const minsr_hamiltonian* H, int Ns, const uint8_t* sigma,
                const double* logpsi, const void* states, const double* site, double* eloc,
                hipStream_t s, int which) {
  (void)logpsi;
  if (Ns == 0) return MINSR_OK;
  if (m->f64) return eloc_t<double>(m, m->wd, H, Ns, sigma, states, site, eloc, s, which);
  return eloc_t<float>(m, m->wf, H, Ns, sigma, states, site, eloc, s, which);
}

// ------------------------------------------------------------ statistics
// E = mean eps, Var = mean |eps - E|^2 (Eq. energy), and optionally
// eps' = 2 (Re(eps - E); Im(eps - E)) / sqrt(Ns) (Eq. real-valued), in a
// fixed-order single-workgroup reduction.
__global__ __launch_bounds__(1024) void k_stats(const double* eloc, int Ns, int cplx,
                                                double* stats, double* epsp, uint32_t* status) {
  __shared__ double sr[1024], si[1024];
  const int t = threadIdx.x;
  double re = 0.0, im = 0.0;
  for (int s = t; s < Ns; s += 1024) { re += eloc[2 * s]; im += eloc[2 * s + 1]; }
  sr[t] = re; si[t] = im;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (t < w) { sr[t] += sr[t + w]; si[t] += si[t + w]; }
    __syncthreads();
  }
  const double Er = sr[0] / Ns, Ei = si[0] / Ns;
  __syncthreads();
  double v = 0.0;
  bool finite = true;
  for (int s = t; s < Ns; s += 1024) {
    double dr = eloc[2 * s] - Er, di = eloc[2 * s + 1] - Ei;
    v += dr * dr + di * di;
    if (!isfinite(eloc[2 * s]) || !isfinite(eloc[2 * s + 1])) finite = false;
    if (epsp) {
      const double sc = 2.0 / sqrt((double)Ns);
      epsp[s] = sc * dr;
      if (cplx) epsp[Ns + s] = sc * di;
    }
  }
  sr[t] = v;
  si[t] = finite ? 0.0 : 1.0;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if (t < w) { sr[t] += sr[t + w]; si[t] += si[t + w]; }
    __syncthreads();
  }
  if (t == 0) {
    stats[0] = Er; stats[1] = Ei; stats[2] = sr[0] / Ns;
    if (status && si[0] != 0.0) status[0] |= MINSR_ST_NONFINITE_ELOC;
  }
}

int launch_stats(minsr_model* m, int Ns, const double* eloc, double* stats, double* epsp,
                 uint32_t* status, hipStream_t s) {
  if (Ns == 0) return MINSR_OK;
  k_stats<<<1, 1024, 0, s>>>(eloc, Ns, m->cplx, stats, epsp, status);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

}  // namespace minsr
