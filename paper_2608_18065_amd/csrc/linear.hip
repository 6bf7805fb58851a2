// The linear recurrent test model of App. C (Eq. linear_rnn): a real,
// positive autoregressive wave function over N sites with
//   h_0 = 0,  z_i = U h_{i-1} + c,  p_i = softmax(z_i),
//   h_i = W h_{i-1} + V onehot(sigma_i) + b,
//   log Psi = (1/2) sum_i log p_i[sigma_i]
// and theta = (W [H x H], V [H x 2], b [H], U [2 x H], c [2]) row-major in
// that order.  It has no local energies: it exists so that the Jacobian,
// centring and Gram kernels can be checked against properties the paper
// proves for it (the exact gauge zero modes of Prop. 1 and the closed-form
// bias element of Prop. 2), independently of the GRU.
//
// FP64 throughout.  One wavefront per configuration, lane j = hidden unit
// j (d_h <= 64); the recurrent matrix is staged in shared memory once per
// workgroup (transposed for the forward pass, so that each step reads a
// row of the staged matrix across the lanes).  Every sum runs in a fixed
// order, so outputs are bitwise reproducible.
#include "model.hpp"

namespace minsr {

constexpr int LIN_WAVES = 4;

struct LinArgs {
  const double* th;
  int N, Ns;
  const double* uniforms;   // [Ns][N] or null (then Philox(key, counter))
  uint64_t key, counter;
  uint8_t* sigma;           // sampled (mode 0) or read (mode 1)
  double* logpsi;           // [Ns][2]
  double* states;           // [Ns][N][H]: h_{i-1}, the state feeding site i
  double* site;             // [Ns][N][4]: log p_i(0), log p_i(1), 0, 0
};

__device__ inline double lin_softplus(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

template <int H>
__global__ __launch_bounds__(64 * LIN_WAVES) void k_lin_forward(LinArgs a, int mode) {
  __shared__ double Wt[H][H];              // Wt[k][j] = W[j][k]
  __shared__ double hb[LIN_WAVES][2][H];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const double* W = a.th;
  const double* V = W + H * H;
  const double* b = V + 2 * H;
  const double* U = b + H;
  const double* c = U + 2 * H;
  for (int e = tid; e < H * H; e += 64 * LIN_WAVES) Wt[e % H][e / H] = W[e];
  __syncthreads();
  const int s = blockIdx.x * LIN_WAVES + w;
  if (s >= a.Ns) return;
  const int N = a.N;
  const bool act = lane < H;
  const double u0 = act ? U[lane] : 0.0, u1 = act ? U[H + lane] : 0.0;
  const double v0 = act ? V[2 * lane] : 0.0, v1 = act ? V[2 * lane + 1] : 0.0;
  const double bj = act ? b[lane] : 0.0;
  const double c0 = c[0], c1 = c[1];
  double h = 0.0, lp = 0.0;
  U64x4 rw{};
  for (int i = 0; i < N; ++i) {
    const double z0 = wave_sum(u0 * h) + c0;
    const double z1 = wave_sum(u1 * h) + c1;
    const double l0 = -lin_softplus(z1 - z0), l1 = -lin_softplus(z0 - z1);
    int sg;
    if (mode == 0) {
      double u;
      if (a.uniforms) {
        u = a.uniforms[(size_t)s * N + i];
      } else {
        if ((i & 3) == 0) rw = philox4x64_10(a.counter, (uint64_t)s, (uint64_t)(i >> 2), 0, a.key, 0);
        u = u01(rw.w[i & 3]);
      }
      sg = u < exp(l0) ? 0 : 1;
      if (lane == 0) a.sigma[(size_t)s * N + i] = (uint8_t)sg;
    } else {
      sg = a.sigma[(size_t)s * N + i];
    }
    lp += sg ? l1 : l0;
    if (a.states && act) a.states[((size_t)s * N + i) * H + lane] = h;
    if (a.site && lane < 4)
      a.site[((size_t)s * N + i) * 4 + lane] = lane == 0 ? l0 : lane == 1 ? l1 : 0.0;
    // h_i = W h_{i-1} + V e_sigma + b (terms in order of k)
    double* hv = hb[w][i & 1];
    if (act) hv[lane] = h;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (act) {
      double acc = 0.0;
#pragma unroll 8
      for (int k = 0; k < H; ++k) acc = fma(Wt[k][lane], hv[k], acc);
      h = acc + (sg ? v1 : v0) + bj;
    }
  }
  if (lane == 0) {
    a.logpsi[2 * (size_t)s] = 0.5 * lp;
    a.logpsi[2 * (size_t)s + 1] = 0.0;
  }
}

// Reverse accumulation of O = d log Psi / d theta for the configurations
// whose states and conditionals the forward pass stored.  With g_i =
// (e_sigma_i - p_i) / 2 (the softmax score of Eq. softmax_score with the
// 1/2 of log Psi) and a_i the adjoint of h_i (a_N = 0), site i adds
// a_i h_{i-1}^T to dW, a_i to column sigma_i of dV and to db, g_i h_{i-1}^T
// to dU and g_i to dc, and a_{i-1} = W^T a_i + U^T g_i.  Rows are written
// scaled by 1/sqrt(Ns).
template <int H>
__global__ __launch_bounds__(64 * LIN_WAVES) void k_lin_jacobian(LinArgs a, double* O, int Np,
                                                                 double scale) {
  __shared__ double Ws[H][H];              // W row-major
  __shared__ double hbuf[LIN_WAVES][H];
  __shared__ double abuf[LIN_WAVES][2][H];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const double* W = a.th;
  const double* U = W + H * H + 2 * H + H;
  for (int e = tid; e < H * H; e += 64 * LIN_WAVES) Ws[e / H][e % H] = W[e];
  __syncthreads();
  const int s = blockIdx.x * LIN_WAVES + w;
  if (s >= a.Ns) return;
  const int N = a.N;
  const bool act = lane < H;
  const double u0 = act ? U[lane] : 0.0, u1 = act ? U[H + lane] : 0.0;
  double dW[H];
#pragma unroll
  for (int t = 0; t < H; ++t) dW[t] = 0.0;
  double dV0 = 0.0, dV1 = 0.0, db = 0.0, dU0 = 0.0, dU1 = 0.0, dc0 = 0.0, dc1 = 0.0;
  double aj = 0.0;   // adjoint of h_N
  auto wave_sync = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  for (int i = N - 1; i >= 0; --i) {
    const size_t si = (size_t)s * N + i;
    const double hp = act ? a.states[si * H + lane] : 0.0;
    const int sg = a.sigma[si];
    const double p0 = exp(a.site[si * 4]), p1 = exp(a.site[si * 4 + 1]);
    const double g0 = 0.5 * ((sg == 0 ? 1.0 : 0.0) - p0);
    const double g1 = 0.5 * ((sg == 1 ? 1.0 : 0.0) - p1);
    if (act) hbuf[w][lane] = hp;
    double* av = abuf[w][i & 1];
    if (act) av[lane] = aj;
    wave_sync();
    // h_i = W h_{i-1} + V e + b
#pragma unroll
    for (int t = 0; t < H; ++t) dW[t] = fma(aj, hbuf[w][t], dW[t]);
    if (sg) dV1 += aj; else dV0 += aj;
    db += aj;
    // z_i = U h_{i-1} + c
    dU0 = fma(g0, hp, dU0);
    dU1 = fma(g1, hp, dU1);
    dc0 += g0;
    dc1 += g1;
    // a_{i-1} = W^T a_i + U^T g_i (terms in order of r)
    if (act) {
      double acc = 0.0;
#pragma unroll 8
      for (int r = 0; r < H; ++r) acc = fma(Ws[r][lane], av[r], acc);
      aj = acc + fma(u0, g0, u1 * g1);
    }
    wave_sync();   // hbuf is rewritten next
  }
  if (!act) return;
  double* row = O + (size_t)s * Np;
  const int j = lane;
#pragma unroll
  for (int t = 0; t < H; ++t) row[j * H + t] = dW[t] * scale;
  row[H * H + 2 * j] = dV0 * scale;
  row[H * H + 2 * j + 1] = dV1 * scale;
  row[H * H + 2 * H + j] = db * scale;
  row[H * H + 3 * H + j] = dU0 * scale;
  row[H * H + 4 * H + j] = dU1 * scale;
  if (j == 0) {
    row[H * H + 5 * H] = dc0 * scale;
    row[H * H + 5 * H + 1] = dc1 * scale;
  }
}

size_t linear_num_params(int H) { return (size_t)H * H + 5 * (size_t)H + 2; }

template <int H>
static void lin_fwd_launch(const LinArgs& a, int mode, hipStream_t s) {
  const unsigned grid = (unsigned)((a.Ns + LIN_WAVES - 1) / LIN_WAVES);
  k_lin_forward<H><<<grid, 64 * LIN_WAVES, 0, s>>>(a, mode);
}

template <int H>
static void lin_jac_launch(const LinArgs& a, double* O, int Np, double scale, hipStream_t s) {
  const unsigned grid = (unsigned)((a.Ns + LIN_WAVES - 1) / LIN_WAVES);
  k_lin_jacobian<H><<<grid, 64 * LIN_WAVES, 0, s>>>(a, O, Np, scale);
}

int launch_linear_forward(minsr_model* m, int mode, int Ns, const double* uniforms,
                          uint64_t key, uint64_t counter, uint8_t* sigma, double* logpsi,
                          hipStream_t s) {
  if (Ns == 0) return MINSR_OK;
  LinArgs a{m->theta, m->N, Ns, uniforms, key, counter, sigma, logpsi,
            (double*)m->states, m->site};
  switch (m->H) {
    case 8: lin_fwd_launch<8>(a, mode, s); break;
    case 16: lin_fwd_launch<16>(a, mode, s); break;
    case 32: lin_fwd_launch<32>(a, mode, s); break;
    case 64: lin_fwd_launch<64>(a, mode, s); break;
    default: return fail(MINSR_E_UNSUPPORTED, "linear model: hidden width 8, 16, 32 or 64");
  }
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int launch_linear_jacobian(minsr_model* m, int Ns, const uint8_t* sigma, double* O,
                           hipStream_t s) {
  if (Ns == 0) return MINSR_OK;
  LinArgs a{m->theta, m->N, Ns, nullptr, 0, 0, const_cast<uint8_t*>(sigma), nullptr,
            (double*)m->states, m->site};
  const int Np = (int)linear_num_params(m->H);
  const double scale = 1.0 / std::sqrt((double)Ns);
  switch (m->H) {
    case 8: lin_jac_launch<8>(a, O, Np, scale, s); break;
    case 16: lin_jac_launch<16>(a, O, Np, scale, s); break;
    case 32: lin_jac_launch<32>(a, O, Np, scale, s); break;
    case 64: lin_jac_launch<64>(a, O, Np, scale, s); break;
    default: return fail(MINSR_E_UNSUPPORTED, "linear model: hidden width 8, 16, 32 or 64");
  }
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

// Glorot-uniform W, V, U from the model's Philox key (the scheme of the GRU
// models), zero biases
int launch_linear_init(minsr_model* m, hipStream_t s) {
  const long long H = m->H;
  InitBlocks b{};
  auto add = [&](long long off, long long rows, long long cols, bool weight) {
    b.off[b.n] = off;
    b.size[b.n] = rows * cols;
    b.a[b.n] = weight ? std::sqrt(6.0 / (double)(rows + cols)) : 0.0;
    b.n++;
  };
  add(0, H, H, true);                    // W
  add(H * H, H, 2, true);                // V
  add(H * H + 3 * H, 2, H, true);        // U
  return launch_init_blocks(m->theta, (long long)linear_num_params(m->H), b, m->d.init_seed, s);
}

}  // namespace minsr
