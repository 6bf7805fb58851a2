// FP64 pseudo-inverse solve of the sample-space system (App. F): with
// T = V diag(w) V^T, x = sum over w_i > cutoff * max(w) of v_i (v_i^T b) / w_i.
//
//   1. Householder tridiagonalisation T = Q J Q^T in panels of TNB columns
//      (each column: update from the panel, reflector, b <- H b, and the
//      product of the trailing matrix with the reflector; a rank-2 TNB
//      update of the trailing matrix after each panel).  Reflector j is kept
//      in row j of the working copy, to the right of the diagonal.
//   2. Divide and conquer on J (Cuppen's tearing into halves down to single
//      rows; rank-one merges solved through the secular equation, with the
//      eigenvector formula of Gu and Eisenstat).  The eigenvector matrix is
//      never formed: each merge keeps its permutation, deflation rotations
//      and the K x K matrix U of its non-deflated eigenvectors, and vectors
//      are carried up (c = Z^T Q^T b) and down (y = Z t) the tree.
//   3. t = c / w on the kept eigenvalues, y = Z t, x = Q y.
// Each merge runs on one workgroup per node for the sequential parts (sort,
// deflation scan, rotations) and on one wavefront per root or column for the
// secular equations and eigenvectors.
#include "model.hpp"
#include <cmath>
#include <vector>

namespace minsr {

// panel width of the tridiagonalisation: the single-workgroup column
// kernel's dot products with the panel grow with it, the number of
// trailing rank-2 TNB updates with its inverse (8 beat 16 at n = 4096)
constexpr int TNB = 8;
constexpr int PINV_MAX_N = 4096;

// ------------------------------------------------------------ workspace
struct PinvWs {
  // tridiagonalisation
  double *A, *V, *W, *tau, *d, *e, *bq, *g, *s12, *scal, *pc, *pd;
  // divide and conquer, per depth parity (ping-pong)
  double *ev[2], *fr[2], *lr[2], *cv[2], *tv[2];
  // per-merge scratch, indexed by position in [0, n)
  double *es, *dl, *wv, *dlo, *taus, *zh, *uk, *rho, *tk;
  // per-level records (depth l at offset l * n)
  int *perm, *wpos, *rotp, *rotn, *kinfo;   // kinfo: [level][2 * slot]: K, nrot
  double *rotc, *rots;
  double* U;
};

static int depth_of(int n) {
  int D = 0;
  while ((1 << D) < n) ++D;
  return D;
}
static size_t mmax_of(int n, int lev) { return ((size_t)n + ((size_t)1 << lev) - 1) >> lev; }
static size_t u_level_elems(int n, int lev) {
  const size_t mm = mmax_of(n, lev);
  return ((size_t)1 << lev) * mm * mm;
}

size_t pinv_workspace_doubles(int nmax) {
  if (nmax <= 0) return 0;
  const size_t n = (size_t)nmax;
  const int D = depth_of(nmax) + 1;
  size_t u = 0;
  for (int l = 0; l < D; ++l) u += u_level_elems(nmax, l);
  size_t dbl = n * n + 2 * TNB * n + 7 * n + 2 * TNB + 8   // tridiagonalisation
             + 10 * n                                      // ping-pong arrays
             + 11 * n                                      // merge scratch (uk has 3 n)
             + 2 * D * n                                   // rotation coefficients
             + u;
  size_t ints = 4 * (size_t)D * n + 2 * (size_t)D * 2 * n;
  return dbl + (ints + 1) / 2 + 64;
}

static PinvWs carve(double* base, int n, int nmax) {
  PinvWs w;
  const size_t N = (size_t)nmax;
  const int D = depth_of(nmax) + 1;
  double* p = base;
  auto take = [&](size_t k) { double* r = p; p += k; return r; };
  w.A = take(N * N);
  w.V = take(TNB * N); w.W = take(TNB * N);
  w.tau = take(N); w.d = take(N); w.e = take(N); w.bq = take(N); w.g = take(N);
  w.s12 = take(2 * TNB); w.scal = take(8); w.pc = take(N); w.pd = take(N);
  for (int i = 0; i < 2; ++i) { w.ev[i] = take(N); w.fr[i] = take(N); w.lr[i] = take(N);
                                w.cv[i] = take(N); w.tv[i] = take(N); }
  w.es = take(N); w.dl = take(N); w.wv = take(N); w.dlo = take(N); w.taus = take(N);
  w.zh = take(N); w.uk = take(3 * N); w.rho = take(N); w.tk = take(N);
  w.rotc = take((size_t)D * N); w.rots = take((size_t)D * N);
  size_t u = 0;
  for (int l = 0; l < D; ++l) u += u_level_elems(nmax, l);
  w.U = take(u);
  int* q = reinterpret_cast<int*>(p);
  w.perm = q; q += (size_t)D * N;
  w.wpos = q; q += (size_t)D * N;
  w.rotp = q; q += (size_t)D * N;
  w.rotn = q; q += (size_t)D * N;
  w.kinfo = q;
  (void)n;
  return w;
}

// ------------------------------------------------------------ helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
  return v;
}
// sum over a workgroup of up to 1024 threads; every thread gets the result
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}
__device__ double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = red[0];
  for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
  return s;
}

// node `slot` of depth `lev`: halving from the root [0, n)
__device__ __host__ inline void node_of(int n, int lev, int slot, int& lo, int& m) {
  lo = 0; m = n;
  for (int b = lev - 1; b >= 0; --b) {
    const int half = m / 2;
    if ((slot >> b) & 1) { lo += half; m -= half; }
    else m = half;
  }
}

// ================================================== tridiagonalisation
struct TriArgs {
  double *A, *V, *W, *tau, *d, *e, *bq, *g, *s12, *pc, *pd;
  int n;
};

constexpr int TBS = 1024;
constexpr int TPT = PINV_MAX_N / TBS;      // rows per thread in single-workgroup kernels

// Column j at position p of its panel, one workgroup.  With the product
// g = (A - V W^T - W V^T) v_{j-1} and its partial dots g.v from the previous
// column's multi-workgroup kernel, w_{j-1} = tau g + alpha v with
// alpha = -tau^2/2 g.v is finalised elementwise; column j (whose panel terms
// up to q = p - 2 the same kernel subtracted) receives the q = p - 1 term;
// then the reflector, b <- H b, and s1 = W^T v, s2 = V^T v over q < p.
__global__ __launch_bounds__(TBS) void k_tri_col(TriArgs a, int j, int p, int npd) {
  __shared__ double red[TBS / 64];
  __shared__ double sh[4];
  __shared__ double vsh[PINV_MAX_N], wsh[PINV_MAX_N], vlsh[PINV_MAX_N];
  __shared__ double gpart[32];
  const int n = a.n, tid = threadIdx.x;
  double col[TPT], wl[TPT], vl[TPT];
  // every global operand of this thread's rows is requested up front, so
  // the kernel waits for memory once rather than once per phase
  double gl_[TPT], pc_[TPT], bq_[TPT];
  const double* vprev = a.V + (size_t)(p > 0 ? p - 1 : 0) * n;
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    const int i = j + tid + TBS * u;
    const bool ok = i < n;
    vl[u] = (ok && p > 0) ? vprev[i] : 0.0;
    gl_[u] = (ok && p > 0) ? a.g[i] : 0.0;
    pc_[u] = ok ? (p > 0 ? a.pc[i] : a.A[(size_t)j * n + i]) : 0.0;
    bq_[u] = ok ? a.bq[i] : 0.0;
  }
  if (p > 0) {
    const double tp = a.tau[j - 1];
    double sp = 0.0;
    for (int k = tid; k < npd; k += TBS) sp += a.pd[k];
    const double alpha = -0.5 * tp * tp * block_sum(sp, red);
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      const int i = j + tid + TBS * u;
      wl[u] = 0.0;
      if (i < n) {
        wl[u] = tp * gl_[u] + alpha * vl[u];
        a.W[(size_t)(p - 1) * n + i] = wl[u];
      }
    }
    if (tid == 0) { sh[1] = wl[0]; sh[2] = vl[0]; }      // row j
    __syncthreads();
    const double Wj = sh[1], Vj = sh[2];
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      const int i = j + tid + TBS * u;
      col[u] = i < n ? pc_[u] - (vl[u] * Wj + wl[u] * Vj) : 0.0;
    }
  } else {
#pragma unroll
    for (int u = 0; u < TPT; ++u) { col[u] = pc_[u]; wl[u] = 0.0; }
  }
  if (tid == 0) a.d[j] = col[0];
  if (j == n - 1) return;
  // reflector for x = col[j+1 ..]: alpha = x_0, sigma^2 = |x_1..|^2
  if (tid == 1) sh[0] = col[0];          // row j + 1 is owned by thread 1
  double ps = 0.0;
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    const int i = j + tid + TBS * u;
    if (i >= j + 2 && i < n) ps += col[u] * col[u];
  }
  const double sig2 = block_sum(ps, red);   // its barriers publish sh[0]
  const double alpha = sh[0];
  double t, beta, sc;
  if (sig2 == 0.0) { t = 0.0; beta = alpha; sc = 0.0; }
  else {
    beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
    t = (beta - alpha) / beta;
    sc = 1.0 / (alpha - beta);
  }
  if (tid == 0) { a.e[j] = beta; a.tau[j] = t; }
  double v[TPT];
  double pb = 0.0;
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    const int i = j + tid + TBS * u;
    double vi = 0.0;
    if (i == j + 1) vi = 1.0;
    else if (i > j + 1 && i < n) vi = col[u] * sc;
    v[u] = vi;
    if (i > j && i < n) {
      a.V[(size_t)p * n + i] = vi;
      a.A[(size_t)j * n + i] = vi;
      pb += vi * bq_[u];
    }
  }
  const double vb = t * block_sum(pb, red);
#pragma unroll
  for (int u = 0; u < TPT; ++u) {
    const int i = j + tid + TBS * u;
    if (i > j && i < n) a.bq[i] = bq_[u] - vb * v[u];
  }
  // s1[q] = W[q] . v, s2[q] = V[q] . v over rows > j, q < p: thread group
  // g (32 threads) owns one of the 2p values and strides over the rows, so
  // every load is coalesced within the group and each value needs a single
  // 32-lane reduction; v and the finalised column p - 1 come from LDS
  if (p > 0) {
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
      const int i = j + tid + TBS * u;
      if (i < n) { vsh[i - j] = v[u]; wsh[i - j] = wl[u]; vlsh[i - j] = vl[u]; }
    }
    __syncthreads();
    // 32 groups of 32 threads; each of the 2p values gets gpv groups that
    // split its rows; four independent accumulators keep loads in flight
    const int grp = tid >> 5, gl = tid & 31;
    const int nval = 2 * p, gpv = nval >= 32 ? 1 : 32 / nval;
    const int val = grp / gpv, sub = grp % gpv;
    double acc = 0.0;
    if (val < nval) {
      const bool isw = val < p;
      const int q = isw ? val : val - p;
      const double* colp = (isw ? a.W : a.V) + (size_t)q * n;
      const double* xs = (q == p - 1) ? (isw ? wsh : vlsh) : nullptr;
      const int stride = 32 * gpv;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int i = j + 1 + sub * 32 + gl;
      for (; i + 3 * stride < n; i += 4 * stride) {
        const double x0 = xs ? xs[i - j] : colp[i];
        const double x1 = xs ? xs[i + stride - j] : colp[i + stride];
        const double x2 = xs ? xs[i + 2 * stride - j] : colp[i + 2 * stride];
        const double x3 = xs ? xs[i + 3 * stride - j] : colp[i + 3 * stride];
        a0 = fma(x0, vsh[i - j], a0);
        a1 = fma(x1, vsh[i + stride - j], a1);
        a2 = fma(x2, vsh[i + 2 * stride - j], a2);
        a3 = fma(x3, vsh[i + 3 * stride - j], a3);
      }
      for (; i < n; i += stride) a0 = fma(xs ? xs[i - j] : colp[i], vsh[i - j], a0);
      acc = (a0 + a1) + (a2 + a3);
#pragma unroll
      for (int m = 16; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 32);
    }
    if (gl == 0) gpart[grp] = acc;
    __syncthreads();
    if (tid < nval) {
      double r = 0.0;
      for (int k = 0; k < gpv; ++k) r += gpart[tid * gpv + k];
      a.s12[tid < p ? tid : TNB + (tid - p)] = r;
    }
  }
}

// Rows i > j, one wavefront per row: g[i] = (A v)[i] - sum_{q<p} V_q[i] s1[q]
// + W_q[i] s2[q]; per-workgroup partial dots g.v; and, when the next column
// is in the same panel, its entries pc[i] = A[i][j+1] - sum_{q<p} (V_q[i]
// W_q[j+1] + W_q[i] V_q[j+1]).
__global__ __launch_bounds__(256) void k_tri_gemv(TriArgs a, int j, int p, int want_pc) {
  __shared__ double pdw[4];
  const int n = a.n, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = j + 1 + blockIdx.x * 4 + wv;
  const double* v = a.V + (size_t)p * n;
  double dot = 0.0;
  if (i < n) {
    const double* row = a.A + (size_t)i * n;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int c = j + 1 + lane;
    // sixteen loads in flight per step, then eight, four, one; element t of
    // this lane goes to accumulator t % 4 in every wide step, so the sums
    // are those of the narrower steps alone
    for (; c + 960 < n; c += 1024) {
      double r[16], x[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) { r[q] = row[c + 64 * q]; x[q] = v[c + 64 * q]; }
#pragma unroll
      for (int q = 0; q < 16; q += 4) {
        s0 = fma(r[q], x[q], s0); s1 = fma(r[q + 1], x[q + 1], s1);
        s2 = fma(r[q + 2], x[q + 2], s2); s3 = fma(r[q + 3], x[q + 3], s3);
      }
    }
    for (; c + 448 < n; c += 512) {
      double r[8], x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) { r[q] = row[c + 64 * q]; x[q] = v[c + 64 * q]; }
      s0 = fma(r[0], x[0], s0); s1 = fma(r[1], x[1], s1); s2 = fma(r[2], x[2], s2); s3 = fma(r[3], x[3], s3);
      s0 = fma(r[4], x[4], s0); s1 = fma(r[5], x[5], s1); s2 = fma(r[6], x[6], s2); s3 = fma(r[7], x[7], s3);
    }
    for (; c + 192 < n; c += 256) {
      const double r0 = row[c], r1 = row[c + 64], r2 = row[c + 128], r3 = row[c + 192];
      const double v0 = v[c], v1 = v[c + 64], v2 = v[c + 128], v3 = v[c + 192];
      s0 = fma(r0, v0, s0); s1 = fma(r1, v1, s1); s2 = fma(r2, v2, s2); s3 = fma(r3, v3, s3);
    }
    for (; c < n; c += 64) s0 = fma(row[c], v[c], s0);
    double corr = 0.0, pcc = 0.0;
    if (lane < p) {
      const double vq = a.V[(size_t)lane * n + i], wq = a.W[(size_t)lane * n + i];
      corr = vq * a.s12[lane] + wq * a.s12[TNB + lane];
      if (want_pc)
        pcc = vq * a.W[(size_t)lane * n + j + 1] + wq * a.V[(size_t)lane * n + j + 1];
    }
    const double gi = wave_sum(((s0 + s1) + (s2 + s3)) - corr);
    if (want_pc) {
      const double pcs = wave_sum(pcc);
      if (lane == 0) a.pc[i] = row[j + 1] - pcs;
    }
    if (lane == 0) a.g[i] = gi;
    dot = gi * v[i];
  }
  if (lane == 0) pdw[wv] = dot;
  __syncthreads();
  if (threadIdx.x == 0) a.pd[blockIdx.x] = (pdw[0] + pdw[1]) + (pdw[2] + pdw[3]);
}

// last column of a panel: w = tau g + alpha v over rows i > jp
__global__ __launch_bounds__(TBS) void k_tri_fin(TriArgs a, int jp, int pp, int npd) {
  __shared__ double red[TBS / 64];
  const int n = a.n, tid = threadIdx.x;
  const double tp = a.tau[jp];
  double sp = 0.0;
  for (int k = tid; k < npd; k += TBS) sp += a.pd[k];
  const double alpha = -0.5 * tp * tp * block_sum(sp, red);
  const double* v = a.V + (size_t)pp * n;
  for (int i = jp + 1 + tid; i < n; i += TBS) a.W[(size_t)pp * n + i] = tp * a.g[i] + alpha * v[i];
}

// A[i][c] -= sum_q V[q][i] W[q][c] + W[q][i] V[q][c], i, c >= j1: 64 x 64
// tiles on the FP64 matrix cores.  Wave w takes rows 16 w .. 16 w + 15 of
// the tile as four 16 x 16 blocks; the product's K index runs over the 2 TNB
// panel columns [V W] against [W V] (zero beyond nb and beyond n).  Lane l
// of v_mfma_f64_16x16x4 supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and holds D[l / 16 + 4 e][l % 16] in element e.
typedef double f64x4_e __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_tri_syr2k(double* A, const double* V, const double* W,
                                                   int n, int j1, int nb) {
  __shared__ double Vi[TNB][64], Wi[TNB][64], Vc[TNB][64], Wc[TNB][64];
  const int r0 = j1 + blockIdx.y * 64, c0 = j1 + blockIdx.x * 64, tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < TNB * 64; e += 256) {
    const int q = e / 64, k = e % 64;
    const bool okq = q < nb;
    Vi[q][k] = (okq && r0 + k < n) ? V[(size_t)q * n + r0 + k] : 0.0;
    Wi[q][k] = (okq && r0 + k < n) ? W[(size_t)q * n + r0 + k] : 0.0;
    Vc[q][k] = (okq && c0 + k < n) ? V[(size_t)q * n + c0 + k] : 0.0;
    Wc[q][k] = (okq && c0 + k < n) ? W[(size_t)q * n + c0 + k] : 0.0;
  }
  // this lane's 16 elements of the tile, requested before the barrier
  f64x4_e acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = r0 + 16 * w + (lane >> 4) + 4 * e, c = c0 + 16 * cb + (lane & 15);
      acc[cb][e] = (r < n && c < n) ? A[(size_t)r * n + c] : 0.0;
    }
  __syncthreads();
  const int i = 16 * w + (lane & 15);
#pragma unroll
  for (int ks = 0; ks < 2 * TNB; ks += 4) {
    const int k = ks + (lane >> 4);
    const double a = k < TNB ? Vi[k][i] : Wi[k - TNB][i];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int c = 16 * cb + (lane & 15);
      const double b = k < TNB ? Wc[k][c] : Vc[k - TNB][c];
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a, b, acc[cb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = r0 + 16 * w + (lane >> 4) + 4 * e, c = c0 + 16 * cb + (lane & 15);
      if (r < n && c < n) A[(size_t)r * n + c] = acc[cb][e];
    }
}

__global__ void k_pinv_copy(const double* T, double* A, size_t nn, const double* b, double* bq,
                            int n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) A[i] = T[i];
  if (i < (size_t)n) bq[i] = b[i];
}

// x = H_0 H_1 ... H_{n-2} y: reflectors applied last-first, one workgroup
__global__ __launch_bounds__(TBS) void k_tri_back(const double* A, const double* tau,
                                                  const double* y, double* x, int n) {
  __shared__ double ys[PINV_MAX_N];
  __shared__ double red[TBS / 64];
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += TBS) ys[i] = y[i];
  __syncthreads();
  for (int j = n - 2; j >= 0; --j) {
    const double t = tau[j];
    if (t == 0.0) continue;                        // uniform across the workgroup
    const double* v = A + (size_t)j * n;
    double pv = 0.0;
    for (int i = j + 1 + tid; i < n; i += TBS) pv += v[i] * ys[i];
    const double s = t * block_sum(pv, red);
    for (int i = j + 1 + tid; i < n; i += TBS) ys[i] -= s * v[i];
    __syncthreads();
  }
  for (int i = tid; i < n; i += TBS) x[i] = ys[i];
}

// ================================================== divide and conquer
struct DcArgs {
  PinvWs w;
  int n, nmax, D;
  size_t ubase;     // U offset of the level
  size_t umm;       // slot stride of U at the level (mmax^2)
  double cutoff;
  uint32_t* status;
};

// scale J to unit max norm; leaves of depth D: torn diagonal, first/last
// rows 1, right-hand side b' = Q^T b
__global__ __launch_bounds__(TBS) void k_dc_init(DcArgs a) {
  __shared__ double red[TBS / 64];
  const int n = a.n, tid = threadIdx.x;
  double mx = 0.0;
  for (int i = tid; i < n; i += TBS) {
    mx = fmax(mx, fabs(a.w.d[i]));
    if (i < n - 1) mx = fmax(mx, fabs(a.w.e[i]));
  }
  mx = block_max(mx, red);
  // a non-finite entry (NaN compares false) makes the result meaningless:
  // flag it; the later kernels stay in bounds either way
  bool bad = !(mx <= 1.7976931348623157e308);
  if (bad && tid == 0 && a.status) atomicOr(a.status, MINSR_ST_EIG_NOCONV);
  const double scale = (mx > 0.0 && !bad) ? mx : 1.0;
  const double inv = 1.0 / scale;
  const int P = a.D & 1;
  for (int i = tid; i < n; i += TBS) {
    const double ei = i < n - 1 ? a.w.e[i] * inv : 0.0;
    const double em = i > 0 ? a.w.e[i - 1] * inv : 0.0;
    a.w.es[i] = ei;
    a.w.ev[P][i] = a.w.d[i] * inv - fabs(em) - fabs(ei);
    a.w.fr[P][i] = 1.0;
    a.w.lr[P][i] = 1.0;
    a.w.cv[P][i] = a.w.bq[i];
  }
  if (tid == 0) a.w.scal[0] = scale;
}

constexpr int DCB = 1024;   // workgroup of the per-node kernels

// One workgroup per node of depth lev: gather the children's eigenvalues and
// rank-one vector, sort, deflate (small z, then close pairs by a rotation),
// record the permutation, positions and rotations, and carry the first/last
// rows and c into the node's basis up to the K x K block.
__global__ __launch_bounds__(DCB) void k_dc_prep(DcArgs a, int lev) {
  extern __shared__ double sm[];
  __shared__ double red[DCB / 64];
  __shared__ int sK, sR;
  const int n = a.n, tid = threadIdx.x, slot = blockIdx.x;
  int lo, m;
  node_of(n, lev, slot, lo, m);
  if (m == 0) return;
  const int Pc = (lev + 1) & 1, P = lev & 1;
  const PinvWs& w = a.w;
  int* kinfo = w.kinfo + (size_t)lev * 4 * a.nmax;
  if (m == 1) {
    if (tid == 0) {
      w.ev[P][lo] = w.ev[Pc][lo];
      w.fr[P][lo] = 1.0;
      w.lr[P][lo] = 1.0;
      w.cv[P][lo] = w.cv[Pc][lo];
      kinfo[2 * slot] = -1;
      kinfo[2 * slot + 1] = 0;
    }
    return;
  }
  double* sd = sm;            // [m] d, sorted
  double* sz = sm + m;        // [m] z, sorted
  double* s3 = sm + 2 * m;    // [m] scratch
  int* sidx = reinterpret_cast<int*>(sm + 3 * m);   // [m]
  const int m1 = m / 2;
  const double beta = w.es[lo + m1 - 1];
  const double rho = 2.0 * fabs(beta);
  const double sg = beta >= 0.0 ? 1.0 : -1.0;
  int* perm = w.perm + (size_t)lev * a.nmax + lo;
  int* wpos = w.wpos + (size_t)lev * a.nmax + lo;
  int* rotp = w.rotp + (size_t)lev * a.nmax + lo;
  int* rotn = w.rotn + (size_t)lev * a.nmax + lo;
  double* rotc = w.rotc + (size_t)lev * a.nmax + lo;
  double* rots = w.rots + (size_t)lev * a.nmax + lo;
  // rank sort of the children's eigenvalues (ties by index)
  for (int i = tid; i < m; i += DCB) {
    const double v = w.ev[Pc][lo + i];
    s3[i] = v == v ? v : INFINITY;     // NaN ranks as +inf, so ranks stay a permutation
  }
  __syncthreads();
  for (int i = tid; i < m; i += DCB) {
    const double di = s3[i];
    int r = 0;
    for (int k = 0; k < m; ++k) {
      const double dk = s3[k];
      r += (dk < di) || (dk == di && k < i);
    }
    sidx[r] = i;
  }
  __syncthreads();
  double mx = 0.0;
  for (int r = tid; r < m; r += DCB) {
    const int i = sidx[r];
    perm[r] = i;
    sd[r] = s3[i];
    const double zi = (i < m1 ? w.lr[Pc][lo + i] : sg * w.fr[Pc][lo + i]) * 0.70710678118654752440;
    sz[r] = zi;
    mx = fmax(mx, fmax(fabs(sd[r]), fabs(zi)));
  }
  mx = block_max(mx, red);
  const double tol = 8.0 * 2.220446049250313e-16 * mx;
  // deflation scan (sequential)
  if (tid == 0) {
    int K = 0, nd = 0, nr = 0, pj = -1;
    // deflated positions are collected from the top of wpos downwards and
    // reversed afterwards, so wpos = [non-deflated ..., deflated ...]
    for (int nj = 0; nj < m; ++nj) {
      if (rho * fabs(sz[nj]) <= tol) { wpos[m - 1 - nd] = nj; ++nd; continue; }
      if (pj < 0) { pj = nj; continue; }
      double s_ = sz[pj], c_ = sz[nj];
      const double tt = hypot(c_, s_);
      const double t = sd[nj] - sd[pj];
      c_ /= tt; s_ = -s_ / tt;
      if (fabs(t * c_ * s_) <= tol) {
        sz[nj] = tt; sz[pj] = 0.0;
        rotp[nr] = pj; rotn[nr] = nj; rotc[nr] = c_; rots[nr] = s_; ++nr;
        const double dp = sd[pj], dn = sd[nj];
        sd[pj] = dp * c_ * c_ + dn * s_ * s_;
        sd[nj] = dp * s_ * s_ + dn * c_ * c_;
        wpos[m - 1 - nd] = pj; ++nd;
        pj = nj;
      } else {
        wpos[K++] = pj;
        pj = nj;
      }
    }
    if (pj >= 0) wpos[K++] = pj;
    // deflated entries were stored in reverse scan order
    for (int a0 = K, b0 = m - 1; a0 < b0; ++a0, --b0) {
      const int t = wpos[a0]; wpos[a0] = wpos[b0]; wpos[b0] = t;
    }
    sK = K; sR = nr;
    kinfo[2 * slot] = K;
    kinfo[2 * slot + 1] = nr;
    w.rho[lo] = rho;
  }
  __syncthreads();
  const int K = sK, nr = sR;
  for (int k = tid; k < m; k += DCB) {
    const int p = wpos[k];
    if (k < K) { w.dl[lo + k] = sd[p]; w.wv[lo + k] = sz[p]; }
    else w.ev[P][lo + k] = sd[p];
  }
  // carry fr = [fr_left; 0], lr = [0; lr_right], c into working order,
  // rotate, reorder to k order; deflated parts are the node's outputs
  __syncthreads();
  for (int vsel = 0; vsel < 3; ++vsel) {
    for (int r = tid; r < m; r += DCB) {
      const int i = perm[r];
      double val;
      if (vsel == 0) val = i < m1 ? w.fr[Pc][lo + i] : 0.0;
      else if (vsel == 1) val = i >= m1 ? w.lr[Pc][lo + i] : 0.0;
      else val = w.cv[Pc][lo + i];
      s3[r] = val;
    }
    __syncthreads();
    if (tid == 0) {
      for (int t = 0; t < nr; ++t) {
        const int pa = rotp[t], pb = rotn[t];
        const double c_ = rotc[t], s_ = rots[t];
        const double wa = s3[pa], wb = s3[pb];
        s3[pa] = c_ * wa + s_ * wb;
        s3[pb] = -s_ * wa + c_ * wb;
      }
    }
    __syncthreads();
    double* outv = vsel == 0 ? w.fr[P] : (vsel == 1 ? w.lr[P] : w.cv[P]);
    for (int k = tid; k < m; k += DCB) {
      const double val = s3[wpos[k]];
      if (k < K) w.uk[(size_t)vsel * a.nmax + lo + k] = val;
      else outv[lo + k] = val;
    }
    __syncthreads();
  }
}

// Secular equation 1 + rho sum_i w_i^2 / (dl_i - lambda) = 0 for root j of
// every node at depth lev, by bisection in tau = lambda - dl_origin.  One
// wavefront per root; the node's poles and weights are staged in LDS.
constexpr int SEC_WAVES = 16;
__global__ __launch_bounds__(64 * SEC_WAVES) void k_dc_secular(DcArgs a, int lev) {
  extern __shared__ double sm[];
  const int slot = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
  int lo, m;
  node_of(a.n, lev, slot, lo, m);
  const int* kinfo = a.w.kinfo + (size_t)lev * 4 * a.nmax;
  if (m < 2) return;
  const int K = kinfo[2 * slot];
  const int j0 = blockIdx.x * SEC_WAVES;
  if (K <= 0 || j0 >= K) return;
  double* pd = sm;
  double* pw = sm + K;
  for (int i = tid; i < K; i += 64 * SEC_WAVES) {
    pd[i] = a.w.dl[lo + i];
    const double wi = a.w.wv[lo + i];
    pw[i] = wi * wi;
  }
  __syncthreads();
  const int j = j0 + (tid >> 6);
  if (j >= K) return;
  const double rho = a.w.rho[lo];
  int o;
  double tl, th;
  if (j < K - 1) {
    const double mid = 0.5 * (pd[j] + pd[j + 1]);
    double s = 0.0;
    for (int i = lane; i < K; i += 64) s += pw[i] / (pd[i] - mid);
    s = wave_sum(s);
    if (1.0 + rho * s > 0.0) { o = j; tl = 0.0; th = mid - pd[j]; }
    else { o = j + 1; tl = mid - pd[j + 1]; th = 0.0; }
  } else {
    double s = 0.0;
    for (int i = lane; i < K; i += 64) s += pw[i];
    s = wave_sum(s);
    o = j; tl = 0.0; th = rho * s;
  }
  const double dorg = pd[o];
  for (int it = 0; it < 400; ++it) {
    const double tm = 0.5 * (tl + th);
    if (tm == tl || tm == th) break;
    double s = 0.0;
    for (int i = lane; i < K; i += 64) s += pw[i] / ((pd[i] - dorg) - tm);
    s = wave_sum(s);
    if (1.0 + rho * s < 0.0) tl = tm; else th = tm;
  }
  if (lane == 0) {
    const double tau = 0.5 * (tl + th);
    a.w.dlo[lo + j] = dorg;
    a.w.taus[lo + j] = tau;
    a.w.ev[lev & 1][lo + j] = dorg + tau;
  }
}

// Gu-Eisenstat: |zhat_i|^2 = (lambda_{K-1} - d_i)/rho
//   * prod_{j<i} (lambda_j - d_i)/(d_j - d_i) * prod_{i<=j<K-1} (lambda_j - d_i)/(d_{j+1} - d_i)
__global__ __launch_bounds__(256) void k_dc_zhat(DcArgs a, int lev) {
  const int slot = blockIdx.y;
  int lo, m;
  node_of(a.n, lev, slot, lo, m);
  if (m < 2) return;
  const int K = a.w.kinfo[(size_t)lev * 4 * a.nmax + 2 * slot];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= K) return;
  const double* dl = a.w.dl + lo;
  const double* dlo = a.w.dlo + lo;
  const double* ta = a.w.taus + lo;
  const double di = dl[i];
  double prod = ((dlo[K - 1] - di) + ta[K - 1]) / a.w.rho[lo];
  for (int j = 0; j < K - 1; ++j) {
    const double num = (dlo[j] - di) + ta[j];
    const double den = (j < i ? dl[j] : dl[j + 1]) - di;
    prod *= num / den;
  }
  a.w.zh[lo + i] = copysign(sqrt(fmax(prod, 0.0)), a.w.wv[lo + i]);
}

// eigenvector columns of the non-deflated block: u_k = zhat_k / (d_k - lambda_col),
// normalised, stored column-major (K x K) in the node's U slot; the node's
// first/last rows and c follow as dot products with the carried vectors.
__global__ __launch_bounds__(256) void k_dc_ucols(DcArgs a, int lev) {
  const int slot = blockIdx.y, lane = threadIdx.x & 63;
  int lo, m;
  node_of(a.n, lev, slot, lo, m);
  if (m < 2) return;
  const int K = a.w.kinfo[(size_t)lev * 4 * a.nmax + 2 * slot];
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= K) return;
  const double* dl = a.w.dl + lo;
  const double* zh = a.w.zh + lo;
  const double dorg = a.w.dlo[lo + col], tau = a.w.taus[lo + col];
  double nn = 0.0;
  for (int k = lane; k < K; k += 64) {
    const double u = zh[k] / ((dl[k] - dorg) - tau);
    nn += u * u;
  }
  const double rn = 1.0 / sqrt(wave_sum(nn));
  double* U = a.w.U + a.ubase + (size_t)slot * a.umm + (size_t)col * K;
  const size_t N = a.nmax;
  double f = 0.0, l = 0.0, c = 0.0;
  for (int k = lane; k < K; k += 64) {
    const double u = zh[k] / ((dl[k] - dorg) - tau) * rn;
    U[k] = u;
    f += u * a.w.uk[lo + k];
    l += u * a.w.uk[N + lo + k];
    c += u * a.w.uk[2 * N + lo + k];
  }
  f = wave_sum(f); l = wave_sum(l); c = wave_sum(c);
  if (lane == 0) {
    const int P = lev & 1;
    a.w.fr[P][lo + col] = f;
    a.w.lr[P][lo + col] = l;
    a.w.cv[P][lo + col] = c;
  }
}

// root: t = c / lambda on the kept eigenvalues (lambda > cutoff * lambda_max)
__global__ __launch_bounds__(TBS) void k_dc_root(DcArgs a) {
  __shared__ double red[TBS / 64];
  const int n = a.n, tid = threadIdx.x;
  double mx = -INFINITY;
  for (int i = tid; i < n; i += TBS) mx = fmax(mx, a.w.ev[0][i]);
  mx = block_max(mx, red);
  const double scale = a.w.scal[0];
  const double thr = a.cutoff * mx;
  for (int i = tid; i < n; i += TBS) {
    const double lam = a.w.ev[0][i];
    a.w.tv[0][i] = (lam > thr && lam > 0.0) ? a.w.cv[0][i] / (lam * scale) : 0.0;
  }
}

// down the tree, node at depth lev: tk = U t (k < K), then working order,
// rotations in reverse, scatter to the children's positions
__global__ __launch_bounds__(256) void k_dc_down_gemv(DcArgs a, int lev) {
  const int slot = blockIdx.y;
  int lo, m;
  node_of(a.n, lev, slot, lo, m);
  if (m < 2) return;
  const int K = a.w.kinfo[(size_t)lev * 4 * a.nmax + 2 * slot];
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= m) return;
  const double* t = a.w.tv[lev & 1] + lo;
  double s;
  if (k < K) {
    const double* U = a.w.U + a.ubase + (size_t)slot * a.umm;
    s = 0.0;
    for (int c = 0; c < K; ++c) s = fma(U[(size_t)c * K + k], t[c], s);
  } else {
    s = t[k];
  }
  a.w.tk[lo + k] = s;
}

__global__ __launch_bounds__(DCB) void k_dc_down_post(DcArgs a, int lev) {
  extern __shared__ double sm[];
  const int slot = blockIdx.x, tid = threadIdx.x;
  int lo, m;
  node_of(a.n, lev, slot, lo, m);
  if (m == 0) return;
  const int Pn = (lev + 1) & 1;
  if (m == 1) {
    if (tid == 0) a.w.tv[Pn][lo] = a.w.tv[lev & 1][lo];
    return;
  }
  const int* kinfo = a.w.kinfo + (size_t)lev * 4 * a.nmax;
  const int nr = kinfo[2 * slot + 1];
  const int* perm = a.w.perm + (size_t)lev * a.nmax + lo;
  const int* wpos = a.w.wpos + (size_t)lev * a.nmax + lo;
  const int* rotp = a.w.rotp + (size_t)lev * a.nmax + lo;
  const int* rotn = a.w.rotn + (size_t)lev * a.nmax + lo;
  const double* rotc = a.w.rotc + (size_t)lev * a.nmax + lo;
  const double* rots = a.w.rots + (size_t)lev * a.nmax + lo;
  double* tw = sm;
  for (int k = tid; k < m; k += DCB) tw[wpos[k]] = a.w.tk[lo + k];
  __syncthreads();
  if (tid == 0) {
    for (int t = nr - 1; t >= 0; --t) {
      const int pa = rotp[t], pb = rotn[t];
      const double c_ = rotc[t], s_ = rots[t];
      const double wa = tw[pa], wb = tw[pb];
      tw[pa] = c_ * wa - s_ * wb;
      tw[pb] = s_ * wa + c_ * wb;
    }
  }
  __syncthreads();
  for (int p = tid; p < m; p += DCB) a.w.tv[Pn][lo + perm[p]] = tw[p];
}

// ================================================== driver
// steps 1 and 2 (tridiagonalisation with b carried along, then the divide
// and conquer merges up to the root), shared by the solve and the spectrum
static int pinv_forward(int n, const double* T, const double* b, const PinvWs& w, int nmax,
                        double cutoff, uint32_t* status, hipStream_t s, DcArgs& da,
                        std::vector<size_t>& ubase) {
  TriArgs ta{w.A, w.V, w.W, w.tau, w.d, w.e, w.bq, w.g, w.s12, w.pc, w.pd, n};
  const size_t nn = (size_t)n * n;
  k_pinv_copy<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(T, w.A, nn, b, w.bq, n);
  MINSR_CHECK_LAUNCH();
  // 1. tridiagonalisation
  int npd = 0;
  for (int j0 = 0; j0 < n; j0 += TNB) {
    const int nb = std::min(TNB, n - j0);
    for (int p = 0; p < nb; ++p) {
      const int j = j0 + p;
      k_tri_col<<<1, TBS, 0, s>>>(ta, j, p, npd);
      MINSR_CHECK_LAUNCH();
      if (j < n - 1) {
        npd = (n - j - 1 + 3) / 4;
        k_tri_gemv<<<(unsigned)npd, 256, 0, s>>>(ta, j, p, p + 1 < nb ? 1 : 0);
        MINSR_CHECK_LAUNCH();
      }
    }
    const int j1 = j0 + nb;
    if (j1 < n) {
      k_tri_fin<<<1, TBS, 0, s>>>(ta, j1 - 1, nb - 1, npd);
      MINSR_CHECK_LAUNCH();
      const unsigned tiles = (unsigned)((n - j1 + 63) / 64);
      k_tri_syr2k<<<dim3(tiles, tiles), 256, 0, s>>>(w.A, w.V, w.W, n, j1, nb);
      MINSR_CHECK_LAUNCH();
    }
  }
  // 2. divide and conquer, leaves at depth D
  const int D = depth_of(n);
  da = DcArgs{w, n, nmax, D, 0, 0, cutoff, status};
  k_dc_init<<<1, TBS, 0, s>>>(da);
  MINSR_CHECK_LAUNCH();
  ubase.assign(D + 1, 0);
  {
    size_t u = 0;
    for (int l = 0; l <= D; ++l) { ubase[l] = u; u += u_level_elems(n, l); }
  }
  for (int lev = D - 1; lev >= 0; --lev) {
    da.ubase = ubase[lev];
    const size_t mm = mmax_of(n, lev);
    da.umm = mm * mm;
    const unsigned nodes = 1u << lev;
    const size_t shm_prep = mm * 3 * sizeof(double) + mm * sizeof(int);
    k_dc_prep<<<nodes, DCB, shm_prep, s>>>(da, lev);
    MINSR_CHECK_LAUNCH();
    k_dc_secular<<<dim3((unsigned)((mm + SEC_WAVES - 1) / SEC_WAVES), nodes), 64 * SEC_WAVES,
                   mm * 2 * sizeof(double), s>>>(da, lev);
    MINSR_CHECK_LAUNCH();
    k_dc_zhat<<<dim3((unsigned)((mm + 255) / 256), nodes), 256, 0, s>>>(da, lev);
    MINSR_CHECK_LAUNCH();
    k_dc_ucols<<<dim3((unsigned)((mm + 3) / 4), nodes), 256, 0, s>>>(da, lev);
    MINSR_CHECK_LAUNCH();
  }
  return MINSR_OK;
}

static int pinv_check(int n, const double* eig, size_t eig_elems, int nmax) {
  if (n > PINV_MAX_N)
    return fail(MINSR_E_UNSUPPORTED, "pseudo-inverse / spectrum: n = " + std::to_string(n) +
                                         " above " + std::to_string(PINV_MAX_N));
  if (!eig || eig_elems < pinv_workspace_doubles(nmax) || n > nmax)
    return fail(MINSR_E_INVALID_ARG, "pseudo-inverse workspace missing or too small");
  return MINSR_OK;
}

// the eigenvalues at the root (unscaled), in ascending order: position of
// entry i = number of entries below it, ties broken by index
__global__ __launch_bounds__(256) void k_eig_sorted(const double* ev, const double* scal, int n,
                                                    double* w) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double v = ev[i];
  int r = 0;
  for (int j = 0; j < n; ++j) {
    const double u = ev[j];
    r += (u < v || (u == v && j < i)) ? 1 : 0;
  }
  w[r] = v * scal[0];
}

// App. E: (w_min, w_max, kappa_2(T + lambda I), d = -log10(kappa_2 eps)),
// T positive semidefinite (w_min taken as max(w_min, 0))
__global__ void k_condition(const double* w, int n, double lambda, double eps, double* cond) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double wmin = w[0], wmax = w[n - 1];
  const double den = fmax(wmin, 0.0) + lambda;
  const double k = den > 0.0 ? (wmax + lambda) / den : INFINITY;
  cond[0] = wmin;
  cond[1] = wmax;
  cond[2] = k;
  cond[3] = isfinite(k) ? -log10(k * eps) : -INFINITY;
}

int launch_spectrum(int n, const double* T, double lambda, double eps, double* w_out,
                    double* cond, double* eig, size_t eig_elems, int nmax, uint32_t* status,
                    hipStream_t s) {
  if (n == 0) return MINSR_OK;
  int rc = pinv_check(n, eig, eig_elems, nmax);
  if (rc) return rc;
  PinvWs w = carve(eig, n, nmax);
  DcArgs da{};
  std::vector<size_t> ubase;
  // the carried vector plays no part in the eigenvalues: the first row of T
  rc = pinv_forward(n, T, T, w, nmax, 0.0, status, s, da, ubase);
  if (rc) return rc;
  k_eig_sorted<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(w.ev[0], w.scal, n, w_out);
  MINSR_CHECK_LAUNCH();
  if (cond) {
    k_condition<<<1, 64, 0, s>>>(w_out, n, lambda, eps, cond);
    MINSR_CHECK_LAUNCH();
  }
  return MINSR_OK;
}

int launch_pinv_solve(int n, double* T, double cutoff, const double* b, double* x, double* eig,
                      size_t eig_elems, int nmax, uint32_t* status, hipStream_t s) {
  if (n == 0) return MINSR_OK;
  int rc = pinv_check(n, eig, eig_elems, nmax);
  if (rc) return rc;
  PinvWs w = carve(eig, n, nmax);
  DcArgs da{};
  std::vector<size_t> ubase;
  rc = pinv_forward(n, T, b, w, nmax, cutoff, status, s, da, ubase);
  if (rc) return rc;
  const int D = da.D;
  // 3. weights at the root, then down the tree
  k_dc_root<<<1, TBS, 0, s>>>(da);
  MINSR_CHECK_LAUNCH();
  for (int lev = 0; lev < D; ++lev) {
    da.ubase = ubase[lev];
    const size_t mm = mmax_of(n, lev);
    da.umm = mm * mm;
    const unsigned nodes = 1u << lev;
    k_dc_down_gemv<<<dim3((unsigned)((mm + 255) / 256), nodes), 256, 0, s>>>(da, lev);
    MINSR_CHECK_LAUNCH();
    k_dc_down_post<<<nodes, DCB, mm * sizeof(double), s>>>(da, lev);
    MINSR_CHECK_LAUNCH();
  }
  // 4. x = Q y
  k_tri_back<<<1, TBS, 0, s>>>(w.A, w.tau, w.tv[D & 1], x, n);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

}  // namespace minsr
