// Per-sample log-derivatives d log Psi(sigma^(s)) / d theta (Sec. 2.3,
// Alg. 1 step 5) by a hand-written reverse pass through the GRU of App. A.
//
// One workgroup owns SG samples.  Threads (p, j) of a sample own hidden
// unit j; the P "parts" p split the columns of the weight gradients and
// the rows of the reverse matrix-vector products, so every thread keeps
// its share of the sample's gradient (3 H/P values per gate matrix row j,
// plus U1/U2 in 2D) in registers for the whole pass and writes it once.
//
// 1D: hidden states are checkpointed every C sites; each segment is
// recomputed forward (with the same arithmetic as the sampling kernel, so
// any C gives bitwise identical rows) into an LDS tape and then reversed.
// With C = 1 and the sampler's gate tape the forward products are skipped:
// the gate values are read back instead of recomputed (same values).
// 2D: every hidden state is stored; the reverse pass recomputes one site
// at a time from its two predecessors and keeps the adjoints of the last
// 2 Lx states in an LDS window (a state feeds its right/left neighbour
// and the state one row up).
#include "model.hpp"
#include <cmath>
#include <type_traits>

namespace minsr {

template <typename T> struct VecJ;
template <> struct VecJ<float> { typedef float4 type; static constexpr int V = 4; };
template <> struct VecJ<double> { typedef double2 type; static constexpr int V = 2; };

__device__ inline float j_exp(float x) { return expf(x); }
__device__ inline double j_exp(double x) { return exp(x); }
__device__ inline float j_tanh(float x) { return tanhf(x); }
__device__ inline double j_tanh(double x) { return tanh(x); }
__device__ inline float j_log1p(float x) { return log1pf(x); }
__device__ inline double j_log1p(double x) { return log1p(x); }
template <typename T> __device__ inline T j_sigmoid(T x) { return T(1) / (T(1) + j_exp(-x)); }

template <typename T> struct JacArgs {
  Work<T> w;
  Layout L;
  int N, Ns, C, zero_mag, cplx;
  const int* nbr;
  const uint8_t* sigma;
  const T* states;       // [Ns][N][H]; 1D: rows k with (k+1) % C == 0 are read
  const T* gates;        // 1D, C == 1, optional: [Ns][N][4][H] u, r, g, ht of the sampler
  T* dp;                 // deferred gradients: [nseeds][Ns][N][3][H] gate adjoints
  const double* site;    // 1D real FP32 models, optional: [Ns][N][4] the
                         // forward pass's log p(0), log p(1) per site (the head's
                         // conditionals, masked as in sampling)
  T* O;                  // [rows][Np]
  T scale;               // 1 / sqrt(Ns)
  int W2;                // 2D adjoint window
};

constexpr int SEGMAX = 16;

// WL: the gate weights (forward and transposed packings) are staged in LDS
// once per workgroup and shared by its samples, instead of being streamed
// from L2 at every site (FP32, 1D, d_h <= 64, checkpoint stride <= 4).
template <int H, int P, bool WL = false> struct JShape {
  static constexpr int TPS = H * P;                        // threads per sample
  static constexpr int NT0 = TPS < 64 ? 64 : TPS;
  static constexpr int NT = WL ? (NT0 * 4 > 256 ? NT0 : NT0 * 4) : NT0;
  static constexpr int SG = NT / TPS;                      // samples per block
  static constexpr int NW = H > 64 ? H / 64 : 1;           // waves per p-subgroup
};
constexpr int SEGMAX_WL = 4;

template <int H> struct JReduce {
  template <typename T> __device__ static T run(T v) {
    constexpr int W = H < 64 ? H : 64;
#pragma unroll
    for (int m = W / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
  }
};

typedef __attribute__((ext_vector_type(16))) float f32x16_j;

// W_u, W_r, W_h blocks of one row (deferred gradients): for gate q,
// dW_q[j][c] = sum over sites k of dp_q[k][j] h_{k-1}[c] (h_{-1} = 0), a
// [H x N] x [N x H] product on v_mfma_f32_32x32x2_f32 (lane l supplies
// A[l % 32][l / 32] and B[l / 32][l % 32]; element e of lane l is row
// 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32).  Wave w of nw takes every
// nw-th of the 3 (H / 32)^2 output blocks.
template <int H>
__device__ void wgrad_row(const JacArgs<float>& a, int row, int s, int lane, int w, int nw) {
  constexpr int NB = H / 32, NBLK = 3 * NB * NB, ds = 2;
  const int N = a.N;
  const float* dp = a.dp + (size_t)row * N * 3 * H;
  const float* st = a.states + (size_t)s * N * H;
  float* o = a.O + (size_t)row * a.L.Np;
  const int kl = lane >> 5, cl = lane & 31;
  // items (block of this wave, group of 64 sites) in order; the operands of
  // the next item (clamped addresses, masked values) are requested before
  // the current item's 32 products, so a wave waits for memory about once
  // per row rather than once per 16 sites
  const int ng = (N + 63) / 64;
  const int nblk = w < NBLK ? (NBLK - 1 - w) / nw + 1 : 0;
  const int nitem = nblk * ng;
  auto load = [&](int item, float (&av)[32], float (&bv)[32]) {
    const int b = w + (item / ng) * nw, k64 = 64 * (item % ng);
    const int q = b / (NB * NB), jb = (b / NB) % NB, cb = b % NB;
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const int k = k64 + 2 * u + kl;
      const float x = dp[((size_t)min(k, N - 1) * 3 + q) * H + jb * 32 + cl];
      const float y = st[(size_t)max(min(k, N) - 1, 0) * H + cb * 32 + cl];
      av[u] = k < N ? x : 0.f;
      bv[u] = (k >= 1 && k < N) ? y : 0.f;
    }
  };
  float av[32], bv[32], an[32], bn[32];
  if (nitem > 0) load(0, av, bv);
  f32x16_j acc;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.f;
  for (int it = 0; it < nitem; ++it) {
    const bool more = it + 1 < nitem;
    if (more) load(it + 1, an, bn);
#pragma unroll
    for (int u = 0; u < 32; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u], bv[u], acc, 0, 0, 0);
    if (it % ng == ng - 1) {
      const int b = w + (it / ng) * nw;
      const int q = b / (NB * NB), jb = (b / NB) % NB, cb = b % NB;
      const size_t off = q == 0 ? a.L.Wu : q == 1 ? a.L.Wr : a.L.Wh;
      const int ldq = q < 2 ? H + ds : H;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int jr = jb * 32 + 8 * (e / 4) + 4 * kl + e % 4;
        o[off + (size_t)jr * ldq + cb * 32 + cl] = acc[e] * a.scale;
        acc[e] = 0.f;
      }
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < 32; ++u) { av[u] = an[u]; bv[u] = bn[u]; }
    }
  }
}

// GD (deferred gradients; FP32 1D with the gate tape): the W_u, W_r, W_h
// blocks of the row are not accumulated here; the reverse pass stores the
// gate adjoints of every site and k_jac_wgrad (wgrad_row) then forms those
// blocks as products over the sites on the matrix cores.  The reverse
// weights of the thread's unit stay in registers.
template <typename T, int H, int DIM, int P, bool WL = false, bool GD = false>
__global__ __launch_bounds__((JShape<H, P, WL>::NT)) void k_jacobian(JacArgs<T> a) {
  using VT = typename VecJ<T>::type;
  constexpr int V = VecJ<T>::V;
  constexpr int NT = JShape<H, P, WL>::NT, SG = JShape<H, P, WL>::SG;
  constexpr int NW = JShape<H, P, WL>::NW;
  constexpr int HP = H + V;
  constexpr int CP = H / P;           // gradient columns per part
  constexpr int SEGN = DIM == 1 ? (WL ? SEGMAX_WL : SEGMAX) : 1;
  constexpr int NWV = WL ? (H / V) * H * 3 : 1;        // staged weight vectors per packing
  __shared__ VT wlf[NWV], wlb[NWV];
  constexpr int WMAX = DIM == 2 ? 32 : 1;
  constexpr int ds = DIM == 1 ? 2 : 4;

  __shared__ __align__(16) T tx[SG][SEGN + 1][HP];     // cell inputs; tx[kk+1] = h_k (1D)
  __shared__ __align__(16) T thh[DIM == 2 ? SG : 1][HP];
  __shared__ __align__(16) T thv[DIM == 2 ? SG : 1][HP];
  __shared__ T town[SG][SEGN][4][H];                   // u, r, g, ht per unit
  __shared__ T thead[SG][SEGN][4];                     // p0, p1, a0, a1
  __shared__ __align__(16) T dbuf[SG][4][HP];          // dpu, dpr, dg, dh' broadcast
  __shared__ T pbuf[SG][P][2][H];                      // partial sums of reverse products
  __shared__ T dacc[DIM == 2 ? SG : 1][WMAX][H];       // 2D adjoint window
  __shared__ T red[NT / 64][4];
  constexpr int RCH = H < 16 ? H : 16;                  // rows per output chunk
  constexpr int TPS = H * P;                            // threads per sample
  __shared__ T stg[SG][RCH][H + 4];                     // output staging

  const int tid = threadIdx.x;
  const int sg = tid / (H * P);
  const int p = (tid / H) % P;
  const int j = tid % H;
  const int wave = tid / 64;
  const int s = blockIdx.x * SG + sg;
  const bool act = s < a.Ns;
  const int sid = act ? s : 0;
  const int N = a.N;
  const Work<T> w = a.w;
  const VT* fw = reinterpret_cast<const VT*>(w.fw);
  const VT* bw = reinterpret_cast<const VT*>(w.bw);
  if constexpr (WL) {
    for (int e = threadIdx.x; e < NWV; e += NT) { wlf[e] = fw[e]; wlb[e] = bw[e]; }
    __syncthreads();
  }
  auto FW = [&](int idx) -> VT {
    if constexpr (WL) return wlf[idx]; else return fw[idx];
  };
  auto BW = [&](int idx) -> VT {
    if constexpr (WL) return wlb[idx]; else return bw[idx];
  };
  VT bwr[GD ? 3 * (H / V) : 1];
  if constexpr (GD) {
#pragma unroll
    for (int i = 0; i < 3 * (H / V); ++i) bwr[i] = bw[((i / 3) * H + j) * 3 + i % 3];
  }
  const VT* f2 = reinterpret_cast<const VT*>(w.f2);
  const VT* b2 = reinterpret_cast<const VT*>(w.b2);
  const uint8_t* sig = a.sigma + (size_t)sid * N;
  const T* st = a.states + (size_t)sid * N * H;
  // N <= 64: the sample's spins as the bits of one word, read once (all
  // loads in flight together), so no site waits on a load for its spin
  uint64_t smask = 0;
  if (N <= 64) {
#pragma unroll
    for (int q0 = 0; q0 < 64; q0 += 16) {
      uint8_t v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = sig[min(q0 + u, N - 1)];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (q0 + u < N) smask |= (uint64_t)(v[u] & 1) << (q0 + u);
    }
  }
  auto spin = [&](int q) -> int { return N <= 64 ? (int)((smask >> q) & 1u) : (int)sig[q]; };
  // the per-site exchanges go through shared memory only; a workgroup of one
  // wave orders them with a wavefront fence, which (unlike a workgroup
  // barrier) does not also wait for its outstanding global loads and stores
  auto site_sync = [&]() {
    if constexpr (NT == 64) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  };

  const T bu = w.bias[j], br = w.bias[H + j], bh = w.bias[2 * H + j], bi = w.bias[3 * H + j];
  const T U0 = w.head[j], U1v = w.head[H + j];
  const T P0 = w.head[2 * H + j], P1 = w.head[3 * H + j];
  const T c0 = w.headb[0], c1 = w.headb[1], cp0 = w.headb[2], cp1 = w.headb[3];
  const T PI = (T)3.14159265358979323846;
  const size_t Np = a.L.Np;

  const int nseeds = a.cplx ? 2 : 1;
  for (int seed = 0; seed < nseeds; ++seed) {
    // ---- accumulators (this thread's share of the sample's row)
    constexpr int CPG = GD ? 1 : CP;
    T gWu[CPG], gWr[CPG], gWh[CPG], gU1[DIM == 2 ? CP : 1], gU2[DIM == 2 ? CP : 1];
#pragma unroll
    for (int c = 0; c < CPG; ++c) gWu[c] = gWr[c] = gWh[c] = (T)0;
    if constexpr (DIM == 2) {
#pragma unroll
      for (int c = 0; c < CP; ++c) gU1[c] = gU2[c] = (T)0;
    }
    T gxu[ds], gxr[ds], gxi[ds];
#pragma unroll
    for (int c = 0; c < ds; ++c) gxu[c] = gxr[c] = gxi[c] = (T)0;
    T gbu = 0, gbr = 0, gbh = 0, gbi = 0, gH0 = 0, gH1 = 0, gc0 = 0, gc1 = 0;

    T dcarry = (T)0;   // 1D: adjoint of h_{k} arriving from site k+1
    if (DIM == 2) {
      for (int i = 0; i < WMAX; ++i) if (p == 0) dacc[sg][i][j] = (T)0;
    }

    const int C = DIM == 1 ? a.C : 1;
    const int nseg = (N + C - 1) / C;
    // 1D: the checkpoint a segment starts from is requested one segment
    // ahead, so its load overlaps the previous segment's work
    auto ckpt = [&](int sgi) -> T {
      const int kss = sgi * C;
      return (sgi < 0 || kss == 0) ? (T)0 : st[(size_t)(kss - 1) * H + j];
    };
    T hnext = (DIM == 1 && p == 0) ? ckpt(nseg - 1) : (T)0;
    // with the sampler's gate tape (C == 1) the segment of one site needs no
    // gate products: its gates and state are requested one site ahead
    const bool tape = DIM == 1 && a.gates != nullptr;
    const T* gt = tape ? a.gates + (size_t)sid * N * 4 * H : nullptr;
    T gnx[4] = {(T)0, (T)0, (T)0, (T)0}, hnx = (T)0;
    // the head's conditionals of the same pass: no reductions over the units
    const bool hsite = DIM == 1 && a.site != nullptr && seed == 0;
    const double* sit = hsite ? a.site + (size_t)sid * N * 4 : nullptr;
    double lsn0 = 0.0, lsn1 = 0.0;
    auto tape_fetch = [&](int k) {
#pragma unroll
      for (int q = 0; q < 4; ++q) gnx[q] = gt[((size_t)k * 4 + q) * H + j];
      hnx = st[(size_t)k * H + j];
      if (hsite) { lsn0 = sit[4 * k]; lsn1 = sit[4 * k + 1]; }
    };
    if (tape) tape_fetch(N - 1);
    for (int segi = nseg - 1; segi >= 0; --segi) {
      const int ks = segi * C;
      const int len = (ks + C <= N) ? C : N - ks;
      const T hck = hnext;
      if (DIM == 1 && p == 0) hnext = ckpt(segi - 1);
      T gcur[4] = {gnx[0], gnx[1], gnx[2], gnx[3]};
      const T hcur = hnx;
      const double lsc0 = lsn0, lsc1 = lsn1;
      if (tape && segi > 0) tape_fetch(segi - 1);

      // zero-magnetisation counts of sigma_{<ks}
      int nup = 0, ndn = 0;
      if (a.zero_mag)
        for (int k = 0; k < ks; ++k) { nup += spin(k) == 0; ndn += spin(k) == 1; }

      if (DIM == 1) {
        // ---- forward recompute of the segment from its checkpoint
        if (p == 0) tx[sg][0][j] = hck;
        site_sync();
        for (int kk = 0; kk < len; ++kk) {
          const int k = ks + kk;
          T u, rr, ag, ht, hn;
          if (tape) {
            u = gcur[0]; rr = gcur[1]; ag = gcur[2]; ht = gcur[3];
            hn = hcur;
          } else {
            const int sprev = k > 0 ? spin(k - 1) : -1;
            T au = bu, ar = br, agg = bh, ai = bi;
            if (sprev >= 0) {
              au += w.xc[(0 * ds + sprev) * H + j];
              ar += w.xc[(1 * ds + sprev) * H + j];
              ai += w.xc[(2 * ds + sprev) * H + j];
            }
#pragma unroll 4
            for (int k4 = 0; k4 < H / V; ++k4) {
              const VT wu = FW((k4 * H + j) * 3 + 0);
              const VT wr = FW((k4 * H + j) * 3 + 1);
              const VT wg = FW((k4 * H + j) * 3 + 2);
              const T* wus = reinterpret_cast<const T*>(&wu);
              const T* wrs = reinterpret_cast<const T*>(&wr);
              const T* wgs = reinterpret_cast<const T*>(&wg);
              const VT xv = *reinterpret_cast<const VT*>(&tx[sg][kk][k4 * V]);
              const T* xs = reinterpret_cast<const T*>(&xv);
#pragma unroll
              for (int v = 0; v < V; ++v) {
                au = fma(wus[v], xs[v], au);
                ar = fma(wrs[v], xs[v], ar);
                agg = fma(wgs[v], xs[v], agg);
              }
            }
            const T hprev = tx[sg][kk][j];
            u = j_sigmoid(au);
            rr = j_sigmoid(ar);
            ag = agg;
            ht = j_tanh(rr * ag + ai);
            hn = ((T)1 - u) * hprev + u * ht;
          }
          T z0 = (T)0, z1 = (T)0, q0 = (T)0, q1 = (T)0;
          if (!hsite) {
            z0 = JReduce<H>::run(U0 * hn); z1 = JReduce<H>::run(U1v * hn);
            if (a.cplx) { q0 = JReduce<H>::run(P0 * hn); q1 = JReduce<H>::run(P1 * hn); }
          }
          if (NW > 1 && !hsite) {
            if ((tid & 63) == 0) { red[wave][0] = z0; red[wave][1] = z1; red[wave][2] = q0; red[wave][3] = q1; }
          }
          if (p == 0) {
            tx[sg][kk + 1][j] = hn;
            town[sg][kk][0][j] = u; town[sg][kk][1][j] = rr;
            town[sg][kk][2][j] = ag; town[sg][kk][3][j] = ht;
          }
          site_sync();
          if (NW > 1 && !hsite) {
            const int w0 = (tid / H) * NW;   // first wave of this p-subgroup
            T s0 = red[w0][0], s1 = red[w0][1], s2 = red[w0][2], s3 = red[w0][3];
            for (int i = 1; i < NW; ++i) { s0 += red[w0 + i][0]; s1 += red[w0 + i][1]; s2 += red[w0 + i][2]; s3 += red[w0 + i][3]; }
            z0 = s0; z1 = s1; q0 = s2; q1 = s3;
          }
          if (j == 0 && p == 0 && !hsite) {
            const T zz0 = z0 + c0, zz1 = z1 + c1;
            const T mx = zz0 > zz1 ? zz0 : zz1;
            const T d = zz0 > zz1 ? zz1 - zz0 : zz0 - zz1;
            const T lse = mx + j_log1p(j_exp(d));
            T p0 = j_exp(zz0 - lse), p1 = j_exp(zz1 - lse);
            if (a.zero_mag) {
              if (nup >= N / 2) { p0 = 0; p1 = 1; }
              else if (ndn >= N / 2) { p0 = 1; p1 = 0; }
            }
            thead[sg][kk][0] = p0; thead[sg][kk][1] = p1;
            thead[sg][kk][2] = q0 + cp0; thead[sg][kk][3] = q1 + cp1;
          }
          nup += spin(k) == 0; ndn += spin(k) == 1;
          if (NW > 1) __syncthreads();
        }
        site_sync();
      }

      // ---- reverse through the segment
      for (int kk = len - 1; kk >= 0; --kk) {
        const int k = ks + kk;
        const int sk = spin(k);
        T u, rr, ag, ht, hprev, hk;
        int kh = -1, kv = -1, sh = -1, sv = -1;
        if (DIM == 1) {
          u = town[sg][kk][0][j]; rr = town[sg][kk][1][j];
          ag = town[sg][kk][2][j]; ht = town[sg][kk][3][j];
          hprev = tx[sg][kk][j];
          hk = tx[sg][kk + 1][j];
        } else {
          // recompute site k from its stored predecessors
          kh = a.nbr[2 * k]; kv = a.nbr[2 * k + 1];
          sh = kh >= 0 ? spin(kh) : -1;
          sv = kv >= 0 ? spin(kv) : -1;
          if (p == 0) {
            thh[sg][j] = kh >= 0 ? st[(size_t)kh * H + j] : (T)0;
            thv[sg][j] = kv >= 0 ? st[(size_t)kv * H + j] : (T)0;
          }
          __syncthreads();
          T hin = (T)0;
#pragma unroll 2
          for (int k4 = 0; k4 < H / V; ++k4) {
            const VT w1 = f2[(k4 * H + j) * 2 + 0];
            const VT w2 = f2[(k4 * H + j) * 2 + 1];
            const T* w1s = reinterpret_cast<const T*>(&w1);
            const T* w2s = reinterpret_cast<const T*>(&w2);
            const VT x1 = *reinterpret_cast<const VT*>(&thh[sg][k4 * V]);
            const VT x2 = *reinterpret_cast<const VT*>(&thv[sg][k4 * V]);
            const T* x1s = reinterpret_cast<const T*>(&x1);
            const T* x2s = reinterpret_cast<const T*>(&x2);
#pragma unroll
            for (int v = 0; v < V; ++v) hin = fma(w1s[v], x1s[v], hin);
#pragma unroll
            for (int v = 0; v < V; ++v) hin = fma(w2s[v], x2s[v], hin);
          }
          if (p == 0) tx[sg][0][j] = hin;
          __syncthreads();
          T au = bu, ar = br, agg = bh, ai = bi;
          if (sh >= 0) {
            au += w.xc[(0 * ds + sh) * H + j];
            ar += w.xc[(1 * ds + sh) * H + j];
            ai += w.xc[(2 * ds + sh) * H + j];
          }
          if (sv >= 0) {
            au += w.xc[(0 * ds + 2 + sv) * H + j];
            ar += w.xc[(1 * ds + 2 + sv) * H + j];
            ai += w.xc[(2 * ds + 2 + sv) * H + j];
          }
#pragma unroll 2
          for (int k4 = 0; k4 < H / V; ++k4) {
            const VT wu = FW((k4 * H + j) * 3 + 0);
            const VT wr = FW((k4 * H + j) * 3 + 1);
            const VT wg = FW((k4 * H + j) * 3 + 2);
            const T* wus = reinterpret_cast<const T*>(&wu);
            const T* wrs = reinterpret_cast<const T*>(&wr);
            const T* wgs = reinterpret_cast<const T*>(&wg);
            const VT xv = *reinterpret_cast<const VT*>(&tx[sg][0][k4 * V]);
            const T* xs = reinterpret_cast<const T*>(&xv);
#pragma unroll
            for (int v = 0; v < V; ++v) {
              au = fma(wus[v], xs[v], au);
              ar = fma(wrs[v], xs[v], ar);
              agg = fma(wgs[v], xs[v], agg);
            }
          }
          u = j_sigmoid(au);
          rr = j_sigmoid(ar);
          ag = agg;
          ht = j_tanh(rr * ag + ai);
          hprev = hin;
          hk = ((T)1 - u) * hprev + u * ht;
          // head of site k (its conditional depends on the counts of sigma_{<k})
          T z0 = JReduce<H>::run(U0 * hk), z1 = JReduce<H>::run(U1v * hk);
          T q0 = (T)0, q1 = (T)0;
          if (a.cplx) { q0 = JReduce<H>::run(P0 * hk); q1 = JReduce<H>::run(P1 * hk); }
          if (NW > 1) {
            if ((tid & 63) == 0) { red[wave][0] = z0; red[wave][1] = z1; red[wave][2] = q0; red[wave][3] = q1; }
            __syncthreads();
            const int w0 = (tid / H) * NW;
            T s0 = red[w0][0], s1 = red[w0][1], s2 = red[w0][2], s3 = red[w0][3];
            for (int i = 1; i < NW; ++i) { s0 += red[w0 + i][0]; s1 += red[w0 + i][1]; s2 += red[w0 + i][2]; s3 += red[w0 + i][3]; }
            z0 = s0; z1 = s1; q0 = s2; q1 = s3;
          }
          if (j == 0 && p == 0) {
            int cu = 0, cd = 0;
            if (a.zero_mag) for (int q = 0; q < k; ++q) { cu += spin(q) == 0; cd += spin(q) == 1; }
            const T zz0 = z0 + c0, zz1 = z1 + c1;
            const T mx = zz0 > zz1 ? zz0 : zz1;
            const T d = zz0 > zz1 ? zz1 - zz0 : zz0 - zz1;
            const T lse = mx + j_log1p(j_exp(d));
            T p0 = j_exp(zz0 - lse), p1 = j_exp(zz1 - lse);
            if (a.zero_mag) {
              if (cu >= N / 2) { p0 = 0; p1 = 1; }
              else if (cd >= N / 2) { p0 = 1; p1 = 0; }
            }
            thead[sg][0][0] = p0; thead[sg][0][1] = p1;
            thead[sg][0][2] = q0 + cp0; thead[sg][0][3] = q1 + cp1;
          }
          __syncthreads();
        }
        const int kt = DIM == 1 ? kk : 0;
        // output-head adjoint for this seed
        T dz0, dz1;
        T dh;
        if (seed == 0) {
          T hp0, hp1;
          if (hsite) {
            hp0 = j_exp((T)(tape ? lsc0 : sit[4 * k]));
            hp1 = j_exp((T)(tape ? lsc1 : sit[4 * k + 1]));
          } else {
            hp0 = thead[sg][kt][0];
            hp1 = thead[sg][kt][1];
          }
          dz0 = (T)0.5 * ((sk == 0 ? (T)1 : (T)0) - hp0);
          dz1 = (T)0.5 * ((sk == 1 ? (T)1 : (T)0) - hp1);
          dh = dz0 * U0 + dz1 * U1v;
        } else {
          const T a0 = thead[sg][kt][2], a1 = thead[sg][kt][3];
          const T e0 = (T)1 + fabs(a0), e1 = (T)1 + fabs(a1);
          dz0 = sk == 0 ? PI / (e0 * e0) : (T)0;
          dz1 = sk == 1 ? PI / (e1 * e1) : (T)0;
          dh = dz0 * P0 + dz1 * P1;
        }
        gH0 += dz0 * hk; gH1 += dz1 * hk;
        gc0 += dz0; gc1 += dz1;
        if (DIM == 1) dh += dcarry;
        else dh += dacc[sg][k % a.W2][j];

        // cell reverse (own unit)
        const T dht = dh * u;
        const T du = dh * (ht - hprev);
        const T dhin_d = dh * ((T)1 - u);
        const T da = dht * ((T)1 - ht * ht);
        const T dr = da * ag;
        const T dg = da * rr;
        const T dpu = du * u * ((T)1 - u);
        const T dpr = dr * rr * ((T)1 - rr);
        if (p == 0) { dbuf[sg][0][j] = dpu; dbuf[sg][1][j] = dpr; dbuf[sg][2][j] = dg; }
        if constexpr (GD) {
          if (act) {
            T* d = a.dp + ((((size_t)seed * a.Ns + s) * N + k) * 3) * H;
            d[j] = dpu; d[H + j] = dpr; d[2 * H + j] = dg;
          }
        }
        gbu += dpu; gbr += dpr; gbh += dg; gbi += da;
        if (DIM == 1) {
          if (k > 0) {
            const int sp = spin(k - 1);
            gxu[sp] += dpu; gxr[sp] += dpr; gxi[sp] += da;
          }
        } else {
          if (sh >= 0) { gxu[sh] += dpu; gxr[sh] += dpr; gxi[sh] += da; }
          if (sv >= 0) { gxu[2 + sv] += dpu; gxr[2 + sv] += dpr; gxi[2 + sv] += da; }
        }
        // outer products with the cell input, columns of part p
        if constexpr (!GD) {
          const T* xrow = DIM == 1 ? &tx[sg][kk][p * CP] : &tx[sg][0][p * CP];
#pragma unroll
          for (int c4 = 0; c4 < CP / V; ++c4) {
            const VT xv = *reinterpret_cast<const VT*>(xrow + c4 * V);
            const T* xs = reinterpret_cast<const T*>(&xv);
#pragma unroll
            for (int v = 0; v < V; ++v) {
              gWu[c4 * V + v] = fma(dpu, xs[v], gWu[c4 * V + v]);
              gWr[c4 * V + v] = fma(dpr, xs[v], gWr[c4 * V + v]);
              gWh[c4 * V + v] = fma(dg, xs[v], gWh[c4 * V + v]);
            }
          }
        }
        site_sync();
        // reverse product into the cell input: rows i of part p; four
        // partial sums so that several weight loads are in flight
        T partv[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll (GD ? H / V : 4)
        for (int i4 = p * CP / V; i4 < (p + 1) * CP / V; ++i4) {
          const VT wu = GD ? bwr[(i4 * 3 + 0) % (GD ? 3 * (H / V) : 1)] : BW((i4 * H + j) * 3 + 0);
          const VT wr = GD ? bwr[(i4 * 3 + 1) % (GD ? 3 * (H / V) : 1)] : BW((i4 * H + j) * 3 + 1);
          const VT wg = GD ? bwr[(i4 * 3 + 2) % (GD ? 3 * (H / V) : 1)] : BW((i4 * H + j) * 3 + 2);
          const T* wus = reinterpret_cast<const T*>(&wu);
          const T* wrs = reinterpret_cast<const T*>(&wr);
          const T* wgs = reinterpret_cast<const T*>(&wg);
          const VT d0 = *reinterpret_cast<const VT*>(&dbuf[sg][0][i4 * V]);
          const VT d1 = *reinterpret_cast<const VT*>(&dbuf[sg][1][i4 * V]);
          const VT d2 = *reinterpret_cast<const VT*>(&dbuf[sg][2][i4 * V]);
          const T* d0s = reinterpret_cast<const T*>(&d0);
          const T* d1s = reinterpret_cast<const T*>(&d1);
          const T* d2s = reinterpret_cast<const T*>(&d2);
          T& part = partv[i4 & 3];
#pragma unroll
          for (int v = 0; v < V; ++v) {
            part = fma(wus[v], d0s[v], part);
            part = fma(wrs[v], d1s[v], part);
            part = fma(wgs[v], d2s[v], part);
          }
        }
        const T part = (partv[0] + partv[1]) + (partv[2] + partv[3]);
        T dhin;
        if (P > 1) {
          pbuf[sg][p][0][j] = part;
          __syncthreads();
          dhin = dhin_d;
#pragma unroll
          for (int q = 0; q < P; ++q) dhin += pbuf[sg][q][0][j];
        } else {
          dhin = dhin_d + part;
        }
        if (DIM == 1) {
          dcarry = dhin;
        } else {
          // h' = U1 h_h + U2 h_v: gradients of U1, U2 and adjoints of the predecessors
          if (p == 0) dbuf[sg][3][j] = dhin;
          {
            const T* hhrow = &thh[sg][p * CP];
            const T* hvrow = &thv[sg][p * CP];
#pragma unroll
            for (int c4 = 0; c4 < CP / V; ++c4) {
              const VT xh = *reinterpret_cast<const VT*>(hhrow + c4 * V);
              const VT xv = *reinterpret_cast<const VT*>(hvrow + c4 * V);
              const T* xhs = reinterpret_cast<const T*>(&xh);
              const T* xvs = reinterpret_cast<const T*>(&xv);
#pragma unroll
              for (int v = 0; v < V; ++v) {
                gU1[c4 * V + v] = fma(dhin, xhs[v], gU1[c4 * V + v]);
                gU2[c4 * V + v] = fma(dhin, xvs[v], gU2[c4 * V + v]);
              }
            }
          }
          __syncthreads();
          T ph = (T)0, pv = (T)0;
#pragma unroll 1
          for (int i4 = p * CP / V; i4 < (p + 1) * CP / V; ++i4) {
            const VT w1 = b2[(i4 * H + j) * 2 + 0];
            const VT w2 = b2[(i4 * H + j) * 2 + 1];
            const T* w1s = reinterpret_cast<const T*>(&w1);
            const T* w2s = reinterpret_cast<const T*>(&w2);
            const VT dd = *reinterpret_cast<const VT*>(&dbuf[sg][3][i4 * V]);
            const T* dds = reinterpret_cast<const T*>(&dd);
#pragma unroll
            for (int v = 0; v < V; ++v) {
              ph = fma(w1s[v], dds[v], ph);
              pv = fma(w2s[v], dds[v], pv);
            }
          }
          T dhh = ph, dhv = pv;
          if (P > 1) {
            pbuf[sg][p][0][j] = ph;
            pbuf[sg][p][1][j] = pv;
            __syncthreads();
            dhh = pbuf[sg][0][0][j]; dhv = pbuf[sg][0][1][j];
#pragma unroll
            for (int q = 1; q < P; ++q) { dhh += pbuf[sg][q][0][j]; dhv += pbuf[sg][q][1][j]; }
          }
          if (p == 0) {
            dacc[sg][k % a.W2][j] = (T)0;
            if (kh >= 0) dacc[sg][kh % a.W2][j] += dhh;
            if (kv >= 0) dacc[sg][kv % a.W2][j] += dhv;
          }
        }
        site_sync();
      }
    }

    // ---- write the row: each gradient matrix goes through LDS in chunks of
    // RCH rows so that the workgroup's stores cover contiguous memory
    {
      const Layout& L = a.L;
      const size_t row = (size_t)seed * a.Ns + s;
      T* o = a.O + row * Np;
      const T sc = a.scale;
      const int tps_id = p * H + j;
#define MINSR_JAC_STAGE(ARR, XS, NX, OFF, LD)                                              \
      for (int j0 = 0; j0 < H; j0 += RCH) {                                                \
        if (j >= j0 && j < j0 + RCH) {                                                     \
          _Pragma("unroll") for (int c = 0; c < CP; ++c) stg[sg][j - j0][p * CP + c] = ARR[c]; \
          if ((NX) > 0 && p == 0) {                                                        \
            _Pragma("unroll") for (int c = 0; c < (NX); ++c) stg[sg][j - j0][H + c] = XS[c]; \
          }                                                                                \
        }                                                                                  \
        __syncthreads();                                                                   \
        if (act) {                                                                         \
          const int tot = RCH * (LD);                                                      \
          for (int e = tps_id; e < tot; e += TPS)                                          \
            o[(OFF) + (size_t)j0 * (LD) + e] = stg[sg][e / (LD)][e % (LD)] * sc;          \
        }                                                                                  \
        __syncthreads();                                                                   \
      }
      if constexpr (!GD) {
        MINSR_JAC_STAGE(gWu, gxu, ds, L.Wu, H + ds)
        MINSR_JAC_STAGE(gWr, gxr, ds, L.Wr, H + ds)
        MINSR_JAC_STAGE(gWh, gxu, 0, L.Wh, H)
      } else if (act && p == 0) {
        // the one-hot input columns of W_u, W_r (the H x H blocks follow)
#pragma unroll
        for (int c = 0; c < ds; ++c) {
          o[L.Wu + (size_t)j * (H + ds) + H + c] = gxu[c] * sc;
          o[L.Wr + (size_t)j * (H + ds) + H + c] = gxr[c] * sc;
        }
      }
      if constexpr (DIM == 2) {
        MINSR_JAC_STAGE(gU1, gxu, 0, L.U1, H)
        MINSR_JAC_STAGE(gU2, gxu, 0, L.U2, H)
      }
#undef MINSR_JAC_STAGE
      if (act && p == 0) {
#pragma unroll
        for (int c = 0; c < ds; ++c) o[L.Win + (size_t)j * ds + c] = gxi[c] * sc;
        o[L.bu + j] = gbu * sc; o[L.br + j] = gbr * sc;
        o[L.bh + j] = gbh * sc; o[L.bin + j] = gbi * sc;
        const size_t hU = seed == 0 ? L.U : L.Uphi;
        const size_t zU = seed == 0 ? L.Uphi : L.U;
        o[hU + j] = gH0 * sc; o[hU + H + j] = gH1 * sc;
        if (a.cplx) { o[zU + j] = (T)0; o[zU + H + j] = (T)0; }
        if (j == 0) {
          const size_t hc = seed == 0 ? L.c : L.cphi;
          const size_t zc = seed == 0 ? L.cphi : L.c;
          o[hc] = gc0 * sc; o[hc + 1] = gc1 * sc;
          if (a.cplx) { o[zc] = (T)0; o[zc + 1] = (T)0; }
        }
      }
    }
    __syncthreads();
  }
}

// the W_u, W_r, W_h blocks of every row after the reverse pass: one
// workgroup of four waves per row, many rows in flight (their operand loads
// are latency-bound, so the pass's own tail would serialise them)
template <int H>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_jac_wgrad(JacArgs<float> a) {
  wgrad_row<H>(a, blockIdx.x, blockIdx.x % a.Ns, threadIdx.x & 63, threadIdx.x >> 6, 4);
}

template <int H>
static int launch_wgrad(const JacArgs<float>& a, hipStream_t s) {
  const unsigned rows = (unsigned)(a.Ns * (a.cplx ? 2 : 1));
  k_jac_wgrad<H><<<rows, 256, 0, s>>>(a);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

template <typename T, int H, int DIM, int P, bool WL = false, bool GD = false>
static int launch_jac_t(const JacArgs<T>& a, hipStream_t s) {
  constexpr int NT = JShape<H, P, WL>::NT, SG = JShape<H, P, WL>::SG;
  unsigned grid = (unsigned)((a.Ns + SG - 1) / SG);
  k_jacobian<T, H, DIM, P, WL, GD><<<grid, NT, 0, s>>>(a);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

// parts: threads per hidden unit (0 = built-in choice)
template <typename T, int DIM>
static int jac_dispatch(int H, int parts, const JacArgs<T>& a, hipStream_t s) {
  switch (H) {
    case 8: return launch_jac_t<T, 8, DIM, 1>(a, s);
    case 16: return launch_jac_t<T, 16, DIM, 1>(a, s);
    case 32:
      if constexpr (DIM == 1 && std::is_same<T, float>::value) {
        if (a.dp) {
          const int rc = launch_jac_t<T, 32, DIM, 1, false, true>(a, s);
          return rc ? rc : launch_wgrad<32>(a, s);
        }
        if (a.C <= SEGMAX_WL) return launch_jac_t<T, 32, DIM, 1, true>(a, s);
      }
      return launch_jac_t<T, 32, DIM, 1>(a, s);
    case 64:
      if (parts == 0) parts = DIM == 1 ? 1 : 4;
      if constexpr (DIM == 1 && std::is_same<T, float>::value) {
        if (a.dp && parts == 1) {
          const int rc = launch_jac_t<T, 64, DIM, 1, false, true>(a, s);
          return rc ? rc : launch_wgrad<64>(a, s);
        }
      }
      if constexpr (DIM == 1 && std::is_same<T, float>::value)
        if (parts == 1 && a.C <= SEGMAX_WL) return launch_jac_t<T, 64, DIM, 1, true>(a, s);
      if (parts == 1) return launch_jac_t<T, 64, DIM, 1>(a, s);
      if (parts == 2) return launch_jac_t<T, 64, DIM, 2>(a, s);
      return launch_jac_t<T, 64, DIM, 4>(a, s);
    case 128:
      if (parts == 0) parts = 2;
      if (parts == 1) return launch_jac_t<T, 128, DIM, 1>(a, s);
      if (parts == 2) return launch_jac_t<T, 128, DIM, 2>(a, s);
      return launch_jac_t<T, 128, DIM, 4>(a, s);
  }
  return fail(MINSR_E_UNSUPPORTED, "hidden width must be 8, 16, 32, 64 or 128");
}

template <typename T>
static int jac_t(minsr_model* m, const Work<T>& w, int Ns, const uint8_t* sigma,
                 const void* states, int C, void* O, const void* gates, const double* site,
                 hipStream_t s) {
  JacArgs<T> a{};
  a.w = w; a.L = m->L; a.N = m->N; a.Ns = Ns; a.C = C;
  a.zero_mag = m->d.zero_mag; a.cplx = m->cplx; a.nbr = m->nbr;
  a.sigma = sigma; a.states = (const T*)states; a.O = (T*)O;
  a.gates = (m->dim == 1 && C == 1) ? (const T*)gates : nullptr;
  // deferred weight gradients with the tape (FP32, 1D, d_h 32 or 64)
  a.dp = (a.gates && m->jdp && (m->H == 32 || m->H == 64)) ? (T*)m->jdp : nullptr;
  a.site = (m->dim == 1 && !m->cplx && sizeof(T) == 4) ? site : nullptr;
  a.scale = (T)(1.0 / std::sqrt((double)Ns));
  a.W2 = 2 * m->d.Lx;
  if (m->dim == 1) return jac_dispatch<T, 1>(m->H, m->tune_jac_parts, a, s);
  return jac_dispatch<T, 2>(m->H, m->tune_jac_parts, a, s);
}

int launch_jacobian(minsr_model* m, int Ns, const uint8_t* sigma, const void* states,
                    int ckpt_every, void* O, const double* g, double* vjp_part, hipStream_t s,
                    const void* gates, const double* site) {
  (void)g; (void)vjp_part;
  if (Ns == 0) return MINSR_OK;
  if (m->dim == 2 && 2 * m->d.Lx > 32) return fail(MINSR_E_UNSUPPORTED, "2D lattices need Lx <= 16");
  if (ckpt_every < 1 || ckpt_every > SEGMAX)
    return fail(MINSR_E_INVALID_ARG, "ckpt_every must be in [1, 16]");
  if (m->f64) return jac_t<double>(m, m->wd, Ns, sigma, states, ckpt_every, O, gates, site, s);
  // d_h = 128 chains: sample-batched reverse pass on the matrix cores
  // (an explicit thread split selects the per-sample kernel below)
  if (m->tune_jac_parts == 0 && site && states == m->states && jac_mfma_supported(m, ckpt_every))
    return launch_jacobian_mfma(m, Ns, sigma, ckpt_every, O, site, s);
  return jac_t<float>(m, m->wf, Ns, sigma, states, ckpt_every, O, gates, site, s);
}

}  // namespace minsr
