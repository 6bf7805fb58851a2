// Local energies of FP32 models on the matrix cores (Sec. 2.3, local
// energy; App. A, GRU cells).
//
// A workgroup re-evaluates 32 connected configurations that share their
// first flipped site (one term of the Hamiltonian for 32 samples), so all
// 32 recurrences restart at the same site and advance in lockstep.  At
// every site the gate pre-activations of the 32 sequences are one
// [32 x (H + ds)] x [(H + ds) x 3H] product on the matrix cores: the one-hot
// input steps on v_mfma_f32_32x32x2_f32, the state term on the same FP32
// instruction in 2D and, in 1D (state in [-1, 1]), as three FP16 hi/lo
// products on v_mfma_f32_32x32x16_f16 (described at k_eloc_mfma_w):
// wave w owns hidden units 32w..32w+31 and keeps its B-operand fragments of
// W_u, W_r, W_h and of the one-hot input columns in registers for the whole
// kernel, so the only per-site operand traffic is the 32 x H hidden state
// read from LDS.  The input vector is [h; onehot(sigma)], exactly the
// paper's x = [h; sigma]; its one-hot columns enter as extra K-steps.  The
// elementwise GRU update runs in the accumulator layout (lane l holds unit
// l mod 32 of 16 sequences), the new state goes back to LDS, and each lane
// then reduces the output head for its own sequence.  In 1D every
// re-evaluated site has exactly one one-hot column set, so the packed
// fragments carry the biases of u, r and the input term on those columns,
// and they are pre-scaled (-log2 e for u, r; 2 log2 e for the candidate)
// so that each nonlinearity is one hardware exp2 and one reciprocal.
// 2D models form h' = U1 h_horizontal + U2 h_vertical with one more MFMA
// product per site (B fragments streamed from L2) before the cell.
#include <type_traits>

#include "model.hpp"
#include "mfma16.hpp"

namespace minsr {

typedef __attribute__((ext_vector_type(16))) float f32x16_m;

struct ElocMArgs {
  const float* mw;
  const float* m2;
  const float* bias;
  const float* head;
  const float* headb;
  int N, Ns, zero_mag, cplx, marshall, nchunks, n_items, W, M;
  const int* nbr;
  const uint8_t* subA;
  const uint8_t* sigma;
  const float* states;
  const double* site;
  const int* bonds;
  int n_nn, ham_kind;
  double hx, J1, J2;
  double* contrib;
  float* ring;
  // J1-J2: only samples whose pair is antiparallel are re-evaluated; items
  // are (term, chunk of the compacted list)
  const int* list;      // [M][Ns]
  const int* count;     // [M], then the item count at [M]
  const int* items;     // [items][2]
};

// hardware exp2 and reciprocal (about 1 ulp each): the GRU nonlinearities
// to FP32 accuracy at a fraction of the cost of the library's expf / tanhf
__device__ __forceinline__ float fast_exp(float x) {
  return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
}
__device__ __forceinline__ float fast_sigmoid(float x) {
  return __builtin_amdgcn_rcpf(1.f + fast_exp(-x));
}
// tanh y = 1 - 2 / (1 + e^{2y}); saturates correctly at both ends
__device__ __forceinline__ float fast_tanh(float y) {
  return 1.f - 2.f * __builtin_amdgcn_rcpf(1.f + fast_exp(2.f * y));
}

// log(1 + e^d) for d <= 0 from the hardware exp2 and log2 (1 + e^d lies in
// [1, 2], so the absolute error stays at FP32 rounding level)
__device__ __forceinline__ float fast_log1p_exp(float d) {
  return 0.6931471805599453f * __builtin_amdgcn_logf(1.f + fast_exp(d));
}

__device__ inline f32x16_m mfma_f32(float a, float b, f32x16_m c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

typedef __attribute__((ext_vector_type(8))) _Float16 f16x8_m;
typedef __attribute__((ext_vector_type(2))) _Float16 f16x2_m;
typedef __attribute__((ext_vector_type(2))) float f32x2_m;

__device__ inline f32x16_m mfma_f16(f16x8_m a, f16x8_m b, f32x16_m c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// x = hi + lo with hi = fp16(x) and lo = fp16(x - hi), both rounded to
// nearest; x - hi is exact in FP32, so |x - hi - lo| <= 2^-22 |x| for x in
// the normal FP16 range (smaller values keep an absolute error of 2^-25)
__device__ inline void split_f16(const float (&x)[8], f16x8_m& hi, f16x8_m& lo) {
#pragma unroll
  for (int e = 0; e < 8; e += 2) {   // pairs: one packed conversion each way
    const f32x2_m v = {x[e], x[e + 1]};
    const f16x2_m h = __builtin_convertvector(v, f16x2_m);
    const f16x2_m l = mf16::lo_pair(h, x[e], x[e + 1]);
    hi[e] = h[0]; hi[e + 1] = h[1];
    lo[e] = l[0]; lo[e + 1] = l[1];
  }
}

// One connected configuration being re-evaluated: sample s with the flips of
// Hamiltonian term t (sites f1 and, for an exchange, f2p > f1), restarted at
// site k0 = f1 from the stored hidden state of the unflipped prefix.
struct ElocSeq {
  int t, chunk, navail, f1, f2p, k0, s, nup, ndn, dA, sprev;
  bool act;
  double oldlp, oldph, lp, ph, mel;
  uint64_t smask;
  const int* lst;
  const uint8_t* sg;
};

// sample of row q of an item (row 0's sample for padding rows)
__device__ inline int eloc_row_sample(const ElocMArgs& a, const ElocSeq& e, int q) {
  int i = e.chunk * 32 + q;
  if (i >= e.navail) i = 0;
  return e.lst ? e.lst[i] : i;
}

// item -> (term, chunk of 32 samples), and row `col`'s sequence: its matrix
// element, the old configuration's log-amplitude from k0 on, the spin
// counts of the prefix (zero-magnetisation mask), and the log-amplitude of
// the new configuration up to and including site k0
__device__ inline ElocSeq eloc_begin(const ElocMArgs& a, int item, int col) {
  ElocSeq e;
  const int N = a.N;
  if (a.list) { e.t = a.items[2 * item]; e.chunk = a.items[2 * item + 1]; }
  else { e.t = item / a.nchunks; e.chunk = item % a.nchunks; }
  e.navail = a.list ? a.count[e.t] : a.Ns;
  e.lst = a.list ? a.list + (size_t)e.t * a.Ns : nullptr;
  e.f2p = -1;
  double Jt = 0.0;
  if (a.ham_kind == MINSR_HAM_J1J2) {
    e.f1 = a.bonds[2 * e.t]; e.f2p = a.bonds[2 * e.t + 1];
    Jt = e.t < a.n_nn ? a.J1 : a.J2;
  } else {
    e.f1 = e.t;
  }
  e.k0 = e.f1;
  e.act = e.chunk * 32 + col < e.navail;
  e.s = eloc_row_sample(a, e, col);
  e.sg = a.sigma + (size_t)e.s * N;
  const uint8_t* sg = e.sg;
  const double* st = a.site + (size_t)e.s * N * 4;
  e.nup = 0; e.ndn = 0; e.dA = 0;
  e.oldlp = 0.0; e.oldph = 0.0;
  e.smask = 0;
  // spins (eight sites at a time) and site terms (four) requested before
  // use (clamped addresses, the values beyond the range unused), then taken
  // in site order
  for (int k = 0; k <= e.k0; k += 8) {
    int v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = sg[min(k + u, N - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k + u <= e.k0) {
        const int vv = v[u] ^ (k + u == e.f1 ? 1 : 0);
        e.nup += vv == 0; e.ndn += vv == 1;
      }
  }
  for (int k = e.k0; k < N; k += 4) {
    int v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = sg[min(k + u, N - 1)];
    double lv[4], pv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = min(k + u, N - 1);
      lv[u] = st[4 * kk + v[u]];
      pv[u] = st[4 * kk + 2 + v[u]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k + u < N) {
        e.oldlp += lv[u];
        e.oldph += pv[u];
        if (N <= 64 && k + u > e.k0) e.smask |= (uint64_t)(v[u] & 1) << (k + u);
      }
  }
  const int vflip = sg[e.k0] ^ 1;
  e.lp = st[4 * e.k0 + vflip];
  e.ph = st[4 * e.k0 + 2 + vflip];
  e.sprev = vflip;
  if (a.ham_kind == MINSR_HAM_TFIM) {
    e.mel = -a.hx;
  } else if (a.ham_kind == MINSR_HAM_CLUSTER) {
    const double zl = 1.0 - 2.0 * sg[(e.f1 - 1 + N) % N];
    const double zr = 1.0 - 2.0 * sg[(e.f1 + 1) % N];
    e.mel = -zl * zr;
  } else {
    e.mel = sg[e.f1] != sg[e.f2p] ? 0.5 * Jt : 0.0;
  }
  if (a.marshall) {
    if (a.subA[e.f1]) e.dA += 1 - 2 * sg[e.f1];
    if (e.f2p >= 0 && a.subA[e.f2p]) e.dA += 1 - 2 * sg[e.f2p];
  }
  return e;
}

// output head at site k for this lane's sequence, from its new hidden state
// hrow (units [half H/2, (half + 1) H/2) here, the other half from lane
// l ^ 32), and the running log-amplitude of the new configuration
template <int H>
__device__ inline void eloc_site(const ElocMArgs& a, ElocSeq& e, const float* hrow,
                                 const float (*hw)[H], const float* hb, int half, int k) {
  const float PI = 3.14159265358979323846f;
  const int N = a.N;
  float z0 = 0.f, z1 = 0.f, q0 = 0.f, q1 = 0.f;
#pragma unroll 4
  for (int u4 = 0; u4 < H / 2; u4 += 4) {
    const int u0 = half * (H / 2) + u4;
    const float4 h4 = *reinterpret_cast<const float4*>(&hrow[u0]);
    const float4 w0 = *reinterpret_cast<const float4*>(&hw[0][u0]);
    const float4 w1 = *reinterpret_cast<const float4*>(&hw[1][u0]);
    z0 = fmaf(w0.x, h4.x, z0); z0 = fmaf(w0.y, h4.y, z0); z0 = fmaf(w0.z, h4.z, z0); z0 = fmaf(w0.w, h4.w, z0);
    z1 = fmaf(w1.x, h4.x, z1); z1 = fmaf(w1.y, h4.y, z1); z1 = fmaf(w1.z, h4.z, z1); z1 = fmaf(w1.w, h4.w, z1);
    if (a.cplx) {
      const float4 p0 = *reinterpret_cast<const float4*>(&hw[2][u0]);
      const float4 p1 = *reinterpret_cast<const float4*>(&hw[3][u0]);
      q0 = fmaf(p0.x, h4.x, q0); q0 = fmaf(p0.y, h4.y, q0); q0 = fmaf(p0.z, h4.z, q0); q0 = fmaf(p0.w, h4.w, q0);
      q1 = fmaf(p1.x, h4.x, q1); q1 = fmaf(p1.y, h4.y, q1); q1 = fmaf(p1.z, h4.z, q1); q1 = fmaf(p1.w, h4.w, q1);
    }
  }
  z0 += __shfl_xor(z0, 32, 64);
  z1 += __shfl_xor(z1, 32, 64);
  q0 += __shfl_xor(q0, 32, 64);
  q1 += __shfl_xor(q1, 32, 64);
  const float zz0 = z0 + hb[0], zz1 = z1 + hb[1];
  const float mx = zz0 > zz1 ? zz0 : zz1;
  const float d = zz0 > zz1 ? zz1 - zz0 : zz0 - zz1;
  const float lse = mx + fast_log1p_exp(d);
  float lp0 = zz0 - lse, lp1 = zz1 - lse;
  if (a.zero_mag) {
    if (e.nup >= N / 2) { lp0 = -INFINITY; lp1 = 0.f; }
    else if (e.ndn >= N / 2) { lp0 = 0.f; lp1 = -INFINITY; }
  }
  int v = N <= 64 ? (int)((e.smask >> k) & 1u) : (int)e.sg[k];
  if (k == e.f2p) v ^= 1;
  e.lp += (double)(v == 0 ? lp0 : lp1);
  if (a.cplx) {
    const float aa = v == 0 ? q0 + hb[2] : q1 + hb[3];
    e.ph += (double)(PI * aa / (1.f + fabsf(aa)));
  }
  e.nup += v == 0; e.ndn += v == 1;
  e.sprev = v;
}

// the term's contribution to E_loc of the sample (one lane per sequence)
__device__ inline void eloc_end(const ElocMArgs& a, const ElocSeq& e) {
  const double dre = 0.5 * (e.lp - e.oldlp);
  const double dim_ = (e.ph - e.oldph) + 3.14159265358979323846 * (double)e.dA;
  const double x = e.mel == 0.0 ? 0.0 : exp(dre);
  double* o = a.contrib + ((size_t)e.t * a.Ns + e.s) * 2;
  o[0] = e.mel * x * cos(dim_);
  o[1] = e.mel * x * sin(dim_);
}

template <int H, int DIM>
// 1D d_h <= 64: two waves per SIMD (at most 256 registers each); 2D keeps
// the whole register file for one wave (its split weight fragments, the
// gate-input product and the window of neighbour states)
__global__ __launch_bounds__(64 * (H / 32), (H <= 64 && DIM == 1) ? 2 : 1) void k_eloc_mfma(ElocMArgs a) {
  constexpr int S = 32;
  constexpr int HP = H + 4;
  constexpr int KS = H / 2;
  constexpr int KX = DIM == 1 ? 1 : 2;
  constexpr int NSTEP = 3 * KS + 3 * KX;
  __shared__ __align__(16) float hA[2][S][HP];
  __shared__ __align__(16) float hx[DIM == 2 ? S : 1][2 * H + 4];
  __shared__ __align__(16) float hw[4][H];
  __shared__ float hb[4];
  __shared__ float hmx[2][H / 32];   // 2D: largest |h'| of each wave at a site
  __shared__ int sqs[DIM == 2 ? S : 1];   // 2D: the item's sample of each sequence

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int half = lane >> 5, col = lane & 31;
  const int unit = 32 * w + col;
  const int N = a.N;
  const int NT = blockDim.x;

  // the gate products as FP16 hi/lo fragments (the split described at
  // k_eloc_mfma_w, same register footprint).  The 1D state lies in
  // [-1, 1]; the 2D gate input h' = U1 h_h + U2 h_v does not, so in 2D the
  // split operand is h' 2^-t with t from the site's largest |h'| over the
  // workgroup (t = 0 below 2^14) and the products are scaled back by 2^t
  constexpr bool SPLIT = true;
  constexpr int KJ = H / 16;
  float Wu[SPLIT ? KX : KS + KX], Wr[SPLIT ? KX : KS + KX], Wg[SPLIT ? 1 : KS], Wi[KX];
  f16x8_m Wuh[SPLIT ? KJ : 1], Wul[SPLIT ? KJ : 1], Wrh[SPLIT ? KJ : 1], Wrl[SPLIT ? KJ : 1],
      Wgh[SPLIT ? KJ : 1], Wgl[SPLIT ? KJ : 1];
  __shared__ unsigned wmax_bits;
  int sexp = 0;                         // some column of the workgroup is scaled
  float sdn[3] = {1.f, 1.f, 1.f}, sup[3] = {1.f, 1.f, 1.f};   // this lane's column, per gate
  {
    const float* base = a.mw + (size_t)w * NSTEP * 64 + lane;
    if constexpr (SPLIT) {
      const float* bw = a.mw + (size_t)w * NSTEP * 64;
      // input unit u = 16 j + 8 half + e sits at K-step u % KS, lane half u / KS
      auto wfrag = [&](int j, int e, int g) -> float {
        const int u = 16 * j + 8 * half + e;
        return bw[(size_t)(g * (KS + KX) + u % KS) * 64 + col + 32 * (u / KS)];
      };
      if (tid == 0) wmax_bits = 0u;
      __syncthreads();
      // FP16 holds magnitudes below 65504: the weights of an output column
      // (one unit of one gate) whose largest magnitude reaches 2^14 are
      // split as w 2^-s and that column's products scaled back by 2^s
      // (exact); a column's inputs sit in this lane and in lane ^ 32
      float mx[3] = {0.f, 0.f, 0.f};
      for (int j = 0; j < KJ; ++j)
        for (int e = 0; e < 8; ++e)
          for (int g = 0; g < 3; ++g) mx[g] = fmaxf(mx[g], fabsf(wfrag(j, e, g)));
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        mx[g] = fmaxf(mx[g], __shfl_xor(mx[g], 32, 64));
        const int se = mx[g] >= 16384.f ? min(ilogbf(mx[g]) - 13, 120) : 0;
        sdn[g] = ldexpf(1.f, -se);
        sup[g] = ldexpf(1.f, se);
      }
      // non-negative floats order as their bits
      atomicMax(&wmax_bits, __float_as_uint(fmaxf(mx[0], fmaxf(mx[1], mx[2]))));
      __syncthreads();
      sexp = __uint_as_float(wmax_bits) >= 16384.f ? 1 : 0;
#pragma unroll
      for (int j = 0; j < KJ; ++j) {
        float xu[8], xr[8], xg[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          xu[e] = wfrag(j, e, 0) * sdn[0];
          xr[e] = wfrag(j, e, 1) * sdn[1];
          xg[e] = wfrag(j, e, 2) * sdn[2];
        }
        split_f16(xu, Wuh[j], Wul[j]);
        split_f16(xr, Wrh[j], Wrl[j]);
        split_f16(xg, Wgh[j], Wgl[j]);
      }
#pragma unroll
      for (int s = 0; s < KX; ++s) {
        Wu[s] = base[(size_t)(KS + s) * 64];
        Wr[s] = base[(size_t)(KS + KX + KS + s) * 64];
      }
    } else {
#pragma unroll
      for (int s = 0; s < KS + KX; ++s) Wu[s] = base[(size_t)s * 64];
#pragma unroll
      for (int s = 0; s < KS + KX; ++s) Wr[s] = base[(size_t)(KS + KX + s) * 64];
#pragma unroll
      for (int s = 0; s < KS; ++s) Wg[s] = base[(size_t)(2 * (KS + KX) + s) * 64];
    }
#pragma unroll
    for (int s = 0; s < KX; ++s) Wi[s] = base[(size_t)(2 * (KS + KX) + KS + s) * 64];
  }
  constexpr int XO = SPLIT ? 0 : KS;   // index of the first one-hot fragment in Wu, Wr
  const float bu = a.bias[unit], br = a.bias[H + unit], bh = a.bias[2 * H + unit];
  const float bi = a.bias[3 * H + unit];
  const float bgs = (float)(2.8853900817779268 * (double)bh);   // 2 log2(e) b_h
  for (int i = tid; i < 4 * H; i += NT) hw[i / H][i % H] = a.head[i];
  if (tid < 4) hb[tid] = a.headb[tid];
  __syncthreads();

  const int n_items = a.list ? a.count[a.M] : a.n_items;
  // instantiated with and without the weight scaling (no branch between
  // the products in the common case)
  auto items = [&](auto scaled) {
  for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
    ElocSeq e = eloc_begin(a, item, col);
    const int k0 = e.k0, f1 = e.f1, f2p = e.f2p;
    const uint8_t* sg = e.sg;
    // 2D: this thread's share (sequence i / H, unit i % H for i = tid +
    // 2H m; the block has 2H threads) of the vertical predecessor of site
    // k2, requested a site ahead, unless that predecessor is site k2 - 1
    // (then the state is in shared memory)
    // (four units per request: thread tid takes sequence i / (H / 4), units
    // 4 (i % (H / 4)) .. + 3 for i = tid + 2H m)
    constexpr int PFN = DIM == 2 ? S / 8 : 1;
    float4 pf[PFN];
    if (DIM == 2) {
      if (tid < S) sqs[tid] = eloc_row_sample(a, e, tid);
      __syncthreads();
    }
    auto prefetch_v = [&](int k2) {
      const int kv2 = a.nbr[2 * k2 + 1];
      if (kv2 < 0 || kv2 == k2 - 1) return;
#pragma unroll
      for (int mm = 0; mm < PFN; ++mm) {
        const int i = tid + 2 * H * mm;
        const int q = i / (H / 4), u = 4 * (i % (H / 4));
        const float* src = kv2 <= k0 ? a.states + ((size_t)sqs[q] * N + kv2) * H + u
                                     : a.ring + (((size_t)blockIdx.x * S + q) * a.W + kv2 % a.W) * H + u;
        pf[mm] = *reinterpret_cast<const float4*>(src);
      }
    };
    // the state of the last unflipped site (2D: the horizontal predecessor
    // of site k0 + 1 unless that site starts a row)
    if (k0 + 1 < N) {
      // four units per request, all requested before any is stored
      constexpr int NTL = 64 * (H / 32), PV = S * H / 4 / NTL;   // NTL: the launch's block size
      float4 pv[PV];
#pragma unroll
      for (int m = 0; m < PV; ++m) {
        const int i = tid + NTL * m, q = i / (H / 4), u = 4 * (i % (H / 4));
        const int sq = eloc_row_sample(a, e, q);
        pv[m] = *reinterpret_cast<const float4*>(&a.states[((size_t)sq * N + k0) * H + u]);
      }
#pragma unroll
      for (int m = 0; m < PV; ++m) {
        const int i = tid + NTL * m, q = i / (H / 4), u = 4 * (i % (H / 4));
        *reinterpret_cast<float4*>(&hA[(k0 + 1) & 1][q][u]) = pv[m];
      }
      if (DIM == 2) prefetch_v(k0 + 1);
    }
    __syncthreads();

    for (int k = k0 + 1; k < N; ++k) {
      const int cb = k & 1, nb = cb ^ 1;
      f32x16_m hin;
      int sh = -1, sv = -1;
      if (DIM == 2) {
        const int kh = a.nbr[2 * k], kv = a.nbr[2 * k + 1];
        if (kh >= 0) { sh = sg[kh]; if (kh == f1 || kh == f2p) sh ^= 1; }
        if (kv >= 0) { sv = sg[kv]; if (kv == f1 || kv == f2p) sv ^= 1; }
        // a predecessor at site k - 1 is the state this workgroup wrote to
        // shared memory at the last site (or loaded above for k0 + 1); older
        // ones come from the stored states (at or before k0) or the window
        // (the vertical one, when older, was requested at the last site)
#pragma unroll
        for (int mm = 0; mm < PFN; ++mm) {
          const int i = tid + 2 * H * mm;
          const int q = i / (H / 4), u = 4 * (i % (H / 4));
          const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
          float4 vh = z, vv = z;
          if (kh == k - 1) {
            vh = *reinterpret_cast<const float4*>(&hA[cb][q][u]);
          } else if (kh >= 0) {
            const float* src = kh <= k0 ? a.states + ((size_t)sqs[q] * N + kh) * H + u
                                        : a.ring + (((size_t)blockIdx.x * S + q) * a.W + kh % a.W) * H + u;
            vh = *reinterpret_cast<const float4*>(src);
          }
          if (kv == k - 1) vv = *reinterpret_cast<const float4*>(&hA[cb][q][u]);
          else if (kv >= 0) vv = pf[mm];
          *reinterpret_cast<float4*>(&hx[q][u]) = vh;
          *reinterpret_cast<float4*>(&hx[q][H + u]) = vv;
        }
        mf16::lds_barrier();
        f32x16_m acc;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = 0.f;
        const float* m2 = a.m2 + (size_t)w * H * 64 + lane;
#pragma unroll 4
        for (int s4 = 0; s4 < H; s4 += 4) {
          const float4 av = *reinterpret_cast<const float4*>(&hx[col][s4 + half * H]);
          acc = mfma_f32(av.x, m2[(size_t)(s4 + 0) * 64], acc);
          acc = mfma_f32(av.y, m2[(size_t)(s4 + 1) * 64], acc);
          acc = mfma_f32(av.z, m2[(size_t)(s4 + 2) * 64], acc);
          acc = mfma_f32(av.w, m2[(size_t)(s4 + 3) * 64], acc);
        }
        hin = acc;
        // the next site's vertical predecessor is requested now, after this
        // site's streamed weight loads, so no wait for those also waits for
        // it; it arrives while the gate products and the cell run
        if (k + 1 < N) prefetch_v(k + 1);
        float m = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          hA[cb][(q / 4) * 8 + half * 4 + (q % 4)][unit] = hin[q];
          m = fmaxf(m, fabsf(hin[q]));
        }
        m = mf16::row16_max(m);
        if (lane == 0) {
          const float m1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 16));
          const float m2v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 32));
          const float m3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 48));
          hmx[cb][w] = fmaxf(fmaxf(m, m1), fmaxf(m2v, m3));
        }
        mf16::lds_barrier();
      }
      // gate pre-activations of the 32 sequences for this wave's units (1D:
      // scaled for exp2, biases of u, r and the input term in the one-hot
      // fragments, so those accumulators start from zero)
      f32x16_m au, ar, ag, ai;
      // 2D: the split operand's power-of-two scale at this site
      float hdn = 1.f, hup = 1.f;
      if (DIM == 2) {
        float mx = hmx[cb][0];
#pragma unroll
        for (int v = 1; v < H / 32; ++v) mx = fmaxf(mx, hmx[cb][v]);
        const int t = mx >= 16384.f ? min(ilogbf(mx) - 13, 120) : 0;
        hdn = ldexpf(1.f, -t);
        hup = ldexpf(1.f, t);
      }
      if (DIM == 1) {
#pragma unroll
        for (int q = 0; q < 16; ++q) { au[q] = 0.f; ar[q] = 0.f; ag[q] = bgs * sdn[2]; ai[q] = 0.f; }
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) { au[q] = 0.f; ar[q] = 0.f; ag[q] = 0.f; ai[q] = bi; }
      }
      if constexpr (SPLIT) {
#pragma unroll
        for (int j = 0; j < KJ; ++j) {
          const float4 x0 = *reinterpret_cast<const float4*>(&hA[cb][col][16 * j + 8 * half]);
          const float4 x1 = *reinterpret_cast<const float4*>(&hA[cb][col][16 * j + 8 * half + 4]);
          float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
          if (DIM == 2) {
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] *= hdn;
          }
          f16x8_m ahi, alo;
          split_f16(x, ahi, alo);
          au = mfma_f16(alo, Wuh[j], au); ar = mfma_f16(alo, Wrh[j], ar); ag = mfma_f16(alo, Wgh[j], ag);
          au = mfma_f16(ahi, Wul[j], au); ar = mfma_f16(ahi, Wrl[j], ar); ag = mfma_f16(ahi, Wgl[j], ag);
          au = mfma_f16(ahi, Wuh[j], au); ar = mfma_f16(ahi, Wrh[j], ar); ag = mfma_f16(ahi, Wgh[j], ag);
        }
        if (DIM == 2) {
          // back to the unscaled products, then the biases
          const float su = sup[0] * hup, sr = sup[1] * hup, sgs = sup[2] * hup;
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            au[q] = fmaf(au[q], su, bu); ar[q] = fmaf(ar[q], sr, br); ag[q] = fmaf(ag[q], sgs, bh);
          }
        } else if constexpr (decltype(scaled)::value) {
#pragma unroll
          for (int q = 0; q < 16; ++q) { au[q] *= sup[0]; ar[q] *= sup[1]; ag[q] *= sup[2]; }
        }
      } else {
#pragma unroll
        for (int s4 = 0; s4 < KS; s4 += 4) {
          const float4 av = *reinterpret_cast<const float4*>(&hA[cb][col][s4 + half * KS]);
          au = mfma_f32(av.x, Wu[s4 + 0], au); ar = mfma_f32(av.x, Wr[s4 + 0], ar); ag = mfma_f32(av.x, Wg[s4 + 0], ag);
          au = mfma_f32(av.y, Wu[s4 + 1], au); ar = mfma_f32(av.y, Wr[s4 + 1], ar); ag = mfma_f32(av.y, Wg[s4 + 1], ag);
          au = mfma_f32(av.z, Wu[s4 + 2], au); ar = mfma_f32(av.z, Wr[s4 + 2], ar); ag = mfma_f32(av.z, Wg[s4 + 2], ag);
          au = mfma_f32(av.w, Wu[s4 + 3], au); ar = mfma_f32(av.w, Wr[s4 + 3], ar); ag = mfma_f32(av.w, Wg[s4 + 3], ag);
        }
      }
      // one-hot spin inputs: this lane supplies column c = 2x + half
      if (DIM == 1) {
        const float o = e.sprev == half ? 1.f : 0.f;
        au = mfma_f32(o, Wu[XO], au); ar = mfma_f32(o, Wr[XO], ar); ai = mfma_f32(o, Wi[0], ai);
      } else {
        const float o0 = sh == half ? 1.f : 0.f;
        const float o1 = sv == half ? 1.f : 0.f;
        au = mfma_f32(o0, Wu[XO], au); ar = mfma_f32(o0, Wr[XO], ar); ai = mfma_f32(o0, Wi[0], ai);
        au = mfma_f32(o1, Wu[XO + 1], au); ar = mfma_f32(o1, Wr[XO + 1], ar); ai = mfma_f32(o1, Wi[1], ai);
      }
      // GRU update in the accumulator layout: element q is sequence
      // (q / 4) * 8 + half * 4 + q % 4, unit `unit`
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int row = (q / 4) * 8 + half * 4 + (q % 4);
        const float hp = DIM == 1 ? hA[cb][row][unit] : hin[q];
        float hn;
        if (DIM == 1) {
          // pre-scaled: u = 1 / (1 + 2^au), tanh y = 1 - 2 / (1 + 2^y')
          const float u = __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(au[q]));
          const float rr = __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(ar[q]));
          const float y = fmaf(rr, ag[q], ai[q]);
          const float ht = fmaf(-2.f, __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(y)), 1.f);
          hn = fmaf(u, ht - hp, hp);
        } else {
          const float u = fast_sigmoid(au[q]);
          const float rr = fast_sigmoid(ar[q]);
          const float ht = fast_tanh(rr * ag[q] + ai[q]);
          hn = (1.f - u) * hp + u * ht;
        }
        hA[nb][row][unit] = hn;
        if (DIM == 2) a.ring[(((size_t)blockIdx.x * S + row) * a.W + k % a.W) * H + unit] = hn;
      }
      __syncthreads();
      eloc_site<H>(a, e, &hA[nb][col][0], hw, hb, half, k);
    }
    if (w == 0 && half == 0 && e.act) eloc_end(a, e);
    __syncthreads();
  }
  };
  if (sexp) items(std::true_type{});
  else items(std::false_type{});
}

// 1D models, d_h <= 64: each wave re-evaluates its own item (32 connected
// configurations that share their first flipped site) over all d_h units,
// so a wave never waits for another between sites.  The state products run
// on v_mfma_f32_32x32x16_f16 with every FP32 operand split into an FP16
// pair x = x_hi + x_lo (both rounded to nearest): the three terms
// a_hi b_hi + a_hi b_lo + a_lo b_hi, accumulated in FP32, represent each
// operand to 2^-22 of its size (the omitted a_lo b_lo is below 2^-22 of
// the product), against 2^-24 for FP32 operands, at 3/16 of the matrix-core
// cycles of the FP32 product.  The one-hot input step stays an FP32 product
// (its operand is exactly 0 or 1).  The workgroup's eight waves share one
// copy of the split B-operand fragments of W_u, W_r, W_h and of the one-hot
// columns in shared memory (eight input units per 16-byte read); each wave
// keeps the 32 x d_h state of its sequences in its own buffer,
// updated in place (a wave reads all of it into the matrix products before
// it writes the new state).  Items are dealt by position p: even positions
// take items from the front of the list (term t restarts at site t, so the
// longest first), odd ones from the back, and the two waves that share a
// SIMD take positions 2q and 2q + 1, so their lengths add up to about the
// same everywhere.  Positions beyond the first round come from a counter;
// the last wave to finish resets it for the next launch.
constexpr int EW_WAVES = 8;
// s_getreg operand for the SIMD id (bits 5:4 of HW_ID): any value yields a
// permutation of the first-round positions, the id only balances them
constexpr int HWREG_SIMD_ID = 4 | (4 << 6) | (1 << 11);

template <int H>
__global__ __launch_bounds__(64 * EW_WAVES, 2) void k_eloc_mfma_w(ElocMArgs a, uint32_t* queue) {
  constexpr int S = 32;
  constexpr int HP = H + 4;
  constexpr int KS = H / 2;
  constexpr int NCB = H / 32;              // 32-unit column blocks
  constexpr int NSTEP = 3 * KS + 3;
  constexpr int KJ = H / 16;               // K-steps of the FP16 products
  __shared__ __align__(16) f16x8_m Bh[NCB][3][KJ][2][64];   // u, r, h: hi and lo parts
  __shared__ __align__(16) float Bx[NCB][3][64];            // one-hot step of u, r, input
  __shared__ __align__(16) float hS[EW_WAVES][S][HP];
  __shared__ __align__(16) float hw[4][H];
  __shared__ float hb[4];
  __shared__ float bgs_s[H];
  __shared__ int simd_of[EW_WAVES];
  __shared__ int sqw[EW_WAVES][S];          // samples of the rows of each wave's item
  __shared__ unsigned wmax_bits;
  __shared__ unsigned colmax[NCB][3][32];   // largest |w| of each output column
  __shared__ float csc[2][NCB][3][32];      // its scale 2^-s and 2^s

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (lane == 0) simd_of[w] = (int)(__builtin_amdgcn_s_getreg(HWREG_SIMD_ID) & 3);
  const int half = lane >> 5, col = lane & 31;
  const int N = a.N;
  // FP16 holds magnitudes below 65504 (the state lies in [-1, 1]): the
  // weights of an output column (one unit of one gate) whose largest
  // magnitude reaches 2^14 are staged again as w 2^-s and that column's
  // state products scaled back by 2^s, both exact powers of two
  if (tid == 0) wmax_bits = 0u;
  for (int i = tid; i < NCB * 3 * 32; i += 64 * EW_WAVES) (&colmax[0][0][0])[i] = 0u;
  __syncthreads();
  // B fragment of K-step j, lane l = n + 32 c, element e: input unit
  // u = 16 j + 8 c + e, output unit 32 cb + n.  In the packed FP32 layout
  // that entry sits at K-step u % KS in lane n + 32 (u / KS).
  // scaled == false: stage unscaled and record the column maxima
  auto stage = [&](bool scaled) {
    float mx = 0.f;
    for (int i = tid; i < NCB * 3 * KJ * 64; i += 64 * EW_WAVES) {
      const int l = i % 64, j = (i / 64) % KJ, g = (i / (64 * KJ)) % 3, cb = i / (64 * KJ * 3);
      const int n = l & 31, c = l >> 5;
      const float* base = a.mw + (size_t)cb * NSTEP * 64 + n;
      const int off = g == 0 ? 0 : g == 1 ? KS + 1 : 2 * (KS + 1);
      const float sc = scaled ? csc[0][cb][g][n] : 1.f;
      float x[8], cm = 0.f;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int u = 16 * j + 8 * c + e;
        x[e] = base[(size_t)(off + u % KS) * 64 + 32 * (u / KS)];
        cm = fmaxf(cm, fabsf(x[e]));
        x[e] *= sc;
      }
      // non-negative floats order as their bits
      if (!scaled) atomicMax(&colmax[cb][g][n], __float_as_uint(cm));
      mx = fmaxf(mx, cm);
      split_f16(x, Bh[cb][g][j][0][l], Bh[cb][g][j][1][l]);
    }
    if (!scaled) atomicMax(&wmax_bits, __float_as_uint(mx));
  };
  stage(false);
  for (int i = tid; i < NCB * 3 * 64; i += 64 * EW_WAVES) {
    const int l = i % 64, g = (i / 64) % 3, cb = i / (64 * 3);
    const float* base = a.mw + (size_t)cb * NSTEP * 64 + l;
    const int off = g == 0 ? KS : g == 1 ? 2 * KS + 1 : 3 * KS + 2;
    Bx[cb][g][l] = base[(size_t)off * 64];
  }
  for (int i = tid; i < 4 * H; i += 64 * EW_WAVES) hw[i / H][i % H] = a.head[i];
  for (int i = tid; i < H; i += 64 * EW_WAVES) bgs_s[i] = (float)(2.8853900817779268 * (double)a.bias[2 * H + i]);
  if (tid < 4) hb[tid] = a.headb[tid];
  __syncthreads();
  for (int i = tid; i < NCB * 3 * 32; i += 64 * EW_WAVES) {
    const float cm = __uint_as_float((&colmax[0][0][0])[i]);
    const int se = cm >= 16384.f ? min(ilogbf(cm) - 13, 120) : 0;
    (&csc[0][0][0][0])[i] = ldexpf(1.f, -se);
    (&csc[1][0][0][0])[i] = ldexpf(1.f, se);
  }
  const int sexp = __uint_as_float(wmax_bits) >= 16384.f ? 1 : 0;   // some column is scaled
  __syncthreads();
  if (sexp) {
    stage(true);
    __syncthreads();
  }
  // this lane's column scales of every block and gate
  float sdn[NCB][3], sup[NCB][3];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      sdn[cb][g] = csc[0][cb][g][col];
      sup[cb][g] = csc[1][cb][g][col];
    }

  float (*hA)[HP] = hS[w];
  // the wave's own shared-memory writes visible to all its lanes
  auto wave_sync = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  const int n_items = a.list ? a.count[a.M] : a.n_items;
  // rank of this wave among the workgroup's, ordered by (SIMD, wave)
  int rank = 0;
  {
    const int me = simd_of[w];
#pragma unroll
    for (int v = 0; v < EW_WAVES; ++v) rank += simd_of[v] < me || (simd_of[v] == me && v < w);
  }
  const int first_round = (int)gridDim.x * EW_WAVES;
  // the site loop is instantiated with and without the weight scaling, so
  // the unscaled case carries no branch between its products
  auto items = [&](auto scaled) {
  for (int p = (int)blockIdx.x * EW_WAVES + rank; p < n_items;) {
    const int item = (p & 1) ? n_items - 1 - (p >> 1) : (p >> 1);
    ElocSeq e = eloc_begin(a, item, col);
    const int k0 = e.k0;
    if (k0 + 1 < N) {
      // the prefix states, four units per request: the rows' samples go
      // through shared memory first, then four requests are made before any
      // of them is stored (named values, so they stay in registers)
      if (lane < S) sqw[w][lane] = eloc_row_sample(a, e, lane);
      wave_sync();
      constexpr int PV = S * H / 4 / 64;
      auto ld = [&](int m) {
        const int i = lane + 64 * m, q = i / (H / 4), u = 4 * (i % (H / 4));
        return *reinterpret_cast<const float4*>(&a.states[((size_t)sqw[w][q] * N + k0) * H + u]);
      };
      auto stv = [&](int m, float4 v) {
        const int i = lane + 64 * m, q = i / (H / 4), u = 4 * (i % (H / 4));
        *reinterpret_cast<float4*>(&hA[q][u]) = v;
      };
#pragma unroll
      for (int m0 = 0; m0 < PV; m0 += 4) {
        const float4 p0 = ld(m0), p1 = ld(m0 + 1), p2 = ld(m0 + 2), p3 = ld(m0 + 3);
        stv(m0, p0);
        stv(m0 + 1, p1);
        stv(m0 + 2, p2);
        stv(m0 + 3, p3);
      }
    }
    wave_sync();
    for (int k = k0 + 1; k < N; ++k) {
      f32x16_m au[NCB], ar[NCB], ag[NCB], ai[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const float g0 = bgs_s[32 * cb + col] * sdn[cb][2];
#pragma unroll
        for (int q = 0; q < 16; ++q) { au[cb][q] = 0.f; ar[cb][q] = 0.f; ag[cb][q] = g0; ai[cb][q] = 0.f; }
      }
#pragma unroll
      for (int j = 0; j < KJ; ++j) {
        // A fragment: sequence col, input units 16 j + 8 half .. + 7
        const float4 x0 = *reinterpret_cast<const float4*>(&hA[col][16 * j + 8 * half]);
        const float4 x1 = *reinterpret_cast<const float4*>(&hA[col][16 * j + 8 * half + 4]);
        const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        f16x8_m ahi, alo;
        split_f16(x, ahi, alo);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const f16x8_m uh = Bh[cb][0][j][0][lane], ul = Bh[cb][0][j][1][lane];
          const f16x8_m rh = Bh[cb][1][j][0][lane], rl = Bh[cb][1][j][1][lane];
          const f16x8_m gh = Bh[cb][2][j][0][lane], gl = Bh[cb][2][j][1][lane];
          au[cb] = mfma_f16(alo, uh, au[cb]); ar[cb] = mfma_f16(alo, rh, ar[cb]); ag[cb] = mfma_f16(alo, gh, ag[cb]);
          au[cb] = mfma_f16(ahi, ul, au[cb]); ar[cb] = mfma_f16(ahi, rl, ar[cb]); ag[cb] = mfma_f16(ahi, gl, ag[cb]);
          au[cb] = mfma_f16(ahi, uh, au[cb]); ar[cb] = mfma_f16(ahi, rh, ar[cb]); ag[cb] = mfma_f16(ahi, gh, ag[cb]);
        }
      }
      if constexpr (decltype(scaled)::value) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            au[cb][q] *= sup[cb][0]; ar[cb][q] *= sup[cb][1]; ag[cb][q] *= sup[cb][2];
          }
      }
      {
        const float o = e.sprev == half ? 1.f : 0.f;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          au[cb] = mfma_f32(o, Bx[cb][0][lane], au[cb]);
          ar[cb] = mfma_f32(o, Bx[cb][1][lane], ar[cb]);
          ai[cb] = mfma_f32(o, Bx[cb][2][lane], ai[cb]);
        }
      }
      // GRU update in the accumulator layout, in place: element q of block cb
      // is sequence (q / 4) * 8 + half * 4 + q % 4, unit 32 cb + col
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int unit = 32 * cb + col;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int row = (q / 4) * 8 + half * 4 + (q % 4);
          const float hp = hA[row][unit];
          const float u = __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(au[cb][q]));
          const float rr = __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(ar[cb][q]));
          const float y = fmaf(rr, ag[cb][q], ai[cb][q]);
          const float ht = fmaf(-2.f, __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(y)), 1.f);
          hA[row][unit] = fmaf(u, ht - hp, hp);
        }
      }
      wave_sync();
      eloc_site<H>(a, e, &hA[col][0], hw, hb, half, k);
      wave_sync();   // the head's reads precede the next state's writes
    }
    if (half == 0 && e.act) eloc_end(a, e);
    int next = 0;
    if (lane == 0) next = (int)atomicAdd(&queue[0], 1u);
    p = first_round + __builtin_amdgcn_readfirstlane(next);
  }
  };
  if (sexp) items(std::true_type{});
  else items(std::false_type{});
  // the last wave out resets the counter for the next launch
  if (lane == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t done = atomicAdd(&queue[1], 1u);
    if (done + 1 == gridDim.x * EW_WAVES) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      atomicExch(&queue[0], 0u);
      atomicExch(&queue[1], 0u);
    }
  }
}

// J1-J2 exchange terms vanish unless the pair is antiparallel: per term,
// the samples with sigma_a != sigma_b in ascending order (one workgroup per
// term, block-wide scan); the other samples' contributions are zeroed here.
__global__ __launch_bounds__(1024) void k_eloc_compact(const uint8_t* sigma, const int* bonds,
                                                       int N, int Ns, int* list, int* count,
                                                       double* contrib) {
  __shared__ int wsum[16];
  __shared__ int base;
  const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int fa = bonds[2 * t], fb = bonds[2 * t + 1];
  if (tid == 0) base = 0;
  __syncthreads();
  for (int s0 = 0; s0 < Ns; s0 += 1024) {
    const int s = s0 + tid;
    int flag = 0;
    if (s < Ns) {
      const uint8_t* sg = sigma + (size_t)s * N;
      flag = sg[fa] != sg[fb];
      if (!flag) {
        contrib[((size_t)t * Ns + s) * 2] = 0.0;
        contrib[((size_t)t * Ns + s) * 2 + 1] = 0.0;
      }
    }
    // inclusive scan within the wave, then across waves
    int x = flag;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int off = base;
    for (int i = 0; i < wv; ++i) off += wsum[i];
    if (flag) list[(size_t)t * Ns + off + x - 1] = s;
    __syncthreads();
    if (tid == 0) {
      int tot = 0;
      for (int i = 0; i < 16; ++i) tot += wsum[i];
      base += tot;
    }
    __syncthreads();
  }
  if (tid == 0) count[t] = base;
}

// item table (term, chunk) over the compacted lists; the total goes to count[M]
__global__ __launch_bounds__(1024) void k_eloc_items(int* count, int M, int* items) {
  __shared__ int start[1025];
  const int tid = threadIdx.x;
  if (tid == 0) {
    int acc = 0;
    for (int t = 0; t < M; ++t) { start[t] = acc; acc += (count[t] + 31) / 32; }
    start[M] = acc;
  }
  __syncthreads();
  for (int t = tid; t < M; t += 1024) {
    const int nc = start[t + 1] - start[t];
    for (int c = 0; c < nc; ++c) {
      items[2 * (start[t] + c)] = t;
      items[2 * (start[t] + c) + 1] = c;
    }
  }
  if (tid == 0) count[M] = start[M];
}

bool eloc_mfma_supported(minsr_model* m) {
  return !m->f64 && (m->H == 32 || m->H == 64 || m->H == 128);
}

int launch_eloc_mfma(minsr_model* m, const minsr_hamiltonian* H, int Ns, const uint8_t* sigma,
                     const void* states, const double* site, int M, hipStream_t s) {
  ElocMArgs a{};
  const Work<float>& w = m->wf;
  a.mw = w.mw; a.m2 = w.m2; a.bias = w.bias; a.head = w.head; a.headb = w.headb;
  a.N = m->N; a.Ns = Ns; a.zero_mag = m->d.zero_mag; a.cplx = m->cplx;
  a.marshall = m->d.marshall;
  a.nchunks = (Ns + 31) / 32;
  a.n_items = a.nchunks * M;
  a.W = 2 * m->d.Lx;
  a.nbr = m->nbr; a.subA = m->subA; a.sigma = sigma; a.states = (const float*)states;
  a.site = site; a.bonds = m->bonds; a.n_nn = m->n_nn; a.ham_kind = H->kind;
  a.hx = H->h; a.J1 = H->J; a.J2 = H->J2; a.contrib = m->contrib; a.ring = (float*)m->ring;
  a.M = M;
  if (a.n_items == 0) return MINSR_OK;
  if (H->kind == MINSR_HAM_J1J2) {
    if (M > 1024) return fail(MINSR_E_UNSUPPORTED, "more than 1024 exchange terms");
    k_eloc_compact<<<M, 1024, 0, s>>>(sigma, m->bonds, m->N, Ns, m->elist, m->ecount, m->contrib);
    MINSR_CHECK_LAUNCH();
    k_eloc_items<<<1, 1024, 0, s>>>(m->ecount, M, m->eitems);
    MINSR_CHECK_LAUNCH();
    a.list = m->elist; a.count = m->ecount; a.items = m->eitems;
  }
  if (m->dim == 1 && m->H <= 64) {
    // one workgroup of eight independent waves per compute unit (the shared
    // weights and eight state buffers fill most of its shared memory)
    static int ncu = 0;
    if (ncu == 0) {
      int dev = 0, v = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
        ncu = v;
      else
        ncu = 256;
    }
    unsigned grid = std::min<unsigned>((unsigned)ncu, (unsigned)((a.n_items + EW_WAVES - 1) / EW_WAVES));
    if (m->tune_eloc_grid > 0) grid = std::min<unsigned>(grid, (unsigned)m->tune_eloc_grid);
    if (m->H == 32) k_eloc_mfma_w<32><<<grid, 64 * EW_WAVES, 0, s>>>(a, m->eloc_q);
    else k_eloc_mfma_w<64><<<grid, 64 * EW_WAVES, 0, s>>>(a, m->eloc_q);
    MINSR_CHECK_LAUNCH();
    return MINSR_OK;
  }
  unsigned grid = (unsigned)a.n_items;
  if (m->tune_eloc_grid > 0) grid = std::min<unsigned>(grid, (unsigned)m->tune_eloc_grid);
  if (m->dim == 2) {
    const int cap = m->ring_blocks / 32;
    if (cap < 1) return fail(MINSR_E_SHAPE, "recompute window too small");
    grid = std::min<unsigned>(grid, (unsigned)cap);
  }
  const unsigned nt = 64u * (unsigned)(m->H / 32);
#define MINSR_ELOC_MFMA(HH, DD) k_eloc_mfma<HH, DD><<<grid, nt, 0, s>>>(a)
  if (m->dim == 1) {
    MINSR_ELOC_MFMA(128, 1);
  } else {
    if (m->H == 32) MINSR_ELOC_MFMA(32, 2);
    else if (m->H == 64) MINSR_ELOC_MFMA(64, 2);
    else MINSR_ELOC_MFMA(128, 2);
  }
#undef MINSR_ELOC_MFMA
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

}  // namespace minsr
