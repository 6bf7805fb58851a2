// Per-sample log-derivatives of 1D FP32 models with d_h = 128 on the matrix
// cores (Sec. 2.3, Alg. 1 step 5; the cell of App. A), in two launches.
//
// k_jac_rev: a workgroup takes 16 rows of O at once: 16 samples of a model
// with a real head, or 8 samples times the two outputs (log-modulus and
// phase) of a cRNN.  It walks the chain backwards one checkpoint segment at
// a time: the segment's hidden states are recomputed forward from the stored
// checkpoint into shared memory, then the reverse pass runs site by site.
// At every site the gate pre-activations of the 16 rows are one
// [16 x d_h] x [d_h x 3 d_h] product, recomputed from h_{k-1} (the same
// instructions on the same inputs as the forward recomputation, so the same
// values), and the adjoint of the cell input is one [16 x 3 d_h] x
// [3 d_h x d_h] product with the transposed gate weights.  Both run on
// v_mfma_f32_16x16x32_f16 with every FP32 operand split into an FP16 pair
// x = hi + lo (three products a_hi b_hi + a_hi b_lo + a_lo b_hi, FP32
// accumulation; operands to 2^-22 of their size).  Wave w owns hidden
// units 16w..16w+15 and keeps, for the whole kernel, its B-operand
// fragments of the gate rows of those units (forward) and of the weight
// columns of those units (reverse) in registers.  The gate adjoints of each
// row are scaled by a power of two from the row's largest before they are
// split, so they never leave FP16's range; weight columns reaching 2^14 are
// scaled the same way.  The kernel forms no row of O: it writes the four
// gate adjoints of every (row, site), the head adjoints, and the recomputed
// hidden states of the non-checkpoint sites (into the state buffer).
//
// k_jac_rows: one workgroup per sample assembles its rows of O: the W_u,
// W_r, W_h blocks as sums over sites of gate adjoint x previous state
// (split FP16 products on the matrix cores, each gate row j scaled by a
// power of two from its largest adjoint over the sites), the one-hot input
// columns, W_in and the biases as FP32 sums over sites, and the output head
// from the head adjoints and the states.
#include <cmath>
#include <mutex>

#include "model.hpp"

namespace minsr {

namespace {

typedef __attribute__((ext_vector_type(8))) _Float16 jh8;
typedef __attribute__((ext_vector_type(2))) _Float16 jh2;
typedef __attribute__((ext_vector_type(2))) float jf2;
typedef __attribute__((ext_vector_type(4))) float jf4;

constexpr int JM_H = 128;       // hidden width of this path
constexpr int JM_SEG = 16;      // longest checkpoint segment
constexpr int JM_KMAX = 128;    // longest chain of the row assembly

__device__ __forceinline__ jf4 jmma(jh8 a, jh8 b, jf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// x = hi + lo, both rounded to nearest FP16; x - hi is exact in FP32
__device__ __forceinline__ void jsplit(const float (&x)[8], jh8& hi, jh8& lo) {
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const jf2 v = {x[e], x[e + 1]};
    const jh2 h = __builtin_convertvector(v, jh2);
    const jh2 l = __builtin_convertvector(v - __builtin_convertvector(h, jf2), jh2);
    hi[e] = h[0]; hi[e + 1] = h[1];
    lo[e] = l[0]; lo[e + 1] = l[1];
  }
}

// hardware exp2 and reciprocal (about 1 ulp each)
__device__ __forceinline__ float jsig(float x) {
  return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(-1.4426950408889634f * x));
}
__device__ __forceinline__ float jtanh(float y) {
  return 1.f - 2.f * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(2.8853900817779268f * y));
}

// power-of-two exponent that brings a largest magnitude m into [2^14, 2^15)
__device__ __forceinline__ int jexp_for(float m) {
  return m > 0.f ? min(max(14 - ilogbf(m), -120), 120) : 0;
}

}  // namespace

struct JRevArgs {
  const float* fw;
  const float* bw;
  const float* xc;
  const float* bias;
  const float* head;
  const float* headb;
  int N, Ns, C;
  const uint8_t* sigma;
  float* states;         // [Ns][N][H]: rows k with (k + 1) % C == 0 read, the others written
  const double* site;    // [Ns][N][4]: log p(0), log p(1) of the forward pass (masked)
  float* dpt;            // [rows][N][4][H]: adjoints of the u, r pre-activations, of
                         // W_h h + b_h and of the candidate's pre-activation
  float* dzt;            // [rows][N][2]: adjoints of the two head outputs
};

template <bool CPLX>
__global__ __launch_bounds__(512, 1) void k_jac_rev(JRevArgs a) {
  constexpr int H = JM_H, NW = H / 16, KF = H / 32, KR = 3 * H / 32;
  constexpr int S = CPLX ? 8 : 16;     // samples per workgroup (16 rows)
  constexpr int HP = H + 4;            // state row pitch (floats)
  constexpr int DP = 3 * H + 4;        // gate-adjoint row pitch
  constexpr int SGP = JM_SEG + 1;
  constexpr int NT = 64 * NW;
  extern __shared__ __align__(16) float jsm[];
  const int C = a.C, N = a.N, Ns = a.Ns;
  float* hs = jsm;                                 // [C + 1][S][HP]: h_{ks-1+kk}
  float* dps = hs + (size_t)(C + 1) * S * HP;      // [2][16][DP] gate adjoints of a site
  float* rmx = dps + 2 * 16 * DP;                  // [2][NW][16] their row maxima per wave
  float* dzs = rmx + 2 * NW * 16;                  // [JM_SEG][16][2] head adjoints
  float* cst = dzs + JM_SEG * 32;                  // [13][H] biases and one-hot columns
  int* sgs = reinterpret_cast<int*>(cst + 13 * H); // [S][SGP] sigma_{ks-1+kk}, 2 before site 0

  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int n = l & 15, kq = l >> 4;
  const int j = 16 * w + n;            // this lane's hidden unit (gate row / state column)
  const int s0 = blockIdx.x * S;

  // cst rows: b_u, b_r, b_h, b_in, then for u, r, in the input columns of
  // spin values 0, 1 and zeros (no input at site 0)
  for (int i = tid; i < H; i += NT) {
#pragma unroll
    for (int g = 0; g < 4; ++g) cst[g * H + i] = a.bias[g * H + i];
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      cst[(4 + 3 * g) * H + i] = a.xc[(g * 2 + 0) * H + i];
      cst[(5 + 3 * g) * H + i] = a.xc[(g * 2 + 1) * H + i];
      cst[(6 + 3 * g) * H + i] = 0.f;
    }
  }

  // ---- register-resident B fragments (lane: column n, inputs 8 kq .. 8 kq + 7)
  auto fwv = [&](int g, int row, int i) -> float {   // W_g[row][i]
    return a.fw[((size_t)(i >> 2) * H + row) * 12 + g * 4 + (i & 3)];
  };
  auto bwv = [&](int g, int row, int col) -> float {   // W_g[row][col]
    return a.bw[((size_t)(row >> 2) * H + col) * 12 + g * 4 + (row & 3)];
  };
  jh8 fh[3][KF], fl[3][KF], rh[KR], rl[KR];
  float fup[3], rup;
  {
    // forward: B[k][n] = W_g[j][32 t + 8 kq + e]
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      float mx = 0.f;
#pragma unroll
      for (int t = 0; t < KF; ++t)
#pragma unroll
        for (int e = 0; e < 8; ++e) mx = fmaxf(mx, fabsf(fwv(g, j, 32 * t + 8 * kq + e)));
      mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
      mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
      // a weight column reaching 2^14 is split as w 2^-s, its products scaled back
      const int se = mx >= 16384.f ? min(ilogbf(mx) - 13, 120) : 0;
      const float dn = ldexpf(1.f, -se);
      fup[g] = ldexpf(1.f, se);
#pragma unroll
      for (int t = 0; t < KF; ++t) {
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = fwv(g, j, 32 * t + 8 * kq + e) * dn;
        jsplit(x, fh[g][t], fl[g][t]);
      }
    }
    // reverse: B[k][n] = W_g[32 (t % KF) + 8 kq + e][j], g = t / KF
    float mx = 0.f;
#pragma unroll
    for (int t = 0; t < KR; ++t)
#pragma unroll
      for (int e = 0; e < 8; ++e) mx = fmaxf(mx, fabsf(bwv(t / KF, 32 * (t % KF) + 8 * kq + e, j)));
    mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
    mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
    const int se = mx >= 16384.f ? min(ilogbf(mx) - 13, 120) : 0;
    const float dn = ldexpf(1.f, -se);
    rup = ldexpf(1.f, se);
#pragma unroll
    for (int t = 0; t < KR; ++t) {
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = bwv(t / KF, 32 * (t % KF) + 8 * kq + e, j) * dn;
      jsplit(x, rh[t], rl[t]);
    }
  }
  // this lane's rows are 4 kq + e; with a cRNN rows 8..15 are the phase
  // outputs of the samples of rows 0..7, so a lane's four rows share a head
  const int seedL = CPLX ? (kq >> 1) : 0;
  const float hd0 = a.head[(seedL ? 2 : 0) * H + j];
  const float hd1 = a.head[(seedL ? 3 : 1) * H + j];
  __syncthreads();

  // gate pre-activation products of the 16 rows from the states in hb (the
  // A row of lane l is row n, i.e. sample n mod S)
  auto gates = [&](const float* hb, jf4 (&acc)[3]) {
#pragma unroll
    for (int g = 0; g < 3; ++g) acc[g] = jf4{0.f, 0.f, 0.f, 0.f};
    const float* src = hb + (n % S) * HP + 8 * kq;
#pragma unroll
    for (int t = 0; t < KF; ++t) {
      const float4 x0 = *reinterpret_cast<const float4*>(src + 32 * t);
      const float4 x1 = *reinterpret_cast<const float4*>(src + 32 * t + 4);
      const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
      jh8 ah, al;
      jsplit(x, ah, al);
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        acc[g] = jmma(al, fh[g][t], acc[g]);
        acc[g] = jmma(ah, fl[g][t], acc[g]);
        acc[g] = jmma(ah, fh[g][t], acc[g]);
      }
      // keep the scheduler from hoisting every K-step's operand loads (the
      // weight fragments leave few registers for them)
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  // the cell of row 4 kq + e, unit j, previous spin sp
  auto cell = [&](const jf4 (&acc)[3], int e, int sp, float& u, float& r, float& ag, float& ht) {
    float au = fmaf(acc[0][e], fup[0], cst[j]);
    float ar = fmaf(acc[1][e], fup[1], cst[H + j]);
    ag = fmaf(acc[2][e], fup[2], cst[2 * H + j]);
    const float ai = cst[3 * H + j] + cst[(10 + sp) * H + j];
    au += cst[(4 + sp) * H + j];
    ar += cst[(7 + sp) * H + j];
    u = jsig(au);
    r = jsig(ar);
    ht = jtanh(fmaf(r, ag, ai));
  };

  float carry[4] = {0.f, 0.f, 0.f, 0.f};   // adjoint of h_k arriving from site k + 1

  const int nseg = (N + C - 1) / C;
  for (int segi = nseg - 1; segi >= 0; --segi) {
    const int ks = segi * C;
    const int len = min(C, N - ks);
    const bool last_ck = (ks + len) % C == 0;   // the segment's last state is stored
    const int nf = last_ck ? len - 1 : len;     // states recomputed forward
    for (int i = tid; i < S * H; i += NT) {
      const int s = i / H, u = i % H;
      const size_t sg = (size_t)min(s0 + s, Ns - 1);
      hs[s * HP + u] = ks > 0 ? a.states[(sg * N + ks - 1) * H + u] : 0.f;
      if (last_ck) hs[((size_t)len * S + s) * HP + u] = a.states[(sg * N + ks + len - 1) * H + u];
    }
    for (int i = tid; i < S * (len + 1); i += NT) {
      const int s = i / (len + 1), kk = i % (len + 1);
      const int k = ks - 1 + kk;
      sgs[s * SGP + kk] = k >= 0 ? (int)(a.sigma[(size_t)min(s0 + s, Ns - 1) * N + k] & 1) : 2;
    }
    __syncthreads();

    // ---- forward recomputation of the segment's states
    for (int kk = 0; kk < nf; ++kk) {
      jf4 acc[3];
      gates(hs + (size_t)kk * S * HP, acc);
      if (!CPLX || kq < 2) {
        const int k = ks + kk;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int sm = 4 * kq + e;
          float u, r, ag, ht;
          cell(acc, e, sgs[sm * SGP + kk], u, r, ag, ht);
          const float hp = hs[((size_t)kk * S + sm) * HP + j];
          const float hn = fmaf(u, ht - hp, hp);
          hs[((size_t)(kk + 1) * S + sm) * HP + j] = hn;
          if (s0 + sm < Ns) a.states[((unsigned)(s0 + sm) * N + k) * H + j] = hn;
        }
      }
      __syncthreads();
    }

    // ---- head adjoints of the segment's sites
    if constexpr (CPLX) {
      for (int p = w; p < len * S; p += NW) {
        const int kk = p / S, s = p % S;
        const float* hr = hs + ((size_t)(kk + 1) * S + s) * HP;
        float v0 = hr[l] * a.head[2 * H + l];
        float v1 = hr[l] * a.head[3 * H + l];
        v0 = fmaf(hr[l + 64], a.head[2 * H + l + 64], v0);
        v1 = fmaf(hr[l + 64], a.head[3 * H + l + 64], v1);
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
          v0 += __shfl_xor(v0, o, 64);
          v1 += __shfl_xor(v1, o, 64);
        }
        if (l == 0) {
          const int k = ks + kk;
          const int sk = sgs[s * SGP + kk + 1];
          const double* st = a.site + ((size_t)min(s0 + s, Ns - 1) * N + k) * 4;
          const float z0 = 0.5f * ((sk == 0 ? 1.f : 0.f) - expf((float)st[0]));
          const float z1 = 0.5f * ((sk == 1 ? 1.f : 0.f) - expf((float)st[1]));
          const float e0 = 1.f + fabsf(v0 + a.headb[2]), e1 = 1.f + fabsf(v1 + a.headb[3]);
          const float PI = 3.14159265358979323846f;
          const float q0 = sk == 0 ? PI / (e0 * e0) : 0.f;
          const float q1 = sk == 1 ? PI / (e1 * e1) : 0.f;
          dzs[(kk * 16 + s) * 2 + 0] = z0;
          dzs[(kk * 16 + s) * 2 + 1] = z1;
          dzs[(kk * 16 + 8 + s) * 2 + 0] = q0;
          dzs[(kk * 16 + 8 + s) * 2 + 1] = q1;
          if (s0 + s < Ns) {
            float* d0 = a.dzt + ((size_t)(s0 + s) * N + k) * 2;
            float* d1 = a.dzt + ((size_t)(Ns + s0 + s) * N + k) * 2;
            d0[0] = z0; d0[1] = z1; d1[0] = q0; d1[1] = q1;
          }
        }
      }
    } else {
      for (int p = tid; p < len * S; p += NT) {
        const int kk = p / S, s = p % S;
        const int k = ks + kk;
        const int sk = sgs[s * SGP + kk + 1];
        const double* st = a.site + ((size_t)min(s0 + s, Ns - 1) * N + k) * 4;
        const float z0 = 0.5f * ((sk == 0 ? 1.f : 0.f) - expf((float)st[0]));
        const float z1 = 0.5f * ((sk == 1 ? 1.f : 0.f) - expf((float)st[1]));
        dzs[(kk * 16 + s) * 2 + 0] = z0;
        dzs[(kk * 16 + s) * 2 + 1] = z1;
        if (s0 + s < Ns) {
          float* d0 = a.dzt + ((size_t)(s0 + s) * N + k) * 2;
          d0[0] = z0; d0[1] = z1;
        }
      }
    }
    __syncthreads();

    // ---- reverse through the segment
    for (int kk = len - 1; kk >= 0; --kk) {
      const int k = ks + kk, buf = k & 1;
      jf4 acc[3];
      gates(hs + (size_t)kk * S * HP, acc);
      float* db = dps + (size_t)buf * 16 * DP;
      float dhd[4];
      float mloc[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = 4 * kq + e;
        const int sm = rr % S;
        float u, r, ag, ht;
        cell(acc, e, sgs[sm * SGP + kk], u, r, ag, ht);
        const float hp = hs[((size_t)kk * S + sm) * HP + j];
        const float dz0 = dzs[(kk * 16 + rr) * 2 + 0], dz1 = dzs[(kk * 16 + rr) * 2 + 1];
        const float dh = fmaf(dz1, hd1, fmaf(dz0, hd0, carry[e]));
        const float dht = dh * u;
        const float du = dh * (ht - hp);
        dhd[e] = dh * (1.f - u);
        const float da = dht * (1.f - ht * ht);
        const float dr = da * ag;
        const float dg = da * r;
        const float dpu = du * u * (1.f - u);
        const float dpr = dr * r * (1.f - r);
        db[rr * DP + j] = dpu;
        db[rr * DP + H + j] = dpr;
        db[rr * DP + 2 * H + j] = dg;
        mloc[e] = fmaxf(fabsf(dpu), fmaxf(fabsf(dpr), fabsf(dg)));
        if (s0 + sm < Ns) {
          const unsigned grow = (CPLX ? (rr >> 3) * Ns : 0) + s0 + sm;
          float* tp = a.dpt + ((grow * N + k) * 4) * H + j;
          tp[0] = dpu; tp[H] = dpr; tp[2 * H] = dg; tp[3 * H] = da;
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) mloc[e] = fmaxf(mloc[e], __shfl_xor(mloc[e], o, 16));
      if (n == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) rmx[(buf * NW + w) * 16 + 4 * kq + e] = mloc[e];
      }
      __syncthreads();

      // adjoint of h_{k-1}: [16 x 3 d_h] x [3 d_h x d_h] with row n scaled by 2^ex
      float mx = 0.f;
#pragma unroll
      for (int v = 0; v < NW; ++v) mx = fmaxf(mx, rmx[(buf * NW + v) * 16 + n]);
      const int ex = jexp_for(mx);
      const float sc = ldexpf(1.f, ex);
      jf4 racc = {0.f, 0.f, 0.f, 0.f};
      const float* arow = db + n * DP + 8 * kq;
#pragma unroll
      for (int t = 0; t < KR; ++t) {
        const float4 x0 = *reinterpret_cast<const float4*>(arow + 32 * t);
        const float4 x1 = *reinterpret_cast<const float4*>(arow + 32 * t + 4);
        const float x[8] = {x0.x * sc, x0.y * sc, x0.z * sc, x0.w * sc,
                            x1.x * sc, x1.y * sc, x1.z * sc, x1.w * sc};
        jh8 ah, al;
        jsplit(x, ah, al);
        racc = jmma(al, rh[t], racc);
        racc = jmma(ah, rl[t], racc);
        racc = jmma(ah, rh[t], racc);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float inv = ldexpf(1.f, -__shfl(ex, 4 * kq + e, 64));
        carry[e] = fmaf(racc[e] * rup, inv, dhd[e]);
      }
    }
  }
}

struct JRowsArgs {
  Layout L;
  int N, Ns;
  const uint8_t* sigma;
  const float* states;
  const float* dpt;
  const float* dzt;
  float* O;
  float scale;           // 1 / sqrt(Ns)
};

template <bool CPLX>
__global__ __launch_bounds__(256, 2) void k_jac_rows(JRowsArgs a) {
  constexpr int H = JM_H, KM = JM_KMAX, AP = KM + 8;
  __shared__ __align__(16) _Float16 ahi[H][AP], alo[H][AP];   // A = adjoints^T, [j][k]
  __shared__ float xch[4][H];      // the upper half's max, sum, one-hot sums
  __shared__ float exs[H];         // 2^-E of gate row j
  __shared__ int sgl[KM];
  const int N = a.N, Ns = a.Ns;
  const int s = blockIdx.x;
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int n = l & 15, kq = l >> 4;
  const int KT = (N + 31) / 32;    // K-steps of 32 sites
  const Layout& L = a.L;
  const float sc = a.scale;

  for (int k = tid; k < KM; k += 256) sgl[k] = k < N ? (int)(a.sigma[(size_t)s * N + k] & 1) : 0;

  // B fragments: B[k][i] = h_{k-1}[i] (zero for k = 0 and k >= N),
  // k = 32 t + 8 kq + e, i = 32 w + 16 ut + n
  const float* hst = a.states + (size_t)s * N * H;
  jh8 bh[2][KM / 32], bl[2][KM / 32];
#pragma unroll
  for (int ut = 0; ut < 2; ++ut)
#pragma unroll
    for (int t = 0; t < KM / 32; ++t) {
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 32 * t + 8 * kq + e;
        x[e] = (k >= 1 && k < N) ? hst[(size_t)(k - 1) * H + 32 * w + 16 * ut + n] : 0.f;
      }
      jsplit(x, bh[ut][t], bl[ut][t]);
    }

  // staging thread: gate row j, sites [64 kb, 64 kb + 64)
  const int jr = tid & (H - 1), kb = tid >> 7;
  const int nseed = CPLX ? 2 : 1;
  for (int seed = 0; seed < nseed; ++seed) {
    const size_t row = (size_t)seed * Ns + s;
    float* o = a.O + row * L.Np;
    const float* tp = a.dpt + row * N * 4 * H;
    for (int q = 0; q < 4; ++q) {
      // load this thread's adjoints, their sums and largest magnitude
      float v[64];
      float sa = 0.f, s0v = 0.f, s1v = 0.f, mx = 0.f;
#pragma unroll
      for (int m = 0; m < 64; ++m) {
        const int k = 64 * kb + m;
        v[m] = k < N ? tp[((size_t)k * 4 + q) * H + jr] : 0.f;
      }
#pragma unroll
      for (int m = 0; m < 64; ++m) {
        const int k = 64 * kb + m;
        sa += v[m];
        if (k >= 1 && k < N) {
          if (sgl[k - 1] == 0) s0v += v[m];
          else s1v += v[m];
        }
        mx = fmaxf(mx, fabsf(v[m]));
      }
      if (kb == 1) {
        xch[0][jr] = mx; xch[1][jr] = sa; xch[2][jr] = s0v; xch[3][jr] = s1v;
      }
      __syncthreads();
      if (kb == 0) {
        mx = fmaxf(mx, xch[0][jr]);
        sa += xch[1][jr]; s0v += xch[2][jr]; s1v += xch[3][jr];
        // one-hot input columns and biases
        if (q == 0) {
          o[L.Wu + (size_t)jr * (H + 2) + H] = s0v * sc;
          o[L.Wu + (size_t)jr * (H + 2) + H + 1] = s1v * sc;
          o[L.bu + jr] = sa * sc;
        } else if (q == 1) {
          o[L.Wr + (size_t)jr * (H + 2) + H] = s0v * sc;
          o[L.Wr + (size_t)jr * (H + 2) + H + 1] = s1v * sc;
          o[L.br + jr] = sa * sc;
        } else if (q == 2) {
          o[L.bh + jr] = sa * sc;
        } else {
          o[L.Win + (size_t)jr * 2] = s0v * sc;
          o[L.Win + (size_t)jr * 2 + 1] = s1v * sc;
          o[L.bin + jr] = sa * sc;
        }
        xch[0][jr] = mx;
      }
      if (q == 3) {
        __syncthreads();
        break;
      }
      __syncthreads();
      // scaled split into the A tile (rows j, sites k)
      const int E = jexp_for(xch[0][jr]);
      const float up = ldexpf(1.f, E);
      if (kb == 0) exs[jr] = ldexpf(1.f, -E);
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) {
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = v[8 * c8 + e] * up;
        jh8 hi, lo;
        jsplit(x, hi, lo);
        *reinterpret_cast<jh8*>(&ahi[jr][64 * kb + 8 * c8]) = hi;
        *reinterpret_cast<jh8*>(&alo[jr][64 * kb + 8 * c8]) = lo;
      }
      __syncthreads();

      // W_q block: D[j][i] = sum_k A[j][k] B[k][i]; wave w takes columns
      // 32 w .. 32 w + 31, all rows in tiles of 16
      const size_t off = q == 0 ? L.Wu : q == 1 ? L.Wr : L.Wh;
      const int ldq = q < 2 ? H + 2 : H;
#pragma unroll 1
      for (int mt = 0; mt < H / 16; ++mt) {
        jf4 acc[2] = {jf4{0.f, 0.f, 0.f, 0.f}, jf4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int t = 0; t < KM / 32; ++t) {
          if (t < KT) {
            const jh8 ah = *reinterpret_cast<const jh8*>(&ahi[16 * mt + n][32 * t + 8 * kq]);
            const jh8 al = *reinterpret_cast<const jh8*>(&alo[16 * mt + n][32 * t + 8 * kq]);
#pragma unroll
            for (int ut = 0; ut < 2; ++ut) {
              acc[ut] = jmma(al, bh[ut][t], acc[ut]);
              acc[ut] = jmma(ah, bl[ut][t], acc[ut]);
              acc[ut] = jmma(ah, bh[ut][t], acc[ut]);
            }
          }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = 16 * mt + 4 * kq + e;
          const float f = exs[j] * sc;
#pragma unroll
          for (int ut = 0; ut < 2; ++ut)
            o[off + (size_t)j * ldq + 32 * w + 16 * ut + n] = acc[ut][e] * f;
        }
      }
      __syncthreads();
    }

    // output head: d/dU[c][j] = sum_k dz_k[c] h_k[j], d/dc[c] = sum_k dz_k[c]
    {
      const float* dz = a.dzt + row * N * 2;
      const int c = kb, j = jr;
      float gh = 0.f;
      for (int k = 0; k < N; ++k) gh = fmaf(dz[2 * k + c], hst[(size_t)k * H + j], gh);
      const size_t hU = seed == 0 ? L.U : L.Uphi;
      o[hU + (size_t)c * H + j] = gh * sc;
      if (CPLX) o[(seed == 0 ? L.Uphi : L.U) + (size_t)c * H + j] = 0.f;
      if (tid < 2) {
        float gc = 0.f;
        for (int k = 0; k < N; ++k) gc += dz[2 * k + tid];
        o[(seed == 0 ? L.c : L.cphi) + tid] = gc * sc;
        if (CPLX) o[(seed == 0 ? L.cphi : L.c) + tid] = 0.f;
      }
    }
  }
}

// ---- launch

size_t jac_mfma_tape_elems(int dim, int f64, int H, int N, int cplx, size_t max_Ns) {
  if (dim != 1 || f64 || H != JM_H || N > JM_KMAX) return 0;
  const size_t rows = (cplx ? 2 : 1) * max_Ns;
  return rows * (size_t)N * 4 * H + rows * (size_t)N * 2;
}

static size_t rev_smem(int C, bool cplx) {
  const int S = cplx ? 8 : 16;
  return sizeof(float) * ((size_t)(C + 1) * S * (JM_H + 4) + 2 * 16 * (3 * JM_H + 4) +
                          2 * (JM_H / 16) * 16 + JM_SEG * 32 + 13 * JM_H) +
         sizeof(int) * (size_t)S * (JM_SEG + 1);
}

bool jac_mfma_supported(const minsr_model* m, int C) {
  if (!m->jtape || m->dim != 1 || m->f64 || m->H != JM_H || m->N > JM_KMAX) return false;
  // the reverse kernel addresses the tape and the states with 32-bit offsets
  if ((size_t)2 * m->d.max_Ns * m->N * 4 * JM_H >= ((size_t)1 << 32)) return false;
  if (C < 1 || C > JM_SEG) return false;
  return rev_smem(C, m->cplx != 0) <= 160 * 1024;
}

template <bool CPLX>
static int launch_rev_rows(minsr_model* m, int Ns, const uint8_t* sigma, int C, float* O,
                           const double* site, hipStream_t s) {
  const int S = CPLX ? 8 : 16;
  const int N = m->N, H = JM_H;
  const size_t rows = (size_t)(CPLX ? 2 : 1) * Ns;
  float* dpt = (float*)m->jtape;
  float* dzt = dpt + rows * N * 4 * H;
  JRevArgs r{};
  r.fw = m->wf.fw; r.bw = m->wf.bw; r.xc = m->wf.xc; r.bias = m->wf.bias;
  r.head = m->wf.head; r.headb = m->wf.headb;
  r.N = N; r.Ns = Ns; r.C = C;
  r.sigma = sigma; r.states = (float*)m->states; r.site = site;
  r.dpt = dpt; r.dzt = dzt;
  const size_t sm = rev_smem(C, CPLX);
  // more than 64 KiB of dynamic shared memory: allowed once per process,
  // before the first launch (outside any stream capture of later calls)
  static std::once_flag once;
  hipError_t attr = hipSuccess;
  std::call_once(once, [&] {
    attr = hipFuncSetAttribute((const void*)k_jac_rev<CPLX>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  });
  MINSR_HIP(attr);
  k_jac_rev<CPLX><<<(unsigned)((Ns + S - 1) / S), 512, sm, s>>>(r);
  MINSR_CHECK_LAUNCH();
  JRowsArgs q{};
  q.L = m->L; q.N = N; q.Ns = Ns; q.sigma = sigma; q.states = (const float*)m->states;
  q.dpt = dpt; q.dzt = dzt; q.O = O;
  q.scale = (float)(1.0 / std::sqrt((double)Ns));
  k_jac_rows<CPLX><<<(unsigned)Ns, 256, 0, s>>>(q);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int launch_jacobian_mfma(minsr_model* m, int Ns, const uint8_t* sigma, int C, void* O,
                         const double* site, hipStream_t s) {
  if (Ns == 0) return MINSR_OK;
  if (!jac_mfma_supported(m, C) || !site)
    return fail(MINSR_E_UNSUPPORTED, "matrix-core Jacobian: 1D FP32 d_h = 128, N <= 128");
  if (m->cplx) return launch_rev_rows<true>(m, Ns, sigma, C, (float*)O, site, s);
  return launch_rev_rows<false>(m, Ns, sigma, C, (float*)O, site, s);
}

}  // namespace minsr
