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
#include "mfma16.hpp"

namespace minsr {

namespace {

using namespace mf16;

constexpr int JM_H = 128;       // hidden width of this path
constexpr int JM_SEG = 16;      // longest checkpoint segment
constexpr int JM_KMAX = 128;    // longest chain of the row assembly

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

// NL: the last NL K-steps of the reverse product take their weight fragments
// from shared memory instead of registers (as many as the segment length
// leaves room for), so the fragments and the working set fit the register file
template <bool CPLX, int NL>
__global__ __launch_bounds__(512, 1) void k_jac_rev(JRevArgs a) {
  constexpr int H = JM_H, NW = H / 16, KF = H / 32, KR = 3 * H / 32;
  constexpr int KRR = KR - NL;         // reverse K-steps with register fragments
  constexpr int S = CPLX ? 8 : 16;     // samples per workgroup (16 rows)
  constexpr int HQ = H + 8;            // state row pitch (halves)
  constexpr int DQ = 3 * H + 8;        // gate-adjoint row pitch (halves)
  constexpr int SGP = JM_SEG + 1;
  constexpr int NT = 64 * NW;
  extern __shared__ __align__(16) unsigned char jsm[];
  const int C = a.C, N = a.N, Ns = a.Ns;
  // states h_{ks-1+kk} and the scaled gate adjoints of a site, both as FP16
  // hi/lo halves (the products' A operands, split once when written)
  _Float16* hsh = reinterpret_cast<_Float16*>(jsm);     // [C + 1][S][HQ]
  _Float16* hsl = hsh + (size_t)(C + 1) * S * HQ;
  _Float16* dph = hsl + (size_t)(C + 1) * S * HQ;       // [16][DQ]
  _Float16* dpl = dph + 16 * DQ;
  h16x8* rfr = reinterpret_cast<h16x8*>(dpl + 16 * DQ);     // [NL][hi, lo][NW][64]
  float* rmx = reinterpret_cast<float*>(rfr + NL * 2 * NW * 64);   // [16][NW] row maxima
  float* dzs = rmx + 16 * NW;                      // [JM_SEG][16][2] head adjoints
  float* cst = dzs + JM_SEG * 32;                  // [21][H] + 2, rows described below
  int* sgs = reinterpret_cast<int*>(cst + 21 * H + 2); // [S][SGP] sigma_{ks-1+kk}, 2 before site 0

  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int n = l & 15, kq = l >> 4;
  const int j = 16 * w + n;            // this lane's hidden unit (gate row / state column)
  const int s0 = blockIdx.x * S;

  // cst rows: 0-3 b_u, b_r, b_h, b_in; 4-12 for u, r, in the input columns
  // of spin values 0, 1 and zeros (no input at site 0); 13-15 the forward
  // column scales of u, r, h; 16 the reverse column scales; 17-20 U, U_phi;
  // then c_phi
  for (int i = tid; i < 4 * H; i += NT) cst[17 * H + i] = a.head[i];
  if (tid < 2) cst[21 * H + tid] = a.headb[2 + tid];
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

  // ---- B fragments (lane: column n, inputs 8 kq .. 8 kq + 7)
  auto fwv = [&](int g, int row, int i) -> float {   // W_g[row][i]
    return a.fw[((size_t)(i >> 2) * H + row) * 12 + g * 4 + (i & 3)];
  };
  auto bwv = [&](int g, int row, int col) -> float {   // W_g[row][col]
    return a.bw[((size_t)(row >> 2) * H + col) * 12 + g * 4 + (row & 3)];
  };
  h16x8 fh[3][KF], fl[3][KF], rh[KRR], rl[KRR];
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
      if (kq == 0) cst[(13 + g) * H + j] = ldexpf(1.f, se);
#pragma unroll
      for (int t = 0; t < KF; ++t) {
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = fwv(g, j, 32 * t + 8 * kq + e) * dn;
        split16(x, fh[g][t], fl[g][t]);
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
    if (kq == 0) cst[16 * H + j] = ldexpf(1.f, se);
#pragma unroll
    for (int t = 0; t < KR; ++t) {
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = bwv(t / KF, 32 * (t % KF) + 8 * kq + e, j) * dn;
      if (t < KRR) {
        split16(x, rh[t < KRR ? t : 0], rl[t < KRR ? t : 0]);
      } else {
        h16x8 hi, lo;
        split16(x, hi, lo);
        rfr[((t - KRR) * 2 + 0) * NW * 64 + w * 64 + l] = hi;
        rfr[((t - KRR) * 2 + 1) * NW * 64 + w * 64 + l] = lo;
      }
    }
  }
  // this lane's rows are 4 kq + e; with a cRNN rows 8..15 are the phase
  // outputs of the samples of rows 0..7, so a lane's four rows share a head
  const int seedL = CPLX ? (kq >> 1) : 0;
  const float* hdw = cst + (17 + 2 * seedL) * H + j;   // this lane's head weights
  lds_barrier();

  // state value of (buffer kk, sample s, unit u) and its split store
  auto hget = [&](int kk, int s, int u) -> float {
    const size_t o = ((size_t)kk * S + s) * HQ + u;
    return (float)hsh[o] + (float)hsl[o];
  };
  auto hput = [&](int kk, int s, int u, float v) {
    const size_t o = ((size_t)kk * S + s) * HQ + u;
    const _Float16 hi = (_Float16)v;
    hsh[o] = hi;
    hsl[o] = (_Float16)(v - (float)hi);
  };
  // gate pre-activation products of the 16 rows from state buffer kk (the
  // A row of lane l is row n, i.e. sample n mod S)
  auto gates = [&](int kk, f32x4v (&acc)[3]) {
#pragma unroll
    for (int g = 0; g < 3; ++g) acc[g] = f32x4v{0.f, 0.f, 0.f, 0.f};
    const size_t o = ((size_t)kk * S + (n % S)) * HQ + 8 * kq;
#pragma unroll
    for (int t = 0; t < KF; ++t) {
      const h16x8 ah = *reinterpret_cast<const h16x8*>(hsh + o + 32 * t);
      const h16x8 al = *reinterpret_cast<const h16x8*>(hsl + o + 32 * t);
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        acc[g] = mma16(al, fh[g][t], acc[g]);
        acc[g] = mma16(ah, fl[g][t], acc[g]);
        acc[g] = mma16(ah, fh[g][t], acc[g]);
      }
    }
  };
  // the cell of row 4 kq + e, unit j, previous spin sp
  auto cell = [&](const f32x4v (&acc)[3], int e, int sp, float& u, float& r, float& ag, float& ht) {
    float au = fmaf(acc[0][e], cst[13 * H + j], cst[j]);
    float ar = fmaf(acc[1][e], cst[14 * H + j], cst[H + j]);
    ag = fmaf(acc[2][e], cst[15 * H + j], cst[2 * H + j]);
    // input columns of both spin values read unconditionally (no shared-
    // memory load waits on the spin), the one for sp selected
    const float xu0 = cst[4 * H + j], xu1 = cst[5 * H + j];
    const float xr0 = cst[7 * H + j], xr1 = cst[8 * H + j];
    const float xi0 = cst[10 * H + j], xi1 = cst[11 * H + j];
    const float ai = cst[3 * H + j] + (sp == 0 ? xi0 : sp == 1 ? xi1 : 0.f);
    au += sp == 0 ? xu0 : sp == 1 ? xu1 : 0.f;
    ar += sp == 0 ? xr0 : sp == 1 ? xr1 : 0.f;
    u = sigm_hw(au);
    r = sigm_hw(ar);
    ht = tanh_hw(fmaf(r, ag, ai));
  };

  float carry[4] = {0.f, 0.f, 0.f, 0.f};   // adjoint of h_k arriving from site k + 1

  const int nseg = (N + C - 1) / C;
  for (int segi = nseg - 1; segi >= 0; --segi) {
    const int ks = segi * C;
    const int len = min(C, N - ks);
    const bool last_ck = (ks + len) % C == 0;   // the segment's last state is stored
    const int nf = last_ck ? len - 1 : len;     // states recomputed forward
    {
      // every global load of the staging issued before any is used
      constexpr int PT = S * H / NT;             // states per thread
      float hv0[PT], hv1[PT];
#pragma unroll
      for (int q = 0; q < PT; ++q) {
        const int i = tid + q * NT, s = i / H, u = i % H;
        const size_t sg = (size_t)min(s0 + s, Ns - 1);
        hv0[q] = ks > 0 ? a.states[(sg * N + ks - 1) * H + u] : 0.f;
        hv1[q] = last_ck ? a.states[(sg * N + ks + len - 1) * H + u] : 0.f;
      }
      const bool sit = tid < S * (len + 1);
      const int s = tid / (len + 1), kk = tid % (len + 1);
      const int k = ks - 1 + kk;
      const size_t sg = (size_t)min(s0 + s, Ns - 1);
      int sk = 2;
      double l0 = 0.0, l1 = 0.0;
      if (sit && k >= 0) sk = (int)(a.sigma[sg * N + k] & 1);
      if (sit && k >= ks) {
        const double* st = a.site + (sg * N + k) * 4;
        l0 = st[0];
        l1 = st[1];
      }
#pragma unroll
      for (int q = 0; q < PT; ++q) {
        const int i = tid + q * NT;
        hput(0, i / H, i % H, hv0[q]);
        if (last_ck) hput(len, i / H, i % H, hv1[q]);
      }
      if (sit) {
        sgs[s * SGP + kk] = sk;
        // log-modulus head adjoints of site k: (delta - p) / 2 from the
        // forward pass's (masked) conditionals
        if (k >= ks) {
          const float z0 = 0.5f * ((sk == 0 ? 1.f : 0.f) - expf((float)l0));
          const float z1 = 0.5f * ((sk == 1 ? 1.f : 0.f) - expf((float)l1));
          dzs[((kk - 1) * 16 + s) * 2 + 0] = z0;
          dzs[((kk - 1) * 16 + s) * 2 + 1] = z1;
          if (s0 + s < Ns) {
            float* d0 = a.dzt + ((size_t)(s0 + s) * N + k) * 2;
            d0[0] = z0; d0[1] = z1;
          }
        }
      }
    }
    lds_barrier();

    // ---- forward recomputation of the segment's states
    for (int kk = 0; kk < nf; ++kk) {
      f32x4v acc[3];
      gates(kk, acc);
      if (!CPLX || kq < 2) {
        const int k = ks + kk;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int sm = 4 * kq + e;
          float u, r, ag, ht;
          cell(acc, e, sgs[sm * SGP + kk], u, r, ag, ht);
          const float hp = hget(kk, sm, j);
          const float hn = fmaf(u, ht - hp, hp);
          hput(kk + 1, sm, j, hn);
          if (s0 + sm < Ns) a.states[((unsigned)(s0 + sm) * N + k) * H + j] = hn;
        }
      }
      lds_barrier();
    }

    // ---- phase-head adjoints of the segment's sites (cRNN; the log-modulus
    // ones come from the forward pass's conditionals, staged above)
    if constexpr (CPLX) {
      // four lanes per (site, sample), 32 units each
      const int p = tid >> 2, qd = tid & 3;
      const bool on = p < len * S;     // len * S <= 128: one pass
      const int kk = on ? p / S : 0, s = p % S;
      const float* hph = cst + 19 * H;
      float v0 = 0.f, v1 = 0.f;
#pragma unroll 8
      for (int u = 32 * qd; u < 32 * qd + 32; ++u) {
        const float hv = hget(kk + 1, s, u);
        v0 = fmaf(hv, hph[u], v0);
        v1 = fmaf(hv, hph[H + u], v1);
      }
      v0 = quad_sum(v0);
      v1 = quad_sum(v1);
      if (on && qd == 0) {
        const int k = ks + kk;
        const int sk = sgs[s * SGP + kk + 1];
        const float e0 = 1.f + fabsf(v0 + cst[21 * H]), e1 = 1.f + fabsf(v1 + cst[21 * H + 1]);
        const float PI = 3.14159265358979323846f;
        const float q0 = sk == 0 ? PI / (e0 * e0) : 0.f;
        const float q1 = sk == 1 ? PI / (e1 * e1) : 0.f;
        dzs[(kk * 16 + 8 + s) * 2 + 0] = q0;
        dzs[(kk * 16 + 8 + s) * 2 + 1] = q1;
        if (s0 + s < Ns) {
          float* d1 = a.dzt + ((size_t)(Ns + s0 + s) * N + k) * 2;
          d1[0] = q0; d1[1] = q1;
        }
      }
      lds_barrier();
    }

    // ---- reverse through the segment
    // the gate products of site k - 1 are issued together with the reverse
    // product of site k (independent work for the matrix cores)
    f32x4v acc[3];
    gates(len - 1, acc);
    for (int kk = len - 1; kk >= 0; --kk) {
      const int k = ks + kk;
      float dp[4][3], dhd[4], mloc[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rr = 4 * kq + e;
        const int sm = rr % S;
        float u, r, ag, ht;
        cell(acc, e, sgs[sm * SGP + kk], u, r, ag, ht);
        const float hp = hget(kk, sm, j);
        const float dz0 = dzs[(kk * 16 + rr) * 2 + 0], dz1 = dzs[(kk * 16 + rr) * 2 + 1];
        const float dh = fmaf(dz1, hdw[H], fmaf(dz0, hdw[0], carry[e]));
        const float dht = dh * u;
        const float du = dh * (ht - hp);
        dhd[e] = dh * (1.f - u);
        const float da = dht * (1.f - ht * ht);
        const float dr = da * ag;
        const float dg = da * r;
        const float dpu = du * u * (1.f - u);
        const float dpr = dr * r * (1.f - r);
        dp[e][0] = dpu; dp[e][1] = dpr; dp[e][2] = dg;
        mloc[e] = fmaxf(fabsf(dpu), fmaxf(fabsf(dpr), fabsf(dg)));
        if (s0 + sm < Ns) {
          const unsigned grow = (CPLX ? (rr >> 3) * Ns : 0) + s0 + sm;
          float* tp = a.dpt + ((grow * N + k) * 4) * H + j;
          tp[0] = dpu; tp[H] = dpr; tp[2 * H] = dg; tp[3 * H] = da;
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) mloc[e] = row16_max(mloc[e]);
      if (n == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) rmx[(4 * kq + e) * NW + w] = mloc[e];
      }
      lds_barrier();
      // each row scaled by a power of two from its largest gate adjoint,
      // then split into the A operand of the reverse product
      int ex[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float4 m0 = *reinterpret_cast<const float4*>(rmx + (4 * kq + e) * NW);
        const float4 m1 = *reinterpret_cast<const float4*>(rmx + (4 * kq + e) * NW + 4);
        const float mx = fmaxf(fmaxf(fmaxf(m0.x, m0.y), fmaxf(m0.z, m0.w)),
                               fmaxf(fmaxf(m1.x, m1.y), fmaxf(m1.z, m1.w)));
        ex[e] = pow2_exp_for(mx);
        const float sc = ldexpf(1.f, ex[e]);
#pragma unroll
        for (int g = 0; g < 3; ++g) {
          const float v = dp[e][g] * sc;
          const _Float16 hi = (_Float16)v;
          dph[(4 * kq + e) * DQ + g * H + j] = hi;
          dpl[(4 * kq + e) * DQ + g * H + j] = (_Float16)(v - (float)hi);
        }
      }
      lds_barrier();

      if (kk > 0) gates(kk - 1, acc);
      // adjoint of h_{k-1}: [16 x 3 d_h] x [3 d_h x d_h]; three independent
      // accumulation chains, one per split product
      f32x4v rc0 = {0.f, 0.f, 0.f, 0.f}, rc1 = rc0, rc2 = rc0;
      const _Float16* ahp = dph + n * DQ + 8 * kq;
      const _Float16* alp = dpl + n * DQ + 8 * kq;
#pragma unroll
      for (int t = 0; t < KR; ++t) {
        const h16x8 ah = *reinterpret_cast<const h16x8*>(ahp + 32 * t);
        const h16x8 al = *reinterpret_cast<const h16x8*>(alp + 32 * t);
        h16x8 bh, bl;
        if (t < KRR) {
          bh = rh[t < KRR ? t : 0];
          bl = rl[t < KRR ? t : 0];
        } else {
          bh = rfr[((t - KRR) * 2 + 0) * NW * 64 + w * 64 + l];
          bl = rfr[((t - KRR) * 2 + 1) * NW * 64 + w * 64 + l];
        }
        rc0 = mma16(al, bh, rc0);
        rc1 = mma16(ah, bl, rc1);
        rc2 = mma16(ah, bh, rc2);
      }
      const f32x4v racc = (rc0 + rc1) + rc2;
      const float rs = cst[16 * H + j];
#pragma unroll
      for (int e = 0; e < 4; ++e) carry[e] = fmaf(racc[e] * rs, ldexpf(1.f, -ex[e]), dhd[e]);
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
  __shared__ float dzl[2][KM][2];  // head adjoints of both outputs
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
  h16x8 bh[2][KM / 32], bl[2][KM / 32];
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
      split16(x, bh[ut][t], bl[ut][t]);
    }

  // staging thread: gate row j, sites [64 kb, 64 kb + 64)
  const int jr = tid & (H - 1), kb = tid >> 7;
  const int nseed = CPLX ? 2 : 1;

  // output head: d/dU[c][j] = sum_k dz_k[c] h_k[j], d/dc[c] = sum_k dz_k[c]
  // (each output's own head; the other head of a cRNN row is zero)
  for (int i = tid; i < nseed * KM * 2; i += 256) {
    const int sd = i / (KM * 2), r = i % (KM * 2);
    dzl[sd][r >> 1][r & 1] = (r >> 1) < N ? a.dzt[((size_t)sd * Ns + s) * N * 2 + r] : 0.f;
  }
  lds_barrier();
  {
    float hv[64];
#pragma unroll
    for (int m = 0; m < 64; ++m) {
      const int k = 64 * kb + m;
      hv[m] = k < N ? hst[(size_t)k * H + jr] : 0.f;
    }
    float g[2][2] = {{0.f, 0.f}, {0.f, 0.f}};
#pragma unroll
    for (int m = 0; m < 64; ++m)
#pragma unroll
      for (int sd = 0; sd < (CPLX ? 2 : 1); ++sd) {
        g[sd][0] = fmaf(dzl[sd][64 * kb + m][0], hv[m], g[sd][0]);
        g[sd][1] = fmaf(dzl[sd][64 * kb + m][1], hv[m], g[sd][1]);
      }
    if (kb == 1) {
      xch[0][jr] = g[0][0]; xch[1][jr] = g[0][1]; xch[2][jr] = g[1][0]; xch[3][jr] = g[1][1];
    }
    lds_barrier();
    if (kb == 0) {
      float* o0 = a.O + (size_t)s * L.Np;
      o0[L.U + jr] = (g[0][0] + xch[0][jr]) * sc;
      o0[L.U + H + jr] = (g[0][1] + xch[1][jr]) * sc;
      if (CPLX) {
        float* o1 = a.O + ((size_t)Ns + s) * L.Np;
        o0[L.Uphi + jr] = 0.f;
        o0[L.Uphi + H + jr] = 0.f;
        o1[L.Uphi + jr] = (g[1][0] + xch[2][jr]) * sc;
        o1[L.Uphi + H + jr] = (g[1][1] + xch[3][jr]) * sc;
        o1[L.U + jr] = 0.f;
        o1[L.U + H + jr] = 0.f;
      }
    }
    if (w == 0) {
      float c[2][2];
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          float v = sd < nseed ? dzl[sd][l][q] + dzl[sd][l + 64][q] : 0.f;
#pragma unroll
          for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
          c[sd][q] = v;
        }
      if (l == 0) {
        float* o0 = a.O + (size_t)s * L.Np;
        o0[L.c] = c[0][0] * sc;
        o0[L.c + 1] = c[0][1] * sc;
        if (CPLX) {
          float* o1 = a.O + ((size_t)Ns + s) * L.Np;
          o0[L.cphi] = 0.f; o0[L.cphi + 1] = 0.f;
          o1[L.cphi] = c[1][0] * sc; o1[L.cphi + 1] = c[1][1] * sc;
          o1[L.c] = 0.f; o1[L.c + 1] = 0.f;
        }
      }
    }
    lds_barrier();
  }
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
      lds_barrier();
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
        lds_barrier();
        break;
      }
      lds_barrier();
      // scaled split into the A tile (rows j, sites k)
      const int E = pow2_exp_for(xch[0][jr]);
      const float up = ldexpf(1.f, E);
      if (kb == 0) exs[jr] = ldexpf(1.f, -E);
#pragma unroll
      for (int c8 = 0; c8 < 8; ++c8) {
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = v[8 * c8 + e] * up;
        h16x8 hi, lo;
        split16(x, hi, lo);
        *reinterpret_cast<h16x8*>(&ahi[jr][64 * kb + 8 * c8]) = hi;
        *reinterpret_cast<h16x8*>(&alo[jr][64 * kb + 8 * c8]) = lo;
      }
      lds_barrier();

      // W_q block: D[j][i] = sum_k A[j][k] B[k][i]; wave w takes columns
      // 32 w .. 32 w + 31, all rows in tiles of 16
      const size_t off = q == 0 ? L.Wu : q == 1 ? L.Wr : L.Wh;
      const int ldq = q < 2 ? H + 2 : H;
#pragma unroll 1
      for (int mt = 0; mt < H / 16; ++mt) {
        f32x4v acc[2] = {f32x4v{0.f, 0.f, 0.f, 0.f}, f32x4v{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int t = 0; t < KM / 32; ++t) {
          if (t < KT) {
            const h16x8 ah = *reinterpret_cast<const h16x8*>(&ahi[16 * mt + n][32 * t + 8 * kq]);
            const h16x8 al = *reinterpret_cast<const h16x8*>(&alo[16 * mt + n][32 * t + 8 * kq]);
#pragma unroll
            for (int ut = 0; ut < 2; ++ut) {
              acc[ut] = mma16(al, bh[ut][t], acc[ut]);
              acc[ut] = mma16(ah, bl[ut][t], acc[ut]);
              acc[ut] = mma16(ah, bh[ut][t], acc[ut]);
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
      lds_barrier();
    }
  }
}

// ---- launch

size_t jac_mfma_tape_elems(int dim, int f64, int H, int N, int cplx, size_t max_Ns) {
  if (dim != 1 || f64 || H != JM_H || N > JM_KMAX) return 0;
  const size_t rows = (cplx ? 2 : 1) * max_Ns;
  return rows * (size_t)N * 4 * H + rows * (size_t)N * 2;
}

static size_t rev_smem(int C, bool cplx, int NL) {
  const int S = cplx ? 8 : 16, NW = JM_H / 16;
  return 2 * sizeof(_Float16) * ((size_t)(C + 1) * S * (JM_H + 8) + 16 * (3 * JM_H + 8)) +
         (size_t)NL * 2 * NW * 64 * 16 +
         sizeof(float) * ((size_t)16 * NW + JM_SEG * 32 + 21 * JM_H + 2) +
         sizeof(int) * (size_t)S * (JM_SEG + 1);
}

constexpr size_t JM_LDS = 160 * 1024;

// register fragments moved to shared memory: as many as fit (at most 4)
static int rev_nl(int C, bool cplx) {
  for (int NL = 4; NL > 0; --NL)
    if (rev_smem(C, cplx, NL) <= JM_LDS) return NL;
  return 0;
}

bool jac_mfma_supported(const minsr_model* m, int C) {
  if (!m->jtape || m->dim != 1 || m->f64 || m->H != JM_H || m->N > JM_KMAX) return false;
  // the reverse kernel addresses the tape and the states with 32-bit offsets
  if ((size_t)2 * m->d.max_Ns * m->N * 4 * JM_H >= ((size_t)1 << 32)) return false;
  if (C < 1 || C > JM_SEG) return false;
  return rev_smem(C, m->cplx != 0, 0) <= JM_LDS;
}

template <bool CPLX, int NL>
static int launch_rev(const JRevArgs& r, int Ns, hipStream_t s) {
  const int S = CPLX ? 8 : 16;
  // more than 64 KiB of dynamic shared memory: allowed once per process,
  // before the first launch (outside any stream capture of later calls)
  static std::once_flag once;
  hipError_t attr = hipSuccess;
  std::call_once(once, [&] {
    attr = hipFuncSetAttribute((const void*)k_jac_rev<CPLX, NL>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)JM_LDS);
  });
  MINSR_HIP(attr);
  k_jac_rev<CPLX, NL><<<(unsigned)((Ns + S - 1) / S), 512, rev_smem(r.C, CPLX, NL), s>>>(r);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

template <bool CPLX>
static int launch_rev_rows(minsr_model* m, int Ns, const uint8_t* sigma, int C, float* O,
                           const double* site, hipStream_t s) {
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
  int rc = MINSR_OK;
  switch (rev_nl(C, CPLX)) {
    case 4: rc = launch_rev<CPLX, 4>(r, Ns, s); break;
    case 3: rc = launch_rev<CPLX, 3>(r, Ns, s); break;
    case 2: rc = launch_rev<CPLX, 2>(r, Ns, s); break;
    case 1: rc = launch_rev<CPLX, 1>(r, Ns, s); break;
    default: rc = launch_rev<CPLX, 0>(r, Ns, s); break;
  }
  if (rc) return rc;
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
