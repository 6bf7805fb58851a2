// Exact autoregressive sampling of 1D FP32 models with d_h = 64 or 128 on
// the matrix cores (Sec. 2, Eqs. 3-7, with the cell of App. A; the samples
// of Alg. 1).
//
// A workgroup draws 16 sequences together, one wave for every 16 hidden
// units.  At each site the gate pre-activations of the 16 sequences are one
// [3 d_h x d_h] x [d_h x 16] product on v_mfma_f32_16x16x32_f16: wave w keeps
// for the whole kernel the A-operand fragments of the rows of W_u, W_r and
// W_h of its units, each row scaled by a power of two that brings its
// largest entry into [2^14, 2^15) and split into an FP16 pair x = hi + lo;
// the hidden states of the 16 sequences are the B operand, scaled by 2^14
// and split the same way when written to shared memory.  The three
// products a_lo b_hi + a_hi b_lo + a_hi b_hi (FP32 accumulation) carry the
// operands to 2^-22 of their size.  In the accumulator layout a lane holds
// four hidden units of one sequence, so the GRU update runs in registers;
// the new state is stored as the next product's operand, and the lane's
// share of the output head (the two logits and, for a complex head, the two
// phase pre-activations) is summed over the four lanes of its sequence by
// cross-lane exchanges and over the waves through shared memory in a fixed
// order.  After the single barrier of a site the next site's products are
// issued first; while they run, every lane forms the conditional of its
// sequence and draws its spin with the uniform of (sequence, site),
// generated into shared memory before the site loop from the same
// Philox4x64-10 stream as every other sampler.  The drawn spin then
// selects the input columns the next cell adds to the products.
#include "model.hpp"
#include "mfma16.hpp"

namespace minsr {

namespace {

using namespace mf16;

constexpr int SM_SEQ = 16;          // sequences per workgroup (the product's N)
constexpr int SM_NMAX = 256;        // longest chain (uniforms held in shared memory)
constexpr float SM_HSCALE = 16384.f;   // 2^14: |h| <= 1 enters FP16 as |h| 2^14

}  // namespace

struct SampMArgs {
  const float* fw;       // packed gate weights [k/4][j][3][4]
  const float* xc;       // input columns [3][2][H]: u, r, candidate input
  const float* bias;     // [4][H]: b_u, b_r, b_h, b_in
  const float* head;     // [4][H]: U rows, then U_phi rows
  const float* headb;    // [4]
  int N, Ns, zero_mag, cplx, marshall, store_every;
  const uint8_t* subA;
  const double* uniforms;        // optional [Ns][N]
  uint64_t key, counter;
  const uint64_t* counter_ptr;   // if set, the counter is read from here
  uint32_t* zero_word;           // if set, cleared by the first thread
  uint8_t* sigma;        // [Ns][N]
  double* logpsi;        // [Ns][2]
  float* states;         // optional [Ns][N][H]
  float* gates;          // optional [Ns][N][4][H]: u, r, candidate pre-activation, candidate
  double* site;          // optional [Ns][N][4]: log p(0), log p(1), phi(0), phi(1)
};

template <int H>
__global__ __launch_bounds__(4 * H) void k_sample_mfma(SampMArgs a) {
  constexpr int NW = H / 16, KB = H / 32, HP = H + 8;
  __shared__ __align__(16) _Float16 hsh[2][SM_SEQ][HP];
  __shared__ __align__(16) _Float16 hsl[2][SM_SEQ][HP];
  __shared__ __align__(16) float4 part[2][NW][SM_SEQ];
  __shared__ double uni[SM_SEQ][SM_NMAX];
  __shared__ uint8_t subA[SM_NMAX];

  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int col = l & 15, grp = l >> 4;
  const int N = a.N;
  const int s = blockIdx.x * SM_SEQ + col;
  const bool act = s < a.Ns;
  const uint64_t ctr = a.counter_ptr ? *a.counter_ptr : a.counter;
  if (a.zero_word && blockIdx.x == 0 && tid == 0) a.zero_word[0] = 0u;

  // uniforms of the workgroup's sequences: Philox block b of sequence s
  // holds the uniforms of sites 4b .. 4b + 3 (sequences past Ns repeat the
  // last one; nothing of theirs is written)
  const int nblk = (N + 3) / 4;
  for (int i = tid; i < SM_SEQ * nblk; i += 4 * H) {
    const int c = i % SM_SEQ, b = i / SM_SEQ;
    const int sc = min((int)blockIdx.x * SM_SEQ + c, a.Ns - 1);
    if (a.uniforms) {
      for (int e = 0; e < 4 && 4 * b + e < N; ++e)
        uni[c][4 * b + e] = a.uniforms[(size_t)sc * N + 4 * b + e];
    } else {
      const U64x4 r = philox4x64_10(ctr, (uint64_t)sc, (uint64_t)b, 0, a.key, 0);
      for (int e = 0; e < 4 && 4 * b + e < N; ++e) uni[c][4 * b + e] = u01(r.w[e]);
    }
  }
  for (int i = tid; i < N; i += 4 * H) subA[i] = a.marshall ? a.subA[i] : 0;
  for (int i = tid; i < SM_SEQ * HP; i += 4 * H) {
    (&hsh[0][0][0])[i] = (_Float16)0.f;
    (&hsl[0][0][0])[i] = (_Float16)0.f;
  }

  // A fragments: row 16 w + col of W_q, inputs 32 kb + 8 grp + e
  h16x8 wah[3][KB], wal[3][KB];
  float dsc[3][4];   // 2^-(row exponent + 14) of the accumulator rows 4 grp + v
  {
    const int ja = 16 * w + col;
    const float4* fw4 = reinterpret_cast<const float4*>(a.fw);
    float wv[3][KB][8];
    float mx[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
          const int k4 = 8 * kb + 2 * grp + hf;
          const float4 v = fw4[((size_t)k4 * H + ja) * 3 + q];
          wv[q][kb][4 * hf + 0] = v.x; wv[q][kb][4 * hf + 1] = v.y;
          wv[q][kb][4 * hf + 2] = v.z; wv[q][kb][4 * hf + 3] = v.w;
          mx[q] = fmaxf(mx[q], fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      mx[q] = fmaxf(mx[q], __shfl_xor(mx[q], 16));
      mx[q] = fmaxf(mx[q], __shfl_xor(mx[q], 32));
      const int e = pow2_exp_for(mx[q]);
      const float sc = ldexpf(1.f, e);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        float x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = wv[q][kb][i] * sc;
        split16(x, wah[q][kb], wal[q][kb]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) dsc[q][v] = ldexpf(1.f, -(__shfl(e, 4 * grp + v) + 14));
    }
  }

  // constants of the lane's units j = 16 w + 4 grp + v
  const int j0 = 16 * w + 4 * grp;
  auto ld4 = [&](const float* p, float (&d)[4]) {
    const float4 v = *reinterpret_cast<const float4*>(p + j0);
    d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
  };
  float bu[4], br[4], bh[4], bi[4], xu0[4], xu1[4], xr0[4], xr1[4], xi0[4], xi1[4];
  float U0[4], U1[4], P0[4], P1[4];
  ld4(a.bias, bu); ld4(a.bias + H, br); ld4(a.bias + 2 * H, bh); ld4(a.bias + 3 * H, bi);
  ld4(a.xc, xu0); ld4(a.xc + H, xu1); ld4(a.xc + 2 * H, xr0); ld4(a.xc + 3 * H, xr1);
  ld4(a.xc + 4 * H, xi0); ld4(a.xc + 5 * H, xi1);
  ld4(a.head, U0); ld4(a.head + H, U1); ld4(a.head + 2 * H, P0); ld4(a.head + 3 * H, P1);
  const float c0 = a.headb[0], c1 = a.headb[1], cp0 = a.headb[2], cp1 = a.headb[3];
  const float PI = 3.14159265358979323846f;
  const bool cplx = a.cplx != 0;
  const bool wr = w == 0 && grp == 0 && act;   // the lane that writes its sequence's outputs
  // every load of the set-up complete before the site loop: the loop's
  // global accesses are stores only, and no wait inside it may then count
  // the stores still in flight (vmcnt covers loads and stores alike)
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  __syncthreads();

  float h[4] = {0.f, 0.f, 0.f, 0.f};
  double lp = 0.0, ph = 0.0;
  int nup = 0, ndn = 0, nA = 0, sp = -1;
  // conditional of site k - 1 from the head sums the waves left in part[],
  // and the draw of its spin (every lane of the sequence draws the same)
  auto draw = [&](int k) {
    const int pb = k & 1;
    float4 zs = part[pb][0][col];
#pragma unroll
    for (int i = 1; i < NW; ++i) {
      const float4 t = part[pb][i][col];
      zs.x += t.x; zs.y += t.y; zs.z += t.z; zs.w += t.w;
    }
    const float zz0 = zs.x + c0, zz1 = zs.y + c1;
    const float mxz = fmaxf(zz0, zz1);
    const float d = -fabsf(zz0 - zz1);
    const float lse = mxz + 0.6931471805599453f *
                                __builtin_amdgcn_logf(1.f + __builtin_amdgcn_exp2f(1.4426950408889634f * d));
    float lp0 = zz0 - lse, lp1 = zz1 - lse;
    if (a.zero_mag) {
      const int half = N / 2;
      if (nup >= half) { lp0 = -INFINITY; lp1 = 0.f; }
      else if (ndn >= half) { lp0 = 0.f; lp1 = -INFINITY; }
    }
    float ph0 = 0.f, ph1 = 0.f;
    if (cplx) {
      const float aa0 = zs.z + cp0, aa1 = zs.w + cp1;
      ph0 = PI * aa0 * __builtin_amdgcn_rcpf(1.f + fabsf(aa0));
      ph1 = PI * aa1 * __builtin_amdgcn_rcpf(1.f + fabsf(aa1));
    }
    const double p0 = (double)__builtin_amdgcn_exp2f(1.4426950408889634f * lp0);
    const int v = uni[col][k] < p0 ? 0 : 1;
    lp += (double)(v == 0 ? lp0 : lp1);
    ph += (double)(v == 0 ? ph0 : ph1);
    nup += v == 0;
    ndn += v == 1;
    nA += subA[k] ? v : 0;
    sp = v;
    if (wr) {
      a.sigma[(size_t)s * N + k] = (uint8_t)v;
      if (a.site) {
        double* st = a.site + ((size_t)s * N + k) * 4;
        st[0] = (double)lp0; st[1] = (double)lp1; st[2] = (double)ph0; st[3] = (double)ph1;
      }
    }
  };
  for (int k = 0; k < N; ++k) {
    const int cb = k & 1, nb = cb ^ 1;
    // gate products of site k on h_k, issued before the spin of site k - 1
    // is drawn: the matrix cores run while the draw takes the vector units
    h16x8 bhi[KB], blo[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      bhi[kb] = *reinterpret_cast<const h16x8*>(&hsh[cb][col][32 * kb + 8 * grp]);
      blo[kb] = *reinterpret_cast<const h16x8*>(&hsl[cb][col][32 * kb + 8 * grp]);
    }
    f32x4v acc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      acc[q] = f32x4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        acc[q] = mma16(wal[q][kb], bhi[kb], acc[q]);
        acc[q] = mma16(wah[q][kb], blo[kb], acc[q]);
        acc[q] = mma16(wah[q][kb], bhi[kb], acc[q]);
      }
    }
    if (k > 0) draw(k - 1);
    // the cell for units j0 + v of this lane's sequence
    float hn[4], gu[4], gr[4], ag[4], gt[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float iu = sp == 0 ? xu0[v] : sp == 1 ? xu1[v] : 0.f;
      const float ir = sp == 0 ? xr0[v] : sp == 1 ? xr1[v] : 0.f;
      const float ii = sp == 0 ? xi0[v] : sp == 1 ? xi1[v] : 0.f;
      const float au = fmaf(acc[0][v], dsc[0][v], bu[v] + iu);
      const float ar = fmaf(acc[1][v], dsc[1][v], br[v] + ir);
      ag[v] = fmaf(acc[2][v], dsc[2][v], bh[v]);
      gu[v] = sigm_hw(au);
      gr[v] = sigm_hw(ar);
      gt[v] = tanh_hw(fmaf(gr[v], ag[v], bi[v] + ii));
      hn[v] = fmaf(gu[v], gt[v], (1.f - gu[v]) * h[v]);
    }
    {
      float x[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) x[v] = hn[v] * SM_HSCALE;
      h16x4 hi, lo;
      split16(x, hi, lo);
      *reinterpret_cast<h16x4*>(&hsh[nb][col][j0]) = hi;
      *reinterpret_cast<h16x4*>(&hsl[nb][col][j0]) = lo;
    }
    // output head: this lane's four units, then the four lanes of the
    // sequence, then (after the barrier) the waves in order
    float z0 = U0[0] * hn[0], z1 = U1[0] * hn[0], q0 = 0.f, q1 = 0.f;
#pragma unroll
    for (int v = 1; v < 4; ++v) {
      z0 = fmaf(U0[v], hn[v], z0);
      z1 = fmaf(U1[v], hn[v], z1);
    }
    if (cplx) {
      q0 = P0[0] * hn[0];
      q1 = P1[0] * hn[0];
#pragma unroll
      for (int v = 1; v < 4; ++v) {
        q0 = fmaf(P0[v], hn[v], q0);
        q1 = fmaf(P1[v], hn[v], q1);
      }
    }
    z0 = sum_xor32(sum_xor16(z0));
    z1 = sum_xor32(sum_xor16(z1));
    if (cplx) {
      q0 = sum_xor32(sum_xor16(q0));
      q1 = sum_xor32(sum_xor16(q1));
    }
    if (grp == 0) part[cb][w][col] = make_float4(z0, z1, q0, q1);
    if (act) {
      const size_t row = (size_t)s * N + k;
      if (a.states && (k + 1) % a.store_every == 0)
        *reinterpret_cast<float4*>(a.states + row * H + j0) = make_float4(hn[0], hn[1], hn[2], hn[3]);
      if (a.gates) {
        float* g = a.gates + row * 4 * H + j0;
        *reinterpret_cast<float4*>(g) = make_float4(gu[0], gu[1], gu[2], gu[3]);
        *reinterpret_cast<float4*>(g + H) = make_float4(gr[0], gr[1], gr[2], gr[3]);
        *reinterpret_cast<float4*>(g + 2 * H) = make_float4(ag[0], ag[1], ag[2], ag[3]);
        *reinterpret_cast<float4*>(g + 3 * H) = make_float4(gt[0], gt[1], gt[2], gt[3]);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) h[i] = hn[i];
    lds_barrier();
  }
  draw(N - 1);
  if (wr) {
    a.logpsi[2 * s] = 0.5 * lp;
    a.logpsi[2 * s + 1] = ph + 3.14159265358979323846 * (double)nA;
  }
}

bool sample_mfma_supported(const minsr_model* m) {
  return !m->f64 && !m->linear && m->dim == 1 && (m->H == 64 || m->H == 128) &&
         m->N <= SM_NMAX;
}

int launch_sample_mfma(minsr_model* m, int Ns, const double* uniforms, uint64_t key,
                       uint64_t counter, const uint64_t* counter_ptr, uint8_t* sigma,
                       double* logpsi, void* states, int store_every, double* site, void* gates,
                       uint32_t* zero_word, hipStream_t s) {
  if (Ns <= 0) return MINSR_OK;
  if (!sample_mfma_supported(m)) return fail(MINSR_E_UNSUPPORTED, "matrix-core sampler: shape");
  if (store_every < 1) return fail(MINSR_E_INVALID_ARG, "store_every >= 1");
  const Work<float>& w = m->wf;
  SampMArgs a{};
  a.fw = w.fw; a.xc = w.xc; a.bias = w.bias; a.head = w.head; a.headb = w.headb;
  a.N = m->N; a.Ns = Ns; a.zero_mag = m->d.zero_mag; a.cplx = m->cplx;
  a.marshall = m->d.marshall; a.store_every = store_every;
  a.subA = m->subA;
  a.uniforms = uniforms; a.key = key; a.counter = counter; a.counter_ptr = counter_ptr;
  a.zero_word = zero_word;
  a.sigma = sigma; a.logpsi = logpsi;
  a.states = (float*)states;
  a.gates = store_every == 1 ? (float*)gates : nullptr;
  a.site = site;
  const unsigned grid = (unsigned)((Ns + SM_SEQ - 1) / SM_SEQ);
  if (m->H == 64) k_sample_mfma<64><<<grid, 256, 0, s>>>(a);
  else k_sample_mfma<128><<<grid, 512, 0, s>>>(a);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

}  // namespace minsr
