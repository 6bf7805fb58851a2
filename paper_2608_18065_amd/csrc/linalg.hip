// Dense stages of one minSR iteration (Eqs. real-valued, minsrR; Alg. 1
// steps 6-9; App. B):
//   centring of O and conversion to the step's precision,
//   the sample-space Gram T = O' O'^T of the n x Np sample-major matrix,
//   the regularised FP64 (or FP32) Cholesky solve (T + lambda I) x = eps',
//   dtheta = eta O'^T x, momentum and the parameter update.
// Every reduction runs in a fixed order: results are bitwise reproducible.
#include "model.hpp"
#include "mfma16.hpp"
#include <algorithm>
#include <type_traits>
#include <cmath>

namespace minsr {

// ================================================================ centring
template <typename TI>
__global__ void k_colsum_part(const TI* O, int rows_per_block, int nrc, int RC, size_t Np,
                              double* part) {
  // part[(blk * nrc + chunk) * Np + col] = sum of the chunk's rows
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  const int blk = blockIdx.z, chunk = blockIdx.y;
  const int r0 = chunk * RC;
  const int r1 = min(rows_per_block, r0 + RC);
  const TI* base = O + ((size_t)blk * rows_per_block) * Np + col;
  // eight rows' loads in flight, then summed in row order
  double s = 0.0;
  for (int r = r0; r < r1; r += 8) {
    TI v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = base[(size_t)min(r + u, r1 - 1) * Np];   // tail rows repeat, unused
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (r + u < r1) s += (double)v[u];
  }
  part[((size_t)blk * nrc + chunk) * Np + col] = s;
}

__global__ void k_colmean(const double* part, int nrc, int rows_per_block, int nblocks, size_t Np,
                          double* mean) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  for (int b = 0; b < nblocks; ++b) {
    // four partial sums so that several loads are in flight
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    int c = 0;
    for (; c + 8 <= nrc; c += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[((size_t)b * nrc + c + u) * Np + col];
#pragma unroll
      for (int u = 0; u < 8; ++u) s4[u & 3] += v[u];
    }
    for (; c + 4 <= nrc; c += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) s4[u] += part[((size_t)b * nrc + c + u) * Np + col];
    }
    for (; c < nrc; ++c) s4[0] += part[((size_t)b * nrc + c) * Np + col];
    mean[(size_t)b * Np + col] = ((s4[0] + s4[1]) + (s4[2] + s4[3])) / rows_per_block;
  }
}

template <typename TO> __device__ inline TO cvt_out(double v);
template <> __device__ inline double cvt_out<double>(double v) { return v; }
template <> __device__ inline float cvt_out<float>(double v) { return (float)v; }
template <> __device__ inline __hip_bfloat16 cvt_out<__hip_bfloat16>(double v) {
  return __float2bfloat16((float)v);
}

// centred value in the input precision (FP32 rows are centred in FP32
// against the FP64 mean rounded to FP32), then rounded to the output type
// Rlo (BF16 output only, may be null): the rounding remainder
// bf16(v - float(bf16(v))), so that hi + lo carries v to about 16 bits
template <typename TI, typename TO>
__global__ void k_center(const TI* O, int rows_per_block, int RC, size_t Np, const double* mean,
                         TO* R, size_t ldo, TO* Rlo) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ldo) return;
  const int blk = blockIdx.z, chunk = blockIdx.y;
  const int r0 = chunk * RC;
  const int r1 = min(rows_per_block, r0 + RC);
  const size_t oo = ((size_t)blk * rows_per_block) * ldo + col;
  if (col >= Np) {   // zero padding of the output rows
    for (int r = r0; r < r1; ++r) {
      R[oo + (size_t)r * ldo] = cvt_out<TO>(0.0);
      if (Rlo) Rlo[oo + (size_t)r * ldo] = cvt_out<TO>(0.0);
    }
    return;
  }
  const TI mu = mean ? (TI)mean[(size_t)blk * Np + col] : (TI)0;
  const size_t off = ((size_t)blk * rows_per_block) * Np + col;
  for (int r = r0; r < r1; r += 8) {   // eight rows' loads in flight
    TI x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = O[off + (size_t)min(r + u, r1 - 1) * Np];   // tail rows repeat, unused
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (r + u >= r1) break;
      const TI v = x[u] - mu;
      const TO hi = cvt_out<TO>((double)v);
      R[oo + (size_t)(r + u) * ldo] = hi;
      if (Rlo) Rlo[oo + (size_t)(r + u) * ldo] = cvt_out<TO>((double)v - (double)(float)hi);
    }
  }
}

template <typename TI>
static int center_t(int rows_per_block, int nblocks, size_t Np, const TI* O, void* R,
                    int out_dtype, double* colpart, double* colmean, size_t ldo, void* Rlo,
                    hipStream_t s) {
  const int RC = 32;
  const int nrc = (rows_per_block + RC - 1) / RC;
  dim3 grid((unsigned)((Np + 255) / 256), (unsigned)nrc, (unsigned)nblocks);
  if (colmean) {
    k_colsum_part<TI><<<grid, 256, 0, s>>>(O, rows_per_block, nrc, RC, Np, colpart);
    MINSR_CHECK_LAUNCH();
    k_colmean<<<(unsigned)((Np + 255) / 256), 256, 0, s>>>(colpart, nrc, rows_per_block, nblocks,
                                                          Np, colmean);
    MINSR_CHECK_LAUNCH();
  }
  dim3 ogrid((unsigned)((ldo + 255) / 256), (unsigned)nrc, (unsigned)nblocks);
  switch (out_dtype) {
    case MINSR_F64:
      k_center<TI, double><<<ogrid, 256, 0, s>>>(O, rows_per_block, RC, Np, colmean, (double*)R, ldo, nullptr);
      break;
    case MINSR_F32:
      k_center<TI, float><<<ogrid, 256, 0, s>>>(O, rows_per_block, RC, Np, colmean, (float*)R, ldo, nullptr);
      break;
    case MINSR_BF16:
      k_center<TI, __hip_bfloat16><<<ogrid, 256, 0, s>>>(O, rows_per_block, RC, Np, colmean,
                                                          (__hip_bfloat16*)R, ldo,
                                                          (__hip_bfloat16*)Rlo);
      break;
    default:
      return fail(MINSR_E_INVALID_ARG, "unknown output dtype");
  }
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int launch_center(int rows_per_block, int nblocks, size_t Np, const void* O, int in_f64, void* R,
                  int out_dtype, double* colpart, double* colmean, size_t ldo, hipStream_t s,
                  void* Rlo) {
  if (rows_per_block == 0 || Np == 0) return MINSR_OK;
  if (in_f64)
    return center_t<double>(rows_per_block, nblocks, Np, (const double*)O, R, out_dtype, colpart,
                            colmean, ldo, Rlo, s);
  return center_t<float>(rows_per_block, nblocks, Np, (const float*)O, R, out_dtype, colpart,
                         colmean, ldo, Rlo, s);
}

// ================================================================== Gram
// Lower-triangular tile pairs (ti >= tj) of T = R R^T; split-K over the
// Np columns; partial tiles reduced in a fixed order and mirrored.
__device__ inline void pair_decode(int p, int& ti, int& tj) {
  int t = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while ((t + 1) * (t + 2) / 2 <= p) ++t;
  while (t * (t + 1) / 2 > p) --t;
  ti = t;
  tj = p - t * (t + 1) / 2;
}

// Work order of the Gram's tile pairs: blocks of GB x GB tiles (lower-
// triangular blocks, each block's pairs row by row), so the workgroups that
// run together on one XCD read few distinct row tiles of R and share them
// in that XCD's L2.  Work item q -> tile pair (ti, tj), ti >= tj.
constexpr int GB = 8;
__device__ inline void pair_blocked(int q, int nt, int& ti, int& tj) {
  const int nb = (nt + GB - 1) / GB;
  for (int I = 0; I < nb; ++I) {
    const int rows = min(GB, nt - GB * I);
    for (int J = 0; J <= I; ++J) {
      const int cols = min(GB, nt - GB * J);
      const int cnt = I == J ? rows * (rows + 1) / 2 : rows * cols;
      if (q < cnt) {
        if (I == J) {
          int r = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
          while ((r + 1) * (r + 2) / 2 <= q) ++r;
          while (r * (r + 1) / 2 > q) --r;
          ti = GB * I + r;
          tj = GB * J + (q - r * (r + 1) / 2);
        } else {
          ti = GB * I + q / cols;
          tj = GB * J + q % cols;
        }
        return;
      }
      q -= cnt;
    }
  }
  ti = tj = 0;
}

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(16))) float f32x16_t;

// BF16 MFMA tile kernel: 128 x 128 output tile per workgroup (8 waves,
// 32 x 64 each as 1 x 2 blocks of v_mfma_f32_32x32x16_bf16, so two waves
// share each SIMD and hide each other's latency), K staged
// through two LDS buffers: the next stage's global loads are in flight
// while the current stage feeds the matrix cores.  Rows of R have a stride
// ld that is a multiple of 64, zero-padded past Np.
// SPLIT: R = hi + lo (two BF16 arrays); the tile is hi hi^T + hi lo^T +
// lo hi^T + lo lo^T, the exact Gram of hi + lo, so T stays positive
// semidefinite up to accumulation error.  (lo is the BF16 residual of R,
// about 2^-8 of it, so lo lo^T is about 2^-16 of T: leaving it out subtracts
// a positive semidefinite matrix of that size, which made T + lambda I
// indefinite for lambda = 1e-3 once |T| grew to a few hundred.)
// The FP32 accumulators are added into FP64 ones every 128 (split) or 256
// (one product) input columns and restarted, so no FP32 sum runs longer;
// the partial tiles are written in FP64 (rounding them to FP32 put an error
// of about 2^-24 |T| on every element, whose 2-norm reached 6e-7 |T|_max).
constexpr int GT = 128;
constexpr int GFLUSH = 4;   // stages of 64 columns per flush (one product)

constexpr int GNT = 512;

// one tile pair over one K range: work item `item` of a Gram with npairs
// tile pairs (item = split * npairs + position in the blocked pair order)
template <bool SPLIT>
__device__ __forceinline__ void gram_tile(const __hip_bfloat16* R, const __hip_bfloat16* Rlo,
                                          int n, size_t ld, size_t kchunk, double* part,
                                          int npairs, int item) {
  // 64 columns per stage: the next stage's loads have a whole stage of
  // products (about 2000 matrix-core cycles per SIMD) to arrive in
  constexpr int GK = 64, GKP = GK + 8;
  constexpr int FLUSH = SPLIT ? GFLUSH / 2 : GFLUSH;
  constexpr int NOP = SPLIT ? 2 : 1;
  __shared__ __align__(16) __hip_bfloat16 As[2][NOP][GT][GKP];
  __shared__ __align__(16) __hip_bfloat16 Bs[2][NOP][GT][GKP];
  const int split = item / npairs;
  int ti, tj;
  pair_blocked(item % npairs, (n + GT - 1) / GT, ti, tj);
  const int pair = ti * (ti + 1) / 2 + tj;   // the partial tile's slot
  const size_t k0 = (size_t)split * kchunk;
  const size_t k1 = min(ld, k0 + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 64;
  f32x16_t acc[1][2];
  double accd[1][2][16];
#pragma unroll
  for (int a = 0; a < 1; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) { acc[a][b][e] = 0.f; accd[a][b][e] = 0.0; }
  auto flush = [&]() {
#pragma unroll
    for (int a = 0; a < 1; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 16; ++e) { accd[a][b][e] += (double)acc[a][b][e]; acc[a][b][e] = 0.f; }
  };

  const int arow0 = ti * GT, brow0 = tj * GT;
  constexpr int CPT = GT * (GK / 8) / GNT;
  uint4 ra[NOP][CPT], rb[NOP][CPT];
  auto load = [&](size_t kk) {
#pragma unroll
    for (int o = 0; o < NOP; ++o) {
      const __hip_bfloat16* M = o == 0 ? R : Rlo;
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        const int c = tid + GNT * i, r = c / (GK / 8), q = (c % (GK / 8)) * 8;
        const int xa = arow0 + r, xb = brow0 + r;
        ra[o][i] = xa < n ? *reinterpret_cast<const uint4*>(M + (size_t)xa * ld + kk + q) : make_uint4(0, 0, 0, 0);
        rb[o][i] = xb < n ? *reinterpret_cast<const uint4*>(M + (size_t)xb * ld + kk + q) : make_uint4(0, 0, 0, 0);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int o = 0; o < NOP; ++o)
#pragma unroll
      for (int i = 0; i < CPT; ++i) {
        const int c = tid + GNT * i, r = c / (GK / 8), q = (c % (GK / 8)) * 8;
        *reinterpret_cast<uint4*>(&As[buf][o][r][q]) = ra[o][i];
        *reinterpret_cast<uint4*>(&Bs[buf][o][r][q]) = rb[o][i];
      }
  };
  if (k0 < k1) {
    load(k0);
    store(0);
  }
  __syncthreads();
  int cur = 0, stages = 0;
  for (size_t kk = k0; kk < k1; kk += GK) {
    const bool more = kk + GK < k1;
    if (more) load(kk + GK);
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
      bf16x8_t fa[NOP][1], fb[NOP][2];
#pragma unroll
      for (int o = 0; o < NOP; ++o) {
#pragma unroll
        for (int a = 0; a < 1; ++a)
          fa[o][a] = *reinterpret_cast<const bf16x8_t*>(&As[cur][o][wm + a * 32 + (lane & 31)][ks + (lane >> 5) * 8]);
#pragma unroll
        for (int b = 0; b < 2; ++b)
          fb[o][b] = *reinterpret_cast<const bf16x8_t*>(&Bs[cur][o][wn + b * 32 + (lane & 31)][ks + (lane >> 5) * 8]);
      }
#pragma unroll
      for (int a = 0; a < 1; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0][a], fb[0][b], acc[a][b], 0, 0, 0);
          if (SPLIT) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[0][a], fb[NOP - 1][b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[NOP - 1][a], fb[0][b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[NOP - 1][a], fb[NOP - 1][b], acc[a][b], 0, 0, 0);
          }
        }
    }
    if (++stages == FLUSH) { flush(); stages = 0; }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  flush();
  // write the partial tile: acc element e of lane l is row
  // (e / 4) * 8 + (l / 32) * 4 + e % 4, column l % 32 of its 32 x 32 block
  double* out = part + ((size_t)split * npairs + pair) * GT * GT;
#pragma unroll
  for (int a = 0; a < 1; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = wm + a * 32 + (e / 4) * 8 + (lane >> 5) * 4 + (e % 4);
        const int c = wn + b * 32 + (lane & 31);
        out[r * GT + c] = accd[a][b][e];
      }
}

// workgroups are dealt to the eight XCDs in turn (linear id mod 8); each
// XCD takes a contiguous run of work items, so the pairs that read the same
// rows over the same K range share that XCD's L2
__device__ __forceinline__ int xcd_item(int lin, int total) {
  const int xcd = lin % 8;
  return xcd * (total / 8) + min(xcd, total % 8) + lin / 8;
}

template <bool SPLIT>
__global__ __launch_bounds__(GNT) void k_gram_bf16(const __hip_bfloat16* R,
                                                   const __hip_bfloat16* Rlo, int n, size_t ld,
                                                   size_t kchunk, double* part) {
  const int npairs = gridDim.x, total = npairs * gridDim.y;
  gram_tile<SPLIT>(R, Rlo, n, ld, kchunk, part, npairs,
                   xcd_item(blockIdx.x + blockIdx.y * npairs, total));
}

// the Grams of several instances (BF16 split form) in one launch: the work
// items of instance j are [item0, item0 + npairs S) of the grid, each
// instance with its own split, so every partial tile equals the one of the
// instance's own launch; the reduction likewise over (instance, pair,
// 32 x 32 sub-tile)
__global__ __launch_bounds__(GNT) void k_gram_bf16_grouped(const GramJob* jobs, int njobs,
                                                           int total) {
  const int item = xcd_item(blockIdx.x, total);
  int j = 0;
  while (j + 1 < njobs && item >= jobs[j + 1].item0) ++j;
  const GramJob& g = jobs[j];
  gram_tile<true>(static_cast<const __hip_bfloat16*>(g.R), static_cast<const __hip_bfloat16*>(g.Rlo),
                  g.n, g.ld, g.kchunk, g.part, g.npairs, item - g.item0);
}

// FP32 MFMA tile kernel (the FP32 form): 128 x 128 output tile per
// workgroup (4 waves, 64 x 64 each as 2 x 2 blocks of
// v_mfma_f32_32x32x2_f32, lane l supplying A[l % 32][l / 32] and
// B[l / 32][l % 32]), FP32 accumulation over the workgroup's K range like
// the form's other arithmetic, K staged 32 columns at a time through two
// shared-memory buffers while the next stage's loads are in flight.
constexpr int FK = 32, FKP = FK + 1;

__global__ __launch_bounds__(256, 2) void k_gram_f32(const float* R, int n, size_t ld,
                                                     size_t kchunk, float* part) {
  __shared__ float As[2][GT][FKP];
  __shared__ float Bs[2][GT][FKP];
  const int npairs = gridDim.x, total = npairs * gridDim.y;
  const int lin = blockIdx.x + blockIdx.y * npairs, xcd = lin % 8;
  const int item = xcd * (total / 8) + min(xcd, total % 8) + lin / 8;
  const int split = item / npairs;
  int ti, tj;
  pair_blocked(item % npairs, (n + GT - 1) / GT, ti, tj);
  const int pair = ti * (ti + 1) / 2 + tj;
  const size_t k0 = (size_t)split * kchunk;
  const size_t k1 = min(ld, k0 + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f32x16_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[a][b][e] = 0.f;
  const int arow0 = ti * GT, brow0 = tj * GT;
  constexpr int CPT = GT * (FK / 4) / 256;   // float4 per thread and operand
  float4 ra[CPT], rb[CPT];
  auto load = [&](size_t kk) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int c = tid + 256 * i, r = c / (FK / 4), q = (c % (FK / 4)) * 4;
      const int xa = arow0 + r, xb = brow0 + r;
      ra[i] = xa < n ? *reinterpret_cast<const float4*>(R + (size_t)xa * ld + kk + q) : make_float4(0, 0, 0, 0);
      rb[i] = xb < n ? *reinterpret_cast<const float4*>(R + (size_t)xb * ld + kk + q) : make_float4(0, 0, 0, 0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int c = tid + 256 * i, r = c / (FK / 4), q = (c % (FK / 4)) * 4;
      As[buf][r][q] = ra[i].x; As[buf][r][q + 1] = ra[i].y;
      As[buf][r][q + 2] = ra[i].z; As[buf][r][q + 3] = ra[i].w;
      Bs[buf][r][q] = rb[i].x; Bs[buf][r][q + 1] = rb[i].y;
      Bs[buf][r][q + 2] = rb[i].z; Bs[buf][r][q + 3] = rb[i].w;
    }
  };
  if (k0 < k1) {
    load(k0);
    store(0);
  }
  __syncthreads();
  int cur = 0;
  const int lr = lane & 31, lk = lane >> 5;
  for (size_t kk = k0; kk < k1; kk += FK) {
    const bool more = kk + FK < k1;
    if (more) load(kk + FK);
#pragma unroll
    for (int ks = 0; ks < FK; ks += 2) {
      float fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) fa[a] = As[cur][wm + a * 32 + lr][ks + lk];
#pragma unroll
      for (int b = 0; b < 2; ++b) fb[b] = Bs[cur][wn + b * 32 + lr][ks + lk];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  // acc element e of lane l is row (e / 4) * 8 + (l / 32) * 4 + e % 4,
  // column l % 32 of its 32 x 32 block
  float* out = part + ((size_t)split * npairs + pair) * GT * GT;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = wm + a * 32 + (e / 4) * 8 + (lane >> 5) * 4 + (e % 4);
        const int c = wn + b * 32 + (lane & 31);
        out[r * GT + c] = acc[a][b][e];
      }
}

// Vector SYRK tile kernel for FP32 / FP64 inputs: 64 x 64 tile, 256
// threads with 4 x 4 outputs each, K staged 16 at a time.
constexpr int VT_ = 64, VK = 16;

template <typename TI, typename TA>
__global__ __launch_bounds__(256) void k_gram_vec(const TI* R, int n, size_t Np, size_t kchunk,
                                                  TA* part) {
  __shared__ TA As[VK][VT_ + 1];
  __shared__ TA Bs[VK][VT_ + 1];
  int ti, tj;
  pair_decode(blockIdx.x, ti, tj);
  const int split = blockIdx.y;
  const size_t k0 = (size_t)split * kchunk;
  const size_t k1 = min(Np, k0 + kchunk);
  const int tid = threadIdx.x;
  const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
  TA acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (TA)0;
  const int arow0 = ti * VT_, brow0 = tj * VT_;
  for (size_t kk = k0; kk < k1; kk += VK) {
    TA va[VT_ * VK / 256], vb[VT_ * VK / 256];
#pragma unroll
    for (int i = 0; i < VT_ * VK / 256; ++i) {
      const int e = tid + 256 * i, r = e / VK, q = e % VK;
      const size_t col = kk + q;
      const int ra = arow0 + r, rb = brow0 + r;
      va[i] = (col < k1 && ra < n) ? (TA)R[(size_t)ra * Np + col] : (TA)0;
      vb[i] = (col < k1 && rb < n) ? (TA)R[(size_t)rb * Np + col] : (TA)0;
    }
#pragma unroll
    for (int i = 0; i < VT_ * VK / 256; ++i) {
      const int e = tid + 256 * i, r = e / VK, q = e % VK;
      As[q][r] = va[i];
      Bs[q][r] = vb[i];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < VK; ++q) {
      TA av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[q][tr + a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[q][tc + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  TA* out = part + ((size_t)split * gridDim.x + blockIdx.x) * VT_ * VT_;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) out[(tr + a) * VT_ + tc + b] = acc[a][b];
}

// sum the split-K partials in split order; write T (lower and mirror)
template <typename TA, typename TT>
__device__ __forceinline__ void gram_reduce_tile(const TA* part, int npairs, int nsplit,
                                                 int tile, int n, TT* T, int pair, int sub) {
  // one 32 x 32 sub-tile per workgroup: partials summed in split order, the
  // tile written row-wise and its mirror through a shared-memory transpose,
  // so both stores are coalesced rows
  __shared__ TT sh[32][33];
  const int nsub = tile / 32;
  const int sr = sub / nsub, sc = sub % nsub;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  int ti, tj;
  pair_decode(pair, ti, tj);
  // partials summed in split order, eight splits' loads in flight
  TA s[4] = {(TA)0, (TA)0, (TA)0, (TA)0};
  for (int k0 = 0; k0 < nsplit; k0 += 8) {
    TA v[4][8];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int lr = sr * 32 + ty + 8 * q, lc = sc * 32 + tx;
        const int k = min(k0 + u, nsplit - 1);   // tail splits repeat, unused
        v[q][u] = part[((size_t)k * npairs + pair) * tile * tile + lr * tile + lc];
      }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k0 + u < nsplit) s[q] += v[q][u];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int lr = sr * 32 + ty + 8 * q, lc = sc * 32 + tx;
    const int r = ti * tile + lr, c = tj * tile + lc;
    sh[ty + 8 * q][tx] = (TT)s[q];
    if (r < n && c < n && (ti != tj || c <= r)) T[(size_t)r * n + c] = (TT)s[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int lr = sr * 32 + tx, lc = sc * 32 + ty + 8 * q;   // element (lr, lc) to T[c][r]
    const int r = ti * tile + lr, c = tj * tile + lc;
    if (r < n && c < n && (ti != tj || c <= r)) T[(size_t)c * n + r] = sh[tx][ty + 8 * q];
  }
}

template <typename TA, typename TT>
__global__ __launch_bounds__(256) void k_gram_reduce(const TA* part, int npairs, int nsplit,
                                                     int tile, int n, TT* T) {
  gram_reduce_tile<TA, TT>(part, npairs, nsplit, tile, n, T, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_gram_reduce_grouped(const GramJob* jobs, int njobs) {
  constexpr int SUB = GRAM_SUBTILES;
  static_assert(SUB == (GT / 32) * (GT / 32), "sub-tiles of a Gram tile");
  int j = 0;
  while (j + 1 < njobs && (int)blockIdx.x >= jobs[j + 1].ritem0) ++j;
  const GramJob& g = jobs[j];
  const int r = blockIdx.x - g.ritem0;
  gram_reduce_tile<double, double>(g.part, g.npairs, g.S, GT, g.n, g.T, r / SUB, r % SUB);
}

constexpr int MAX_SPLIT = 64;

// split-K factor: requested, else enough for ~1024 workgroups; at most
// MAX_SPLIT, 4096 workgroups in total, and chunks of >= 256 columns
static int pick_split(int npairs, size_t Np, int want) {
  // default: about 4096 workgroups, at most 8 partial tiles per pair
  int S = want > 0 ? want : std::min(8, (4096 + npairs - 1) / npairs);
  const int by_grid = std::max(1, (4096 + npairs - 1) / npairs);
  int maxS = (int)std::max<size_t>(1, std::min<size_t>(MAX_SPLIT, Np / 256));
  maxS = std::min(maxS, by_grid);
  return std::max(1, std::min(S, maxS));
}

// workspace for the largest split any setting may request
size_t gram_partial_bytes(int n, size_t Np, int dtype) {
  const int tile = dtype == MINSR_F64 ? VT_ : GT;
  const int nt = (n + tile - 1) / tile;
  const int npairs = nt * (nt + 1) / 2;
  const int S = std::max(pick_split(npairs, Np, 0), pick_split(npairs, Np, MAX_SPLIT));
  const size_t el = dtype == MINSR_F32 ? 4 : 8;
  return (size_t)S * npairs * tile * tile * el;
}

// split-K factor and K range per workgroup: the MFMA tile kernel holds one
// workgroup per CU (FP64 accumulators), so by default the split (1..8)
// minimises rounds of the grid over the CUs times the K range of one
// workgroup
static void gram_plan(int npairs, size_t Np, size_t ld, int dtype, int want_split, int& S,
                      size_t& kchunk) {
  int want = want_split;
  if (dtype == MINSR_BF16 && want_split <= 0) {
    static int ncu = 0;
    if (ncu == 0) {
      int dev = 0, v = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
        ncu = v;
      else
        ncu = 256;
    }
    double best = 1e300;
    for (int q = 1; q <= 8; ++q) {
      const double cost = (double)((npairs * q + ncu - 1) / ncu) / q;
      if (cost < best * (1.0 - 1e-9)) { best = cost; want = q; }
    }
  }
  S = pick_split(npairs, Np, want);
  const size_t kgran = dtype == MINSR_BF16 ? 64 : dtype == MINSR_F32 ? FK : VK;
  kchunk = (ld + S - 1) / S;
  kchunk = (kchunk + kgran - 1) / kgran * kgran;
}

int gram_job(int n, size_t Np, const void* R, const void* Rlo, double* T, float* gpart,
             size_t gpart_elems, int want_split, GramJob* job) {
  const size_t ld = (Np + 63) / 64 * 64;
  const int nt = (n + GT - 1) / GT;
  const int npairs = nt * (nt + 1) / 2;
  int S = 0;
  size_t kchunk = 0;
  gram_plan(npairs, Np, ld, MINSR_BF16, want_split, S, kchunk);
  if ((size_t)S * npairs * GT * GT * 8 > gpart_elems * sizeof(float))
    return fail(MINSR_E_SHAPE, "Gram workspace too small");
  *job = GramJob{R, Rlo, reinterpret_cast<double*>(gpart), T, ld, kchunk, n, npairs, S, 0, 0, 0};
  return MINSR_OK;
}

int launch_gram_grouped(const GramJob* dev_jobs, int njobs, int items, int ritems,
                        hipStream_t s) {
  if (njobs == 0 || items == 0) return MINSR_OK;
  k_gram_bf16_grouped<<<(unsigned)items, GNT, 0, s>>>(dev_jobs, njobs, items);
  MINSR_CHECK_LAUNCH();
  k_gram_reduce_grouped<<<(unsigned)ritems, 256, 0, s>>>(dev_jobs, njobs);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int launch_gram(int n, size_t Np, const void* R, int dtype, double* T, float* gpart,
                size_t gpart_elems, hipStream_t s, int which, const void* Rlo, int want_split) {
  // R rows have the padded stride ld = round_up(Np, 64); the padding is zero
  const size_t ld = (Np + 63) / 64 * 64;
  if (n == 0) return MINSR_OK;
  const int tile = dtype == MINSR_F64 ? VT_ : GT;
  const int nt = (n + tile - 1) / tile;
  const int npairs = nt * (nt + 1) / 2;
  int S = 0;
  size_t kchunk = 0;
  gram_plan(npairs, Np, ld, dtype, want_split, S, kchunk);
  const size_t need = (size_t)S * npairs * tile * tile * (dtype == MINSR_F32 ? 4 : 8);
  if (need > gpart_elems * sizeof(float)) return fail(MINSR_E_SHAPE, "Gram workspace too small");
  dim3 grid((unsigned)npairs, (unsigned)S);
  dim3 rgrid((unsigned)((tile / 32) * (tile / 32)), (unsigned)npairs);
  if (dtype == MINSR_BF16) {
    double* dp = reinterpret_cast<double*>(gpart);
    if (which & 1) {
      if (Rlo)
        k_gram_bf16<true><<<grid, GNT, 0, s>>>((const __hip_bfloat16*)R,
                                               (const __hip_bfloat16*)Rlo, n, ld, kchunk, dp);
      else
        k_gram_bf16<false><<<grid, GNT, 0, s>>>((const __hip_bfloat16*)R, nullptr, n, ld, kchunk,
                                                dp);
      MINSR_CHECK_LAUNCH();
    }
    if (which & 2) k_gram_reduce<double, double><<<rgrid, 256, 0, s>>>(dp, npairs, S, tile, n, T);
  } else if (dtype == MINSR_F32) {
    if (which & 1) {
      k_gram_f32<<<grid, 256, 0, s>>>((const float*)R, n, ld, kchunk, gpart);
      MINSR_CHECK_LAUNCH();
    }
    if (which & 2) k_gram_reduce<float, float><<<rgrid, 256, 0, s>>>(gpart, npairs, S, tile, n, (float*)T);
  } else {
    double* dp = reinterpret_cast<double*>(gpart);
    if (which & 1) {
      k_gram_vec<double, double><<<grid, 256, 0, s>>>((const double*)R, n, ld, kchunk, dp);
      MINSR_CHECK_LAUNCH();
    }
    if (which & 2) k_gram_reduce<double, double><<<rgrid, 256, 0, s>>>(dp, npairs, S, tile, n, T);
  }
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

// ============================================================= Cholesky
// Right-looking tiled Cholesky of A = T + lambda I (lower, row-major, tiles
// of 64) into a separate buffer, so T survives, with the forward
// substitution L y = b folded in.  FP64 runs the whole factorisation in one
// launch (k_chol_persist_f64, below).  FP32 takes one launch per block
// column k:
//   every workgroup updates one trailing tile A_ij -= L_ik L_jk^T (i >= j > k);
//   the workgroup of the next diagonal tile then factors it, forms the
//   inverse of its factor and the block y_{k+1} = inv(L) b_{k+1}, and
//   publishes them through a flag;
//   the workgroups of the tiles below it wait for the flag, finish their
//   panel tile L_i,k+1 = A_i,k+1 inv(L_k+1,k+1)^T and subtract
//   L_i,k+1 y_k+1 from their block of b.
// Roles come from a ticket taken when a workgroup starts, so the ticket-0
// workgroup (the factoring one) is resident before anyone waits on it.
// The backward substitution L^T x = y runs last, with the stored inverses.
constexpr int CB = 64;

__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
// 1/sqrt(d) from the hardware estimate and Newton steps
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-(d * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}
// 1/sqrt(d) from the hardware estimate y (relative error below 2^-24 on
// this chip, measured) and one third-order step y (1 + e/2 + 3 e^2 / 8),
// e = 1 - d y^2: the truncation error is about 5 e^3 / 16 < 2^-70, so the
// result is FP64-accurate in five dependent operations
__device__ __forceinline__ double rsqrt_h(double d) {
  const double y = __builtin_amdgcn_rsq(d);
  const double e = fma(-(d * y), y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}
__device__ __forceinline__ float rsqrt_nr(float d) {
  float y = __builtin_amdgcn_rsqf(d);
  const float e = fmaf(-(d * y), y, 1.0f);
  return fmaf(0.5f * y, e, y);
}

// Factor the 64 x 64 tile Lt (rows < nb valid, lower triangle read) with a
// workgroup of four wavefronts; every thread must call it.  Wave w keeps, for
// row `lane`, the sixteen columns [16w, 16w + 16) in registers.  Panel P
// (the columns of wave P) is factored by wave P alone, the pivot column
// reaching the other lanes through readlane; the later waves then subtract
// the rank-16 product of the panel, read from shared memory.  The inverse
// follows blockwise: each wave inverts its 16 x 16 diagonal block with the
// same register broadcasts, the blocks below by Z_QP = -Z_QQ sum_R L_QR Z_RP.
// Writes L to A and to Lt (zero above the diagonal), inv(L) to Di and Is.
template <typename TT>
__device__ void factor_block(TT (*Lt)[CB + 1], TT (*Pn)[CB], TT (*Is)[CB + 1], int nb, TT* A,
                             int n, int k0, TT* Di, uint32_t* status) {
  constexpr int PB = 16;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  TT f[PB];
#pragma unroll
  for (int k = 0; k < PB; ++k) {
    const int q = PB * w + k;
    f[k] = lane < nb ? (q <= lane ? Lt[lane][q] : (TT)0) : (lane == q ? (TT)1 : (TT)0);
  }
  bool bad = false;
  __syncthreads();
  for (int P = 0; P < CB / PB; ++P) {
    if (w == P) {
#pragma unroll
      for (int cc = 0; cc < PB; ++cc) {
        const int c = PB * P + cc;
        TT d = lane_bcast(f[cc], c);
        if (!(d > (TT)0)) { bad = true; d = (TT)1; }
        const TT rp = rsqrt_nr(d);
        const TT lc = (lane == c) ? d * rp : f[cc] * rp;
        f[cc] = lc;
        const TT nl = lane > c ? -lc : (TT)0;
#pragma unroll
        for (int kk = cc + 1; kk < PB; ++kk) f[kk] = fma(nl, lane_bcast(lc, PB * P + kk), f[kk]);
      }
#pragma unroll
      for (int cc = 0; cc < PB; ++cc) Pn[lane][cc] = f[cc];
    }
    __syncthreads();
    if (w > P) {
      TT own[PB];
#pragma unroll
      for (int cc = 0; cc < PB; ++cc) own[cc] = Pn[lane][cc];
#pragma unroll
      for (int k = 0; k < PB; ++k) {
        const int q = PB * w + k;
        TT s = (TT)0;
#pragma unroll
        for (int cc = 0; cc < PB; ++cc) s = fma(own[cc], Pn[q][cc], s);
        f[k] -= s;
      }
    }
    __syncthreads();
  }
  if (bad && lane == 0 && status) atomicOr(status, MINSR_ST_NOT_PD);
  // L to shared memory and A
#pragma unroll
  for (int k = 0; k < PB; ++k) {
    const int q = PB * w + k;
    const TT v = q <= lane ? f[k] : (TT)0;
    Lt[lane][q] = v;
    if (q <= lane && lane < nb) A[(size_t)(k0 + lane) * n + k0 + q] = v;
  }
  // inverse of this wave's diagonal block: lane 16w + j keeps column j
  {
    TT z[PB];
#pragma unroll
    for (int i = 0; i < PB; ++i) z[i] = (PB * w + i == lane) ? (TT)1 : (TT)0;
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const TT lii = lane_bcast(f[i], PB * w + i);
      const TT zi = z[i] / lii;
      z[i] = zi;
#pragma unroll
      for (int q = i + 1; q < PB; ++q) z[q] = fma(-lane_bcast(f[i], PB * w + q), zi, z[q]);
    }
    if (lane >= PB * w && lane < PB * (w + 1)) {
#pragma unroll
      for (int i = 0; i < PB; ++i) Is[PB * w + i][lane] = z[i];
    }
  }
  // the other blocks start at zero (the ones below are filled next)
  for (int e = tid; e < CB * CB; e += 256) {
    const int i = e / CB, j = e % CB;
    if (i / PB != j / PB) Is[i][j] = (TT)0;
  }
  __syncthreads();
  // blocks below the diagonal, one level of Q - P at a time
  TT* tmp = &Pn[0][0];   // [3][16][16]
  for (int lv = 1; lv < CB / PB; ++lv) {
    const int nblk = CB / PB - lv;
    for (int e = tid; e < nblk * PB * PB; e += 256) {
      const int b = e / (PB * PB), i = (e / PB) % PB, j = e % PB;
      const int P = b, Q = b + lv;
      TT s = (TT)0;
      for (int R = P; R < Q; ++R)
        for (int k = 0; k < PB; ++k) s = fma(Lt[PB * Q + i][PB * R + k], Is[PB * R + k][PB * P + j], s);
      tmp[e] = s;
    }
    __syncthreads();
    for (int e = tid; e < nblk * PB * PB; e += 256) {
      const int b = e / (PB * PB), i = (e / PB) % PB, j = e % PB;
      const int P = b, Q = b + lv;
      TT s = (TT)0;
      for (int k = 0; k < PB; ++k) s = fma(Is[PB * Q + i][PB * Q + k], tmp[b * PB * PB + k * PB + j], s);
      Is[PB * Q + i][PB * P + j] = -s;
    }
    __syncthreads();
  }
  for (int e = tid; e < CB * CB; e += 256) {
    const int i = e / CB, j = e % CB;
    Di[e] = (i < nb && j < nb) ? Is[i][j] : (TT)0;
  }
}

struct CholArgs {
  const void* T;        // source matrix (read while a tile is first touched)
  void* A;              // factor
  void* Dinv;           // [nblk][64][64]
  void* y;              // [n] right-hand side, overwritten by L^-1 b block by block
  uint32_t* sync;       // [2][nblk + 1]: tickets, then flags
  uint32_t* status;
  double lambda;
  const double* lam_dev;  // if set, the shift actually used (FP64 one-launch kernel)
  int n, nblk;
  uint32_t* abort;        // set by the first wait that gives up
  uint32_t spin_limit;    // polls before a wait gives up
};

// A wait on a flag another workgroup publishes, bounded: after `limit`
// polls, or as soon as some wait of the launch has given up (the abort
// word), it stops waiting, sets MINSR_ST_SOLVE_TIMEOUT and the abort word,
// and returns false.  Every wait of the launch then ends, so the kernel
// exits whatever happened to the publishing workgroup; the solve's result
// is invalid and the status word says so.  Relaxed polls (an acquiring load
// would invalidate this CU's caches at every poll); the caller fences once.
__device__ inline bool bounded_wait(const uint32_t* f, uint32_t* abort, uint32_t limit,
                                    uint32_t* status) {
  uint32_t polls = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
    ++polls;
    if (polls >= limit ||
        ((polls & 63u) == 0u &&
         __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
      if (status) atomicOr(status, MINSR_ST_SOLVE_TIMEOUT);
      __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}
constexpr uint32_t DEFAULT_SPIN_LIMIT = 1u << 22;

// Block column k of the factorisation (k = -1: the first block column,
// read straight from T).
template <typename TT>
__global__ __launch_bounds__(256) void k_chol_step(CholArgs a, int k) {
  __shared__ TT Li[CB][CB + 1];
  __shared__ TT Lj[CB][CB + 1];
  __shared__ __align__(16) TT Lc[CB][CB];
  __shared__ TT yb[CB];
  __shared__ int tk;
  const int n = a.n, tid = threadIdx.x;
  TT* A = reinterpret_cast<TT*>(a.A);
  const TT* Tm = reinterpret_cast<const TT*>(a.T);
  TT* y = reinterpret_cast<TT*>(a.y);
  uint32_t* tickets = a.sync;
  uint32_t* flags = a.sync + (a.nblk + 1);
  const int kk = k + 1;                  // block column being finished
  if (tid == 0)
    tk = (int)__hip_atomic_fetch_add(&tickets[kk], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int ticket = tk;
  int ti, tj;
  if (k < 0) { ti = ticket; tj = 0; }
  else { pair_decode(ticket, ti, tj); ti += kk; tj += kk; }
  const int r0 = ti * CB, c0 = tj * CB;
  const bool fresh = k <= 0;             // tile not written before: read T + lambda I
  const TT* src = fresh ? Tm : A;
  const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;

  // current tile values (lower part of diagonal tiles only)
  TT t[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const int r = r0 + tr + x, c = c0 + tc + z;
      TT val = (TT)0;
      if (r < n && c < n && (ti != tj || c <= r)) {
        val = src[(size_t)r * n + c];
        if (fresh && r == c) val += (TT)a.lambda;
      }
      t[x][z] = val;
    }
  if (k >= 0) {
    // A_ij -= L_ik L_jk^T
    const int k0 = k * CB;
    {
      TT vi[CB * CB / 256], vj[CB * CB / 256];
#pragma unroll
      for (int i = 0; i < CB * CB / 256; ++i) {
        const int e = tid + 256 * i, r = e / CB, q = e % CB;
        vi[i] = (r0 + r < n) ? A[(size_t)(r0 + r) * n + k0 + q] : (TT)0;
        vj[i] = (c0 + r < n) ? A[(size_t)(c0 + r) * n + k0 + q] : (TT)0;
      }
#pragma unroll
      for (int i = 0; i < CB * CB / 256; ++i) {
        const int e = tid + 256 * i, r = e / CB, q = e % CB;
        Li[r][q] = vi[i];
        Lj[r][q] = vj[i];
      }
    }
    __syncthreads();
    TT acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int z = 0; z < 4; ++z) acc[x][z] = (TT)0;
#pragma unroll 4
    for (int q = 0; q < CB; ++q) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int z = 0; z < 4; ++z) acc[x][z] = fma(Li[tr + x][q], Lj[tc + z][q], acc[x][z]);
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int z = 0; z < 4; ++z) t[x][z] -= acc[x][z];
    __syncthreads();   // Li, Lj are reused below
  }

  if (tj != kk) {
    // plain trailing tile
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int z = 0; z < 4; ++z) {
        const int r = r0 + tr + x, c = c0 + tc + z;
        if (r < n && c < n && (ti != tj || c <= r)) A[(size_t)r * n + c] = t[x][z];
      }
    return;
  }

  const int kb0 = kk * CB, nb = min(CB, n - kb0);
  TT* Di = reinterpret_cast<TT*>(a.Dinv) + (size_t)kk * CB * CB;
  if (ti == kk) {
    // diagonal tile: factor, invert, y_kk = inv(L) b_kk, publish
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int z = 0; z < 4; ++z) Li[tr + x][tc + z] = t[x][z];
    if (tid < CB) yb[tid] = tid < nb ? y[kb0 + tid] : (TT)0;
    __syncthreads();
    factor_block<TT>(Li, Lc, Lj, nb, A, n, kb0, Di, a.status);
    __syncthreads();
    // y_kk = inv(L) b_kk with the inverse from shared memory, 4 threads a row
    {
      const int row = tid / 4, part = tid % 4;
      TT s = (TT)0;
      if (row < nb)
        for (int q = part; q <= row; q += 4) s = fma(Lj[row][q], yb[q], s);
      s += __shfl_xor(s, 1, 4);
      s += __shfl_xor(s, 2, 4);
      if (part == 0 && row < nb) y[kb0 + row] = s;
    }
    if (kk + 1 < a.nblk) {
      // every wave's stores complete (a workgroup barrier alone does not wait
      // for global stores), then one agent-scope release: a single L2
      // write-back instead of one per wave
      __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
      __syncthreads();
      if (tid == 0) __hip_atomic_store(&flags[kk], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }

  // panel tile below the diagonal: wait for the factor of block kk
  if (tid == 0) {
    bounded_wait(&flags[kk], a.abort, a.spin_limit, a.status);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  // the acquire invalidated this CU's L1 and its L2 for every wave
  __syncthreads();
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int z = 0; z < 4; ++z) Li[tr + x][tc + z] = t[x][z];
#pragma unroll
  for (int i = 0; i < CB * CB / 256; ++i) {
    const int e = tid + 256 * i, r = e / CB, q = e % CB;
    Lj[r][q] = Di[e];
  }
  if (tid < CB) yb[tid] = y[kb0 + tid < n ? kb0 + tid : 0];
  __syncthreads();
  TT l[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int z = 0; z < 4; ++z) l[x][z] = (TT)0;
#pragma unroll 4
  for (int q = 0; q < CB; ++q) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int z = 0; z < 4; ++z) l[x][z] = fma(Li[tr + x][q], Lj[tc + z][q], l[x][z]);
  }
  TT s[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    s[x] = (TT)0;
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const int r = r0 + tr + x, c = tc + z;
      const bool ok = r < n && c < nb;
      if (ok) A[(size_t)r * n + kb0 + c] = l[x][z];
      s[x] = fma(ok ? l[x][z] : (TT)0, yb[c], s[x]);
    }
  }
  // the 16 threads of a row group hold the 64 columns of rows tr..tr+3
#pragma unroll
  for (int x = 0; x < 4; ++x) {
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) s[x] += __shfl_xor(s[x], m, 16);
  }
  if (tid % 16 == 0) {
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int r = r0 + tr + x;
      if (r < n) y[r] -= s[x];
    }
  }
}

// ------------------------------------------- FP64 path on the matrix cores
// The same algorithm for FP64 with every tile product (trailing updates,
// panel products, the blocked inverse) on the 16 x 16 x 4 FP64 MFMA.  Lane l
// of a wavefront supplies A[l % 16][l / 16] and B[l / 16][l % 16] of the
// product and receives D[l / 16 + 4 v][l % 16] in element v.
typedef double f64x4_t __attribute__((ext_vector_type(4)));
constexpr int LDT = CB + 1;   // row stride of the shared tiles (odd: rows fall in distinct banks)

__device__ __forceinline__ int mrow(int lane, int v) { return (lane >> 4) + 4 * v; }

// acc (+/-)= X[xr + i][k0 + k] Y[yr + j][k0 + k] summed over k < K, for the
// 16 x 16 block (i, j)
template <int K, bool NEG>
__device__ __forceinline__ f64x4_t mm_nt(f64x4_t acc, const double (*X)[LDT], int xr,
                                         const double (*Y)[LDT], int yr, int k0, int lane) {
#pragma unroll
  for (int s = 0; s < K; s += 4) {
    const double xa = X[xr + (lane & 15)][k0 + s + (lane >> 4)];
    const double yb = Y[yr + (lane & 15)][k0 + s + (lane >> 4)];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(NEG ? -xa : xa, yb, acc, 0, 0, 0);
  }
  return acc;
}

// Factor the 64 x 64 tile S (lower triangle; rows >= nb are made identity
// rows) in place and write inv(L) into Z, with four wavefronts.  Panels of
// 16 columns are factored by wave 0 alone, two columns at a time (row
// `lane` in registers, the pair's columns reaching the other lanes through
// readlane and the scratch columns lb[2][64]); after each panel the four
// waves subtract its rank-16 product from the 16 x 16 blocks of the
// trailing lower triangle on the MFMA.  The inverse is blockwise: wave w
// inverts diagonal block w by forward substitution (lane j: column j), then
// level by level Z_QP = -Z_QQ sum_{P <= R < Q} L_QR Z_RP, one block per
// wave.  L stays in S (the caller stores it); inv(L) goes to Z and to Di
// (zero outside the leading nb x nb block).
// `during_first_panel` runs on waves 1..3 while wave 0 factors the first
// panel (it may complete columns 16.. of S); with `fill` false the caller has
// already made the rows >= nb identity rows.  `pub` (may be null) is
// released once the barrier after the first panel has seen every wave's
// earlier global stores complete: the caller's stores are published off
// wave 0's path.
template <typename F>
__device__ void factor_block_f64(double (*S)[LDT], double (*Z)[LDT], double (*Tm)[16][17],
                                 double* rinv, double* lb, int nb, int k0, double* Di,
                                 uint32_t* status, bool fill, F&& during_first_panel,
                                 uint32_t* pub) {
  constexpr int PB = 16, NB = CB / 16;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  if (fill && nb < CB) {   // the last, partial block only
    for (int e = tid; e < CB * CB; e += 256) {
      const int r = e / CB, c = e % CB;
      if (r >= nb && c <= r) S[r][c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
  }
  // the blockwise inverse, on the calling wave: Z_bb of diagonal block b
  // (lane j: column j by forward substitution, the terms of each row taken in
  // order of m, column by column so the dependent chain is one fma deep);
  // Tm[slot] = sum_{P <= R < Q} L_QR Z_RP; Z_QP = -Z_QQ Tm[slot]
  auto diag_inv = [&](int b) {
    if (lane < 16) {
      const int b0 = 16 * b, j = lane;
      double z[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) z[i] = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        z[m] *= rinv[b0 + m];
#pragma unroll
        for (int i = m + 1; i < 16; ++i) z[i] = fma(-S[b0 + i][b0 + m], z[m], z[i]);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) Z[b0 + i][b0 + j] = z[i];
    }
  };
  auto lprod = [&](int Q, int P, int slot) {
    f64x4_t t = {0.0, 0.0, 0.0, 0.0};
    for (int R = P; R < Q; ++R) {
#pragma unroll
      for (int s = 0; s < 16; s += 4) {
        const double la = S[16 * Q + (lane & 15)][16 * R + s + (lane >> 4)];
        const double zb = Z[16 * R + s + (lane >> 4)][16 * P + (lane & 15)];
        t = __builtin_amdgcn_mfma_f64_16x16x4f64(la, zb, t, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Tm[slot][mrow(lane, v)][lane & 15] = t[v];
  };
  auto zprod = [&](int Q, int P, int slot) {
    f64x4_t u = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 16; s += 4) {
      const double za = Z[16 * Q + (lane & 15)][16 * Q + s + (lane >> 4)];
      const double tb = Tm[slot][s + (lane >> 4)][lane & 15];
      u = __builtin_amdgcn_mfma_f64_16x16x4f64(-za, tb, u, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Z[16 * Q + mrow(lane, v)][16 * P + (lane & 15)] = u[v];
  };
  auto wave_fence = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };

  // block (Q, R) of S less the product of panel Pp's columns
  auto trail = [&](int Q, int R, int Pp) {
    f64x4_t t;
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = S[16 * Q + mrow(lane, v)][16 * R + (lane & 15)];
    t = mm_nt<PB, true>(t, S, 16 * Q, S, 16 * R, PB * Pp, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) S[16 * Q + mrow(lane, v)][16 * R + (lane & 15)] = t[v];
  };
  // Panel P is factored by wave 0 after it has applied panel P - 1's
  // product to its own column block; meanwhile waves 1..3 apply that
  // product to the blocks right of it and form the parts of the inverse
  // that blocks < P already fix: Z_00 under panel 1; Z_11 and L_10 Z_00
  // under panel 2; Z_22, Z_10 and L_21 Z_11 under panel 3; the last rows of
  // blocks follow.  Every block receives the panel products in panel order,
  // so the factor does not depend on which wave applies them.  One barrier
  // per panel.  (The pivots of a pair form a dependent chain of about 580
  // cycles, measured; taking the far columns' updates off wave 0 onto a
  // helper wave did not shorten it.)
  bool bad = false;
  for (int P = 0; P < CB / PB; ++P) {
    const int p0 = PB * P;
    if (w == 0) {
      if (P > 0) {
        for (int Q = P; Q < NB; ++Q) trail(Q, P, P - 1);
        wave_fence();   // the updated blocks are read back across lanes below
      }
      double f[PB];
#pragma unroll
      for (int cc = 0; cc < PB; ++cc) f[cc] = S[lane][p0 + cc];
      // columns in pairs: with d0 = A_cc, a10 = A_c+1,c, d1 = A_c+1,c+1 and
      // det = d0 d1 - a10^2, 1/L_cc = rsqrt(d0) and 1/L_c+1,c+1 =
      // sqrt(d0) rsqrt(det) come from two independent chains; rows above the
      // pair are left as they are (upper triangle, cleared below)
#pragma unroll
      for (int cc = 0; cc < PB; cc += 2) {
        const int c = p0 + cc;
        const double d0 = lane_bcast(f[cc], c);
        const double a10 = lane_bcast(f[cc], c + 1);
        const double d1 = lane_bcast(f[cc + 1], c + 1);
        const double det = fma(-a10, a10, d0 * d1);
        // a pivot <= 0 or NaN is recorded off the dependent chain; its NaNs
        // then run through the factor, which the status word marks invalid
        bad |= !(d0 > 0.0) || !(det > 0.0);
        const double inv0 = rsqrt_h(d0);
        const double invdet = rsqrt_h(det);
        const double inv1 = (d0 * inv0) * invdet;
        const double l10 = a10 * inv0;
        const double lc0 = f[cc] * inv0;                       // lane c: sqrt(d0)
        const double lc1 = fma(-lc0, l10, f[cc + 1]) * inv1;   // lane c + 1: sqrt(det / d0)
        f[cc] = lc0;
        f[cc + 1] = lc1;
        if (lane == 0) {   // inv0, inv1 are the same on every lane
          rinv[c] = inv0;
          rinv[c + 1] = inv1;
        }
        // rank-2 update: the next pair's columns by readlane (short chain),
        // the others with the two columns broadcast through shared memory
        if (cc + 2 < PB) {
          lb[lane] = lc0;
          lb[CB + lane] = lc1;
          const double b0 = lane_bcast(lc0, c + 2), b1 = lane_bcast(lc1, c + 2);
          const double e0 = lane_bcast(lc0, c + 3), e1 = lane_bcast(lc1, c + 3);
          f[cc + 2] = fma(-lc1, b1, fma(-lc0, b0, f[cc + 2]));
          f[cc + 3] = fma(-lc1, e1, fma(-lc0, e0, f[cc + 3]));
#pragma unroll
          for (int kk = cc + 4; kk < PB; ++kk)
            f[kk] = fma(-lc1, lb[CB + p0 + kk], fma(-lc0, lb[p0 + kk], f[kk]));
        }
      }
#pragma unroll
      for (int cc = 0; cc < PB; ++cc) S[lane][p0 + cc] = lane >= p0 + cc ? f[cc] : 0.0;
    } else {
      if (P == 1 && pub && tid == 192)
        __hip_atomic_store(pub, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      if (P > 0) {
        // blocks (Q, R), Q >= R >= P + 1, of panel P - 1's trailing update
        const int R0 = P + 1, nr = NB - R0;
        for (int pi = w - 1; pi < nr * (nr + 1) / 2; pi += 3) {
          int q = 0, rem = pi;
          while (rem > q) { rem -= q + 1; ++q; }
          trail(R0 + q, R0 + rem, P - 1);
        }
      }
      if (P == 0) {
        during_first_panel();
      } else if (P == 1) {
        if (w == 1) diag_inv(0);
      } else if (P == 2) {
        if (w == 1) diag_inv(1);
        else if (w == 2) lprod(1, 0, 0);
      } else {
        if (w == 1) {
          diag_inv(2);
          zprod(1, 0, 0);
        } else if (w == 3) {
          lprod(2, 1, 2);
        }
      }
    }
    __syncthreads();
  }
  if (bad && lane == 0 && status) atomicOr(status, MINSR_ST_NOT_PD);
  // the last rows of blocks: Z_33, Z_20 (L_20 Z_00 + L_21 Z_10 first),
  // Z_21 and L_32 Z_22, then Z_30, Z_31, Z_32
  if (w == 0) {
    diag_inv(3);
  } else if (w == 1) {
    lprod(2, 0, 1);
    wave_fence();
    zprod(2, 0, 1);
  } else if (w == 2) {
    zprod(2, 1, 2);
  } else {
    lprod(3, 2, 3);
  }
  __syncthreads();
  if (w == 1) {
    lprod(3, 0, 0);
    wave_fence();
    zprod(3, 0, 0);
  } else if (w == 2) {
    lprod(3, 1, 1);
    wave_fence();
    zprod(3, 1, 1);
  } else if (w == 3) {
    zprod(3, 2, 3);
  }
  __syncthreads();
  {
    double zv[CB * CB / 256];
#pragma unroll
    for (int q = 0; q < CB * CB / 256; ++q) {
      const int e = tid + 256 * q;
      zv[q] = Z[e / CB][e % CB];
    }
#pragma unroll
    for (int q = 0; q < CB * CB / 256; ++q) {
      const int e = tid + 256 * q, i = e / CB, j = e % CB;
      Di[e] = (i < nb && j < nb && i / 16 >= j / 16) ? zv[q] : 0.0;
    }
  }
}

// FP64, the whole factorisation in one launch, tiles held in registers from
// their first read of T + lambda I to their final value.  Roles come from a
// ticket: ticket 0 factors block 0; then, block column k by block column k,
// one workgroup takes the pair of tiles (k+1, k) and (k+1, k+1), and one
// workgroup each panel tile (i, k), i >= k + 2.  A workgroup only waits for
// tiles of earlier columns or for the diagonal block of its own column, all
// of which took earlier tickets, so every wait ends whether or not the whole
// grid is resident.  Tiles apply the updates A -= L_ik L_jk^T of earlier
// columns as their panel tiles are published (flag per tile); a panel tile
// then waits for its diagonal block, forms L_ij = A_ij inv(L_jj)^T, stores
// it with its contribution L_ij y_j to the forward substitution, and
// publishes.  The pair workgroup of block j applies its own L_j,j-1 to the
// diagonal tile from shared memory, so the step from one diagonal block to
// the next crosses workgroups once; it then factors, inverts and solves its
// block of L y = b from the contributions of the tiles of row j (summed in
// the order of k) and publishes the block.
__global__ __launch_bounds__(256) void k_chol_persist_f64(CholArgs a, uint32_t* ctl,
                                                          double* cpart) {
  __shared__ double X[CB][LDT];
  __shared__ double Y[CB][LDT];
  __shared__ double Tm[4][16][17];
  __shared__ double rinv[CB];
  __shared__ double lb[2 * CB];
  __shared__ double yb[CB];
  __shared__ double cown[CB];
  __shared__ int tk;
  const int n = a.n, nblk = a.nblk, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  double* A = reinterpret_cast<double*>(a.A);
  const double* T0 = reinterpret_cast<const double*>(a.T);
  double* y = reinterpret_cast<double*>(a.y);
  uint32_t* dflag = ctl + 1;              // [nblk]: diagonal block j published
  uint32_t* pflag = ctl + 1 + nblk;       // [nblk][nblk]: panel tile (i, j) published
  if (tid == 0)
    tk = (int)__hip_atomic_fetch_add(&ctl[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  // the panel tile (pi, pj), if any, and the diagonal block jd, if any
  bool has_panel = false, has_diag = true;
  int pi = 0, pj = 0, jd = 0;
  if (tk > 0) {
    int k = 0, rem = tk - 1;
    while (rem >= nblk - k - 1) { rem -= nblk - k - 1; ++k; }
    has_panel = true;
    pj = k;
    pi = k + 1 + rem;
    has_diag = rem == 0;
    jd = k + 1;
  }
  const double lam = a.lam_dev ? *a.lam_dev : a.lambda;
  // relaxed polls (an acquiring load would invalidate this CU's caches at
  // every poll, slowing the many waiting tiles' neighbours), one acquire
  // fence once the flag is seen
  auto wait_flag = [&](const uint32_t* f) {
    if (tid == 0) {
      bounded_wait(f, a.abort, a.spin_limit, a.status);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
  };
  auto publish = [&](uint32_t* f) {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's stores are complete
    __syncthreads();
    if (tid == 0) __hip_atomic_store(f, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  };
  // tile (r0, c0) of T + lambda I in the MFMA result layout (wave w: rows
  // 16w.., four 16 x 16 blocks), the diagonal tile lower triangle only
  auto load_tile = [&](f64x4_t (&t)[4], int r0, int c0, bool diag) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * w + mrow(lane, v), col = c0 + 16 * c + (lane & 15);
        double val = T0[(size_t)min(r, n - 1) * n + min(col, n - 1)];
        if (r == col) val += lam;
        t[c][v] = (r < n && col < n && (!diag || col <= r)) ? val : 0.0;
      }
  };
  auto tile_to_lds = [&](const f64x4_t (&t)[4], double (*M)[LDT]) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) M[16 * w + mrow(lane, v)][16 * c + (lane & 15)] = t[c][v];
  };

  f64x4_t tp[4], td[4];
  if (has_panel) load_tile(tp, pi * CB, pj * CB, false);
  if (has_diag) load_tile(td, jd * CB, jd * CB, true);
  // updates of columns k < pj, in order of k; the pair workgroup's diagonal
  // tile takes L_jd,k L_jd,k^T from the same rows
  const int nk = has_panel ? pj : 0;
  for (int k = 0; k < nk; ++k) {
    wait_flag(&pflag[pi * nblk + k]);
    wait_flag(&pflag[pj * nblk + k]);
    const int k0 = k * CB, ri = pi * CB, rj = pj * CB;
    {
      double vi[CB * CB / 256], vj[CB * CB / 256];
#pragma unroll
      for (int q = 0; q < CB * CB / 256; ++q) {
        const int e = tid + 256 * q, r = e / CB, cc = e % CB;
        const double xi = A[(size_t)min(ri + r, n - 1) * n + k0 + cc];
        vi[q] = (ri + r < n) ? xi : 0.0;
        vj[q] = A[(size_t)(rj + r) * n + k0 + cc];   // pj < pi: a full block
      }
#pragma unroll
      for (int q = 0; q < CB * CB / 256; ++q) {
        const int e = tid + 256 * q, r = e / CB, cc = e % CB;
        X[r][cc] = vi[q];
        Y[r][cc] = vj[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) tp[c] = mm_nt<CB, true>(tp[c], X, 16 * w, Y, 16 * c, 0, lane);
    if (has_diag) {
#pragma unroll
      for (int c = 0; c < 4; ++c) td[c] = mm_nt<CB, true>(td[c], X, 16 * w, X, 16 * c, 0, lane);
    }
    __syncthreads();   // X, Y are rewritten next
  }
  // b_jd less the contributions L_jd,k y_k, k < jd - 1, of the panel tiles of
  // row jd (published with their flags, seen above), summed in order of k
  // while the diagonal block jd - 1 is still being factored
  const int kbd = jd * CB, nb = min(CB, n - kbd);
  double bpart = 0.0;
  if (has_diag && tid < CB) {
    bpart = tid < nb ? y[kbd + tid] : 0.0;
    const int kmax = jd - 1;
    for (int k0 = 0; k0 < kmax; k0 += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = cpart[((size_t)jd * nblk + min(k0 + u, kmax - 1)) * CB + tid];
#pragma unroll
      for (int u = 0; u < 8; ++u) bpart -= k0 + u < kmax ? v[u] : 0.0;
    }
  }

  if (has_panel) {
    // L = A_pi,pj inv(L_pj,pj)^T and its contribution L y_pj
    const int kb0 = pj * CB;   // pj < pi <= nblk - 1: a full block
    wait_flag(&dflag[pj]);
    tile_to_lds(tp, X);
    {
      const double* Di = reinterpret_cast<const double*>(a.Dinv) + (size_t)pj * CB * CB;
      double dv[CB * CB / 256];
#pragma unroll
      for (int q = 0; q < CB * CB / 256; ++q) dv[q] = Di[tid + 256 * q];
#pragma unroll
      for (int q = 0; q < CB * CB / 256; ++q) Y[(tid + 256 * q) / CB][(tid + 256 * q) % CB] = dv[q];
    }
    if (tid < CB) yb[tid] = y[kb0 + tid];
    __syncthreads();
    const int r0 = pi * CB;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    // inv(L) is block lower triangular: column block c of L takes the first
    // 16 (c + 1) columns of the tile
    f64x4_t l[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) l[c] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    l[0] = mm_nt<16, false>(l[0], X, 16 * w, Y, 0, 0, lane);
    l[1] = mm_nt<32, false>(l[1], X, 16 * w, Y, 16, 0, lane);
    l[2] = mm_nt<48, false>(l[2], X, 16 * w, Y, 32, 0, lane);
    l[3] = mm_nt<64, false>(l[3], X, 16 * w, Y, 48, 0, lane);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = 16 * c + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * w + mrow(lane, v);
        if (r < n) A[(size_t)r * n + kb0 + col] = l[c][v];
        s[v] = fma(r < n ? l[c][v] : 0.0, yb[col], s[v]);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int m = 1; m < 16; m <<= 1) s[v] += __shfl_xor(s[v], m, 16);
    }
    if (!has_diag) {
      if ((lane & 15) == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          cpart[((size_t)pi * nblk + pj) * CB + 16 * w + mrow(lane, v)] = s[v];
      }
      publish(&pflag[pi * nblk + pj]);
      return;
    }
    // the pair workgroup: keep the contribution, subtract L L^T from the
    // diagonal tile (rows beyond n of L are zero); L is published during the
    // factorisation's first panel, so the barriers up to there order shared
    // memory only and do not wait for its stores
    if ((lane & 15) == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) cown[16 * w + mrow(lane, v)] = s[v];
    }
    mf16::lds_barrier();   // X, Y, yb are no longer read
    tile_to_lds(l, X);
    mf16::lds_barrier();
    // column block 0 of L L^T now; the other lower blocks while wave 0
    // factors the first panel (L stays in X until then)
    td[0] = mm_nt<CB, true>(td[0], X, 16 * w, X, 0, 0, lane);
  }

  // the diagonal block jd: factor (in Y, the inverse in X), invert, and
  // solve its block of L y = b; rows >= nb become identity rows as they are
  // written
  const int kb0 = kbd;
  double* Di = reinterpret_cast<double*>(a.Dinv) + (size_t)jd * CB * CB;
  auto put_block = [&](const f64x4_t& t, int c) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * w + mrow(lane, v), col = 16 * c + (lane & 15);
      Y[r][col] = r < nb ? t[v] : (r == col ? 1.0 : 0.0);
    }
  };
  mf16::lds_barrier();   // Y is rewritten
  if (has_panel) {
    put_block(td[0], 0);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) put_block(td[c], c);
  }
  if (tid < CB) {
    const double r = jd > 0 ? bpart - cown[tid] : bpart;
    yb[tid] = tid < nb ? r : 0.0;
  }
  mf16::lds_barrier();
  // waves 1..3: the rest of L L^T for their lower blocks (1 <= c <= w)
  auto rest = [&]() {
    if (!has_panel) return;
#pragma unroll
    for (int c = 1; c < 4; ++c)
      if (c <= w) {
        td[c] = mm_nt<CB, true>(td[c], X, 16 * w, X, 16 * c, 0, lane);
        put_block(td[c], c);
      }
  };
  factor_block_f64(Y, X, Tm, rinv, lb, nb, kb0, Di, a.status, false, rest,
                   has_panel ? &pflag[pi * nblk + pj] : nullptr);
  mf16::lds_barrier();   // the inverse's stores complete under the solve below
  {
    // y_jd = inv(L) yb: four threads per row, terms q = part, part + 4, ...
    // up to the diagonal (X above the diagonal blocks is not cleared)
    const int row = tid / 4, part = tid % 4;
    double zr[CB / 4], yq[CB / 4];
#pragma unroll
    for (int u = 0; u < CB / 4; ++u) {
      zr[u] = X[row][part + 4 * u];
      yq[u] = yb[part + 4 * u];
    }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < CB / 4; ++u) s = fma(part + 4 * u <= row ? zr[u] : 0.0, yq[u], s);
    s += __shfl_xor(s, 1, 4);
    s += __shfl_xor(s, 2, 4);
    if (part == 0 && row < nb) y[kb0 + row] = s;
  }
  if (jd + 1 < nblk) publish(&dflag[jd]);
  // the diagonal block of L, which no tile of this factorisation reads
#pragma unroll
  for (int q = 0; q < CB * CB / 256; ++q) {
    const int e = tid + 256 * q, i = e / CB, j = e % CB;
    if (j <= i && i < nb) A[(size_t)(kb0 + i) * n + kb0 + j] = Y[i][j];
  }
}

// sync words and b -> y (one kernel, safe inside captured graphs).  If
// lam_out or a report pointer is set, workgroup 0 also sums the diagonal of
// T (tr T, fixed order) and forms the shift
//   lambda_eff = max(lambda, rel_tr * tr T)      (rel_tr = 0: lambda)
// with lambda = *lam_in when lam_in is set (a shift computed on the device)
// into lam_out, MINSR_ST_SHIFT_FLOOR in *status when the floor is the
// larger, and tr T and lambda_eff into rep_tn / rep_lam.  The floor bounds
// the accumulation error of a low-precision Gram: each entry of the
// computed T is within gamma sqrt(T_ii T_jj) of the exact one, so its
// spectral-norm error is at most gamma tr T.
// x entries not yet computed by the backward substitution hold a signalling
// NaN: arithmetic only ever yields quiet NaNs, so no computed x equals it,
// and a waiting workgroup polls the entries themselves (one round trip for
// flag and data)
constexpr uint64_t X_UNSET = 0x7FF40000DEAD0001ull;

template <typename TT>
__global__ __launch_bounds__(256) void k_chol_prep(uint32_t* sync, int nsync, const double* b,
                                                   TT* y, int n, const TT* T, double lambda,
                                                   double rel_tr, double* lam_out,
                                                   uint64_t* xmark, double* rep_tn,
                                                   double* rep_lam, uint32_t* status,
                                                   const double* lam_in) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nsync) sync[i] = 0u;
  if (i < n) y[i] = (TT)b[i];
  if (i < n) xmark[i] = X_UNSET;
  if ((lam_out || rep_tn || rep_lam) && blockIdx.x == 0) {
    __shared__ double red[256];
    double tr = 0.0;
    for (int k0 = threadIdx.x; k0 < n; k0 += 256 * 8) {   // eight loads in flight
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = min(k0 + 256 * u, n - 1);
        v[u] = (double)T[(size_t)k * n + k];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (k0 + 256 * u < n) tr += v[u];
    }
    red[threadIdx.x] = tr;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double fl = rel_tr * red[0];
      double lam = lam_in ? lam_in[0] : lambda;
      if (rel_tr > 0.0 && fl > lam) {
        lam = fl;
        if (status) atomicOr(status, MINSR_ST_SHIFT_FLOOR);
      }
      if (lam_out) lam_out[0] = lam;
      if (rep_tn) rep_tn[0] = red[0];
      if (rep_lam) rep_lam[0] = lam;
    }
  }
}

// the report of a pseudo-inverse step: tr T and the shift 0
__global__ __launch_bounds__(256) void k_report_trace(const double* T, int n, double* rep_tn,
                                                      double* rep_lam) {
  __shared__ double red[256];
  double tr = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) tr += T[(size_t)k * n + k];
  red[threadIdx.x] = tr;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (rep_tn) rep_tn[0] = red[0];
    if (rep_lam) rep_lam[0] = 0.0;
  }
}

int launch_report_trace(int n, const double* T, double* rep_tn, double* rep_lam, hipStream_t s) {
  if (n == 0 || (!rep_tn && !rep_lam)) return MINSR_OK;
  k_report_trace<<<1, 256, 0, s>>>(T, n, rep_tn, rep_lam);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

// Backward substitution L^T x = y by one workgroup per block of 64:
//   x_k = inv(L_kk)^T (y_k - sum_{j>k} L_jk^T x_j).
// The workgroup with ticket t takes block k = nblk - 1 - t, so it only waits
// for blocks whose workgroups started before it.  It keeps inv(L_kk) in
// shared memory, adds the products L_jk^T x_j for j = nblk-1 down to k+1 in
// that fixed order as the x_j are published (the tile of the next j is
// requested before waiting), then publishes x_k: its entries are stored
// atomically over the unset marks the waiting workgroups poll.
template <typename TT>
__global__ __launch_bounds__(256) void k_trsv_back_mt(const TT* A, int n, const TT* Dinv,
                                                      const TT* y, double* x, uint32_t* bsync,
                                                      int nblk, uint32_t* abort,
                                                      uint32_t spin_limit, uint32_t* status) {
  __shared__ TT Dk[CB][CB + 1];
  __shared__ TT xj[CB];
  __shared__ TT part[4][CB];
  __shared__ TT rb[CB];
  __shared__ int tk;
  uint32_t* ticket_ctr = bsync;
  const int tid = threadIdx.x, c = tid & 63, g = tid >> 6;
  if (tid == 0)
    tk = (int)__hip_atomic_fetch_add(ticket_ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int kb = nblk - 1 - tk;
  const int k0 = kb * CB, nb = min(CB, n - k0);
  const TT* Di = Dinv + (size_t)kb * CB * CB;
  {
    TT dv[CB * CB / 256];   // all loads in flight before the first store
#pragma unroll
    for (int i = 0; i < CB * CB / 256; ++i) dv[i] = Di[tid + 256 * i];
#pragma unroll
    for (int i = 0; i < CB * CB / 256; ++i) Dk[(tid + 256 * i) / CB][(tid + 256 * i) % CB] = dv[i];
  }
  TT acc = (TT)0;
  TT l[16];
  auto fetch = [&](int j) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      // clamped and unguarded, so that all sixteen loads are in flight: rows
      // beyond n meet zeros in xj, columns beyond nb are never used
      const int r = j * CB + 16 * g + u;
      l[u] = A[(size_t)min(r, n - 1) * n + k0 + min(c, nb - 1)];
    }
  };
  if (kb + 1 < nblk) fetch(nblk - 1);
  for (int j = nblk - 1; j > kb; --j) {
    if (tid < CB) {
      TT v = (TT)0;
      if (j * CB + tid < n) {
        const uint64_t* xp = reinterpret_cast<const uint64_t*>(x) + j * CB + tid;
        uint64_t bits;
        uint32_t polls = 0;
        // bounded as in bounded_wait: a wait that gives up keeps the mark
        // (a NaN) and flags the solve as failed
        while ((bits = __hip_atomic_load(xp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == X_UNSET) {
          ++polls;
          if (polls >= spin_limit ||
              ((polls & 63u) == 0u &&
               __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
            if (status) atomicOr(status, MINSR_ST_SOLVE_TIMEOUT);
            __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        v = (TT)__longlong_as_double((long long)bits);
      }
      xj[tid] = v;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) acc = fma(l[u], xj[16 * g + u], acc);
    if (j - 1 > kb) fetch(j - 1);
    __syncthreads();   // xj is rewritten next iteration
  }
  part[g][c] = acc;
  __syncthreads();
  if (tid < CB) {
    const TT s = (part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid]);
    rb[tid] = tid < nb ? y[k0 + tid] - s : (TT)0;
  }
  __syncthreads();
  // x_k[cc] = sum_{r >= cc} inv(L_kk)[r][cc] rb[r], four threads per cc
  // (thread sb: rows cc + sb, cc + sb + 4, ... below nb; all sixteen reads
  // issued together, rows past the block masked to zero terms)
  {
    const int cc = tid >> 2, sb = tid & 3;
    TT dv[CB / 4], rv[CB / 4];
#pragma unroll
    for (int u = 0; u < CB / 4; ++u) {
      const int r = min(cc + sb + 4 * u, CB - 1);
      dv[u] = Dk[r][cc];
      rv[u] = rb[r];
    }
    TT v = (TT)0;
#pragma unroll
    for (int u = 0; u < CB / 4; ++u) v = fma(cc + sb + 4 * u < nb ? dv[u] : (TT)0, rv[u], v);
    v += __shfl_xor(v, 1, 4);
    v += __shfl_xor(v, 2, 4);
    if (sb == 0 && cc < nb)
      __hip_atomic_store(reinterpret_cast<uint64_t*>(x) + k0 + cc,
                         (uint64_t)__double_as_longlong((double)v), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
}

size_t chol_dinv_elems(int n) { return (size_t)((n + CB - 1) / CB) * CB * CB; }
// sync words: [2 (nblk + 1)] tickets and flags of the launch-per-column
// factorisation (FP32), [nblk + 1] ticket and flags of the backward pass,
// [1 + nblk + nblk^2] ticket, diagonal and panel flags of the one-launch
// factorisation (FP64), then the abort word of the bounded waits
static size_t chol_sync_bwd(int nblk) { return 2 * (size_t)(nblk + 1); }
static size_t chol_sync_one(int nblk) { return 3 * (size_t)(nblk + 1); }
size_t chol_sync_words(int n) {
  const size_t nblk = (size_t)((n + CB - 1) / CB);
  return chol_sync_one((int)nblk) + 1 + nblk + nblk * nblk + 1;
}
// solver vector: y (n, rounded up to whole blocks), then the per-tile
// contributions L_ij y_j of the one-launch factorisation ([nblk][nblk][64])
size_t chol_vec_elems(int n) {
  const size_t nblk = (size_t)((n + CB - 1) / CB);
  return nblk * CB + nblk * nblk * CB + 1;   // + the shift actually used
}

template <typename TT>
static int chol_t(int n, const TT* T, TT* A, TT* Dinv, TT* yv, uint32_t* sync, double lambda,
                  const double* b, double* x, uint32_t* status, hipStream_t s,
                  double lam_floor_rel, double* rep_tn, double* rep_lam,
                  const double* lam_in, uint32_t spin_limit) {
  const int nblk = (n + CB - 1) / CB;
  const int nsync = (int)chol_sync_words(n);
  const int m = std::max(nsync, n);
  uint32_t* abort = sync + nsync - 1;   // cleared with the other sync words
  const uint32_t lim = spin_limit ? spin_limit : DEFAULT_SPIN_LIMIT;
  CholArgs a{T, A, Dinv, yv, sync, status, lambda, nullptr, n, nblk, abort, lim};
  double* lam_slot = nullptr;
  if constexpr (std::is_same<TT, double>::value) {
    if (lam_floor_rel > 0.0 || lam_in) {
      lam_slot = reinterpret_cast<double*>(yv) + chol_vec_elems(n) - 1;
      a.lam_dev = lam_slot;
    }
  }
  k_chol_prep<TT><<<(m + 255) / 256, 256, 0, s>>>(sync, nsync, b, yv, n, T, lambda,
                                                  lam_slot ? lam_floor_rel : 0.0, lam_slot,
                                                  reinterpret_cast<uint64_t*>(x), rep_tn,
                                                  rep_lam, status, lam_in);
  MINSR_CHECK_LAUNCH();
  if constexpr (std::is_same<TT, double>::value) {
    k_chol_persist_f64<<<1 + nblk * (nblk - 1) / 2, 256, 0, s>>>(a, sync + chol_sync_one(nblk),
                                                             yv + (size_t)nblk * CB);
    MINSR_CHECK_LAUNCH();
  } else {
    for (int k = -1; k + 1 < nblk; ++k) {
      const int nt = nblk - k - 1;
      const int grid = k < 0 ? nblk : nt * (nt + 1) / 2;
      k_chol_step<TT><<<grid, 256, 0, s>>>(a, k);
      MINSR_CHECK_LAUNCH();
    }
  }
  k_trsv_back_mt<TT><<<nblk, 256, 0, s>>>(A, n, Dinv, yv, x, sync + chol_sync_bwd(nblk), nblk,
                                          abort, lim, status);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int launch_cholesky_solve(int n, const double* T, double* Lf, double* Dinv, int f32,
                          double lambda, const double* b, double* x, double* yv, uint32_t* sync,
                          uint32_t* status, hipStream_t s, double lam_floor_rel, double* rep_tn,
                          double* rep_lam, const double* lam_in, uint32_t spin_limit) {
  if (n == 0) return MINSR_OK;
  if (f32) {
    if (lam_in) return fail(MINSR_E_UNSUPPORTED, "a device-side shift needs the FP64 solve");
    return chol_t<float>(n, reinterpret_cast<const float*>(T), reinterpret_cast<float*>(Lf),
                         reinterpret_cast<float*>(Dinv), reinterpret_cast<float*>(yv), sync,
                         lambda, b, x, status, s, 0.0, rep_tn, rep_lam, nullptr, spin_limit);
  }
  return chol_t<double>(n, T, Lf, Dinv, yv, sync, lambda, b, x, status, s, lam_floor_rel, rep_tn,
                        rep_lam, lam_in, spin_limit);
}

// ================================================================ update
// dpart[chunk][k] = sum over the chunk's rows a of R[a][k] x[a]  (FP64)
template <typename TR>
__global__ void k_update_part(const TR* R, int n, size_t Np, size_t ld, int RC, const double* x,
                              double* part, const TR* Rlo) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  const int r0 = blockIdx.y * RC, r1 = min(n, r0 + RC);
  double s = 0.0;
  if (Rlo)
    for (int r = r0; r < r1; ++r)
      s += ((double)(float)R[(size_t)r * ld + col] + (double)(float)Rlo[(size_t)r * ld + col]) * x[r];
  else
    for (int r = r0; r < r1; ++r) s += (double)(float)R[(size_t)r * ld + col] * x[r];
  part[(size_t)blockIdx.y * Np + col] = s;
}

// BF16 hi/lo: two adjacent columns per thread (4-byte loads), rows in steps
// of four with their loads issued together; each column's sum runs over the
// rows in order, as above
__global__ void k_update_part_bf16x2(const __hip_bfloat16* R, const __hip_bfloat16* Rlo, int n,
                                     size_t Np, size_t ld, int RC, const double* x, double* part) {
  const size_t col = 2 * ((size_t)blockIdx.x * blockDim.x + threadIdx.x);
  if (col >= Np) return;
  const int r0 = blockIdx.y * RC, r1 = min(n, r0 + RC);
  double s0 = 0.0, s1 = 0.0;
  auto term = [&](int r, double& a0, double& a1) {
    // ld is a multiple of 64 and col even: the pair lies inside the padded row
    const __hip_bfloat162 h = *reinterpret_cast<const __hip_bfloat162*>(R + (size_t)r * ld + col);
    const __hip_bfloat162 l = *reinterpret_cast<const __hip_bfloat162*>(Rlo + (size_t)r * ld + col);
    const double xr = x[r];
    a0 += ((double)__bfloat162float(h.x) + (double)__bfloat162float(l.x)) * xr;
    a1 += ((double)__bfloat162float(h.y) + (double)__bfloat162float(l.y)) * xr;
  };
  int r = r0;
  for (; r + 4 <= r1; r += 4) {
    __hip_bfloat162 h[4], l[4];
    double xr[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      h[u] = *reinterpret_cast<const __hip_bfloat162*>(R + (size_t)(r + u) * ld + col);
      l[u] = *reinterpret_cast<const __hip_bfloat162*>(Rlo + (size_t)(r + u) * ld + col);
      xr[u] = x[r + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s0 += ((double)__bfloat162float(h[u].x) + (double)__bfloat162float(l[u].x)) * xr[u];
      s1 += ((double)__bfloat162float(h[u].y) + (double)__bfloat162float(l[u].y)) * xr[u];
    }
  }
  for (; r < r1; ++r) term(r, s0, s1);
  part[(size_t)blockIdx.y * Np + col] = s0;
  if (col + 1 < Np) part[(size_t)blockIdx.y * Np + col + 1] = s1;
}
template <>
__global__ void k_update_part<double>(const double* R, int n, size_t Np, size_t ld, int RC,
                                      const double* x, double* part, const double* Rlo) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  const int r0 = blockIdx.y * RC, r1 = min(n, r0 + RC);
  double s = 0.0;
  for (int r = r0; r < r1; ++r) s += R[(size_t)r * ld + col] * x[r];
  part[(size_t)blockIdx.y * Np + col] = s;
}

// (bump, if set: the step's Philox counter, advanced once here since every
// read of it this step has happened)
__global__ void k_update_final(const double* part, int nrc, size_t Np, double eta, double* dtheta,
                               uint32_t* status, uint64_t* bump) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (bump && col == 0) bump[0] += 1;
  if (col >= Np) return;
  double s = 0.0;
  for (int c0 = 0; c0 < nrc; c0 += 8) {   // eight partials in flight, summed in order
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)min(c0 + u, nrc - 1) * Np + col];   // tail repeats, unused
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (c0 + u < nrc) s += v[u];
  }
  const double d = eta * s;
  dtheta[col] = d;
  if (!isfinite(d)) atomicOr(status, MINSR_ST_NONFINITE_DTH);
}

__global__ void k_apply(size_t Np, const double* dtheta, double mu, double* m, double* theta,
                        const uint32_t* status) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  if (status[0] & MINSR_ST_ERRORS) return;
  const double mn = mu * m[col] + (1.0 - mu) * dtheta[col];
  m[col] = mn;
  theta[col] -= mn;
}

int launch_update(int n, size_t Np, const void* R, int dtype, const double* x, double eta,
                  double mu, double* dpart, double* dtheta, double* momentum, double* theta,
                  uint32_t* status, int apply, hipStream_t s, const void* Rlo, uint64_t* bump) {
  const int RC = 64;
  const int nrc = (n + RC - 1) / RC;
  dim3 grid((unsigned)((Np + 255) / 256), (unsigned)nrc);
  const size_t ld = (Np + 63) / 64 * 64;
  if (dtype == MINSR_BF16)
    if (Rlo)
      k_update_part_bf16x2<<<dim3((unsigned)((Np + 511) / 512), (unsigned)nrc), 256, 0, s>>>(
          (const __hip_bfloat16*)R, (const __hip_bfloat16*)Rlo, n, Np, ld, RC, x, dpart);
    else
      k_update_part<__hip_bfloat16><<<grid, 256, 0, s>>>((const __hip_bfloat16*)R, n, Np, ld, RC, x,
                                                         dpart, nullptr);
  else if (dtype == MINSR_F32)
    k_update_part<float><<<grid, 256, 0, s>>>((const float*)R, n, Np, ld, RC, x, dpart, nullptr);
  else
    k_update_part<double><<<grid, 256, 0, s>>>((const double*)R, n, Np, ld, RC, x, dpart, nullptr);
  MINSR_CHECK_LAUNCH();
  const unsigned g1 = (unsigned)((Np + 255) / 256);
  k_update_final<<<g1, 256, 0, s>>>(dpart, nrc, Np, eta, dtheta, status, bump);
  MINSR_CHECK_LAUNCH();
  if (apply) {
    k_apply<<<g1, 256, 0, s>>>(Np, dtheta, mu, momentum, theta, status);
    MINSR_CHECK_LAUNCH();
  }
  return MINSR_OK;
}

}  // namespace minsr
