// Dense stages of one minSR iteration (Eqs. real-valued, minsrR; Alg. 1
// steps 6-9; App. B):
//   centring of O and conversion to the step's precision,
//   the sample-space Gram T = O' O'^T of the n x Np sample-major matrix,
//   the regularised FP64 (or FP32) Cholesky solve (T + lambda I) x = eps',
//   dtheta = eta O'^T x, momentum and the parameter update.
// Every reduction runs in a fixed order: results are bitwise reproducible.
#include "model.hpp"
#include <algorithm>
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
  double s = 0.0;
  for (int r = r0; r < r1; ++r) s += (double)base[(size_t)r * Np];
  part[((size_t)blk * nrc + chunk) * Np + col] = s;
}

__global__ void k_colmean(const double* part, int nrc, int rows_per_block, int nblocks, size_t Np,
                          double* mean) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  for (int b = 0; b < nblocks; ++b) {
    double s = 0.0;
    for (int c = 0; c < nrc; ++c) s += part[((size_t)b * nrc + c) * Np + col];
    mean[(size_t)b * Np + col] = s / rows_per_block;
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
template <typename TI, typename TO>
__global__ void k_center(const TI* O, int rows_per_block, int RC, size_t Np, const double* mean,
                         TO* R) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  const int blk = blockIdx.z, chunk = blockIdx.y;
  const int r0 = chunk * RC;
  const int r1 = min(rows_per_block, r0 + RC);
  const TI mu = mean ? (TI)mean[(size_t)blk * Np + col] : (TI)0;
  const size_t off = ((size_t)blk * rows_per_block) * Np + col;
  for (int r = r0; r < r1; ++r) {
    const TI v = O[off + (size_t)r * Np] - mu;
    R[off + (size_t)r * Np] = cvt_out<TO>((double)v);
  }
}

template <typename TI>
static int center_t(int rows_per_block, int nblocks, size_t Np, const TI* O, void* R,
                    int out_dtype, double* colpart, double* colmean, hipStream_t s) {
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
  switch (out_dtype) {
    case MINSR_F64:
      k_center<TI, double><<<grid, 256, 0, s>>>(O, rows_per_block, RC, Np, colmean, (double*)R);
      break;
    case MINSR_F32:
      k_center<TI, float><<<grid, 256, 0, s>>>(O, rows_per_block, RC, Np, colmean, (float*)R);
      break;
    case MINSR_BF16:
      k_center<TI, __hip_bfloat16><<<grid, 256, 0, s>>>(O, rows_per_block, RC, Np, colmean,
                                                         (__hip_bfloat16*)R);
      break;
    default:
      return fail(MINSR_E_INVALID_ARG, "unknown output dtype");
  }
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int launch_center(int rows_per_block, int nblocks, size_t Np, const void* O, int in_f64, void* R,
                  int out_dtype, double* colpart, double* colmean, hipStream_t s) {
  if (rows_per_block == 0 || Np == 0) return MINSR_OK;
  if (in_f64)
    return center_t<double>(rows_per_block, nblocks, Np, (const double*)O, R, out_dtype, colpart,
                            colmean, s);
  return center_t<float>(rows_per_block, nblocks, Np, (const float*)O, R, out_dtype, colpart,
                         colmean, s);
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

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(16))) float f32x16_t;

// BF16 MFMA tile kernel: 128 x 128 output tile per workgroup (4 waves,
// 64 x 64 each as 2 x 2 blocks of v_mfma_f32_32x32x16_bf16), K staged
// through LDS 64 columns at a time.
constexpr int GT = 128, GK = 64, GKP = GK + 8;

__global__ __launch_bounds__(256) void k_gram_bf16(const __hip_bfloat16* R, int n, size_t Np,
                                                   size_t kchunk, float* part) {
  __shared__ __align__(16) __hip_bfloat16 As[GT][GKP];
  __shared__ __align__(16) __hip_bfloat16 Bs[GT][GKP];
  int ti, tj;
  pair_decode(blockIdx.x, ti, tj);
  const int split = blockIdx.y;
  const size_t k0 = (size_t)split * kchunk;
  const size_t k1 = min(Np, k0 + kchunk);
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
  const bool vec_ok = (Np % 8) == 0;
  for (size_t kk = k0; kk < k1; kk += GK) {
    // stage: 128 rows x 64 bf16 per operand = 1024 chunks of 8
    for (int c = tid; c < GT * (GK / 8); c += 256) {
      const int r = c / (GK / 8), q = (c % (GK / 8)) * 8;
      const size_t col = kk + q;
      __hip_bfloat16 va[8], vb[8];
      const int ra = arow0 + r, rb = brow0 + r;
      if (vec_ok && col + 8 <= k1) {
        uint4 xa = make_uint4(0, 0, 0, 0), xb = make_uint4(0, 0, 0, 0);
        if (ra < n) xa = *reinterpret_cast<const uint4*>(R + (size_t)ra * Np + col);
        if (rb < n) xb = *reinterpret_cast<const uint4*>(R + (size_t)rb * Np + col);
        *reinterpret_cast<uint4*>(&As[r][q]) = xa;
        *reinterpret_cast<uint4*>(&Bs[r][q]) = xb;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bool ok = col + e < k1;
          va[e] = (ok && ra < n) ? R[(size_t)ra * Np + col + e] : __float2bfloat16(0.f);
          vb[e] = (ok && rb < n) ? R[(size_t)rb * Np + col + e] : __float2bfloat16(0.f);
          As[r][q + e] = va[e];
          Bs[r][q + e] = vb[e];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < GK; ks += 16) {
      bf16x8_t fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        fa[a] = *reinterpret_cast<const bf16x8_t*>(&As[wm + a * 32 + (lane & 31)][ks + (lane >> 5) * 8]);
#pragma unroll
      for (int b = 0; b < 2; ++b)
        fb[b] = *reinterpret_cast<const bf16x8_t*>(&Bs[wn + b * 32 + (lane & 31)][ks + (lane >> 5) * 8]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // write the partial tile: acc element e of lane l is row
  // (e / 4) * 8 + (l / 32) * 4 + e % 4, column l % 32 of its 32 x 32 block
  float* out = part + ((size_t)split * gridDim.x + blockIdx.x) * GT * GT;
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
    for (int e = tid; e < VT_ * VK; e += 256) {
      const int r = e / VK, q = e % VK;
      const size_t col = kk + q;
      const int ra = arow0 + r, rb = brow0 + r;
      As[q][r] = (col < k1 && ra < n) ? (TA)R[(size_t)ra * Np + col] : (TA)0;
      Bs[q][r] = (col < k1 && rb < n) ? (TA)R[(size_t)rb * Np + col] : (TA)0;
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
__global__ void k_gram_reduce(const TA* part, int npairs, int nsplit, int tile, int n, TT* T) {
  const int pair = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= tile * tile) return;
  int ti, tj;
  pair_decode(pair, ti, tj);
  const int r = ti * tile + e / tile, c = tj * tile + e % tile;
  if (r >= n || c >= n) return;
  if (ti == tj && c > r) return;
  TA s = (TA)0;
  for (int k = 0; k < nsplit; ++k) s += part[((size_t)k * npairs + pair) * tile * tile + e];
  T[(size_t)r * n + c] = (TT)s;
  T[(size_t)c * n + r] = (TT)s;
}

static int pick_split(int npairs, size_t Np, int kgran) {
  int S = (1024 + npairs - 1) / npairs;
  int maxS = (int)std::max<size_t>(1, Np / 512);
  S = std::max(1, std::min(S, maxS));
  (void)kgran;
  return S;
}

size_t gram_partial_bytes(int n, size_t Np, int dtype) {
  const int tile = dtype == MINSR_BF16 ? GT : VT_;
  const int nt = (n + tile - 1) / tile;
  const int npairs = nt * (nt + 1) / 2;
  const int S = pick_split(npairs, Np, 0);
  const size_t el = dtype == MINSR_F64 ? 8 : 4;
  return (size_t)S * npairs * tile * tile * el;
}

int launch_gram(int n, size_t Np, const void* R, int dtype, double* T, float* gpart,
                size_t gpart_elems, hipStream_t s, int which) {
  if (n == 0) return MINSR_OK;
  const int tile = dtype == MINSR_BF16 ? GT : VT_;
  const int nt = (n + tile - 1) / tile;
  const int npairs = nt * (nt + 1) / 2;
  const int S = pick_split(npairs, Np, 0);
  const size_t kgran = dtype == MINSR_BF16 ? GK : VK;
  size_t kchunk = (Np + S - 1) / S;
  kchunk = (kchunk + kgran - 1) / kgran * kgran;
  const size_t need = gram_partial_bytes(n, Np, dtype);
  if (need > gpart_elems * sizeof(float)) return fail(MINSR_E_SHAPE, "Gram workspace too small");
  dim3 grid((unsigned)npairs, (unsigned)S);
  dim3 rgrid((unsigned)((tile * tile + 255) / 256), (unsigned)npairs);
  if (dtype == MINSR_BF16) {
    if (which & 1) {
      k_gram_bf16<<<grid, 256, 0, s>>>((const __hip_bfloat16*)R, n, Np, kchunk, gpart);
      MINSR_CHECK_LAUNCH();
    }
    if (which & 2) k_gram_reduce<float, double><<<rgrid, 256, 0, s>>>(gpart, npairs, S, tile, n, T);
  } else if (dtype == MINSR_F32) {
    if (which & 1) {
      k_gram_vec<float, float><<<grid, 256, 0, s>>>((const float*)R, n, Np, kchunk, gpart);
      MINSR_CHECK_LAUNCH();
    }
    if (which & 2) k_gram_reduce<float, float><<<rgrid, 256, 0, s>>>(gpart, npairs, S, tile, n, (float*)T);
  } else {
    double* dp = reinterpret_cast<double*>(gpart);
    if (which & 1) {
      k_gram_vec<double, double><<<grid, 256, 0, s>>>((const double*)R, n, Np, kchunk, dp);
      MINSR_CHECK_LAUNCH();
    }
    if (which & 2) k_gram_reduce<double, double><<<rgrid, 256, 0, s>>>(dp, npairs, S, tile, n, T);
  }
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

// ============================================================= Cholesky
// Right-looking blocked Cholesky of A = T + lambda I (lower, in place,
// row-major), block 64: factor the diagonal block, solve the panel below
// it, update the trailing lower triangle.
constexpr int CB = 64;

template <typename TT>
__global__ __launch_bounds__(256) void k_potrf_diag(TT* A, int n, int kb, uint32_t* status) {
  __shared__ TT L[CB][CB + 1];
  const int k0 = kb * CB;
  const int nb = min(CB, n - k0);
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * CB; e += 256) {
    const int r = e / CB, c = e % CB;
    L[r][c] = (r < nb && c < nb) ? A[(size_t)(k0 + r) * n + k0 + c] : (TT)0;
  }
  __syncthreads();
  __shared__ int bad;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    if (tid == 0) {
      TT d = L[c][c];
      if (!(d > (TT)0)) { bad = 1; d = (TT)1; }
      L[c][c] = sqrt(d);
    }
    __syncthreads();
    const TT piv = L[c][c];
    for (int r = c + 1 + tid; r < nb; r += 256) L[r][c] /= piv;
    __syncthreads();
    // rank-1 update of the remaining lower triangle
    for (int e = tid; e < CB * CB; e += 256) {
      const int r = e / CB, q = e % CB;
      if (r > c && q > c && q <= r && r < nb) L[r][q] -= L[r][c] * L[q][c];
    }
    __syncthreads();
  }
  for (int e = tid; e < CB * CB; e += 256) {
    const int r = e / CB, c = e % CB;
    if (r < nb && c <= r) A[(size_t)(k0 + r) * n + k0 + c] = L[r][c];
  }
  if (tid == 0 && bad && status) atomicOr(status, MINSR_ST_NOT_PD);
}

// panel rows below the diagonal block: X L_kk^T = A_ik, one row per thread
template <typename TT>
__global__ __launch_bounds__(64) void k_trsm_panel(TT* A, int n, int kb) {
  __shared__ TT L[CB][CB + 1];
  const int k0 = kb * CB;
  const int nb = min(CB, n - k0);
  for (int e = threadIdx.x; e < CB * CB; e += 64) {
    const int r = e / CB, c = e % CB;
    L[r][c] = (r < nb && c <= r) ? A[(size_t)(k0 + r) * n + k0 + c] : (TT)0;
  }
  __syncthreads();
  const int row = k0 + nb + blockIdx.x * 64 + threadIdx.x;
  if (row >= n) return;
  TT x[CB];
  TT* a = A + (size_t)row * n + k0;
#pragma unroll
  for (int c = 0; c < CB; ++c) x[c] = c < nb ? a[c] : (TT)0;
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    if (c < nb) {
      TT v = x[c];
#pragma unroll
      for (int m = 0; m < c; ++m) v -= x[m] * L[c][m];
      x[c] = v / L[c][c];
    }
  }
#pragma unroll
  for (int c = 0; c < CB; ++c) if (c < nb) a[c] = x[c];
}

// trailing update A_ij -= L_ik L_jk^T for the lower tiles i >= j > k
template <typename TT>
__global__ __launch_bounds__(256) void k_syrk_trail(TT* A, int n, int kb) {
  __shared__ TT Li[CB][CB + 1];
  __shared__ TT Lj[CB][CB + 1];
  const int k0 = kb * CB;
  const int nb = min(CB, n - k0);
  const int base = kb + 1;
  int ti, tj;
  pair_decode(blockIdx.x, ti, tj);
  ti += base; tj += base;
  const int r0 = ti * CB, c0 = tj * CB;
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * CB; e += 256) {
    const int r = e / CB, q = e % CB;
    Li[r][q] = (r0 + r < n && q < nb) ? A[(size_t)(r0 + r) * n + k0 + q] : (TT)0;
    Lj[r][q] = (c0 + r < n && q < nb) ? A[(size_t)(c0 + r) * n + k0 + q] : (TT)0;
  }
  __syncthreads();
  const int tr = (tid / 16) * 4, tc = (tid % 16) * 4;
  TT acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (TT)0;
  for (int q = 0; q < CB; ++q) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(Li[tr + a][q], Lj[tc + b][q], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = r0 + tr + a, c = c0 + tc + b;
      if (r < n && c < n && (ti != tj || c <= r)) A[(size_t)r * n + c] -= acc[a][b];
    }
}

// forward (L y = b) and backward (L^T x = y) substitution, one workgroup,
// 64-row blocks: wave 0 solves the diagonal block from LDS (lane r holds
// unknown r, the solved value is broadcast lane to lane), then all threads
// update the rest of the right-hand side.
template <typename TT>
__global__ __launch_bounds__(1024) void k_trsv(const TT* A, int n, const double* b, double* x) {
  extern __shared__ unsigned char smem_raw[];
  TT* y = reinterpret_cast<TT*>(smem_raw);
  __shared__ TT D[CB][CB + 1];
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += 1024) y[i] = (TT)b[i];
  const int nblk = (n + CB - 1) / CB;
  // forward
  for (int kb = 0; kb < nblk; ++kb) {
    const int k0 = kb * CB, nb = min(CB, n - k0);
    for (int e = tid; e < CB * CB; e += 1024) {
      const int r = e / CB, c = e % CB;
      D[r][c] = (r < nb && c < nb) ? A[(size_t)(k0 + r) * n + k0 + c] : (TT)0;
    }
    __syncthreads();
    if (tid < 64) {
      TT v = tid < nb ? y[k0 + tid] : (TT)0;
      for (int c = 0; c < nb; ++c) {
        if (tid == c) v = v / D[c][c];
        const TT yc = __shfl(v, c, 64);
        if (tid > c && tid < nb) v -= D[tid][c] * yc;
      }
      if (tid < nb) y[k0 + tid] = v;
    }
    __syncthreads();
    for (int i = k0 + nb + tid; i < n; i += 1024) {
      TT v = y[i];
      const TT* row = A + (size_t)i * n + k0;
      for (int m = 0; m < nb; ++m) v -= row[m] * y[k0 + m];
      y[i] = v;
    }
    __syncthreads();
  }
  // backward with L^T
  for (int kb = nblk - 1; kb >= 0; --kb) {
    const int k0 = kb * CB, nb = min(CB, n - k0);
    for (int e = tid; e < CB * CB; e += 1024) {
      const int r = e / CB, c = e % CB;
      D[r][c] = (r < nb && c < nb) ? A[(size_t)(k0 + r) * n + k0 + c] : (TT)0;
    }
    __syncthreads();
    if (tid < 64) {
      TT v = tid < nb ? y[k0 + tid] : (TT)0;
      for (int c = nb - 1; c >= 0; --c) {
        if (tid == c) v = v / D[c][c];
        const TT yc = __shfl(v, c, 64);
        if (tid < c) v -= D[c][tid] * yc;
      }
      if (tid < nb) y[k0 + tid] = v;
    }
    __syncthreads();
    for (int i = tid; i < k0; i += 1024) {
      TT v = y[i];
      for (int m = 0; m < nb; ++m) v -= A[(size_t)(k0 + m) * n + i] * y[k0 + m];
      y[i] = v;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += 1024) x[i] = (double)y[i];
}

template <typename TT>
__global__ void k_copy_add_diag(const TT* T, TT* A, size_t nn, int n, double lambda) {
  size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  TT v = T[e];
  if (e / n == e % n) v += (TT)lambda;
  A[e] = v;
}

template <typename TT>
static int chol_t(int n, const TT* T, TT* A, double lambda, const double* b, double* x,
                  uint32_t* status, hipStream_t s) {
  const size_t nn = (size_t)n * n;
  k_copy_add_diag<TT><<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(T, A, nn, n, lambda);
  MINSR_CHECK_LAUNCH();
  const int nblk = (n + CB - 1) / CB;
  for (int kb = 0; kb < nblk; ++kb) {
    k_potrf_diag<TT><<<1, 256, 0, s>>>(A, n, kb, status);
    MINSR_CHECK_LAUNCH();
    const int rows_below = n - (kb * CB + std::min(CB, n - kb * CB));
    if (rows_below > 0) {
      k_trsm_panel<TT><<<(rows_below + 63) / 64, 64, 0, s>>>(A, n, kb);
      MINSR_CHECK_LAUNCH();
      const int nt = nblk - kb - 1;
      k_syrk_trail<TT><<<nt * (nt + 1) / 2, 256, 0, s>>>(A, n, kb);
      MINSR_CHECK_LAUNCH();
    }
  }
  const size_t shm = (size_t)n * sizeof(TT);
  if (shm > 96 * 1024) return fail(MINSR_E_SHAPE, "triangular solve: n too large");
  k_trsv<TT><<<1, 1024, shm, s>>>(A, n, b, x);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

int launch_cholesky_solve(int n, const double* T, double* Lf, int f32, double lambda,
                          const double* b, double* x, uint32_t* status, hipStream_t s) {
  if (n == 0) return MINSR_OK;
  if (f32)
    return chol_t<float>(n, reinterpret_cast<const float*>(T), reinterpret_cast<float*>(Lf),
                         lambda, b, x, status, s);
  return chol_t<double>(n, T, Lf, lambda, b, x, status, s);
}

// ================================================================ update
// dpart[chunk][k] = sum over the chunk's rows a of R[a][k] x[a]  (FP64)
template <typename TR>
__global__ void k_update_part(const TR* R, int n, size_t Np, int RC, const double* x,
                              double* part) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  const int r0 = blockIdx.y * RC, r1 = min(n, r0 + RC);
  double s = 0.0;
  for (int r = r0; r < r1; ++r) s += (double)(float)R[(size_t)r * Np + col] * x[r];
  part[(size_t)blockIdx.y * Np + col] = s;
}
template <>
__global__ void k_update_part<double>(const double* R, int n, size_t Np, int RC, const double* x,
                                      double* part) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  const int r0 = blockIdx.y * RC, r1 = min(n, r0 + RC);
  double s = 0.0;
  for (int r = r0; r < r1; ++r) s += R[(size_t)r * Np + col] * x[r];
  part[(size_t)blockIdx.y * Np + col] = s;
}

__global__ void k_update_final(const double* part, int nrc, size_t Np, double eta, double* dtheta,
                               uint32_t* status) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  double s = 0.0;
  for (int c = 0; c < nrc; ++c) s += part[(size_t)c * Np + col];
  const double d = eta * s;
  dtheta[col] = d;
  if (!isfinite(d)) atomicOr(status, MINSR_ST_NONFINITE_DTH);
}

__global__ void k_apply(size_t Np, const double* dtheta, double mu, double* m, double* theta,
                        const uint32_t* status) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  if (status[0] != 0) return;
  const double mn = mu * m[col] + (1.0 - mu) * dtheta[col];
  m[col] = mn;
  theta[col] -= mn;
}

int launch_update(int n, size_t Np, const void* R, int dtype, const double* x, double eta,
                  double mu, double* dpart, double* dtheta, double* momentum, double* theta,
                  uint32_t* status, int apply, hipStream_t s) {
  const int RC = 64;
  const int nrc = (n + RC - 1) / RC;
  dim3 grid((unsigned)((Np + 255) / 256), (unsigned)nrc);
  if (dtype == MINSR_BF16)
    k_update_part<__hip_bfloat16><<<grid, 256, 0, s>>>((const __hip_bfloat16*)R, n, Np, RC, x, dpart);
  else if (dtype == MINSR_F32)
    k_update_part<float><<<grid, 256, 0, s>>>((const float*)R, n, Np, RC, x, dpart);
  else
    k_update_part<double><<<grid, 256, 0, s>>>((const double*)R, n, Np, RC, x, dpart);
  MINSR_CHECK_LAUNCH();
  const unsigned g1 = (unsigned)((Np + 255) / 256);
  k_update_final<<<g1, 256, 0, s>>>(dpart, nrc, Np, eta, dtheta, status);
  MINSR_CHECK_LAUNCH();
  if (apply) {
    k_apply<<<g1, 256, 0, s>>>(Np, dtheta, mu, momentum, theta, status);
    MINSR_CHECK_LAUNCH();
  }
  return MINSR_OK;
}

// weighted row reduction: out[k] = sum_r part-free  (used by the VJP)
__global__ void k_reduce_rows(const double* w, int rows, size_t Np, const double* O,
                              double* out) {
  size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= Np) return;
  double s = 0.0;
  for (int r = 0; r < rows; ++r) s += w[r] * O[(size_t)r * Np + col];
  out[col] = s;
}

int launch_reduce_rows(int rows, size_t Np, const double* part, double* out, hipStream_t s) {
  (void)rows; (void)Np; (void)part; (void)out; (void)s;
  return MINSR_OK;
}

int launch_pinv_solve(int n, double* T, double cutoff, const double* b, double* x, double* eig,
                      size_t eig_elems, uint32_t* status, hipStream_t s) {
  (void)n; (void)T; (void)cutoff; (void)b; (void)x; (void)eig; (void)eig_elems; (void)status;
  (void)s;
  return fail(MINSR_E_UNSUPPORTED, "pseudo-inverse solve not built yet");
}

}  // namespace minsr
