// The parameter-space metric S = O' O'^T of Eq. SR (N_p x N_p, the real
// part of the quantum geometric tensor estimated from the samples), used by
// the subsampled-QGT study of Prop. 3: S[i][j] = sum over the rows r of the
// centred real form (Re rows, then Im rows) of R[r][i] R[r][j].  FP64
// accumulation; lower-triangle tiles computed and mirrored, so S is exactly
// symmetric; each entry sums its rows in ascending order.
#include "model.hpp"

namespace minsr {

constexpr int QT = 64;      // output tile
constexpr int QK = 32;      // rows per shared-memory chunk

template <typename TR>
__global__ __launch_bounds__(256) void k_param_gram(const TR* R, int rows, int Np, size_t ld,
                                                    double* S) {
  __shared__ double A[QK][QT + 1];
  __shared__ double B[QK][QT + 1];
  // lower-triangle tile (ti >= tj) from the linear block index
  int ti = 0, b = blockIdx.x;
  while (b > ti) { b -= ti + 1; ++ti; }
  const int tj = b;
  const int i0 = ti * QT, j0 = tj * QT;
  const int tid = threadIdx.x, tr = (tid / 16) * 4, tc = (tid % 16) * 4;
  double acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int z = 0; z < 4; ++z) acc[x][z] = 0.0;
  for (int r0 = 0; r0 < rows; r0 += QK) {
    // stage R[r0 .. r0 + QK)[i0 .. i0 + QT) and [j0 .. j0 + QT), zeros outside
    for (int e = tid; e < QK * QT; e += 256) {
      const int rr = e / QT, cc = e % QT, r = r0 + rr;
      const int ci = i0 + cc, cj = j0 + cc;
      A[rr][cc] = (r < rows && ci < Np) ? (double)R[(size_t)r * ld + ci] : 0.0;
      B[rr][cc] = (r < rows && cj < Np) ? (double)R[(size_t)r * ld + cj] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < QK; ++k) {
      double a[4], bb[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) a[x] = A[k][tr + x];
#pragma unroll
      for (int z = 0; z < 4; ++z) bb[z] = B[k][tc + z];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int z = 0; z < 4; ++z) acc[x][z] = fma(a[x], bb[z], acc[x][z]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int z = 0; z < 4; ++z) {
      const int i = i0 + tr + x, j = j0 + tc + z;
      if (i < Np && j < Np && j <= i) {
        S[(size_t)i * Np + j] = acc[x][z];
        S[(size_t)j * Np + i] = acc[x][z];
      }
    }
}

int launch_param_gram(const void* R, int r_f64, int rows, int Np, size_t ld, double* S,
                      hipStream_t s) {
  if (Np <= 0) return MINSR_OK;
  const int nt = (Np + QT - 1) / QT;
  const unsigned grid = (unsigned)(nt * (nt + 1) / 2);
  if (r_f64)
    k_param_gram<double><<<grid, 256, 0, s>>>((const double*)R, rows, Np, ld, S);
  else
    k_param_gram<float><<<grid, 256, 0, s>>>((const float*)R, rows, Np, ld, S);
  MINSR_CHECK_LAUNCH();
  return MINSR_OK;
}

}  // namespace minsr
