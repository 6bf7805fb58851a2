// Shared device/host definitions of the minSR library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstdint>
#include <cstddef>
#include <string>
#include <vector>

#include "../../include/minsr.h"

namespace minsr {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define MINSR_HIP(call)                                                     \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return ::minsr::fail(MINSR_E_DEVICE, std::string(#call) + ": " +      \
                                               hipGetErrorString(e_));      \
  } while (0)

#define MINSR_CHECK_LAUNCH() MINSR_HIP(hipGetLastError())

// ---------------------------------------------------------------- Philox
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64 x 64 -> 128-bit products with Weyl key increments.
struct U64x4 { uint64_t w[4]; };

__host__ __device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  lo = a * b;
  hi = __umul64hi(a, b);
#else
  unsigned __int128 p = (unsigned __int128)a * b;
  lo = (uint64_t)p;
  hi = (uint64_t)(p >> 64);
#endif
}

__host__ __device__ inline U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, hi0, lo0);
    mulhilo64(M1, c2, hi1, lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  U64x4 o; o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
  return o;
}

// top 53 bits of a word, scaled to [0, 1): exact in double
__host__ __device__ inline double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

// ---------------------------------------------------------------- model
// Offsets of the parameter blocks in the flat FP64 vector (row-major).
struct Layout {
  int H, ds, dim, cplx;
  size_t U1, U2, Wu, bu, Wr, br, Wh, bh, Win, bin, U, c, Uphi, cphi, Np;
};
Layout make_layout(int dim, int H, int cplx);

// Working copy of the parameters in the compute precision T, laid out
// for the kernels:
//   fw   : forward gate weights, [k/V][j][3][V]: for unit j and input k,
//          the weights of u, r and candidate (Wu, Wr, Wh on h), V = 16/sizeof(T)
//   bw   : the same matrices transposed (row index i, column j) for the
//          reverse pass: [i/V][j][3][V] holds W_q[i][j]
//   f2   : 2D only: [k/V][j][2][V] = U1[j][k], U2[j][k]
//   b2   : 2D only: [i/V][j][2][V] = U1[i][j], U2[i][j]
//   xc   : per unit: Wu[j][H+c], Wr[j][H+c], Win[j][c] for c < ds as
//          [3][ds][H]; then bu, br, bh, bin as [4][H]
//   head : U [2][H], Uphi [2][H], c[2], cphi[2]
//   mw   : FP32 models: MFMA B-operand fragments of the gate weights for the
//          local-energy kernel, [wave][step][64 lanes] (see gru_mfma.hip)
//   m2   : FP32 2D models: the same for [U1 | U2]
template <typename T> struct Work {
  T* fw; T* bw; T* f2; T* b2; T* xc; T* bias; T* head; T* headb; T* mw; T* m2;
};

}  // namespace minsr
