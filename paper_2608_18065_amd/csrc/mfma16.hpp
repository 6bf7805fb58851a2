// Helpers of the 16 x 16 x 32 FP16 matrix-core kernels of FP32 recurrences
// (the Jacobian's reverse pass and row assembly, the sampler): FP32
// operands enter v_mfma_f32_16x16x32_f16 as pairs x = hi + lo of FP16
// values, products a_lo b_hi + a_hi b_lo + a_hi b_hi accumulate in FP32.
//
// Lane layouts of v_mfma_f32_16x16x32_f16 (64 lanes, l = lane):
//   A (16 x 32): lane l holds A[l % 16][8 (l / 16) + e], e = 0..7;
//   B (32 x 16): lane l holds B[8 (l / 16) + e][l % 16], e = 0..7;
//   D (16 x 16): lane l holds D[4 (l / 16) + v][l % 16], v = 0..3.
#pragma once

#include <hip/hip_runtime.h>

namespace minsr {
namespace mf16 {

typedef __attribute__((ext_vector_type(8))) _Float16 h16x8;
typedef __attribute__((ext_vector_type(4))) _Float16 h16x4;
typedef __attribute__((ext_vector_type(2))) _Float16 h16x2;
typedef __attribute__((ext_vector_type(2))) float f32x2v;
typedef __attribute__((ext_vector_type(4))) float f32x4v;

__device__ __forceinline__ f32x4v mma16(h16x8 a, h16x8 b, f32x4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// The low parts fp16(a - hi.x), fp16(b - hi.y) of a pair whose high parts
// hi = fp16(a), fp16(b) are packed in one register, by v_fma_mix with hi read
// as FP16: a - hi is exact in FP32 and is rounded once, so the bits equal
// those of converting the FP32 difference (also for FP16 subnormal and
// overflowing values; compared over 2^21 such pairs on gfx950), in two
// instructions instead of five
__device__ __forceinline__ h16x2 lo_pair(h16x2 hi, float a, float b) {
  const uint32_t hb = __builtin_bit_cast(uint32_t, hi);
  uint32_t m;
  asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(m) : "v"(hb), "v"(a));
  asm("v_fma_mixhi_f16 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
      : "+v"(m) : "v"(hb), "v"(b));
  return __builtin_bit_cast(h16x2, m);
}

// x = hi + lo, both rounded to nearest FP16; x - hi is exact in FP32, so
// |x - hi - lo| <= 2^-22 |x| while lo stays in FP16's normal range
template <int E, typename HV>
__device__ __forceinline__ void split16(const float (&x)[E], HV& hi, HV& lo) {
#pragma unroll
  for (int e = 0; e < E; e += 2) {
    const f32x2v v = {x[e], x[e + 1]};
    const h16x2 h = __builtin_convertvector(v, h16x2);
    const h16x2 l = lo_pair(h, x[e], x[e + 1]);
    hi[e] = h[0]; hi[e + 1] = h[1];
    lo[e] = l[0]; lo[e + 1] = l[1];
  }
}

// logistic function and tanh from the hardware exp2 and reciprocal (about
// 1 ulp each); both saturate correctly
__device__ __forceinline__ float sigm_hw(float x) {
  return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(-1.4426950408889634f * x));
}
__device__ __forceinline__ float tanh_hw(float y) {
  return 1.f - 2.f * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(2.8853900817779268f * y));
}

// workgroup barrier ordering shared-memory accesses only: unlike
// __syncthreads() it does not wait for the wave's outstanding global stores
// (these kernels never read back, within a launch, what they store)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// v[l] + v[l ^ 16] and v[l] + v[l ^ 32]: both lanes of a pair add the same
// two values in the same order (lower row or half first), so they end with
// equal sums; the exchanges are VALU lane swaps, not shared-memory traffic
__device__ __forceinline__ float sum_xor16(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float sum_xor32(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// lane exchanges inside rows of 16 lanes by DPP (no shared-memory crossbar
// round trip): quad_sum adds the partners at distance 1, then 2, exactly as
// an xor butterfly over those distances does; row16_max takes the maximum
// over each row of 16 lanes
template <int CTRL> __device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float quad_sum(float v) {
  v += dpp_f<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  return v;
}
__device__ __forceinline__ float row16_max(float v) {
  v = fmaxf(v, dpp_f<0xB1>(v));
  v = fmaxf(v, dpp_f<0x4E>(v));
  v = fmaxf(v, dpp_f<0x141>(v));   // row_half_mirror
  v = fmaxf(v, dpp_f<0x140>(v));   // row_mirror
  return v;
}

// power-of-two exponent that brings a largest magnitude m into [2^14, 2^15)
__device__ __forceinline__ int pow2_exp_for(float m) {
  return m > 0.f ? min(max(14 - ilogbf(m), -120), 120) : 0;
}

}  // namespace mf16
}  // namespace minsr
