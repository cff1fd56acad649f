// MFMA wrappers for gfx950 (CDNA4) 16x16x4 FP32/FP64 matrix instructions.
//
// Operand layout (both precisions), one 64-lane wavefront:
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
// Output (16 x 16), column = l % 16, four registers r = 0..3 per lane:
//   FP32: row = 4 * (l / 16) + r
//   FP64: row = (l / 16) + 4 * r
#pragma once
#include <hip/hip_runtime.h>

#define TILE 64

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;

template <> struct Mfma<float> {
  typedef f4v acc;
  __device__ static inline acc zero() { acc a = {0.f, 0.f, 0.f, 0.f}; return a; }
  __device__ static inline acc mac(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <> struct Mfma<double> {
  typedef d4v acc;
  __device__ static inline acc zero() { acc a = {0.0, 0.0, 0.0, 0.0}; return a; }
  __device__ static inline acc mac(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// BF16 16x16x32 (gfx950): A lane l holds A[l % 16][8*(l/16) .. 8*(l/16)+7],
// B lane l holds B[8*(l/16) .. +7][l % 16]; output as FP32 16x16x4.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ inline f4v mfma_bf16(bf16x8 a, bf16x8 b, f4v c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

// Split operands travel as 16-bit patterns (us16, eight to a u32x4 register
// quad); H selects what they mean: false = BF16 (8-bit significand, FP32
// range), true = FP16 (11-bit significand, range 2^-24 .. 65504, used with a
// power-of-two scale that puts the largest magnitude just below 2^15).  The
// FP16 16x16x32 MFMA has the BF16 operand and output layout.
typedef unsigned short us16;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <bool H>
__device__ inline f4v mfma_p(u32x4 a, u32x4 b, f4v c) {
  if constexpr (H)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// v = sum of NS parts, each the round-to-nearest-even value of what the
// previous parts left
template <int NS, bool H>
__device__ inline void split_n(float v, us16 *out) {
  float r = v;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    if constexpr (H) {
      const _Float16 h = (_Float16)r;
      out[i] = __builtin_bit_cast(us16, h);
      r -= (float)h;
    } else {
      const __bf16 h = (__bf16)r;
      out[i] = __builtin_bit_cast(us16, h);
      r -= (float)h;
    }
  }
}

// Two-part FP16 split of the products a0 b0 and a1 b1, packed (element 0 in
// the low half): hi = f16(a b) and lo = f16(a b - hi), each from the exact
// product in one mixed-precision FMA (v_fma_mixlo/mixhi_f16 write one half of
// the destination and keep the other), two instructions per value.
__device__ inline void split2_h_pair(float a0, float b0, float a1, float b1, unsigned &hi, unsigned &lo) {
  unsigned h, l;
  asm("v_fma_mixlo_f16 %0, %1, %2, 0\n\t"
      "v_fma_mixhi_f16 %0, %3, %4, 0"
      : "=&v"(h)
      : "v"(a0), "v"(b0), "v"(a1), "v"(b1));
  asm("v_fma_mixlo_f16 %0, %2, %3, -%1 op_sel_hi:[0,0,1]\n\t"
      "v_fma_mixhi_f16 %0, %4, %5, -%1 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
      : "=&v"(l)
      : "v"(h), "v"(a0), "v"(b0), "v"(a1), "v"(b1));
  hi = h;
  lo = l;
}

// Power-of-two scale for a block whose largest magnitude is m: m / scale <
// 2^15 (m = 0 or not finite: 1).  inv_pow2_scale is its exact reciprocal.
__device__ inline float pow2_scale(float m) {
  if (!(m > 0.f) || !(m < INFINITY)) return 1.f;
  int e;
  frexpf(m, &e);   // m < 2^e
  return ldexpf(1.f, e - 15);
}
__device__ inline float inv_pow2_scale(float m) {
  if (!(m > 0.f) || !(m < INFINITY)) return 1.f;
  int e;
  frexpf(m, &e);
  return ldexpf(1.f, 15 - e);
}

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
__device__ inline void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}
