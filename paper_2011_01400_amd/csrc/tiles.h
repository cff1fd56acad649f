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

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
__device__ inline void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}
