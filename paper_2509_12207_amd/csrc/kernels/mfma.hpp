// CDNA4 (gfx950) FP32 matrix-core helpers shared by the contraction kernels.
//
// v_mfma_f32_32x32x2_f32 (wave64): D[32x32] += A[32x2] * B[2x32].
//   lane l supplies A[i][k] with i = l % 32, k = l / 32, and B[k][j] with
//   j = l % 32, k = l / 32;
//   accumulator register r of lane l holds D[row][col] with col = l % 32 and
//   row = 8 * (r / 4) + 4 * (l / 32) + (r % 4).
// 4096 FLOP per instruction, 64 FLOP/clk per SIMD.
#pragma once

#include <hip/hip_runtime.h>

namespace ug {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f32x16 mfma_32x32x2(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Row of accumulator register r for lane l (column is l % 32).
__device__ __forceinline__ int mfma32_row(int r, int lane) {
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.0f;
  return z;
}

}  // namespace ug
