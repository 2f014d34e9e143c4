// bfloat16-split products on the matrix cores (16 x 16 x 16 bfloat16
// instructions with FP32 accumulation), shared by the 1D and 2D stage kernels.
//
// An operand x (an FP32 value, or an FP64 value rounded to FP32) is split into
// a high and a low bfloat16 part, x = hi + lo + d, each rounded to nearest
// even, so |d| <= 2^-16 |x|; a product is formed as lo*hi + hi*lo + hi*hi (the
// small cross terms first, the main product last), dropping lo*lo, which is
// below 2^-16 of the product too.
//
// Operand layout of v_mfma_f32_16x16x16_bf16 (measured on gfx950): lane
// l = i + 16 c holds A[i][4c .. 4c+3] and B[4c .. 4c+3][i] (four bfloat16 each),
// and the result D[4c + r][i] in its register r.
#pragma once

#include <hip/hip_runtime.h>

namespace frsg {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma_bf(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// bfloat16 bits of x rounded to nearest even
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// x = hi + lo for four values at once
__device__ __forceinline__ void split4(const float* x, v4s& hi, v4s& lo) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned short h = bf16_rne(x[i]);
    hi[i] = (short)h;
    lo[i] = (short)bf16_rne(x[i] - __uint_as_float((unsigned)h << 16));
  }
}

// d + A B with both operands split (three products)
__device__ __forceinline__ v4f mfma_split(v4s ah, v4s al, v4s bh, v4s bl, v4f d) {
  d = mfma_bf(al, bh, d);
  d = mfma_bf(ah, bl, d);
  return mfma_bf(ah, bh, d);
}

}  // namespace frsg
