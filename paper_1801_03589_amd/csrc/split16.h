// Split of FP32 operands into two 16-bit values for the split-precision
// products: v = hi + lo with hi = r(v) and lo = r(v - hi), r the
// round-to-nearest-even conversion to bf16 or fp16 (v - hi is exact in FP32).
// A real product is then hi*hi + hi*lo + lo*hi on the 16-bit matrix cores with
// FP32 accumulation.  bf16 keeps 8 bits per part (about 16 in all); fp16 keeps
// 11 (about 22) but has a 5-bit exponent, so its operands are scaled by a power
// of two first (split_shift in kernels.h) and the results by its inverse.
// Values travel as raw 16-bit patterns; the vector type of the bf16
// instructions carries them, and the fp16 instructions take the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace nesa {

typedef __bf16 s16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 h16x8 __attribute__((ext_vector_type(8)));
typedef float s16_f32x4 __attribute__((ext_vector_type(4)));
typedef float s16_f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ unsigned short s16_bf16_rne(float v) {
  const unsigned u = __float_as_uint(v);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

template <int F>
__device__ __forceinline__ void split16(float v, unsigned short& hi, unsigned short& lo) {
  if constexpr (F == SPLIT_FP16) {
    const _Float16 h = (_Float16)v;
    hi = __builtin_bit_cast(unsigned short, h);
    lo = __builtin_bit_cast(unsigned short, (_Float16)(v - (float)h));
  } else {
    hi = s16_bf16_rne(v);
    lo = s16_bf16_rne(v - __uint_as_float((unsigned)hi << 16));
  }
}

// C += A B on one 16x16x32 or 32x32x16 instruction of the format
template <int F>
__device__ __forceinline__ s16_f32x4 mfma16x16x32(s16x8 a, s16x8 b, s16_f32x4 c) {
  if constexpr (F == SPLIT_FP16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h16x8, a), __builtin_bit_cast(h16x8, b), c, 0,
                                                  0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
template <int F>
__device__ __forceinline__ s16_f32x16 mfma32x32x16(s16x8 a, s16x8 b, s16_f32x16 c) {
  if constexpr (F == SPLIT_FP16)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h16x8, a), __builtin_bit_cast(h16x8, b), c, 0,
                                                  0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// scale exponents of a product: the sources' shift from their slot (fp16), and
// the exponent that takes the accumulated result back (ldexp, exact)
template <int F>
__device__ __forceinline__ int split_src_shift(const int* bexp) {
  if constexpr (F == SPLIT_FP16)
    return split_shift(*bexp);
  else
    return 0;
}

}  // namespace nesa
