// BF16 storage for device code: a value is the upper 16 bits of an IEEE binary32,
// rounded to nearest (ties to even) from FP32.  Arithmetic happens in FP32.
#pragma once
#include <hip/hip_runtime.h>

namespace rz {

typedef unsigned short bf16_t;

__device__ __forceinline__ float bf16_to_f(bf16_t b) { return __builtin_bit_cast(float, (unsigned)b << 16); }

// round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ bf16_t f_to_bf16(float f) { return __builtin_bit_cast(bf16_t, (__bf16)f); }

// loads and stores of a storage type S in the compute type T
template <typename T, typename S>
__device__ __forceinline__ T st_load(S v) {
  return (T)v;
}
template <>
__device__ __forceinline__ float st_load<float, bf16_t>(bf16_t v) {
  return bf16_to_f(v);
}
template <typename S, typename T>
__device__ __forceinline__ S st_store(T v) {
  return (S)v;
}
template <>
__device__ __forceinline__ bf16_t st_store<bf16_t, float>(float v) {
  return f_to_bf16(v);
}

}  // namespace rz
