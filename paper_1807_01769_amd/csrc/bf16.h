// bf16.h -- FP32 <-> BF16 conversion on the device (BF16 = the upper 16 bits
// of an IEEE binary32, 8 significant bits).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fs {

// FP32 -> BF16, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ short to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(short h) {
  return __uint_as_float(((uint32_t)(unsigned short)h) << 16);
}

}  // namespace fs
