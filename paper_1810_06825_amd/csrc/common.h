// Shared device/host helpers of the gfx950 frPCA library (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "frpca.h"

#include <string>

namespace frpca {

constexpr int kWave = 64;      // CDNA wavefront width
constexpr int kMaxL = 128;     // largest sketch width l = k + s supported by the kernels

// Panel width: l rounded up to a multiple of 32 so every FP32 row is whole 128-byte lines.
inline int panel_ld(int l) { return (l + 31) / 32 * 32; }

// ---------------------------------------------------------------- BF16 (round to even)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Two consecutive panel elements as float2, from FP32 or BF16 storage.
template <bool BF16>
__device__ __forceinline__ float2 load2(const void* base, size_t idx) {
  if constexpr (BF16) {
    uint32_t w = *reinterpret_cast<const uint32_t*>(static_cast<const uint16_t*>(base) + idx);
    return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xFFFF0000u));
  } else {
    return *reinterpret_cast<const float2*>(static_cast<const float*>(base) + idx);
  }
}
__device__ __forceinline__ void store2_f32(float* base, size_t idx, float2 v) {
  *reinterpret_cast<float2*>(base + idx) = v;
}
__device__ __forceinline__ void store2_bf16(uint16_t* base, size_t idx, float2 v) {
  uint32_t w = (uint32_t)f32_to_bf16(v.x) | ((uint32_t)f32_to_bf16(v.y) << 16);
  *reinterpret_cast<uint32_t*>(base + idx) = w;
}

// ---------------------------------------------------------------- errors
struct Error {
  int code;
  std::string msg;
};

}  // namespace frpca

#define FRPCA_HIP(call)                                                              \
  do {                                                                               \
    hipError_t _e = (call);                                                          \
    if (_e != hipSuccess)                                                            \
      throw ::frpca::Error{FRPCA_EHIP, std::string(#call) + ": " + hipGetErrorString(_e)}; \
  } while (0)

#define FRPCA_CHECK(cond, code, text)                             \
  do {                                                            \
    if (!(cond)) throw ::frpca::Error{(code), std::string(text)}; \
  } while (0)
