// Stored factor values.  L_K and W_K are kept in the precision of the
// Schur-complement updates (FP64, FP32 or the bits of a bfloat16), the
// pivot blocks D_K and S_K always in FP64: the updates read L and W, the
// drop test and the pivot inverse work on FP64 panels, and the apply reads
// L and W in the same precision as the updates.  Offsets are counted in
// values, not bytes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bilu {

constexpr int kValF64 = 0, kValF32 = 1, kValBF16 = 2;

inline int value_bytes(int prec) { return prec == kValF64 ? 8 : prec == kValF32 ? 4 : 2; }

#ifdef __HIP__  // device helpers: HIP sources only (host C++ files include this header too)

// bfloat16 by round-to-nearest-even of the float value (NaN stays NaN).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// One value of type T as a double, and a double stored as T (FP32 by
// round-to-nearest, BF16 through FP32).
__device__ __forceinline__ double as_double(double v) { return v; }
__device__ __forceinline__ double as_double(float v) { return (double)v; }
__device__ __forceinline__ double as_double(uint16_t v) { return (double)bf16_float(v); }
template <class T>
__device__ __forceinline__ T from_double(double v);
template <>
__device__ __forceinline__ double from_double<double>(double v) { return v; }
template <>
__device__ __forceinline__ float from_double<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ uint16_t from_double<uint16_t>(double v) { return bf16_bits((float)v); }

// Untyped access for code that handles every precision at run time (the
// precision is uniform across a launch, so the branch does not diverge).
__device__ __forceinline__ double value_load(const void* base, int prec, int64_t o) {
  if (prec == kValF32) return (double)static_cast<const float*>(base)[o];
  if (prec == kValBF16) return (double)bf16_float(static_cast<const uint16_t*>(base)[o]);
  return static_cast<const double*>(base)[o];
}
__device__ __forceinline__ void value_store(void* base, int prec, int64_t o, double v) {
  if (prec == kValF32)
    static_cast<float*>(base)[o] = (float)v;
  else if (prec == kValBF16)
    static_cast<uint16_t*>(base)[o] = bf16_bits((float)v);
  else
    static_cast<double*>(base)[o] = v;
}

#endif  // __HIP__

}  // namespace bilu
