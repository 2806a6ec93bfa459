// PDF storage types and their compute types.
//
// FP64 storage computes in FP64; FP32, BF16 and FP16 storage compute in FP32.
// Every stored value is the shifted population f - w_q rho_0 (the shift keeps
// the small deviations from the rest state at full relative precision);
// conversions to the 16-bit types round to nearest-even.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Materialise an FP32 value before it is rounded to a 16-bit type, so the
// compiler cannot fuse the last FMA with the conversion in some kernels and
// not in others: every kernel then rounds the same FP32 value once more, and
// the two-array and AA sweeps stay bit-identical.
__device__ __forceinline__ float pin_f32(float v) {
  asm volatile("" : "+v"(v));
  return v;
}

template <class T>
struct Storage;

template <>
struct Storage<double> {
  using R = double;
  static constexpr int code = 0;
  __device__ static R load(const double* p) { return *p; }
  __device__ static void store(double* p, R v) { *p = v; }
  __device__ static void store_nt(double* p, R v) { __builtin_nontemporal_store(v, p); }
};

template <>
struct Storage<float> {
  using R = float;
  static constexpr int code = 1;
  __device__ static R load(const float* p) { return *p; }
  __device__ static void store(float* p, R v) { *p = v; }
  __device__ static void store_nt(float* p, R v) { __builtin_nontemporal_store(v, p); }
};

template <>
struct Storage<__bf16> {
  using R = float;
  static constexpr int code = 2;
  __device__ static R load(const __bf16* p) { return static_cast<float>(*p); }
  __device__ static void store(__bf16* p, R v) { *p = static_cast<__bf16>(pin_f32(v)); }
  __device__ static void store_nt(__bf16* p, R v) {
    __builtin_nontemporal_store(static_cast<__bf16>(pin_f32(v)), p);
  }
};

template <>
struct Storage<_Float16> {
  using R = float;
  static constexpr int code = 3;
  __device__ static R load(const _Float16* p) { return static_cast<float>(*p); }
  __device__ static void store(_Float16* p, R v) { *p = static_cast<_Float16>(pin_f32(v)); }
  __device__ static void store_nt(_Float16* p, R v) {
    __builtin_nontemporal_store(static_cast<_Float16>(pin_f32(v)), p);
  }
};

}  // namespace lbm
