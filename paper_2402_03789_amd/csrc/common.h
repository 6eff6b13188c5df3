// Shared definitions of the libsn HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstdint>
#include <cstddef>

namespace sn {

constexpr int kWave = 64;
constexpr int kNumL = 4;  // feature and harmonic degrees l = 0..3

// Layout of one feature row: degree blocks l = 0..kNumL-1, each [m][channel] with
// the channel index innermost, so every (atom, m) pair is a contiguous row of
// `mul` values and a per-degree channel mixing is a GEMM over those rows.
struct IrrepLayout {
  int mul[kNumL];  // channels per degree (0 when absent)
  int off[kNumL];  // offset of each degree block within the row
  int width;       // total floats per row
};

// A GEMM operand whose logical row r lives at
//   base + (r / nm) * stride + off + (r % nm) * ld
// i.e. the (atom, m) rows of one degree block of a feature row.
struct RowMap {
  int nm;          // rows per atom (2l + 1)
  int ld;          // distance between consecutive m rows of one atom
  int64_t stride;  // distance between atoms
  int64_t off;     // offset of the degree block
  __host__ __device__ inline int64_t operator()(int64_t r) const {
    return (r / nm) * stride + off + (r % nm) * (int64_t)ld;
  }
};

__host__ __device__ inline RowMap plain_rows(int ld) { return RowMap{1, 0, (int64_t)ld, 0}; }

template <typename T> struct Acc { using type = T; };

// bfloat16 storage of per-edge and per-node intermediates in the bfloat16 form (arithmetic
// stays in float32): round to nearest even when stored, exact widening when loaded.
struct bf16_t {
  uint16_t u;
};
__device__ inline float sload(float v) { return v; }
__device__ inline double sload(double v) { return v; }
__device__ inline float sload(bf16_t v) { return __uint_as_float((uint32_t)v.u << 16); }
template <typename S, typename T>
__host__ __device__ inline S sstore(T v) {
  return S(v);
}
template <>
__host__ __device__ inline bf16_t sstore<bf16_t, float>(float v) {
#if defined(__HIP_DEVICE_COMPILE__)
  // gfx950 rounds to nearest even in one instruction (v_cvt_pk_bf16_f32)
  return bf16_t{__builtin_bit_cast(uint16_t, (__bf16)v)};
#else
  uint32_t u = __builtin_bit_cast(uint32_t, v);
  u += 0x7fffu + ((u >> 16) & 1u);
  return bf16_t{(uint16_t)(u >> 16)};
#endif
}
template <>
__host__ __device__ inline bf16_t sstore<bf16_t, double>(double v) {
  return sstore<bf16_t, float>((float)v);
}

__device__ inline float to_f(float v) { return v; }
__device__ inline double to_f(double v) { return v; }

// phi(z) = c z sigmoid(z) and its derivative
template <typename T>
__device__ inline T act(T z, T c) {
  T s = T(1) / (T(1) + exp(-z));
  return c * z * s;
}
template <typename T>
__device__ inline T act_grad(T z, T c) {
  T s = T(1) / (T(1) + exp(-z));
  return c * (s + z * s * (T(1) - s));
}

}  // namespace sn
