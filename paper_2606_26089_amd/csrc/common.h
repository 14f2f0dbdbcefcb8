// Device-side helpers shared by the fmdet kernels (gfx950 / CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // 16-byte register chunk

constexpr int kWave = 64;
constexpr int kXcds = 8;          // MI355X: 8 accelerator complex dies, 32 CUs each
constexpr float kLnEps = 1e-5f;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}

// Transpose-reduction of 32 per-lane values over the 32 lanes of a half wave: afterwards
// v[0] of lane l holds the sum over the 32 lanes of value (l & 31). 31 exchanges instead of
// 5 per value: at each step a lane keeps half of its values and adds its partner's copy.
__device__ __forceinline__ void transpose_reduce32(float (&v)[32], int lane) {
#pragma unroll
  for (int m = 16, n = 32; m >= 1; m >>= 1, n >>= 1) {
    const bool up = (lane & m) != 0;
#pragma unroll
    for (int i = 0; i < n / 2; ++i) {
      const float send = up ? v[i] : v[i + n / 2];
      const float keep = up ? v[i + n / 2] : v[i];
      v[i] = keep + __shfl_xor(send, m, kWave);
    }
  }
}

// Workgroups of a 1-D launch are dealt round-robin to the XCDs (block b runs on XCD b % 8).
// Renumber them so that each XCD owns one contiguous range of logical tiles: neighbouring
// tiles that share an operand then share that XCD's L2. A bijection on [0, n).
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n / kXcds, r = n % kXcds;
  const int xcd = b % kXcds, local = b / kXcds;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

template <typename T> __device__ __forceinline__ T from_f32(float x);
template <> __device__ __forceinline__ float from_f32<float>(float x) { return x; }
template <> __device__ __forceinline__ bf16 from_f32<bf16>(float x) { return (bf16)x; }  // RNE

__device__ __forceinline__ float to_f32(float x) { return x; }
__device__ __forceinline__ float to_f32(bf16 x) { return (float)x; }

// Exact GELU through erf.
__device__ __forceinline__ float gelu_erf(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

// ODE state update of one feature, v being the velocity evaluated at xs. Modes:
// 0 Euler x += h v; 1..4 the four RK4 stages (acc collects k1 + 2 k2 + 2 k3, xs receives
// the next stage input); 5 velocity only (v written to out); 7, 8 the two explicit midpoint
// stages (xs <- x + h/2 v, then x <- x + h v); anything else: no effect.
__device__ __forceinline__ void ode_update(int mode, float h, float v, float* x, float* acc,
                                           float* xs, float* out) {
  switch (mode) {
    case 0: {
      const float xn = fmaf(h, v, *x);
      *x = xn; *xs = xn;
      if (out) *out = xn;
    } break;
    case 1:
      *acc = v;
      *xs = fmaf(0.5f * h, v, *x);
      break;
    case 2:
      *acc = fmaf(2.0f, v, *acc);
      *xs = fmaf(0.5f * h, v, *x);
      break;
    case 3:
      *acc = fmaf(2.0f, v, *acc);
      *xs = fmaf(h, v, *x);
      break;
    case 4: {
      const float xn = fmaf(h * (1.0f / 6.0f), *acc + v, *x);
      *x = xn; *xs = xn;
      if (out) *out = xn;
    } break;
    case 5:
      if (out) *out = v;
      break;
    case 7:
      *xs = fmaf(0.5f * h, v, *x);
      break;
    case 8: {
      const float xn = fmaf(h, v, *x);
      *x = xn; *xs = xn;
      if (out) *out = xn;
    } break;
    default:
      break;
  }
}

}  // namespace fmd
