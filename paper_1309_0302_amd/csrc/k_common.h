// Device helpers shared by the libgodec kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace godec {

__device__ __forceinline__ float bf16_to_f32(uint32_t h) {
  return __uint_as_float(h << 16);
}

// Round-to-nearest-even FP32 -> bfloat16 (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 4 consecutive elements (16-byte aligned for f32/bf16 pairs, 32-byte for f64).
__device__ __forceinline__ void load4(const float* p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void load4(const double* p, double (&o)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}
__device__ __forceinline__ void load4(const uint16_t* p, float (&o)[4]) {
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  o[0] = bf16_to_f32(v.x & 0xffffu); o[1] = bf16_to_f32(v.x >> 16);
  o[2] = bf16_to_f32(v.y & 0xffffu); o[3] = bf16_to_f32(v.y >> 16);
}
__device__ __forceinline__ void load2(const float* p, float (&o)[4]) {
  const float2 v = *reinterpret_cast<const float2*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = 0.f; o[3] = 0.f;
}
__device__ __forceinline__ void load2(const double* p, double (&o)[4]) {
  const double2 v = *reinterpret_cast<const double2*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = 0.0; o[3] = 0.0;
}
__device__ __forceinline__ void load2(const uint16_t* p, float (&o)[4]) {
  const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
  o[0] = bf16_to_f32(v & 0xffffu); o[1] = bf16_to_f32(v >> 16); o[2] = 0.f; o[3] = 0.f;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Cross-block hand-off without a device-wide cache write-back: partial
// results are stored write-through at device (agent) scope and read back
// with device-scope loads; a block waits for its stores to complete before
// it signals arrival with a device-scope atomic.
__device__ __forceinline__ void publish(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void publish_u32(unsigned int* p, unsigned int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double fetch(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned int arrive(unsigned int* p) {
  return __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// s_waitcnt vmcnt(0) (gfx9 encoding: expcnt and lgkmcnt left at their maxima)
__device__ __forceinline__ void stores_done() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// 1 / sqrt(x) for x > 0 from the hardware estimate and two Newton steps
// (each roughly doubles the correct bits), within an ulp or two of the
// correctly rounded value: one short dependent chain where sqrt and a
// division would be two long ones.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// q = a / b and r = a % b for 0 <= a < 2^52 and b >= 1, with rb = 1 / b in
// double precision: the product a * rb is within one of the quotient (its
// relative error is at most 2^-52), so one correction step makes it exact.
// Cheaper than a 64-bit integer division by a runtime divisor.
__device__ __forceinline__ void divmod_nn(int64_t a, int64_t b, double rb, int64_t& q,
                                          int64_t& r) {
  q = (int64_t)((double)a * rb);
  r = a - q * b;
  if (r < 0) {
    q -= 1;
    r += b;
  } else if (r >= b) {
    q += 1;
    r -= b;
  }
}

// Sum of p[0 .. n) in an order fixed by n and the block size alone, so a
// run reproduces its own bits: thread t adds p[t], p[t + B], ... in turn,
// each wave reduces by the butterfly of wave_sum, and thread 0 adds the wave
// sums in wave order.  Every thread of the block must call it (it holds two
// block barriers); the result is returned to every thread.  red: shared
// scratch of at least blockDim.x / 64 + 1 doubles.
__device__ inline double block_sum_fixed(const double* __restrict__ p, int64_t n, double* red) {
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) s += p[e];
  s = wave_sum(s);
  const int nw = (int)(blockDim.x >> 6);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w];
    red[nw] = t;
  }
  __syncthreads();
  return red[nw];
}

// Monotone integer key of |x|: the IEEE bits with the sign cleared.
__device__ __forceinline__ unsigned long long abs_key(float x) {
  return (unsigned long long)(__float_as_uint(x) & 0x7fffffffu);
}
__device__ __forceinline__ unsigned long long abs_key(double x) {
  return (unsigned long long)__double_as_longlong(x) & 0x7fffffffffffffffull;
}

}  // namespace godec
