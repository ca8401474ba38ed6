// Matrix-core pieces shared by the panel kernels: the MFMA operand types and
// the main loop of the transposed panel product Z_out^T = W^T D over one
// block's 128-column strip and row chunk (k_mm_b in k_mfma.hip, and the
// Gram-pass kernel of k_small.hip that adds the Cholesky QR step to it).
//
// Layouts (v_mfma_f32_32x32x{16_bf16, 2_f32}, lane l, l%32 = index on the
// lanes, l/32 = group g): A operand row i = l%32; B operand column
// j = l%32; accumulator register v holds C[8(v/4) + 4g + v%4][l%32].
#pragma once

#include "k_common.h"

namespace godec {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int acc_row(int v, int lane) {
  return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
}

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) {
  return __builtin_bit_cast(bf16x8, v);
}

__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma_f32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Stride (floats per column of D) of the row-chunk partials of Z_out: the
// panel width rounded up to whole float4 groups (the MFMA tile's padding
// rows past it are not stored).
__host__ __device__ constexpr int zpart_stride(int rp) { return rp < 4 ? 4 : (rp + 3) / 4 * 4; }

// Main loop of W^T D over rows [k0, k1) of the 128-column strip at column
// cw: lane n holds columns 4n .. 4n+3 of the strip, one per 32-column MFMA
// tile (acc[t]), so a wave reads each row as one contiguous run.  The bf16
// form takes 16 rows per step (8 per lane group, repacked into pairs).
__device__ __forceinline__ void mmb_loop_bf16(const uint16_t* __restrict__ D, int64_t ldd,
                                              int64_t mpad, const uint16_t* __restrict__ Wt,
                                              int64_t cw, int64_t k0, int64_t k1, int lane,
                                              f32x16 (&acc)[4]) {
  const int n = lane & 31, g = lane >> 5;
  const uint16_t* pd = D + (8 * g) * ldd + cw + 4 * n;
  const uint16_t* pw = Wt + (int64_t)n * mpad + 8 * g;
  for (int64_t kk = k0; kk < k1; kk += 16) {
    // A: W^T[n][kk + 8g .. +7]
    const u32x4 a = *reinterpret_cast<const u32x4*>(pw + kk);
    // B: 8 rows (kk + 8g + s) x 4 columns
    uint2 d[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) d[s] = *reinterpret_cast<const uint2*>(pd + (kk + s) * ldd);
    // repack: tile t gets column 4n + t of the 8 rows (bf16 pairs)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      u32x4 b;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const uint32_t x0 = (t < 2) ? d[2 * h].x : d[2 * h].y;
        const uint32_t x1 = (t < 2) ? d[2 * h + 1].x : d[2 * h + 1].y;
        const uint32_t lo = (t & 1) ? (x0 >> 16) : (x0 & 0xffffu);
        const uint32_t hi = (t & 1) ? (x1 >> 16) : (x1 & 0xffffu);
        b[h] = lo | (hi << 16);
      }
      acc[t] = mfma_bf16(as_bf16x8(a), as_bf16x8(b), acc[t]);
    }
  }
}

// FP32 form: 8 rows per step; slot s pairs row kk + 4g + s on both operands.
// A step's 16 MFMAs take about as long as its loads, so the loads of the
// next step are issued before the MFMAs of the current one (two register
// buffers).
__device__ __forceinline__ void mmb_loop_f32(const float* __restrict__ D, int64_t ldd,
                                             int64_t mpad, const float* __restrict__ Wt,
                                             int64_t cw, int64_t k0, int64_t k1, int lane,
                                             f32x16 (&acc)[4]) {
  const int n = lane & 31, g = lane >> 5;
  const float* pd = D + (4 * g) * ldd + cw + 4 * n;
  const float* pw = Wt + (int64_t)n * mpad + 4 * g;
  if (k0 >= k1) return;
  float4 a = *reinterpret_cast<const float4*>(pw + k0);
  float4 d[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) d[s] = *reinterpret_cast<const float4*>(pd + (k0 + s) * ldd);
  for (int64_t kk = k0; kk < k1; kk += 8) {
    const float av[4] = {a.x, a.y, a.z, a.w};
    float4 dc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) dc[s] = d[s];
    if (kk + 8 < k1) {   // uniform
      a = *reinterpret_cast<const float4*>(pw + kk + 8);
#pragma unroll
      for (int s = 0; s < 4; ++s) d[s] = *reinterpret_cast<const float4*>(pd + (kk + 8 + s) * ldd);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc[0] = mfma_f32(av[s], dc[s].x, acc[0]);
      acc[1] = mfma_f32(av[s], dc[s].y, acc[1]);
      acc[2] = mfma_f32(av[s], dc[s].z, acc[2]);
      acc[3] = mfma_f32(av[s], dc[s].w, acc[3]);
    }
  }
}

// Rows of the chunk [kc0, kc1) taken by wave `wave` (the chunk is split into
// four ranges; `step` = rows per loop step).
__device__ __forceinline__ void mmb_wave_rows(int64_t kc0, int64_t kc1, int wave, int step,
                                              int64_t& k0, int64_t& k1) {
  const int64_t q = ((kc1 - kc0) / 4 + step - 1) / step * step;
  k0 = kc0 + q * wave;
  k1 = (k0 + q) < kc1 ? (k0 + q) : kc1;
}

// Sum of the four waves' tiles in a fixed order ((w0 + w2) + (w1 + w3));
// afterwards wave 0's acc holds the block's sum.  lds: 2 * 64 * 64 floats.
__device__ __forceinline__ void mmb_block_reduce(f32x16 (&acc)[4], float* lds, int wave,
                                                 int lane) {
  float* mine = lds + (int64_t)(wave & 1) * 64 * 64;
  if (wave >= 2) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) mine[(t * 16 + v) * 64 + lane] = acc[t][v];
  }
  __syncthreads();
  if (wave < 2) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[t][v] += mine[(t * 16 + v) * 64 + lane];
  }
  __syncthreads();
  if (wave == 1) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) lds[(t * 16 + v) * 64 + lane] = acc[t][v];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[t][v] += lds[(t * 16 + v) * 64 + lane];
  }
}

}  // namespace godec
