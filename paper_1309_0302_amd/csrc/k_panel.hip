// Tall-skinny panel products over the working copy D = X - S_{t-1}.
//
// Algorithm 1 spends its time in products of D (or D^T) with r-column
// panels (Sec. 3.1: "the time complexity is dominated by matrix
// multiplications").  These kernels stream D row-major with 16-byte vector
// loads, keep the r-wide panel rows in LDS, and accumulate in the panel
// type (FP64, or FP32 for the f32 and bf16 storage modes).
#include "godec_internal.h"
#include "k_common.h"

namespace godec {

// ---------------------------------------------------------------------------
// W = D Z.  Each wave owns NR rows; lanes cover 4 consecutive columns of a
// 256-column chunk whose Z rows are staged in LDS; the partial row sums are
// reduced across the wave with a butterfly at the end.
// ---------------------------------------------------------------------------
template <typename TA, int RP>
constexpr int apply_rows() {
  if (sizeof(TA) == 8) return RP <= 8 ? 4 : (RP <= 16 ? 2 : 1);
  return RP <= 8 ? 8 : (RP <= 16 ? 4 : 3);
}

template <typename TD, typename TA, int RP>
__global__ __launch_bounds__(256) void k_apply(const TD* __restrict__ D,
                                               int64_t ldd, int64_t m,
                                               const TA* __restrict__ Z,
                                               TA* __restrict__ W) {
  constexpr int NR = apply_rows<TA, RP>();
  constexpr int CJ = (sizeof(TA) == 8 && RP > 16) ? 128 : 256;
  constexpr int SUB = CJ / 64;  // columns per lane per chunk (2 or 4)
  __shared__ TA zs[CJ * RP];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * NR;
  TA acc[NR][RP];
#pragma unroll
  for (int a = 0; a < NR; ++a)
#pragma unroll
    for (int c = 0; c < RP; ++c) acc[a][c] = TA(0);

  for (int64_t c0 = 0; c0 < ldd; c0 += CJ) {
    const int64_t ncol = (ldd - c0) < CJ ? (ldd - c0) : CJ;
    __syncthreads();
    for (int e = threadIdx.x; e < CJ * RP; e += 256)
      zs[e] = (e < ncol * RP) ? Z[c0 * RP + e] : TA(0);
    __syncthreads();
    const int64_t j = c0 + (int64_t)lane * SUB;
    if (j < ldd) {
      TA d[NR][4];
#pragma unroll
      for (int a = 0; a < NR; ++a) {
        if (row0 + a < m) {
          if constexpr (SUB == 4)
            load4(D + (row0 + a) * ldd + j, d[a]);
          else
            load2(D + (row0 + a) * ldd + j, d[a]);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) d[a][t] = TA(0);
        }
      }
#pragma unroll
      for (int t = 0; t < SUB; ++t) {
        TA z[RP];
#pragma unroll
        for (int c = 0; c < RP; ++c) z[c] = zs[(lane * SUB + t) * RP + c];
#pragma unroll
        for (int a = 0; a < NR; ++a)
#pragma unroll
          for (int c = 0; c < RP; ++c) acc[a][c] = fma_t(d[a][t], z[c], acc[a][c]);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < NR; ++a)
#pragma unroll
    for (int c = 0; c < RP; ++c) acc[a][c] = wave_sum(acc[a][c]);
#pragma unroll
  for (int a = 0; a < NR; ++a)
#pragma unroll
    for (int c = 0; c < RP; ++c)
      if (((a * RP + c) & 63) == lane && row0 + a < m) W[(row0 + a) * RP + c] = acc[a][c];
}

// ---------------------------------------------------------------------------
// Zpart[chunk] = D[rows of chunk]^T W[rows of chunk].  A block covers 1024
// columns (4 per lane, one 16-byte load per row) and one chunk of rows;
// the W rows of the chunk are staged in LDS and read as broadcasts.
// ---------------------------------------------------------------------------
template <typename TD, typename TA, int RP>
__global__ __launch_bounds__(256) void k_apply_t(const TD* __restrict__ D,
                                                 int64_t ldd, int64_t m,
                                                 const TA* __restrict__ W,
                                                 TA* __restrict__ Zpart,
                                                 int64_t rows_per_chunk) {
  constexpr int RB = 64;
  __shared__ TA ws[RB * RP];
  const int64_t j = (int64_t)blockIdx.x * 1024 + (int64_t)threadIdx.x * 4;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r1 = (r0 + rows_per_chunk) < m ? (r0 + rows_per_chunk) : m;
  TA acc[4][RP];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int c = 0; c < RP; ++c) acc[t][c] = TA(0);
  for (int64_t i0 = r0; i0 < r1; i0 += RB) {
    const int nr = (r1 - i0) < RB ? (int)(r1 - i0) : RB;
    __syncthreads();
    for (int e = threadIdx.x; e < RB * RP; e += 256)
      ws[e] = (e < nr * RP) ? W[i0 * RP + e] : TA(0);
    __syncthreads();
    if (j < ldd) {
      for (int ii = 0; ii < nr; ++ii) {
        TA d[4];
        load4(D + (i0 + ii) * ldd + j, d);
#pragma unroll
        for (int c = 0; c < RP; ++c) {
          const TA w = ws[ii * RP + c];
#pragma unroll
          for (int t = 0; t < 4; ++t) acc[t][c] = fma_t(d[t], w, acc[t][c]);
        }
      }
    }
  }
  if (j < ldd) {
    TA* out = Zpart + ((int64_t)blockIdx.y * ldd + j) * RP;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int c = 0; c < RP; ++c) out[t * RP + c] = acc[t][c];
  }
}

template <typename TA>
__global__ __launch_bounds__(256) void k_reduce_chunks(const TA* __restrict__ Zpart,
                                                       int64_t nchunks,
                                                       int64_t nel,
                                                       TA* __restrict__ Zo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nel) return;
  TA s = TA(0);
  for (int64_t b = 0; b < nchunks; ++b) s += Zpart[b * nel + e];
  Zo[e] = s;
}

// Out = P R^{-1} by forward substitution in FP64 (x R = p row by row, R
// upper triangular in st->Rq, 1/diag in st->dinv, zero on inactive
// columns); optionally also the transposed panel Zt (32 x ldz) in bf16 or
// f32 for the next matrix-core pass, rows >= RP zero.
template <typename TA, int RP, typename TT>
__global__ __launch_bounds__(256) void k_apply_rinv(const TA* __restrict__ P, int64_t rows,
                                                    const SmallState* __restrict__ st,
                                                    TA* __restrict__ Out, TT* __restrict__ Zt,
                                                    int64_t ldz) {
  __shared__ double rs[RP * RP];
  __shared__ double di[RP];
  for (int e = threadIdx.x; e < RP * RP; e += 256) rs[e] = st->Rq[e];
  if (threadIdx.x < RP) di[threadIdx.x] = st->dinv[threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows) return;
  double x[RP];
#pragma unroll
  for (int j = 0; j < RP; ++j) {
    double s = (double)P[i * RP + j];
#pragma unroll
    for (int l = 0; l < j; ++l) s = fma(-x[l], rs[l * RP + j], s);
    x[j] = s * di[j];
  }
#pragma unroll
  for (int j = 0; j < RP; ++j) Out[i * RP + j] = (TA)x[j];
  if (Zt != nullptr) {
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      const float v = j < RP ? (float)x[j] : 0.f;
      if constexpr (sizeof(TT) == 2)
        Zt[(int64_t)j * ldz + i] = f32_to_bf16(v);
      else
        Zt[(int64_t)j * ldz + i] = (TT)v;
    }
  }
}

// Out = P K with K an RP x RP matrix in the panel type.
template <typename TA, int RP>
__global__ __launch_bounds__(256) void k_apply_small(const TA* __restrict__ P,
                                                     int64_t rows,
                                                     const TA* __restrict__ K,
                                                     TA* __restrict__ Out) {
  __shared__ TA ks[RP * RP];
  for (int e = threadIdx.x; e < RP * RP; e += 256) ks[e] = K[e];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows) return;
  TA p[RP], o[RP];
#pragma unroll
  for (int a = 0; a < RP; ++a) { p[a] = P[i * RP + a]; o[a] = TA(0); }
#pragma unroll
  for (int a = 0; a < RP; ++a)
#pragma unroll
    for (int c = 0; c < RP; ++c) o[c] = fma_t(p[a], ks[a * RP + c], o[c]);
#pragma unroll
  for (int c = 0; c < RP; ++c) Out[i * RP + c] = o[c];
}

// dst (rows_pad x RP, panel type) <- src (rows x r, FP64 row-major), with
// the columns at or past st->r_eff and all padding set to zero.
template <typename TA, int RP>
__global__ __launch_bounds__(256) void k_copy_panel(const double* __restrict__ src,
                                                    int64_t rows, int64_t rows_pad,
                                                    int r,
                                                    const SmallState* __restrict__ st,
                                                    TA* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows_pad * RP) return;
  const int64_t i = e / RP;
  const int c = (int)(e % RP);
  const int reff = st->r_eff;
  dst[e] = (i < rows && c < r && c < reff) ? (TA)src[i * r + c] : TA(0);
}

// dst (rows x r, row-major) <- the first r columns of src (rows x RP).
template <typename TA, int RP>
__global__ __launch_bounds__(256) void k_cast_panel(const TA* __restrict__ src, int64_t rows,
                                                    int r, TA* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * r) return;
  const int64_t i = e / r;
  const int c = (int)(e % r);
  dst[e] = src[i * RP + c];
}

// ---------------------------------------------------------------------------
// Host launchers: dispatch on storage type and padded width.
// ---------------------------------------------------------------------------
#define GODEC_RP_SWITCH(rp, ...)                   \
  switch (rp) {                                    \
    case 1: { constexpr int RP = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int RP = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int RP = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int RP = 8; __VA_ARGS__; } break;   \
    case 12: { constexpr int RP = 12; __VA_ARGS__; } break; \
    case 16: { constexpr int RP = 16; __VA_ARGS__; } break; \
    case 20: { constexpr int RP = 20; __VA_ARGS__; } break; \
    case 24: { constexpr int RP = 24; __VA_ARGS__; } break; \
    case 32: { constexpr int RP = 32; __VA_ARGS__; } break; \
    default: break;                                \
  }

template <typename TD, typename TA>
static void apply_t(const Launch& L, int rp, const void* D, int64_t ldd,
                    int64_t m, const void* Z, void* W) {
  GODEC_RP_SWITCH(rp, {
    constexpr int NR = apply_rows<TA, RP>();
    const int64_t blocks = (m + 4 * NR - 1) / (4 * NR);
    hipLaunchKernelGGL((k_apply<TD, TA, RP>), dim3((unsigned)blocks), dim3(256), 0,
                       L.stream, (const TD*)D, ldd, m, (const TA*)Z, (TA*)W);
  });
}

void launch_apply(const Launch& L, DType td, int rp, const void* D,
                  int64_t ldd, int64_t m, const void* Z, void* W) {
  if (td == F64) apply_t<double, double>(L, rp, D, ldd, m, Z, W);
  else if (td == F32) apply_t<float, float>(L, rp, D, ldd, m, Z, W);
  else apply_t<uint16_t, float>(L, rp, D, ldd, m, Z, W);
}

template <typename TD, typename TA>
static void apply_tt(const Launch& L, int rp, const void* D, int64_t ldd,
                     int64_t m, const void* W, void* Zpart, int64_t rpc,
                     int64_t nchunks) {
  GODEC_RP_SWITCH(rp, {
    dim3 grid((unsigned)((ldd + 1023) / 1024), (unsigned)nchunks);
    hipLaunchKernelGGL((k_apply_t<TD, TA, RP>), grid, dim3(256), 0, L.stream,
                       (const TD*)D, ldd, m, (const TA*)W, (TA*)Zpart, rpc);
  });
}

void launch_apply_t(const Launch& L, DType td, int rp, const void* D,
                    int64_t ldd, int64_t m, const void* W, void* Zpart,
                    int64_t rows_per_chunk, int64_t nchunks) {
  if (td == F64) apply_tt<double, double>(L, rp, D, ldd, m, W, Zpart, rows_per_chunk, nchunks);
  else if (td == F32) apply_tt<float, float>(L, rp, D, ldd, m, W, Zpart, rows_per_chunk, nchunks);
  else apply_tt<uint16_t, float>(L, rp, D, ldd, m, W, Zpart, rows_per_chunk, nchunks);
}

void launch_reduce_chunks(const Launch& L, bool f64, int rp, const void* Zpart,
                          int64_t nchunks, int64_t rows, void* Zo) {
  const int64_t nel = rows * rp;
  const unsigned blocks = (unsigned)((nel + 255) / 256);
  if (f64)
    hipLaunchKernelGGL(k_reduce_chunks<double>, dim3(blocks), dim3(256), 0, L.stream,
                       (const double*)Zpart, nchunks, nel, (double*)Zo);
  else
    hipLaunchKernelGGL(k_reduce_chunks<float>, dim3(blocks), dim3(256), 0, L.stream,
                       (const float*)Zpart, nchunks, nel, (float*)Zo);
}

void launch_apply_rinv(const Launch& L, bool f64, int rp, const void* P, int64_t rows,
                       const SmallState* st, void* Out, DType zt_type, void* Zt, int64_t ldz) {
  const unsigned blocks = (unsigned)((rows + 255) / 256);
  GODEC_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((k_apply_rinv<double, RP, double>), dim3(blocks), dim3(256), 0,
                         L.stream, (const double*)P, rows, st, (double*)Out, (double*)nullptr,
                         ldz);
    else if (Zt != nullptr && zt_type == BF16)
      hipLaunchKernelGGL((k_apply_rinv<float, RP, uint16_t>), dim3(blocks), dim3(256), 0,
                         L.stream, (const float*)P, rows, st, (float*)Out, (uint16_t*)Zt, ldz);
    else
      hipLaunchKernelGGL((k_apply_rinv<float, RP, float>), dim3(blocks), dim3(256), 0,
                         L.stream, (const float*)P, rows, st, (float*)Out, (float*)Zt, ldz);
  });
}

void launch_apply_small(const Launch& L, bool f64, int rp, const void* P,
                        int64_t rows, const void* K, void* Out) {
  const unsigned blocks = (unsigned)((rows + 255) / 256);
  GODEC_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((k_apply_small<double, RP>), dim3(blocks), dim3(256), 0,
                         L.stream, (const double*)P, rows, (const double*)K, (double*)Out);
    else
      hipLaunchKernelGGL((k_apply_small<float, RP>), dim3(blocks), dim3(256), 0,
                         L.stream, (const float*)P, rows, (const float*)K, (float*)Out);
  });
}

void launch_copy_panel(const Launch& L, bool f64, int rp, const double* src,
                       int64_t rows, int64_t rows_pad, int r,
                       const SmallState* st, void* dst) {
  const unsigned blocks = (unsigned)((rows_pad * rp + 255) / 256);
  GODEC_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((k_copy_panel<double, RP>), dim3(blocks), dim3(256), 0,
                         L.stream, src, rows, rows_pad, r, st, (double*)dst);
    else
      hipLaunchKernelGGL((k_copy_panel<float, RP>), dim3(blocks), dim3(256), 0,
                         L.stream, src, rows, rows_pad, r, st, (float*)dst);
  });
}

void launch_cast_panel(const Launch& L, bool f64, int rp, const void* src,
                       int64_t rows, int r, void* dst) {
  const unsigned blocks = (unsigned)((rows * r + 255) / 256);
  if (blocks == 0) return;
  GODEC_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((k_cast_panel<double, RP>), dim3(blocks), dim3(256), 0, L.stream,
                         (const double*)src, rows, r, (double*)dst);
    else
      hipLaunchKernelGGL((k_cast_panel<float, RP>), dim3(blocks), dim3(256), 0, L.stream,
                         (const float*)src, rows, r, (float*)dst);
  });
}

}  // namespace godec
