// GreBsmo kernels (Sec. 3.2.1): the fused soft-thresholding pass of Eq. 12 /
// Eq. 13 and the small helpers of the greedy rank step (Algorithm 2).  The
// panel products (D V^T, U^T D), the Cholesky QR steps and the power steps of
// the greedy directions reuse the panel, Gram and matrix-core kernels of the
// BRP path.
#include <hip/hip_runtime.h>

#include "godec_internal.h"
#include "k_common.h"
#include "k_mmb.h"

namespace godec {

namespace {

constexpr int kSoftRows = 16;      // rows per block of the soft pass
constexpr int kSoftCols = 256;     // columns per block (one per thread)

// One block per (16-row, 256-column) tile.  Each thread owns a column j and
// keeps V^T's row j in registers; row i of U is uniform across the block.
// For every element
//   res = X - (U V)_ij,  s = sgn(res) max(|res| - lambda, 0)     (Eq. 12)
//   e = res - s          (the entry of X - U V - S, i.e. dF/dV of Eq. 14)
// MODE 0 writes D = X - s (and e into R when R is given) and the block's
// partial sums of e^2, |s| and the count of nonzero s; MODE 1 writes s to
// Sout (ld lds).
template <typename TA, int RP, int MODE>
__global__ __launch_bounds__(kSoftCols) void kg_soft(const TA* __restrict__ X, int64_t ldx,
                                                      const TA* __restrict__ U,
                                                      const TA* __restrict__ Vt, int64_t m,
                                                      int64_t n, TA lam, TA* __restrict__ D,
                                                      int64_t ldd, TA* __restrict__ R,
                                                      TA* __restrict__ Sout, int64_t lds,
                                                      double* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.y * kSoftCols + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * kSoftRows;
  const int64_t i1 = (i0 + kSoftRows) < m ? (i0 + kSoftRows) : m;
  double e2 = 0.0, l1 = 0.0, cnt = 0.0;
  if (j < n) {
    TA v[RP];
#pragma unroll
    for (int c = 0; c < RP; ++c) v[c] = Vt[j * RP + c];
    for (int64_t i = i0; i < i1; ++i) {
      const TA* u = U + i * RP;
      TA l = TA(0);
#pragma unroll
      for (int c = 0; c < RP; ++c) l = fma_t(u[c], v[c], l);
      const TA x = X[i * ldx + j];
      const TA res = x - l;
      const TA a = fabs(res) - lam;
      const TA s = a > TA(0) ? copysign(a, res) : TA(0);
      if constexpr (MODE == 0) {
        const TA e = res - s;
        D[i * ldd + j] = x - s;
        if (R != nullptr) R[i * ldd + j] = e;
        e2 = fma((double)e, (double)e, e2);
        l1 += fabs((double)s);
        cnt += s != TA(0) ? 1.0 : 0.0;
      } else {
        Sout[i * lds + j] = s;
      }
    }
  }
  if constexpr (MODE == 0) {
    if (part == nullptr) return;   // uniform: no statistics wanted
    __shared__ double red[3][kSoftCols / 64];
    e2 = wave_sum(e2);
    l1 = wave_sum(l1);
    cnt = wave_sum(cnt);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
      red[0][w] = e2;
      red[1][w] = l1;
      red[2][w] = cnt;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < kSoftCols / 64; ++q) t += red[threadIdx.x][q];
      const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
      part[b * 3 + threadIdx.x] = t;
    }
  }
}

// out[0..2] = sums of the nb partial triples, in a fixed order (one block).
__global__ __launch_bounds__(256) void kg_stats_reduce(const double* __restrict__ part,
                                                       int64_t nb, double* __restrict__ out) {
  __shared__ double red[3][256];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t k = threadIdx.x; k < nb; k += 256) {
    a += part[k * 3 + 0];
    b += part[k * 3 + 1];
    c += part[k * 3 + 2];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
#pragma unroll
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

// Vt[:, c0 + c] <- P[:, c] for c < cnt (rows x RP panels).
template <typename TA, int RP>
__global__ __launch_bounds__(256) void kg_put_cols(const TA* __restrict__ P, int64_t rows,
                                                   int c0, int cnt, TA* __restrict__ Vt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * cnt) return;
  const int64_t i = e / cnt;
  const int c = (int)(e % cnt);
  Vt[i * RP + c0 + c] = P[i * RP + c];
}

// V^T (ldd x rp) = sum_ch Zpart[ch] (ldd x zpart_stride(rp)), and its transpose into rows
// j < rp of Zt (32 x ldd, the B operand of the next matrix-core pass).  One
// block per 16 consecutive outputs e = c * rp + j; each of 16 chunk lanes
// adds every 16th chunk (ascending), then the lane sums are added in lane
// order (a fixed order).
constexpr int kZtVals = 16;
constexpr int kZtLanes = 16;
__global__ __launch_bounds__(256) void kg_reduce_zt(const float* __restrict__ Zpart,
                                                    int64_t nch, int64_t ldd, int rp,
                                                    float* __restrict__ Vt,
                                                    float* __restrict__ Zt) {
  __shared__ float red[kZtLanes][kZtVals];
  const int v = threadIdx.x % kZtVals, hl = threadIdx.x / kZtVals;
  const int64_t e = (int64_t)blockIdx.x * kZtVals + v;
  const bool live = e < ldd * rp;
  float s = 0.f;
  if (live) {
    const int zs = zpart_stride(rp);
    const float* p = Zpart + (e / rp) * zs + (e % rp);
    const int64_t step = ldd * zs;
    for (int64_t h = hl; h < nch; h += kZtLanes) s += p[h * step];
  }
  red[hl][v] = s;
  __syncthreads();
  if (hl == 0 && live) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < kZtLanes; ++q) t += red[q][v];
    Vt[e] = t;
    Zt[(e % rp) * ldd + e / rp] = t;
  }
}

}  // namespace

void gb_reduce_zt(const Launch& L, const float* Zpart, int64_t nch, int64_t ldd, int rp,
                  float* Vt, float* Zt) {
  const unsigned b = (unsigned)((ldd * rp + kZtVals - 1) / kZtVals);
  hipLaunchKernelGGL(kg_reduce_zt, dim3(b), dim3(256), 0, L.stream, Zpart, nch, ldd, rp, Vt,
                     Zt);
}

#define GB_RP_SWITCH(rp, ...)                                \
  switch (rp) {                                              \
    case 1: { constexpr int RP = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int RP = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int RP = 4; __VA_ARGS__; } break;   \
    case 8: { constexpr int RP = 8; __VA_ARGS__; } break;   \
    case 12: { constexpr int RP = 12; __VA_ARGS__; } break; \
    case 16: { constexpr int RP = 16; __VA_ARGS__; } break; \
    case 20: { constexpr int RP = 20; __VA_ARGS__; } break; \
    case 24: { constexpr int RP = 24; __VA_ARGS__; } break; \
    case 32: { constexpr int RP = 32; __VA_ARGS__; } break; \
    default: break;                                          \
  }

int64_t gb_soft_blocks(int64_t m, int64_t n) {
  return ((m + kSoftRows - 1) / kSoftRows) * ((n + kSoftCols - 1) / kSoftCols);
}

void gb_soft(const Launch& L, bool f64, int rp, const void* X, int64_t ldx, const void* U,
             const void* Vt, int64_t m, int64_t n, double lam, void* D, int64_t ldd, void* R,
             double* part, double* stats) {
  if (m < 1 || n < 1) return;
  const dim3 grid((unsigned)((m + kSoftRows - 1) / kSoftRows),
                  (unsigned)((n + kSoftCols - 1) / kSoftCols));
  GB_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((kg_soft<double, RP, 0>), grid, dim3(kSoftCols), 0, L.stream,
                         (const double*)X, ldx, (const double*)U, (const double*)Vt, m, n, lam,
                         (double*)D, ldd, (double*)R, (double*)nullptr, (int64_t)0, part);
    else
      hipLaunchKernelGGL((kg_soft<float, RP, 0>), grid, dim3(kSoftCols), 0, L.stream,
                         (const float*)X, ldx, (const float*)U, (const float*)Vt, m, n,
                         (float)lam, (float*)D, ldd, (float*)R, (float*)nullptr, (int64_t)0,
                         part);
  });
  if (stats != nullptr)
    hipLaunchKernelGGL(kg_stats_reduce, dim3(1), dim3(256), 0, L.stream, part,
                       gb_soft_blocks(m, n), stats);
}

void gb_soft_s(const Launch& L, bool f64, int rp, const void* X, int64_t ldx, const void* U,
               const void* Vt, int64_t m, int64_t n, double lam, void* S, int64_t lds) {
  if (m < 1 || n < 1) return;
  const dim3 grid((unsigned)((m + kSoftRows - 1) / kSoftRows),
                  (unsigned)((n + kSoftCols - 1) / kSoftCols));
  GB_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((kg_soft<double, RP, 1>), grid, dim3(kSoftCols), 0, L.stream,
                         (const double*)X, ldx, (const double*)U, (const double*)Vt, m, n, lam,
                         (double*)nullptr, (int64_t)0, (double*)nullptr, (double*)S, lds,
                         (double*)nullptr);
    else
      hipLaunchKernelGGL((kg_soft<float, RP, 1>), grid, dim3(kSoftCols), 0, L.stream,
                         (const float*)X, ldx, (const float*)U, (const float*)Vt, m, n,
                         (float)lam, (float*)nullptr, (int64_t)0, (float*)nullptr, (float*)S,
                         lds, (double*)nullptr);
  });
}

void gb_put_cols(const Launch& L, bool f64, int rp, const void* P, int64_t rows, int c0,
                 int cnt, void* Vt) {
  if (rows < 1 || cnt < 1) return;
  const unsigned blocks = (unsigned)((rows * cnt + 255) / 256);
  GB_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((kg_put_cols<double, RP>), dim3(blocks), dim3(256), 0, L.stream,
                         (const double*)P, rows, c0, cnt, (double*)Vt);
    else
      hipLaunchKernelGGL((kg_put_cols<float, RP>), dim3(blocks), dim3(256), 0, L.stream,
                         (const float*)P, rows, c0, cnt, (float*)Vt);
  });
}

}  // namespace godec
