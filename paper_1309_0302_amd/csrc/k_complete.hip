// GoDec matrix completion (Sec. 2): the S update on a fixed support set in
// place of the cardinality constraint, S_t = P_support(X - L_t).  The L
// update and the D update are those of Algorithm 1; these kernels replace
// the radix selection.
#include <hip/hip_runtime.h>

#include "godec_internal.h"
#include "k_common.h"

namespace godec {

namespace {

constexpr int kNormBlocks = 16384;  // most blocks (= partial sums) of the pass

template <typename T>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

// One pass over X for the whole fixed-support step.  Tiles of 64 rows x 256
// columns (tile t: row block t % nrb, column block t / nrb) are walked
// grid-stride; a thread owns one column and keeps its row of V_L in
// registers (the row of U_L is the same for the whole block).  The rows of
// a tile go in chunks of CR: every thread loads its X entries of the chunk
// together and puts the residuals r = X - (U_L V_L^T) in LDS; then the
// support entries of the chunk's rows inside the tile's columns -- per row
// the contiguous run [row_ptr[i][cb], row_ptr[i][cb + 1]) of the ascending
// list -- are taken by the block in one pass: s_idx, s_val = r, s_x = X, and
// their columns are marked, so that the block partials pall / psel sum r^2
// off / on the support separately (off the support in row order per
// thread).
constexpr int kNormRows = 64;

template <typename T, int RP>
__global__ __launch_bounds__(256) void kc_pass(const T* __restrict__ X, int64_t ldx,
                                               const T* __restrict__ UL,
                                               const T* __restrict__ VL, int64_t m, int64_t n,
                                               int64_t nrb, int64_t ntiles, int64_t ncb,
                                               const int64_t* __restrict__ support,
                                               const int64_t* __restrict__ row_ptr,
                                               int64_t* __restrict__ s_idx,
                                               T* __restrict__ s_val, T* __restrict__ s_x,
                                               double* __restrict__ pall,
                                               double* __restrict__ psel) {
  constexpr int CR = sizeof(T) == 4 ? 16 : 8;   // rows per chunk (LDS: 2 x CR x 256 x T)
  __shared__ T rs[CR][256], xs[CR][256];
  __shared__ unsigned char mk[CR][256];
  __shared__ int64_t rstart[CR];
  __shared__ int rpre[CR + 1];
  __shared__ double red[4];
  double acc = 0.0, accs = 0.0;   // sums of r^2 off and on the support
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t i0 = (t % nrb) * kNormRows;
    const int64_t cb = t / nrb;
    const int64_t j0 = cb * 256;
    const int64_t j = j0 + threadIdx.x;
    const bool live = j < n;
    T v[RP];
#pragma unroll
    for (int c = 0; c < RP; ++c) v[c] = live ? VL[j * RP + c] : T(0);
    const int64_t i1 = (i0 + kNormRows) < m ? (i0 + kNormRows) : m;
    for (int64_t c0 = i0; c0 < i1; c0 += CR) {
      const int nr = (i1 - c0) < CR ? (int)(i1 - c0) : CR;
      // ---- residuals of the chunk (all X loads in flight together) ----
      T x[CR];
#pragma unroll
      for (int rr = 0; rr < CR; ++rr)
        x[rr] = (live && rr < nr) ? X[(c0 + rr) * ldx + j] : T(0);
#pragma unroll
      for (int rr = 0; rr < CR; ++rr) {
        if (rr < nr) {
          const T* u = UL + (c0 + rr) * RP;
          T l = T(0);
#pragma unroll
          for (int c = 0; c < RP; ++c) l = fma_t(u[c], v[c], l);
          rs[rr][threadIdx.x] = x[rr] - l;
          xs[rr][threadIdx.x] = x[rr];
        }
        mk[rr][threadIdx.x] = 0;
      }
      if ((int)threadIdx.x < CR) {
        const int rr = threadIdx.x;
        int len = 0;
        int64_t a = 0;
        if (rr < nr) {
          const int64_t* run = row_ptr + (c0 + rr) * (ncb + 1) + cb;
          a = run[0];
          len = (int)(run[1] - a);
        }
        rstart[rr] = a;
        rpre[rr + 1] = len;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        rpre[0] = 0;
        for (int rr = 0; rr < CR; ++rr) rpre[rr + 1] += rpre[rr];
      }
      __syncthreads();
      // ---- the support entries of the chunk, one pass ----
      const int tot = rpre[CR];
      for (int e = threadIdx.x; e < tot; e += 256) {
        int rr = 0;
        while (rpre[rr + 1] <= e) ++rr;   // at most CR steps
        const int64_t ent = rstart[rr] + (e - rpre[rr]);
        const int64_t id = support[ent];
        const int q = (int)(id - (c0 + rr) * n - j0);
        const T rv = rs[rr][q];
        s_idx[ent] = id;
        s_val[ent] = rv;
        s_x[ent] = xs[rr][q];
        mk[rr][q] = 1;
        accs = fma((double)rv, (double)rv, accs);
      }
      __syncthreads();
      // ---- off the support, in row order ----
      if (live) {
        for (int rr = 0; rr < nr; ++rr)
          if (!mk[rr][threadIdx.x]) {
            const double r = (double)rs[rr][threadIdx.x];
            acc = fma(r, r, acc);
          }
      }
      __syncthreads();   // the next chunk overwrites the staging arrays
    }
  }
  double tot = block_sum<T>(acc, red);
  if (threadIdx.x == 0) pall[blockIdx.x] = tot;
  __syncthreads();
  tot = block_sum<T>(accs, red);
  if (threadIdx.x == 0) psel[blockIdx.x] = tot;
}

// The plan of a fixed-support step: nnz, sum_sel2 = sum of the support
// partials, sum_obs2 = sum of the off-support partials, sum_r2 = both
// (strided per thread, then a tree in LDS: a fixed order).
__global__ __launch_bounds__(256) void kc_finish(const double* __restrict__ psel, int nsel,
                                                 const double* __restrict__ pall, int nall,
                                                 int64_t nnz, SelPlan* __restrict__ plan) {
  __shared__ double ra[256], rb[256];
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nsel; q += 256) a += psel[q];
  for (int q = threadIdx.x; q < nall; q += 256) b += pall[q];
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      ra[threadIdx.x] += ra[threadIdx.x + h];
      rb[threadIdx.x] += rb[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  plan->nnz = nnz;
  plan->sum_sel2 = ra[0];
  plan->sum_obs2 = rb[0];
  plan->sum_r2 = rb[0] + ra[0];
  plan->threshold = 0.0;
  plan->slow = 0;
  plan->overflow = 0;
  plan->mode = SEL_DONE;
}


}  // namespace

#define GC_RP_SWITCH(rp, ...)                                \
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

void launch_fixed_support(const Launch& L, bool f64, int rp, const void* X, int64_t ldx,
                          const void* UL, const void* VL, int64_t m, int64_t n,
                          const int64_t* support, const int64_t* row_ptr, int64_t nnz,
                          int64_t* s_idx, void* s_val, void* s_x, SelPlan* plan,
                          double* scratch) {
  const int64_t nrb = (m + kNormRows - 1) / kNormRows;
  const int64_t ntiles = nrb * ((n + 255) / 256);
  const unsigned ga = (unsigned)(ntiles < kNormBlocks ? ntiles : kNormBlocks);
  double* psel = scratch;
  double* pall = scratch + kNormBlocks;
  GC_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((kc_pass<double, RP>), dim3(ga), dim3(256), 0, L.stream,
                         (const double*)X, ldx, (const double*)UL, (const double*)VL, m, n, nrb,
                         ntiles, (n + 255) / 256, support, row_ptr, s_idx, (double*)s_val,
                         (double*)s_x, pall,
                         psel);
    else
      hipLaunchKernelGGL((kc_pass<float, RP>), dim3(ga), dim3(256), 0, L.stream,
                         (const float*)X, ldx, (const float*)UL, (const float*)VL, m, n, nrb,
                         ntiles, (n + 255) / 256, support, row_ptr, s_idx, (float*)s_val,
                         (float*)s_x, pall,
                         psel);
  });
  hipLaunchKernelGGL(kc_finish, dim3(1), dim3(256), 0, L.stream, psel, (int)ga, pall, (int)ga,
                     nnz, plan);
}

int64_t fixed_support_scratch_doubles() { return 2 * (int64_t)kNormBlocks; }

}  // namespace godec
