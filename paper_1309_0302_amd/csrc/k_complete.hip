// GoDec matrix completion (Sec. 2): the S update on a fixed support set in
// place of the cardinality constraint, S_t = P_support(X - L_t).  The L
// update and the D update are those of Algorithm 1; these kernels replace
// the radix selection.
#include <hip/hip_runtime.h>

#include "godec_internal.h"
#include "k_common.h"

namespace godec {

namespace {

constexpr int kCompBlocks = 2048;   // most blocks (= partial sums) per pass

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

// For every support entry e (ascending linear index id = i n + j):
// r = X_ij - (U_L V_L^T)_ij, s_idx[e] = id, s_val[e] = r, s_x[e] = X_ij;
// part[block] = sum of r^2 over the block's entries.
template <typename T, int RP>
__global__ __launch_bounds__(256) void kc_gather(const T* __restrict__ X, int64_t ldx,
                                                 const T* __restrict__ UL,
                                                 const T* __restrict__ VL, int64_t n,
                                                 const int64_t* __restrict__ support,
                                                 int64_t nnz, int64_t* __restrict__ s_idx,
                                                 T* __restrict__ s_val, T* __restrict__ s_x,
                                                 double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * 256) {
    const int64_t id = support[e];
    const int64_t i = id / n, j = id % n;
    T l = T(0);
#pragma unroll
    for (int c = 0; c < RP; ++c) l = fma_t(UL[i * RP + c], VL[j * RP + c], l);
    const T x = X[i * ldx + j];
    const T r = x - l;
    s_idx[e] = id;
    s_val[e] = r;
    s_x[e] = x;
    acc = fma((double)r, (double)r, acc);
  }
  const double t = block_sum<T>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// part[block] = sum over the block's entries of (X - U_L V_L^T)^2.
template <typename T, int RP>
__global__ __launch_bounds__(256) void kc_res_norm(const T* __restrict__ X, int64_t ldx,
                                                   const T* __restrict__ UL,
                                                   const T* __restrict__ VL, int64_t m,
                                                   int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  const int64_t total = m * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n, j = e % n;
    T l = T(0);
#pragma unroll
    for (int c = 0; c < RP; ++c) l = fma_t(UL[i * RP + c], VL[j * RP + c], l);
    const double r = (double)(X[i * ldx + j] - l);
    acc = fma(r, r, acc);
  }
  const double t = block_sum<T>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// The plan of a fixed-support step: nnz, sum_sel2 = sum of the gather
// partials, sum_r2 = sum of the norm partials (both in block order).
__global__ __launch_bounds__(64) void kc_finish(const double* __restrict__ psel, int nsel,
                                                const double* __restrict__ pall, int nall,
                                                int64_t nnz, SelPlan* __restrict__ plan) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int q = 0; q < nsel; ++q) a += psel[q];
  for (int q = 0; q < nall; ++q) b += pall[q];
  plan->nnz = nnz;
  plan->sum_sel2 = a;
  plan->sum_r2 = b;
  plan->threshold = 0.0;
  plan->slow = 0;
  plan->overflow = 0;
  plan->mode = SEL_DONE;
}

unsigned blocks_of(int64_t work) {
  int64_t g = (work + 255) / 256;
  if (g > kCompBlocks) g = kCompBlocks;
  if (g < 1) g = 1;
  return (unsigned)g;
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
                          const int64_t* support, int64_t nnz, int64_t* s_idx, void* s_val,
                          void* s_x, SelPlan* plan, double* scratch) {
  const unsigned gs = blocks_of(nnz), ga = blocks_of(m * n);
  double* psel = scratch;
  double* pall = scratch + kCompBlocks;
  GC_RP_SWITCH(rp, {
    if (f64) {
      hipLaunchKernelGGL((kc_gather<double, RP>), dim3(gs), dim3(256), 0, L.stream,
                         (const double*)X, ldx, (const double*)UL, (const double*)VL, n, support,
                         nnz, s_idx, (double*)s_val, (double*)s_x, psel);
      hipLaunchKernelGGL((kc_res_norm<double, RP>), dim3(ga), dim3(256), 0, L.stream,
                         (const double*)X, ldx, (const double*)UL, (const double*)VL, m, n,
                         pall);
    } else {
      hipLaunchKernelGGL((kc_gather<float, RP>), dim3(gs), dim3(256), 0, L.stream,
                         (const float*)X, ldx, (const float*)UL, (const float*)VL, n, support,
                         nnz, s_idx, (float*)s_val, (float*)s_x, psel);
      hipLaunchKernelGGL((kc_res_norm<float, RP>), dim3(ga), dim3(256), 0, L.stream,
                         (const float*)X, ldx, (const float*)UL, (const float*)VL, m, n, pall);
    }
  });
  hipLaunchKernelGGL(kc_finish, dim3(1), dim3(64), 0, L.stream, psel, (int)gs, pall, (int)ga,
                     nnz, plan);
}

int64_t fixed_support_scratch_doubles() { return 2 * (int64_t)kCompBlocks; }

}  // namespace godec
