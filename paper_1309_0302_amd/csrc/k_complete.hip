// GoDec matrix completion (Sec. 2): the S update on a fixed support set in
// place of the cardinality constraint, S_t = P_support(X - L_t).  The L
// update and the D update are those of Algorithm 1; these kernels replace
// the radix selection.
#include <hip/hip_runtime.h>

#include "godec_internal.h"
#include "k_common.h"

namespace godec {

namespace {

constexpr int kCompBlocks = 2048;   // most blocks (= partial sums) of the gather
constexpr int kNormBlocks = 16384;  // most blocks of the residual-norm pass

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
                                                 bool small,
                                                 const int64_t* __restrict__ support,
                                                 int64_t nnz, int64_t* __restrict__ s_idx,
                                                 T* __restrict__ s_val, T* __restrict__ s_x,
                                                 double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * 256) {
    const int64_t id = support[e];
    int64_t i, j;
    if (small) {   // m n < 2^32: 32-bit division (uniform branch)
      const uint32_t q = (uint32_t)id / (uint32_t)n;
      i = q;
      j = (int64_t)((uint32_t)id - q * (uint32_t)n);
    } else {
      i = id / n;
      j = id % n;
    }
    T l = T(0);
    if constexpr (sizeof(T) == 4 && RP % 4 == 0) {
      // rows of the panels as 16-byte loads (RP * 4 bytes, 16-byte aligned)
      const float4* u4 = reinterpret_cast<const float4*>(UL + i * RP);
      const float4* v4 = reinterpret_cast<const float4*>(VL + j * RP);
#pragma unroll
      for (int c = 0; c < RP / 4; ++c) {
        const float4 a = u4[c], b = v4[c];
        l = fma_t(a.x, b.x, l);
        l = fma_t(a.y, b.y, l);
        l = fma_t(a.z, b.z, l);
        l = fma_t(a.w, b.w, l);
      }
    } else {
#pragma unroll
      for (int c = 0; c < RP; ++c) l = fma_t(UL[i * RP + c], VL[j * RP + c], l);
    }
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

// part[block] = sum of (X - U_L V_L^T)^2 over the block's tiles of 64 rows
// x 256 columns (tile t: row block t % nrb, column block t / nrb).  A thread
// owns one column and keeps its row of V_L in registers; the row of U_L is
// the same for the whole block, so each entry costs RP FMAs and one load.
constexpr int kNormRows = 64;
template <typename T, int RP>
__global__ __launch_bounds__(256) void kc_res_norm(const T* __restrict__ X, int64_t ldx,
                                                   const T* __restrict__ UL,
                                                   const T* __restrict__ VL, int64_t m,
                                                   int64_t n, int64_t nrb, int64_t ntiles,
                                                   double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t i0 = (t % nrb) * kNormRows;
    const int64_t j = (t / nrb) * 256 + threadIdx.x;
    if (j >= n) continue;
    T v[RP];
#pragma unroll
    for (int c = 0; c < RP; ++c) v[c] = VL[j * RP + c];
    const int64_t i1 = (i0 + kNormRows) < m ? (i0 + kNormRows) : m;
    for (int64_t i = i0; i < i1; ++i) {
      const T* u = UL + i * RP;
      T l = T(0);
#pragma unroll
      for (int c = 0; c < RP; ++c) l = fma_t(u[c], v[c], l);
      const double r = (double)(X[i * ldx + j] - l);
      acc = fma(r, r, acc);
    }
  }
  const double tot = block_sum<T>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// The plan of a fixed-support step: nnz, sum_sel2 = sum of the gather
// partials, sum_r2 = sum of the norm partials (strided per thread, then a
// tree in LDS: a fixed order).
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
  plan->sum_r2 = rb[0];
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
  const unsigned gs = blocks_of(nnz);
  const bool small = m * n <= (int64_t)0xffffffffLL;
  const int64_t nrb = (m + kNormRows - 1) / kNormRows;
  const int64_t ntiles = nrb * ((n + 255) / 256);
  const unsigned ga = (unsigned)(ntiles < kNormBlocks ? ntiles : kNormBlocks);
  double* psel = scratch;
  double* pall = scratch + kCompBlocks;
  GC_RP_SWITCH(rp, {
    if (f64) {
      hipLaunchKernelGGL((kc_gather<double, RP>), dim3(gs), dim3(256), 0, L.stream,
                         (const double*)X, ldx, (const double*)UL, (const double*)VL, n, small,
                         support, nnz, s_idx, (double*)s_val, (double*)s_x, psel);
      hipLaunchKernelGGL((kc_res_norm<double, RP>), dim3(ga), dim3(256), 0, L.stream,
                         (const double*)X, ldx, (const double*)UL, (const double*)VL, m, n,
                         nrb, ntiles, pall);
    } else {
      hipLaunchKernelGGL((kc_gather<float, RP>), dim3(gs), dim3(256), 0, L.stream,
                         (const float*)X, ldx, (const float*)UL, (const float*)VL, n, small,
                         support, nnz, s_idx, (float*)s_val, (float*)s_x, psel);
      hipLaunchKernelGGL((kc_res_norm<float, RP>), dim3(ga), dim3(256), 0, L.stream,
                         (const float*)X, ldx, (const float*)UL, (const float*)VL, m, n, nrb,
                         ntiles, pall);
    }
  });
  hipLaunchKernelGGL(kc_finish, dim3(1), dim3(256), 0, L.stream, psel, (int)gs, pall, (int)ga,
                     nnz, plan);
}

int64_t fixed_support_scratch_doubles() { return (int64_t)kCompBlocks + kNormBlocks; }

}  // namespace godec
