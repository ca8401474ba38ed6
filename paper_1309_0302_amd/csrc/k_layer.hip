// Kernels of the differentiable GoDec layer (backward pass).
//
// With the supports M_t of the forward frozen, each unrolled iteration is
//   D_t = X - S_{t-1},  L_t = f(D_t),  S_t = M_t * (X - L_t),
// and f, the power-scheme BRP update of Algorithm 1 (Sec. 3.1.3, Eq. 6-9),
// equals exactly
//   f(D) = D A^q Q C^a Q^T,   A = D^T D,  Q = orth(A^p A1),  C = Q^T A^p Q,
//   p = 2q + 1,  a = -(p - 1) / (2p)
// (the range of Q is that of Y2; B = D A^q Q is L~ Q2; C^a = (B^T B)^a gives
// the (2q+1)-th root of the core).  Its adjoint is assembled from thin panel
// products (the batched GEMM below) and r x r FP64 algebra (one thread per
// problem): the eigen-function derivative of C^a (Daleckii-Krein), the
// derivative of an orthonormalised range, and the power-chain terms, each of
// rank r.
#include "godec_internal.h"
#include "k_common.h"

#include <algorithm>
#include <type_traits>

namespace godec {

// ---------------------------------------------------------------------------
// Batched GEMM with optional split over K:
//   C[b] = alpha * op(A[b]) op(B[b]) + beta * C[b],  op(A) M x K, op(B) K x N,
// row-major storage; ta: A is stored K x M (op(A) = A^T); tb: B is stored
// N x K.  With nsplit > 1 the K range is cut into nsplit chunks whose
// products go to part[b][s] and are added in order by kl_gemm_reduce.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void kl_gemm(int M, int N, int K, const T* __restrict__ A,
                                               int64_t lda, int64_t sA, int ta,
                                               const T* __restrict__ B, int64_t ldb,
                                               int64_t sB, int tb, T alpha, T beta,
                                               T* __restrict__ C, int64_t ldc, int64_t sC,
                                               int nsplit, T* __restrict__ part) {
  __shared__ T As[16][17];
  __shared__ T Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int b = blockIdx.z / nsplit, s = blockIdx.z % nsplit;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  const int kc = (K + nsplit - 1) / nsplit;
  const int kb = s * kc;
  const int ke = (kb + kc) < K ? (kb + kc) : K;
  const T* Ab = A + (int64_t)b * sA;
  const T* Bb = B + (int64_t)b * sB;
  T acc = T(0);
  for (int k0 = kb; k0 < ke; k0 += 16) {
    if (!ta) {
      const int i = i0 + ty, k = k0 + tx;
      As[ty][tx] = (i < M && k < ke) ? Ab[(int64_t)i * lda + k] : T(0);
    } else {
      const int i = i0 + tx, k = k0 + ty;
      As[tx][ty] = (i < M && k < ke) ? Ab[(int64_t)k * lda + i] : T(0);
    }
    if (!tb) {
      const int k = k0 + ty, j = j0 + tx;
      Bs[ty][tx] = (k < ke && j < N) ? Bb[(int64_t)k * ldb + j] : T(0);
    } else {
      const int k = k0 + tx, j = j0 + ty;
      Bs[tx][ty] = (k < ke && j < N) ? Bb[(int64_t)j * ldb + k] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) acc += As[ty][kk] * Bs[kk][tx];
    __syncthreads();
  }
  const int i = i0 + ty, j = j0 + tx;
  if (i >= M || j >= N) return;
  if (nsplit > 1) {
    part[(((int64_t)b * nsplit + s) * M + i) * N + j] = acc;
  } else {
    T* Cb = C + (int64_t)b * sC;
    const T old = beta != T(0) ? Cb[(int64_t)i * ldc + j] : T(0);
    Cb[(int64_t)i * ldc + j] = alpha * acc + beta * old;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void kl_gemm_reduce(int M, int N, int nsplit,
                                                      const T* __restrict__ part, T alpha,
                                                      T beta, T* __restrict__ C, int64_t ldc,
                                                      int64_t sC) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  T acc = T(0);
  for (int s = 0; s < nsplit; ++s) acc += part[((int64_t)b * nsplit + s) * M * N + e];
  T* Cb = C + (int64_t)b * sC;
  const T old = beta != T(0) ? Cb[(int64_t)i * ldc + j] : T(0);
  Cb[(int64_t)i * ldc + j] = alpha * acc + beta * old;
}

// ---------------------------------------------------------------------------
// Elementwise and sparse helpers (one problem per blockIdx.y).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void kl_fill(T* __restrict__ P, int64_t count, int64_t stride,
                                               T v) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) P[(int64_t)blockIdx.y * stride + e] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void kl_copy(const T* __restrict__ S, T* __restrict__ D,
                                               int64_t count, int64_t stride) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) D[(int64_t)blockIdx.y * stride + e] = S[(int64_t)blockIdx.y * stride + e];
}

// P[idx[e]] = v[e]  (mode 0),  P[idx[e]] += s * v[e]  (mode 1)  over the list
// of problem b (idx/v with batch stride kstride, counts nnz[b]).
template <typename T>
__global__ __launch_bounds__(256) void kl_scatter(T* __restrict__ P, int64_t stride,
                                                  const int64_t* __restrict__ idx,
                                                  const T* __restrict__ v, int64_t kstride,
                                                  const int64_t* __restrict__ nnz, int mode,
                                                  T s) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nnz[b]) return;
  const int64_t at = idx[(int64_t)b * kstride + e];
  const T x = v[(int64_t)b * kstride + e];
  if (mode == 0) P[(int64_t)b * stride + at] = x;
  else P[(int64_t)b * stride + at] += s * x;
}

// out[e] = G[idx[e]] (gather from a dense matrix)
template <typename T>
__global__ __launch_bounds__(256) void kl_gather(const T* __restrict__ G, int64_t stride,
                                                 const int64_t* __restrict__ idx,
                                                 int64_t kstride,
                                                 const int64_t* __restrict__ nnz,
                                                 T* __restrict__ out) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nnz[b]) return;
  out[(int64_t)b * kstride + e] = G[(int64_t)b * stride + idx[(int64_t)b * kstride + e]];
}

// Low-rank update split by a support (one block: RB rows x 256 columns).
//   P = U V^T  (U m x w, V n x w, both with row stride w)
//   X += P off the support,  Lbar = P on the support and 0 off it;
// without a bitmap: X += P everywhere, or X = P when accumulate is 0 (Lbar
// untouched).  Entry (i, j) of the
// support is bit i n + j of the problem's bitmap.  Chunks of CW columns of w
// pass through LDS: V's rows for the block's columns (one per thread, odd
// row stride) and U's rows for the block's rows, transposed so that a thread
// reads four of its RB row values per broadcast.  Each thread owns one column
// and keeps RB sums, added in the order of w.
template <typename T, int RB>
__global__ __launch_bounds__(256) void kl_uvt_update(int m, int n, int w,
                                                     const T* __restrict__ U, int64_t sU,
                                                     const T* __restrict__ V, int64_t sV,
                                                     T* __restrict__ X, int64_t ldx, int64_t sX,
                                                     int accumulate,
                                                     const uint32_t* __restrict__ bits,
                                                     int64_t wstride, T* __restrict__ Lbar,
                                                     int64_t sL) {
  constexpr int CW = sizeof(T) == 8 ? 16 : 32;
  __shared__ T vs[256][CW + 1];
  __shared__ __align__(16) T ut[CW][RB];
  const int b = blockIdx.z, tid = threadIdx.x;
  const int j0 = blockIdx.x * 256, i0 = blockIdx.y * RB;
  const T* Ub = U + (int64_t)b * sU;
  const T* Vb = V + (int64_t)b * sV;
  T acc[RB];
#pragma unroll
  for (int ii = 0; ii < RB; ++ii) acc[ii] = T(0);
  for (int c0 = 0; c0 < w; c0 += CW) {
    const int cw = (w - c0) < CW ? (w - c0) : CW;
    __syncthreads();
#pragma unroll 4
    for (int e = tid; e < 256 * CW; e += 256) {
      const int jj = e / CW, cc = e % CW;
      vs[jj][cc] = (cc < cw && j0 + jj < n) ? Vb[(int64_t)(j0 + jj) * w + c0 + cc] : T(0);
    }
    for (int e = tid; e < RB * CW; e += 256) {
      const int ii = e / CW, cc = e % CW;
      ut[cc][ii] = (cc < cw && i0 + ii < m) ? Ub[(int64_t)(i0 + ii) * w + c0 + cc] : T(0);
    }
    __syncthreads();
    for (int cc = 0; cc < cw; ++cc) {
      const T v = vs[tid][cc];
#pragma unroll
      for (int ii = 0; ii < RB; ++ii) acc[ii] += ut[cc][ii] * v;
    }
  }
  const int j = j0 + tid;
  if (j >= n) return;
  T* Xb = X + (int64_t)b * sX;
#pragma unroll
  for (int ii = 0; ii < RB; ++ii) {
    const int i = i0 + ii;
    if (i < m) {
      T* x = Xb + (int64_t)i * ldx + j;
      if (bits) {
        const int64_t e = (int64_t)i * n + j;
        const bool on = (bits[(int64_t)b * wstride + (e >> 5)] >> (unsigned)(e & 31)) & 1u;
        if (!on) *x += acc[ii];
        Lbar[(int64_t)b * sL + e] = on ? acc[ii] : T(0);
      } else {
        *x = accumulate ? *x + acc[ii] : acc[ii];
      }
    }
  }
}

// FP32 form of kl_uvt_update on the matrix cores: a block covers 64 rows x
// 128 columns, each wave one 16-row tile against the 8 column tiles, with
// v_mfma_f32_16x16x4f32 over chunks of 32 columns of w.  In k-step s of a
// chunk, lane l (row or column l%16, g = l/16) supplies column 8g + s of the
// chunk, so that each lane reads eight consecutive values of its U or V row
// (two 16-byte loads when VEC: w a multiple of four).  Lane l receives the
// product at column l%16 and rows 4g + v, v < 4, of its tile.
typedef float kl_f32x4 __attribute__((ext_vector_type(4)));

template <bool VEC>
__device__ __forceinline__ void uvt_row8(const float* __restrict__ row, bool ok, int c, int w,
                                         float (&v)[8]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) v[s] = 0.f;
  if (!ok) return;
  if (VEC) {
    if (c + 8 <= w) {
      const float4 x = *reinterpret_cast<const float4*>(row + c);
      const float4 y = *reinterpret_cast<const float4*>(row + c + 4);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
      v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
    } else if (c + 4 <= w) {
      const float4 x = *reinterpret_cast<const float4*>(row + c);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
  } else {
#pragma unroll
    for (int s = 0; s < 8; ++s)
      if (c + s < w) v[s] = row[c + s];
  }
}

constexpr int kUvtTiles = 8;   // 16-column tiles per wave (a block: 64 rows x 128 columns)

template <bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void kl_uvt_mfma(
    int m, int n, int w,
                                                   const float* __restrict__ U, int64_t sU,
                                                   const float* __restrict__ V, int64_t sV,
                                                   float* __restrict__ X, int64_t ldx,
                                                   int64_t sX, int accumulate,
                                                   const uint32_t* __restrict__ bits,
                                                   int64_t wstride, float* __restrict__ Lbar,
                                                   int64_t sL) {
  constexpr int NT = kUvtTiles;
  const int b = blockIdx.z, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, g = lane >> 4;
  const int r0 = blockIdx.y * 64 + wave * 16;
  const int j0 = blockIdx.x * (16 * NT);
  const float* Ub = U + (int64_t)b * sU;
  const float* Vb = V + (int64_t)b * sV;
  float* Xb = X + (int64_t)b * sX;
  const uint32_t* Bb = bits ? bits + (int64_t)b * wstride : nullptr;
  // Epilogue operands in batches of EB tiles; each next batch's loads are
  // issued before the current batch's stores (so that waiting for loads never
  // waits for stores).
  constexpr int EB = 2;
  float xv[2][EB][4];
  uint32_t wv[2][EB][4];
  auto load_batch = [&](int t0, float (&xs)[EB][4], uint32_t (&ws)[EB][4]) {
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int j = j0 + 16 * (t0 + u) + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = r0 + 4 * g + v;
        const bool ok = i < m && j < n;
        const int64_t e = (int64_t)i * n + j;
        xs[u][v] = (ok && (accumulate || Bb)) ? Xb[(int64_t)i * ldx + j] : 0.f;
        ws[u][v] = (ok && Bb) ? Bb[e >> 5] : 0u;
      }
    }
  };
  kl_f32x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = kl_f32x4{0.f, 0.f, 0.f, 0.f};
  const int urow = r0 + li;
  for (int c0 = 0; c0 < w; c0 += 32) {
    const int ks = (w - c0) < 8 ? (w - c0) : 8;  // k-steps with a valid column
    float a[8];
    uvt_row8<VEC>(Ub + (int64_t)urow * w, urow < m, c0 + 8 * g, w, a);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int vrow = j0 + 16 * t + li;
      float bv[8];
      uvt_row8<VEC>(Vb + (int64_t)vrow * w, vrow < n, c0 + 8 * g, w, bv);
#pragma unroll
      for (int s = 0; s < 8; ++s)
        if (s < ks) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bv[s], acc[t], 0, 0, 0);
    }
  }
  load_batch(0, xv[0], wv[0]);
#pragma unroll
  for (int k = 0; k < NT / EB; ++k) {
    if (k + 1 < NT / EB) load_batch(EB * (k + 1), xv[(k + 1) & 1], wv[(k + 1) & 1]);
#pragma unroll
    for (int u = 0; u < EB; ++u) {
      const int t = EB * k + u;
      const int j = j0 + 16 * t + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = r0 + 4 * g + v;
        if (i < m && j < n) {
          float* x = Xb + (int64_t)i * ldx + j;
          const float val = acc[t][v];
          const float old = xv[k & 1][u][v];
          if (Bb) {
            const int64_t e = (int64_t)i * n + j;
            const bool on = (wv[k & 1][u][v] >> (unsigned)(e & 31)) & 1u;
            if (!on) *x = old + val;
            Lbar[(int64_t)b * sL + e] = on ? val : 0.f;
          } else {
            *x = accumulate ? old + val : val;
          }
        }
      }
    }
  }
}

// D = X (count entries per problem; 16-byte vectors when vec is set) and,
// when bits is given, zero the problem's bitmap words.
template <typename T>
__global__ __launch_bounds__(256) void kl_rebuild_d(const T* __restrict__ X, T* __restrict__ D,
                                                    int64_t count, int vec,
                                                    uint32_t* __restrict__ bits, int64_t words) {
  constexpr int VW = 16 / sizeof(T);
  using V4 = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (bits && e < words) bits[(int64_t)b * words + e] = 0u;
  if (vec) {
    if (e < count / VW)
      reinterpret_cast<V4*>(D + (int64_t)b * count)[e] =
          reinterpret_cast<const V4*>(X + (int64_t)b * count)[e];
  } else if (e < count) {
    D[(int64_t)b * count + e] = X[(int64_t)b * count + e];
  }
}

// D[idx[e]] -= v[e] over the list of problem b and set the entry's bit.
template <typename T>
__global__ __launch_bounds__(256) void kl_sub_mark(T* __restrict__ D, int64_t stride,
                                                   const int64_t* __restrict__ idx,
                                                   const T* __restrict__ v, int64_t kstride,
                                                   const int64_t* __restrict__ nnz,
                                                   uint32_t* __restrict__ bits, int64_t words) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nnz[b]) return;
  const int64_t at = idx[(int64_t)b * kstride + e];
  D[(int64_t)b * stride + at] -= v[(int64_t)b * kstride + e];
  atomicOr(&bits[(int64_t)b * words + (at >> 5)], 1u << (unsigned)(at & 31));
}

// Copy panel P0 (rows x r, ld r) into columns [c0, c0 + r) of a rows x w
// panel, and P1 (when given) into columns [c0 + r, c0 + 2r).
template <typename T>
__global__ __launch_bounds__(256) void kl_put_cols(const T* __restrict__ P0,
                                                   const T* __restrict__ P1, int64_t sP, int r,
                                                   T* __restrict__ O, int64_t sO, int w, int c0,
                                                   int64_t rows) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * r) return;
  const int64_t i = e / r;
  const int c = (int)(e % r);
  T* o = O + (int64_t)b * sO + i * w + c0 + c;
  o[0] = P0[(int64_t)b * sP + e];
  if (P1) o[r] = P1[(int64_t)b * sP + e];
}


// ---------------------------------------------------------------------------
// Tall-skinny products (the panel passes of the backward).
//
// kl_ts_nn: C[b] = alpha A[b] B[b] + beta C[b] with A M x K (row-major, one
// thread per row) and B K x NC (NC <= 8, K <= kTsMaxK, row stride ldb) staged
// in LDS; column j of the product uses column (j + rot) mod NC of B.
// kl_ts_tn: the K-chunk partials of A[b]^T B[b] with A stored K x M (one
// thread per column of A, rows of the chunk read coalesced) and B K x NC;
// kl_ts_reduce adds the chunks in order.
// ---------------------------------------------------------------------------
constexpr int kTsMaxK = 512;
constexpr int kTsChunk = 256;

template <typename T, int NC>
__global__ __launch_bounds__(256) void kl_ts_nn(int M, int K, const T* __restrict__ A,
                                                int64_t lda, int64_t sA, const T* __restrict__ B,
                                                int64_t ldb, int64_t sB, int rot, T alpha,
                                                T beta, T* __restrict__ C, int64_t ldc,
                                                int64_t sC) {
  __shared__ T bs[kTsMaxK * NC];
  const int b = blockIdx.y, tid = threadIdx.x;
  const T* Bb = B + (int64_t)b * sB;
  for (int e = tid; e < K * NC; e += 256) {
    const int k = e / NC, j = e % NC;
    bs[e] = Bb[(int64_t)k * ldb + (j + rot) % NC];
  }
  __syncthreads();
  const int i = blockIdx.x * 256 + tid;
  if (i >= M) return;
  const T* a = A + (int64_t)b * sA + (int64_t)i * lda;
  T acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = T(0);
  for (int k = 0; k < K; ++k) {
    const T x = a[k];
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j] += x * bs[k * NC + j];
  }
  T* c = C + (int64_t)b * sC + (int64_t)i * ldc;
#pragma unroll
  for (int j = 0; j < NC; ++j) c[j] = alpha * acc[j] + (beta != T(0) ? beta * c[j] : T(0));
}

template <typename T, int NC>
__global__ __launch_bounds__(256) void kl_ts_tn(int M, int K, int chunk, const T* __restrict__ A,
                                                int64_t lda, int64_t sA, const T* __restrict__ B,
                                                int64_t sB, T* __restrict__ part) {
  __shared__ T bs[kTsChunk * NC];
  const int b = blockIdx.z, ch = blockIdx.y, tid = threadIdx.x;
  const int k0 = ch * chunk;
  const int kn = (K - k0) < chunk ? (K - k0) : chunk;
  const T* Bb = B + (int64_t)b * sB + (int64_t)k0 * NC;
  for (int e = tid; e < kn * NC; e += 256) bs[e] = Bb[e];
  __syncthreads();
  const int c = blockIdx.x * 256 + tid;
  if (c >= M) return;
  const T* a = A + (int64_t)b * sA + (int64_t)k0 * lda + c;
  T acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = T(0);
  for (int k = 0; k < kn; ++k) {
    const T x = a[(int64_t)k * lda];
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j] += x * bs[k * NC + j];
  }
  T* o = part + (((int64_t)b * gridDim.y + ch) * M + c) * NC;
#pragma unroll
  for (int j = 0; j < NC; ++j) o[j] = acc[j];
}

template <typename T>
__global__ __launch_bounds__(256) void kl_ts_reduce(int M, int NC, int nch,
                                                    const T* __restrict__ part, T alpha, T beta,
                                                    T* __restrict__ C, int64_t ldc, int64_t sC) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * NC) return;
  T s = T(0);
  const T* pe = part + (int64_t)b * nch * M * NC + e;
  const int64_t st = (int64_t)M * NC;
  int ch = 0;
  for (; ch + 8 <= nch; ch += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = pe[(ch + u) * st];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; ch < nch; ++ch) s += pe[ch * st];
  const int64_t i = e / NC, j = e % NC;
  T* c = C + (int64_t)b * sC + i * ldc + j;
  *c = alpha * s + (beta != T(0) ? beta * *c : T(0));
}

// kl_inner: C[b] = alpha P[b]^T P2[b] for two NC-column panels of `rows` rows
// (ld NC), one block per chunk of kInnerRows rows; each thread sums its rows,
// the wave sums go through fixed-order lane exchanges, then the four waves
// add in order.  With one chunk the block writes C; otherwise it writes its
// chunk's partial for kl_ts_reduce.
constexpr int kInnerRows = 4096;

template <typename T, int NC>
__global__ __launch_bounds__(256) void kl_inner(int rows, const T* __restrict__ P,
                                                int64_t sP, const T* __restrict__ P2,
                                                int64_t sP2, T alpha, T beta,
                                                T* __restrict__ C, int64_t ldc, int64_t sC,
                                                T* __restrict__ part) {
  __shared__ T red[4][NC * NC];
  const int b = blockIdx.y, ch = blockIdx.x, tid = threadIdx.x;
  const int r0 = ch * kInnerRows;
  const int r1 = (rows - r0) < kInnerRows ? rows : r0 + kInnerRows;
  const T* pb = P + (int64_t)b * sP;
  const T* qb = P2 + (int64_t)b * sP2;
  T acc[NC][NC];
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[i][j] = T(0);
  for (int row = r0 + tid; row < r1; row += 256) {
    T x[NC], y[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      x[i] = pb[(int64_t)row * NC + i];
      y[i] = qb[(int64_t)row * NC + i];
    }
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
      for (int j = 0; j < NC; ++j) acc[i][j] += x[i] * y[j];
  }
#pragma unroll
  for (int i = 0; i < NC; ++i)
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      T v = acc[i][j];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      acc[i][j] = v;
    }
  const int wave = tid >> 6, lane = tid & 63;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
      for (int j = 0; j < NC; ++j) red[wave][i * NC + j] = acc[i][j];
  }
  __syncthreads();
  if (tid >= NC * NC) return;
  const T s = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
  if (gridDim.x == 1) {
    T* c = C + (int64_t)b * sC + (tid / NC) * ldc + tid % NC;
    *c = alpha * s + (beta != T(0) ? beta * *c : T(0));
  } else {
    part[((int64_t)b * gridDim.x + ch) * NC * NC + tid] = s;
  }
}

#define GODEC_NC_SWITCH(nc, ...)                              \
  switch (nc) {                                               \
    case 1: { constexpr int NC = 1; __VA_ARGS__; } break;     \
    case 2: { constexpr int NC = 2; __VA_ARGS__; } break;     \
    case 3: { constexpr int NC = 3; __VA_ARGS__; } break;     \
    case 4: { constexpr int NC = 4; __VA_ARGS__; } break;     \
    case 5: { constexpr int NC = 5; __VA_ARGS__; } break;     \
    case 6: { constexpr int NC = 6; __VA_ARGS__; } break;     \
    case 7: { constexpr int NC = 7; __VA_ARGS__; } break;     \
    case 8: { constexpr int NC = 8; __VA_ARGS__; } break;     \
    default: break;                                           \
  }

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
template <typename T>
void lk_gemm_t(const Launch& L, int nb, int M, int N, int K, const T* A, int64_t lda,
               int64_t sA, int ta, const T* B, int64_t ldb, int64_t sB, int tb, T alpha, T beta,
               T* C, int64_t ldc, int64_t sC, T* part, int64_t part_cap) {
  // r x r inner products of two panels
  if (ta && !tb && M <= 8 && N == M && lda == M && ldb == N) {
    const int nch = (K + kInnerRows - 1) / kInnerRows;
    if (nch == 1 || (int64_t)nb * nch * M * N <= part_cap) {
      const dim3 grid((unsigned)std::max(nch, 1), (unsigned)nb);
      GODEC_NC_SWITCH(N, hipLaunchKernelGGL((kl_inner<T, NC>), grid, dim3(256), 0, L.stream, K,
                                            A, sA, B, sB, alpha, beta, C, ldc, sC, part));
      if (nch > 1) {
        const dim3 g2((unsigned)((M * N + 255) / 256), (unsigned)nb);
        hipLaunchKernelGGL(kl_ts_reduce<T>, g2, dim3(256), 0, L.stream, M, N, nch,
                           (const T*)part, alpha, beta, C, ldc, sC);
      }
      return;
    }
  }
  // tall-skinny cases: a long panel times a small N-column one
  if (!ta && !tb && N <= 8 && K <= kTsMaxK && ldb == N && M >= 256) {
    const dim3 grid((unsigned)((M + 255) / 256), (unsigned)nb);
    GODEC_NC_SWITCH(N, hipLaunchKernelGGL((kl_ts_nn<T, NC>), grid, dim3(256), 0, L.stream, M, K,
                                          A, lda, sA, B, ldb, sB, 0, alpha, beta, C, ldc, sC));
    return;
  }
  // K chunks of kTsChunk rows, halved (down to 32) while the launch has
  // fewer than four blocks per compute unit and the partials fit
  int chunk = kTsChunk;
  const int64_t mb = (M + 255) / 256;
  auto nch_of = [&](int c) { return (K + c - 1) / c; };
  while (chunk > 32 && nb * mb * nch_of(chunk) < 4 * (int64_t)L.num_cu &&
         (int64_t)nb * nch_of(chunk / 2) * M * N <= part_cap)
    chunk /= 2;
  const int nch_ts = nch_of(chunk);
  if (ta && !tb && N <= 8 && ldb == N && M >= 64 && (int64_t)nb * nch_ts * M * N <= part_cap) {
    const dim3 grid((unsigned)mb, (unsigned)nch_ts, (unsigned)nb);
    GODEC_NC_SWITCH(N, hipLaunchKernelGGL((kl_ts_tn<T, NC>), grid, dim3(256), 0, L.stream, M, K,
                                          chunk, A, lda, sA, B, sB, part));
    const dim3 g2((unsigned)(((int64_t)M * N + 255) / 256), (unsigned)nb);
    hipLaunchKernelGGL(kl_ts_reduce<T>, g2, dim3(256), 0, L.stream, M, N, nch_ts, (const T*)part,
                       alpha, beta, C, ldc, sC);
    return;
  }
  const int tiles = ((M + 15) / 16) * ((N + 15) / 16) * nb;
  int nsplit = 1;
  if (tiles < 1024 && K > 512) {
    nsplit = std::min(64, (K + 511) / 512);
    while (nsplit > 1 && (int64_t)nb * nsplit * M * N > part_cap) --nsplit;
  }
  dim3 grid((unsigned)((N + 15) / 16), (unsigned)((M + 15) / 16), (unsigned)(nb * nsplit));
  hipLaunchKernelGGL(kl_gemm<T>, grid, dim3(256), 0, L.stream, M, N, K, A, lda, sA, ta, B, ldb,
                     sB, tb, alpha, beta, C, ldc, sC, nsplit, part);
  if (nsplit > 1) {
    dim3 g2((unsigned)(((int64_t)M * N + 255) / 256), (unsigned)nb);
    hipLaunchKernelGGL(kl_gemm_reduce<T>, g2, dim3(256), 0, L.stream, M, N, nsplit,
                       (const T*)part, alpha, beta, C, ldc, sC);
  }
}

void lk_gemm(const Launch& L, bool f64, int nb, int M, int N, int K, const void* A, int64_t lda,
             int64_t sA, int ta, const void* B, int64_t ldb, int64_t sB, int tb, double alpha,
             double beta, void* C, int64_t ldc, int64_t sC, void* part, int64_t part_cap) {
  if (f64)
    lk_gemm_t<double>(L, nb, M, N, K, (const double*)A, lda, sA, ta, (const double*)B, ldb, sB,
                      tb, alpha, beta, (double*)C, ldc, sC, (double*)part, part_cap);
  else
    lk_gemm_t<float>(L, nb, M, N, K, (const float*)A, lda, sA, ta, (const float*)B, ldb, sB, tb,
                     (float)alpha, (float)beta, (float*)C, ldc, sC, (float*)part, part_cap);
}

static dim3 g1(int64_t count, int nb) { return dim3((unsigned)((count + 255) / 256), (unsigned)nb); }

void lk_fill(const Launch& L, bool f64, int nb, void* P, int64_t count, int64_t stride, double v) {
  if (f64) hipLaunchKernelGGL(kl_fill<double>, g1(count, nb), dim3(256), 0, L.stream, (double*)P, count, stride, v);
  else hipLaunchKernelGGL(kl_fill<float>, g1(count, nb), dim3(256), 0, L.stream, (float*)P, count, stride, (float)v);
}

void lk_copy(const Launch& L, bool f64, int nb, const void* S, void* D, int64_t count, int64_t stride) {
  if (f64) hipLaunchKernelGGL(kl_copy<double>, g1(count, nb), dim3(256), 0, L.stream, (const double*)S, (double*)D, count, stride);
  else hipLaunchKernelGGL(kl_copy<float>, g1(count, nb), dim3(256), 0, L.stream, (const float*)S, (float*)D, count, stride);
}

void lk_scatter(const Launch& L, bool f64, int nb, void* P, int64_t stride, const int64_t* idx,
                const void* v, int64_t kstride, int64_t kmax, const int64_t* nnz, int mode,
                double s) {
  if (f64)
    hipLaunchKernelGGL(kl_scatter<double>, g1(kmax, nb), dim3(256), 0, L.stream, (double*)P, stride, idx,
                       (const double*)v, kstride, nnz, mode, s);
  else
    hipLaunchKernelGGL(kl_scatter<float>, g1(kmax, nb), dim3(256), 0, L.stream, (float*)P, stride, idx,
                       (const float*)v, kstride, nnz, mode, (float)s);
}

void lk_gather(const Launch& L, bool f64, int nb, const void* G, int64_t stride, const int64_t* idx,
               int64_t kstride, int64_t kmax, const int64_t* nnz, void* out) {
  if (f64)
    hipLaunchKernelGGL(kl_gather<double>, g1(kmax, nb), dim3(256), 0, L.stream, (const double*)G, stride,
                       idx, kstride, nnz, (double*)out);
  else
    hipLaunchKernelGGL(kl_gather<float>, g1(kmax, nb), dim3(256), 0, L.stream, (const float*)G, stride,
                       idx, kstride, nnz, (float*)out);
}

void lk_rebuild_d(const Launch& L, bool f64, int nb, const void* X, void* D, int64_t count,
                  uint32_t* bits, int64_t words) {
  const int64_t vw = f64 ? 2 : 4;
  const bool vec = count % vw == 0 && (uintptr_t)X % 16 == 0 && (uintptr_t)D % 16 == 0;
  const int64_t th = std::max<int64_t>(vec ? count / vw : count, bits ? words : 0);
  if (f64)
    hipLaunchKernelGGL(kl_rebuild_d<double>, g1(th, nb), dim3(256), 0, L.stream,
                       (const double*)X, (double*)D, count, (int)vec, bits, words);
  else
    hipLaunchKernelGGL(kl_rebuild_d<float>, g1(th, nb), dim3(256), 0, L.stream, (const float*)X,
                       (float*)D, count, (int)vec, bits, words);
}

void lk_sub_mark(const Launch& L, bool f64, int nb, void* D, int64_t stride, const int64_t* idx,
                 const void* v, int64_t kstride, int64_t kmax, const int64_t* nnz,
                 uint32_t* bits, int64_t words) {
  if (f64)
    hipLaunchKernelGGL(kl_sub_mark<double>, g1(kmax, nb), dim3(256), 0, L.stream, (double*)D,
                       stride, idx, (const double*)v, kstride, nnz, bits, words);
  else
    hipLaunchKernelGGL(kl_sub_mark<float>, g1(kmax, nb), dim3(256), 0, L.stream, (float*)D,
                       stride, idx, (const float*)v, kstride, nnz, bits, words);
}

bool lk_dmul_rot(const Launch& L, bool f64, int nb, int M, int N, int K, const void* A,
                 int64_t lda, int64_t sA, const void* B, int64_t ldb, int64_t sB, int rot,
                 void* C, int64_t ldc, int64_t sC) {
  if (N > 8 || K > kTsMaxK || M < 256) return false;
  const dim3 grid((unsigned)((M + 255) / 256), (unsigned)nb);
  if (f64) {
    GODEC_NC_SWITCH(N, hipLaunchKernelGGL((kl_ts_nn<double, NC>), grid, dim3(256), 0, L.stream,
                                          M, K, (const double*)A, lda, sA, (const double*)B, ldb,
                                          sB, rot, 1.0, 0.0, (double*)C, ldc, sC));
  } else {
    GODEC_NC_SWITCH(N, hipLaunchKernelGGL((kl_ts_nn<float, NC>), grid, dim3(256), 0, L.stream, M,
                                          K, (const float*)A, lda, sA, (const float*)B, ldb, sB,
                                          rot, 1.0f, 0.0f, (float*)C, ldc, sC));
  }
  return true;
}

void lk_uvt_update(const Launch& L, bool f64, int nb, int m, int n, int w, const void* U,
                   int64_t sU, const void* V, int64_t sV, void* X, int64_t ldx, int64_t sX,
                   int accumulate, const uint32_t* bits, int64_t wstride, void* Lbar,
                   int64_t sL) {
  constexpr int RB = 32;
  if (f64) {
    const dim3 grid((unsigned)((n + 255) / 256), (unsigned)((m + RB - 1) / RB), (unsigned)nb);
    hipLaunchKernelGGL((kl_uvt_update<double, RB>), grid, dim3(256), 0, L.stream, m, n, w,
                       (const double*)U, sU, (const double*)V, sV, (double*)X, ldx, sX,
                       accumulate, bits, wstride, (double*)Lbar, sL);
    return;
  }
  const dim3 grid((unsigned)((n + 16 * kUvtTiles - 1) / (16 * kUvtTiles)),
                  (unsigned)((m + 63) / 64), (unsigned)nb);
  const bool vec = w % 4 == 0 && (uintptr_t)U % 16 == 0 && (uintptr_t)V % 16 == 0 &&
                   sU % 4 == 0 && sV % 4 == 0;
  if (vec)
    hipLaunchKernelGGL(kl_uvt_mfma<true>, grid, dim3(256), 0, L.stream, m, n, w, (const float*)U,
                       sU, (const float*)V, sV, (float*)X, ldx, sX, accumulate, bits, wstride,
                       (float*)Lbar, sL);
  else
    hipLaunchKernelGGL(kl_uvt_mfma<false>, grid, dim3(256), 0, L.stream, m, n, w,
                       (const float*)U, sU, (const float*)V, sV, (float*)X, ldx, sX,
                       accumulate, bits, wstride, (float*)Lbar, sL);
}

void lk_put_cols(const Launch& L, bool f64, int nb, const void* P0, const void* P1, int64_t sP,
                 int r, void* O, int64_t sO, int w, int c0, int64_t rows) {
  if (f64)
    hipLaunchKernelGGL(kl_put_cols<double>, g1(rows * r, nb), dim3(256), 0, L.stream,
                       (const double*)P0, (const double*)P1, sP, r, (double*)O, sO, w, c0, rows);
  else
    hipLaunchKernelGGL(kl_put_cols<float>, g1(rows * r, nb), dim3(256), 0, L.stream,
                       (const float*)P0, (const float*)P1, sP, r, (float*)O, sO, w, c0, rows);
}

}  // namespace godec
