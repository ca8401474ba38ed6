// MSE training (Sec. 4.2.1, Algorithm 4): kernels of one label update and
// of the sparse step's bookkeeping.
//
// The state is E = X - sum_j L^j - S (n x p, row-major, leading dimension
// lde, a multiple of 64) and, per label i, L^i_{Omega_i} = U_i V_i^T with U_i
// (n_i x 8, rows in the order of Omega_i) and V_i (p x 8, orthonormal
// columns, zero past the label's rank).  Label i's residual is
// N = E_{Omega_i} + L^i_{Omega_i}: the rows Omega_i of X minus the other
// labels and S.  Before a label's first update L^i is the initial
// Z_{Omega_i} = (D^{-1} X)_{Omega_i} (D = number of labels of each sample),
// taken from X directly.
//
// The label update (q = 0 bilateral random projection with A2 = Y1) is
//   km_gram / km_gram_v  Y2 partials: per block, sum over its rows of
//                  N_row^T (N_row A1) (first update / updated label)
//   km_reduce_orth Y2 = the partials added in a fixed order (FP64), then,
//                  in the last block to finish, two Cholesky QR rounds with
//                  an FP64 Gram: Q = orth(Y2)
//   km_update      U_row = N_row Q, E_row = N_row - U_row Q^T
// so that L^i_{Omega_i} = N Q Q^T = Y1 (A2^T Y1)^{-1} Y2^T.
//
// A wavefront owns one row at a time: lane l holds columns l + 64 s,
// s < S (p <= 64 S); dot products over the row are wavefront sums.
#include "godec_internal.h"
#include "k_common.h"

namespace godec {

constexpr int kMseRP = 8;          // padded rank of every label
constexpr int kMseWaves = 4;       // wavefronts per block of the row passes

// The update pass stores E and U write-through to memory (device scope), so
// that the kernel's end finds no dirty lines to write back (measured faster
// for its full-row stores; the Y2 pass's partials are stored normally,
// where the 16-byte stores the compiler forms pay more).
template <typename T>
__device__ __forceinline__ void store_wt(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float lane_read(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_read(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Register-only lane exchanges (no LDS crossbar, no address operand):
//   swap32 / swap16: the gfx950 lane-half swaps.  For a pair (x, y) with
//     x kept by lanes whose bit 5 (4) is clear and y by the others, x + y
//     of the two returned registers is the kept value plus the partner's
//     (lane l ^ 32, l ^ 16) copy of it.
//   dpp<CTRL>: the value of a partner lane through a DPP move: row_ror:8
//     (lane l ^ 8), row_half_mirror (l ^ 7 within eight lanes), quad_perm
//     swaps (l ^ 2, l ^ 1).
constexpr int kDppRor8 = 0x128;
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppXor2 = 0x4E;
constexpr int kDppXor1 = 0xB1;
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <bool S32>
__device__ __forceinline__ float swap_sum(float x, float y) {
  const auto r = S32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y),
                                                         false, false)
                     : __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y),
                                                         false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
template <bool S32>
__device__ __forceinline__ double swap_sum(double x, double y) {
  const unsigned long long bx = (unsigned long long)__double_as_longlong(x);
  const unsigned long long by = (unsigned long long)__double_as_longlong(y);
  const auto lo = S32 ? __builtin_amdgcn_permlane32_swap((unsigned)bx, (unsigned)by, false, false)
                      : __builtin_amdgcn_permlane16_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi = S32 ? __builtin_amdgcn_permlane32_swap((unsigned)(bx >> 32),
                                                          (unsigned)(by >> 32), false, false)
                      : __builtin_amdgcn_permlane16_swap((unsigned)(bx >> 32),
                                                          (unsigned)(by >> 32), false, false);
  const double a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  const double b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
  return a + b;
}
// One halving step through a DPP partner: the lane keeps index `up ? y : x`
// and adds the partner's copy of it.
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_halve(T x, T y, bool up) {
  return (up ? y : x) + dpp<CTRL>(up ? x : y);
}

// The eight sums over the wavefront's 64 lanes of the per-lane values
// d[0..7], in three parts:
//   wave_halve8: three halving steps (partners whose lane bit 5, 4, 3
//     differs exchange the half of their values that the partner keeps);
//     lane l is left with a partial of index l >> 3 over the eight lanes
//     that share its bits 2..0, a set disjoint from those of the seven
//     other lanes of its group of eight;
//   wave_bfly8: three butterfly steps over the group (pairs l ^ 7, l ^ 2,
//     l ^ 1), after which every lane l holds the sum of index l >> 3;
//   wave_bcast8: every lane reads the eight sums.
// Ten exchanges where eight separate butterflies take 48, all in registers.
// The order of the additions is fixed by the lane indices, so the sums are
// reproducible.
template <typename T>
__device__ __forceinline__ T wave_halve8(const T (&d)[kMseRP]) {
  const int lane = threadIdx.x & 63;
  T a4[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) a4[i] = swap_sum<true>(d[i], d[i + 4]);
  T a2[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) a2[i] = swap_sum<false>(a4[i], a4[i + 2]);
  return dpp_halve<kDppRor8>(a2[0], a2[1], (lane & 8) != 0);
}
template <typename T>
__device__ __forceinline__ T wave_bfly8(T a) {
  a += dpp<kDppHalfMirror>(a);
  a += dpp<kDppXor2>(a);
  a += dpp<kDppXor1>(a);
  return a;
}
template <typename T>
__device__ __forceinline__ void wave_bcast8(T a, T (&d)[kMseRP]) {
  // lane 32 b2 + 16 b1 + 8 b0 holds the sum of index 4 b2 + 2 b1 + b0
#pragma unroll
  for (int t = 0; t < kMseRP; ++t)
    d[t] = lane_read(a, ((t >> 2) << 5) | (((t >> 1) & 1) << 4) | ((t & 1) << 3));
}
template <typename T>
__device__ __forceinline__ void wave_sum8(T (&d)[kMseRP]) {
  wave_bcast8(wave_bfly8(wave_halve8(d)), d);
}

// Rows of a wavefront are processed in groups: the loads of a group are all
// issued before any of its arithmetic, so a wavefront waits for one memory
// round trip per group instead of one per row.  Groups keep the rows in
// their order, so every sum is added in the same order.  The Y2 pass takes
// 8 FP32 (4 FP64) rows per group and the update pass 2 (measured on the
// 65536 x 512 workload: 1.47 ms per iteration against 1.49 with 4 and 1.50
// with 1); a block covers kMseWaves groups.
template <typename T>
struct MseGroup {
  static constexpr int gram = sizeof(T) == 4 ? 8 : 4;
  static constexpr int update = 2;
};

// Partial sums of Y2 = N^T (N A1) over the block's rows (group h of
// wavefront w holds rows j0 + h * stride, j0 = w + 4 blk, stride =
// 4 gridDim.x); written to part[blockIdx.x] as p_pad x 8.  The launcher
// uses it for a label's first update (FIRST, N from X / D); km_gram_v below
// takes the labels updated before.  Each wavefront
// accumulates its rows in order, then the block adds its four wavefronts in
// order.  A1 and V live in LDS, transposed (entry [t][c]), so lane reads
// are consecutive.  The first group's loads are issued before the panels
// are staged.
template <typename T, int S, bool FIRST>
__global__ __launch_bounds__(256) void km_gram(const T* __restrict__ E, int64_t lde,
                                               const T* __restrict__ X, int64_t ldx,
                                               const T* __restrict__ cnt,
                                               const int64_t* __restrict__ rows, int64_t nrows,
                                               int64_t p, const T* __restrict__ U,
                                               const T* __restrict__ V,
                                               const T* __restrict__ A1,
                                               T* __restrict__ part) {
  constexpr int PP = 64 * S;
  constexpr int G = MseGroup<T>::gram;
  // the panels during the row loop, then the four wavefronts' sums
  __shared__ T lds[kMseWaves * PP * kMseRP];
  T* at = lds;                   // A1^T: kMseRP x PP
  T* vt = lds + PP * kMseRP;     // V^T
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t stride = (int64_t)gridDim.x * kMseWaves;
  T e[G][S], xl[FIRST ? G : 1][FIRST ? S : 1], u[FIRST ? 1 : G][kMseRP], c[G];
  auto load_group = [&](int64_t j0) {
#pragma unroll
    for (int h = 0; h < G; ++h) {
      const int64_t j = j0 + h * stride;
      const bool rv = j < nrows;   // wavefront-uniform
      const int64_t g = rv ? rows[j] : 0;
      c[h] = (FIRST && rv) ? cnt[g] : T(0);
      if constexpr (!FIRST) {
#pragma unroll
        for (int t = 0; t < kMseRP; ++t) u[h][t] = rv ? U[j * kMseRP + t] : T(0);
      }
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int64_t col = lane + 64 * s;
        const bool ok = rv && col < p;
        e[h][s] = ok ? E[g * lde + col] : T(0);
        if constexpr (FIRST) xl[h][s] = ok ? X[g * ldx + col] : T(0);
      }
    }
  };
  int64_t j0 = (int64_t)blockIdx.x * kMseWaves + wave;
  if (j0 < nrows) load_group(j0);
  {
    // every panel load in flight at once, then the transposed LDS stores
    constexpr int NST = PP * kMseRP / 256;
    T av[NST], vv[NST];
#pragma unroll
    for (int k = 0; k < NST; ++k) {
      av[k] = A1[k * 256 + threadIdx.x];
      vv[k] = FIRST ? T(0) : V[k * 256 + threadIdx.x];
    }
#pragma unroll
    for (int k = 0; k < NST; ++k) {
      const int q = k * 256 + threadIdx.x;
      const int cc = q / kMseRP, t = q % kMseRP;
      at[t * PP + cc] = av[k];
      vt[t * PP + cc] = vv[k];
    }
  }
  __syncthreads();
  T acc[S][kMseRP];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int t = 0; t < kMseRP; ++t) acc[s][t] = T(0);
  for (; j0 < nrows; j0 += G * stride) {
    // ---- N rows, then N A1 and the accumulation, row by row ----
#pragma unroll
    for (int h = 0; h < G; ++h) {
      if (j0 + h * stride >= nrows) break;   // wavefront-uniform
      T nrow[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int col = lane + 64 * s;
        T l = T(0);
        if constexpr (FIRST) {
          l = (col < p && c[h] > T(0)) ? xl[h][s] / c[h] : T(0);
        } else {
#pragma unroll
          for (int t = 0; t < kMseRP; ++t) l = fma_t(u[h][t], vt[t * PP + col], l);
        }
        nrow[s] = e[h][s] + l;
      }
      T w[kMseRP];
#pragma unroll
      for (int t = 0; t < kMseRP; ++t) {
        T d = T(0);
#pragma unroll
        for (int s = 0; s < S; ++s) d = fma_t(nrow[s], at[t * PP + lane + 64 * s], d);
        w[t] = d;
      }
      wave_sum8(w);
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int t = 0; t < kMseRP; ++t) acc[s][t] = fma_t(nrow[s], w[t], acc[s][t]);
    }
    if (j0 + G * stride < nrows) load_group(j0 + G * stride);
  }
  __syncthreads();   // the panels are no longer read
  T* red = lds;
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int t = 0; t < kMseRP; ++t)
      red[wave * PP * kMseRP + (lane + 64 * s) * kMseRP + t] = acc[s][t];
  __syncthreads();
  T* out = part + (int64_t)blockIdx.x * PP * kMseRP;
  for (int q = threadIdx.x; q < PP * kMseRP; q += 256) {
    T sum = red[q];
#pragma unroll
    for (int w = 1; w < kMseWaves; ++w) sum += red[w * PP * kMseRP + q];
    out[q] = sum;
  }
}

// The 64 sums over the wavefront's lanes of the per-lane values v[0..63]:
// six halving steps (partners whose lane bit 5, 4, ..., 0 differs exchange
// the half that the partner keeps), after which lane l holds the sum of
// index l.  The order of the additions is fixed by the lane indices.
// The 64 sums over the wavefront's lanes of the per-lane values v[0..63]:
// six halving steps (partners l ^ 32, l ^ 16, l ^ 8 through the register
// exchanges above, then l ^ 7, l ^ 2, l ^ 1 within groups of eight; at the
// step on lane bit b the lane keeps the upper half of the indices when its
// bit b is set), after which lane l holds the sum of index l.  The order
// of the additions is fixed by the lane indices.
template <typename T>
__device__ __forceinline__ T wave_reduce_scatter64(T (&v)[64]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 32; ++i) v[i] = swap_sum<true>(v[i], v[i + 32]);
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = swap_sum<false>(v[i], v[i + 16]);
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = dpp_halve<kDppRor8>(v[i], v[i + 8], (lane & 8) != 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = dpp_halve<kDppHalfMirror>(v[i], v[i + 4], (lane & 4) != 0);
#pragma unroll
  for (int i = 0; i < 2; ++i) v[i] = dpp_halve<kDppXor2>(v[i], v[i + 2], (lane & 2) != 0);
  return dpp_halve<kDppXor1>(v[0], v[1], (lane & 1) != 0);
}

// Y2 pass of a label that has been updated before (L^i = U V^T).  With
// N = E + U V^T,
//   W_row = N_row A1 = E_row A1 + U_row P,                 P = V^T A1 (8 x 8)
//   Y2 = sum_rows N_row^T W_row = sum_rows E_row^T W_row + V M,
//   M = sum_rows U_row^T W_row (8 x 8),
// so the row loop multiplies each entry of E by A1 and by W only; L^i is
// never formed.  Lane l keeps the A1 rows of its columns in registers and
// the entry (l & 7, l >> 3) of P and of M: in the eight-sum reduction of W
// (see wave_sum8) lane l holds, before the last three butterfly steps, a
// partial of W_row[l >> 3] over a set of lanes disjoint from those of the
// other seven lanes of its group, so adding u[l & 7] P[l & 7][l >> 3] there
// adds U_row P exactly once; after them it holds W_row[l >> 3] itself, the
// factor of M's entry.  The block writes its partial of Y2 (its rows'
// E^T W sums plus V M over its rows) to part[blockIdx.x]; row and group
// order as in km_gram.
template <typename T, int S>
__global__ __launch_bounds__(256) void km_gram_v(const T* __restrict__ E, int64_t lde,
                                                 const int64_t* __restrict__ rows,
                                                 int64_t nrows, int64_t p,
                                                 const T* __restrict__ U,
                                                 const T* __restrict__ V,
                                                 const T* __restrict__ A1,
                                                 T* __restrict__ part) {
  constexpr int PP = 64 * S;
  constexpr int G = MseGroup<T>::gram;
  __shared__ T red[kMseWaves * PP * kMseRP];
  __shared__ T pm[kMseWaves * 64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t stride = (int64_t)gridDim.x * kMseWaves;
  T e[G][S], ul[G];
  // Branch-free loads (rows past the end read the last row and are zeroed;
  // E is zero in its padding columns p..p_pad-1), so that all of a group's
  // loads are issued back to back.
  auto load_group = [&](int64_t j0) {
    int64_t g[G];
#pragma unroll
    for (int h = 0; h < G; ++h) {
      const int64_t j = j0 + h * stride;
      g[h] = rows[j < nrows ? j : nrows - 1];
    }
#pragma unroll
    for (int h = 0; h < G; ++h) {
      const int64_t j = j0 + h * stride;
      const bool rv = j < nrows;   // wavefront-uniform
      const T uv = U[(rv ? j : nrows - 1) * kMseRP + (lane & 7)];
      ul[h] = rv ? uv : T(0);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const T ev = E[g[h] * lde + lane + 64 * s];
        e[h][s] = rv ? ev : T(0);
      }
    }
  };
  // the panels are loaded first: the memory counters complete in issue
  // order, so P can be formed, and the rows processed one by one, while
  // later rows are still arriving.
  // A1 rows of the lane's columns (zero past p)
  T a1r[S][kMseRP];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int t = 0; t < kMseRP; ++t) a1r[s][t] = A1[(int64_t)(lane + 64 * s) * kMseRP + t];
  // V and A1 rows of the slices s = wave + 4 k (the columns c = threadIdx.x +
  // 256 k; zero for s >= S): P here, and V again for V M at the end
  constexpr int NV = (S + kMseWaves - 1) / kMseWaves;
  T vr[NV][kMseRP], ar[NV][kMseRP];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int s = wave + kMseWaves * k;
    const bool ok = s < S;   // wavefront-uniform
    const int64_t c = lane + 64 * (ok ? s : S - 1);
#pragma unroll
    for (int t = 0; t < kMseRP; ++t) {
      const T vv = V[c * kMseRP + t];
      const T av = A1[c * kMseRP + t];
      vr[k][t] = ok ? vv : T(0);
      ar[k][t] = ok ? av : T(0);
    }
  }
  int64_t j0 = (int64_t)blockIdx.x * kMseWaves + wave;
  if (j0 < nrows) load_group(j0);
  // P = V^T A1: wavefront w takes the columns of slices s = w, w + 4, ...
  {
    T pv[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) pv[i] = T(0);
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int t1 = 0; t1 < kMseRP; ++t1)
#pragma unroll
        for (int t2 = 0; t2 < kMseRP; ++t2)
          pv[t1 * kMseRP + t2] = fma_t(vr[k][t1], ar[k][t2], pv[t1 * kMseRP + t2]);
    pm[wave * 64 + lane] = wave_reduce_scatter64(pv);   // P_w[t1 * 8 + t2] on lane t1 * 8 + t2
  }
  __syncthreads();
  T pl;
  {
    const int q = (lane & 7) * kMseRP + (lane >> 3);   // P[l & 7][l >> 3]
    pl = pm[q];
#pragma unroll
    for (int w = 1; w < kMseWaves; ++w) pl += pm[w * 64 + q];
  }
  T acc[S][kMseRP];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int t = 0; t < kMseRP; ++t) acc[s][t] = T(0);
  T macc = T(0);
  for (; j0 < nrows; j0 += G * stride) {
#pragma unroll
    for (int h = 0; h < G; ++h) {
      if (j0 + h * stride >= nrows) break;   // wavefront-uniform
      T d[kMseRP];
#pragma unroll
      for (int t = 0; t < kMseRP; ++t) {
        T x = T(0);
#pragma unroll
        for (int s = 0; s < S; ++s) x = fma_t(e[h][s], a1r[s][t], x);
        d[t] = x;
      }
      T a1 = wave_halve8(d);
      a1 = fma_t(ul[h], pl, a1);   // + u[l & 7] P[l & 7][l >> 3]
      a1 = wave_bfly8(a1);
      macc = fma_t(ul[h], a1, macc);   // M[l & 7][l >> 3] += u[l & 7] W[l >> 3]
      T w[kMseRP];
      wave_bcast8(a1, w);
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int t = 0; t < kMseRP; ++t) acc[s][t] = fma_t(e[h][s], w[t], acc[s][t]);
    }
    if (j0 + G * stride < nrows) load_group(j0 + G * stride);
  }
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int t = 0; t < kMseRP; ++t)
      red[wave * PP * kMseRP + (lane + 64 * s) * kMseRP + t] = acc[s][t];
  pm[wave * 64 + lane] = macc;   // M_w[t1][t2] on lane t2 * 8 + t1 (pm is free again)
  __syncthreads();
  T mm[kMseRP][kMseRP];   // the block's M, added over the wavefronts in order
#pragma unroll
  for (int t1 = 0; t1 < kMseRP; ++t1)
#pragma unroll
    for (int t2 = 0; t2 < kMseRP; ++t2) {
      const int q = t2 * kMseRP + t1;
      T m = pm[q];
#pragma unroll
      for (int w = 1; w < kMseWaves; ++w) m += pm[w * 64 + q];
      mm[t1][t2] = m;
    }
  T* out = part + (int64_t)blockIdx.x * PP * kMseRP;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int c = threadIdx.x + 256 * k;
    if (c >= PP) break;
#pragma unroll
    for (int t2 = 0; t2 < kMseRP; ++t2) {
      T sum = red[c * kMseRP + t2];
#pragma unroll
      for (int w = 1; w < kMseWaves; ++w) sum += red[w * PP * kMseRP + c * kMseRP + t2];
      T vm = T(0);
#pragma unroll
      for (int t1 = 0; t1 < kMseRP; ++t1) vm = fma_t(vr[k][t1], mm[t1][t2], vm);
      out[c * kMseRP + t2] = sum + vm;
    }
  }
}

// One Cholesky QR round on the p_pad x 8 panel Y (FP64, LDS, rows padded to
// kOrthLd doubles so that a wavefront's row reads do not collide in the
// banks) by a block of kOrthThreads: Gram in a fixed order, Cholesky with
// the dependent-column rule (a pivot at most tau * G_jj marks column j
// dependent: zero row of R, zero column of the result), Y <- Y R^{-1}.
// `act` holds the columns still in use.  The Gram takes no cross-lane
// sums: thread (seg, a, b) adds Y[c][a] Y[c][b] over the rows c of segment
// seg (four interleaved accumulators), then 64 threads add the eight
// segments in order.  The Cholesky factorisation and the substitution are
// right-looking (each finished column is subtracted from all later ones at
// once), which performs the same additions in the same order as the
// column-by-column form with far shorter dependent chains.  Every loop over
// the 8 columns is unrolled so that all small arrays stay in registers.
constexpr int kOrthThreads = 512;
constexpr int kOrthLd = kMseRP + 1;
template <int PP>
__device__ __forceinline__ void mse_chol_round(double* Y, int r, double tau, int* act, double* gsh,
                               double* red) {
  constexpr int R8 = kMseRP;
  constexpr int LD = kOrthLd;
  constexpr int NE = R8 * (R8 + 1) / 2;   // entries a <= b
  constexpr int NSEG = kOrthThreads / (R8 * R8);
  constexpr int SEG = PP / NSEG;
  static_assert(SEG % 4 == 0, "segment length");
  auto tri = [](int a_, int b_) { return a_ * R8 - a_ * (a_ - 1) / 2 + (b_ - a_); };
  const int tid = threadIdx.x;
  {
    const int ab = tid & (R8 * R8 - 1);
    const int seg = tid / (R8 * R8);
    const int a_ = ab / R8, b_ = ab % R8;
    double g4[4] = {0.0, 0.0, 0.0, 0.0};
    const double* y = Y + seg * SEG * LD;
#pragma unroll 4
    for (int c = 0; c < SEG; c += 4) {
#pragma unroll
      for (int k = 0; k < 4; ++k) g4[k] = fma(y[(c + k) * LD + a_], y[(c + k) * LD + b_], g4[k]);
    }
    const double gv = (a_ < r && b_ < r) ? (g4[0] + g4[1]) + (g4[2] + g4[3]) : 0.0;
    red[seg * R8 * R8 + ab] = gv;
  }
  __syncthreads();
  if (tid < R8 * R8) {
    double t = red[tid];
#pragma unroll
    for (int sg = 1; sg < NSEG; ++sg) t += red[sg * R8 * R8 + tid];
    const int a_ = tid / R8, b_ = tid % R8;
    if (a_ <= b_) gsh[tri(a_, b_)] = t;
  }
  __syncthreads();
  if (tid == 0) {
    // packed upper triangle, entry (a, b) at tri(a, b); G becomes R in place
    double T[NE], gd[R8];
#pragma unroll
    for (int q = 0; q < NE; ++q) T[q] = gsh[q];
#pragma unroll
    for (int j = 0; j < R8; ++j) gd[j] = T[tri(j, j)];
    int am = 0;
#pragma unroll
    for (int j = 0; j < R8; ++j) am |= act[j] ? (1 << j) : 0;
#pragma unroll
    for (int j = 0; j < R8; ++j) {
      // T[j][j..] already has the rows l < j of R subtracted
      const double d = T[tri(j, j)];
      const bool on = j < r && ((am >> j) & 1) && (d > tau * gd[j]) && (gd[j] > 0.0);
      if (!on) {
        am &= ~(1 << j);
#pragma unroll
        for (int b_ = j; b_ < R8; ++b_) T[tri(j, b_)] = 0.0;
        gsh[NE + j] = 0.0;
        continue;
      }
      // 1 / r_jj from a Newton-refined reciprocal square root: the rows of R
      // and the substitution below multiply by it instead of dividing
      const double ir = rsqrt_nr(d);
      T[tri(j, j)] = d * ir;
#pragma unroll
      for (int b_ = j + 1; b_ < R8; ++b_) T[tri(j, b_)] *= ir;
#pragma unroll
      for (int a_ = j + 1; a_ < R8; ++a_)
#pragma unroll
        for (int b_ = a_; b_ < R8; ++b_) T[tri(a_, b_)] -= T[tri(j, a_)] * T[tri(j, b_)];
      gsh[NE + j] = ir;
    }
#pragma unroll
    for (int j = 0; j < R8; ++j) act[j] = (am >> j) & 1;
#pragma unroll
    for (int q = 0; q < NE; ++q) gsh[q] = T[q];
  }
  __syncthreads();
  // Y <- Y R^{-1} on the active columns (forward substitution per row; an
  // inactive column has a zero row of R and a zero result)
  int am = 0;
#pragma unroll
  for (int j = 0; j < R8; ++j) am |= act[j] ? (1 << j) : 0;
  double rr[NE], rinv[R8];
#pragma unroll
  for (int q = 0; q < NE; ++q) rr[q] = gsh[q];
#pragma unroll
  for (int j = 0; j < R8; ++j) rinv[j] = gsh[NE + j];
  for (int c = tid; c < PP; c += kOrthThreads) {
    double sv[R8];
#pragma unroll
    for (int t = 0; t < R8; ++t) sv[t] = Y[c * LD + t];
#pragma unroll
    for (int j = 0; j < R8; ++j) {
      const double qj = ((am >> j) & 1) ? sv[j] * rinv[j] : 0.0;
      sv[j] = qj;
#pragma unroll
      for (int b_ = j + 1; b_ < R8; ++b_) sv[b_] -= qj * rr[tri(j, b_)];
    }
#pragma unroll
    for (int t = 0; t < R8; ++t) Y[c * LD + t] = sv[t];
  }
  __syncthreads();
}

// Y2 from the block partials, in FP64 and a fixed order, then Q = orth(Y2).
// A block of kOrthThreads takes 32 entries of Y2: thread (g, e) adds the
// partials g, g + 16, g + 32, ... of entry e in ascending order (all its
// loads in flight at once), then the sixteen group sums of each entry are
// added in group order and stored write-through at device scope.  The last
// block to arrive (a device-scope counter, reset by that block) reads all
// of Y2 back with device-scope loads and runs the two Cholesky QR rounds.
constexpr int kMseRedEntries = 32;
constexpr int kMseRedGroups = kOrthThreads / kMseRedEntries;
template <typename T, int PP>
__global__ __launch_bounds__(kOrthThreads) void km_reduce_orth(const T* __restrict__ part,
                                                               int nblk, int r,
                                                               double* __restrict__ y2,
                                                               unsigned int* __restrict__ ctl,
                                                               T* __restrict__ Q) {
  constexpr int F = 16;   // partials per group: nblk <= F * kMseRedGroups
  constexpr int PER = PP * kMseRP / kOrthThreads;
  __shared__ double Y[PP * kOrthLd];
  __shared__ double red[kOrthThreads];
  __shared__ double gsh[kMseRP * kMseRP];
  __shared__ int act[kMseRP];
  __shared__ int last;
  const int tid = threadIdx.x;
  {
    const int el = tid % kMseRedEntries, gq = tid / kMseRedEntries;
    const int e = blockIdx.x * kMseRedEntries + el;
    T v[F];
#pragma unroll
    for (int k = 0; k < F; ++k) {
      const int b = gq + kMseRedGroups * k;
      v[k] = b < nblk ? part[(int64_t)b * PP * kMseRP + e] : T(0);
    }
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < F; ++k)
      if (gq + kMseRedGroups * k < nblk) sum += (double)v[k];
    red[gq * kMseRedEntries + el] = sum;
  }
  __syncthreads();
  if (tid < kMseRedEntries) {
    double y = red[tid];
#pragma unroll
    for (int g = 1; g < kMseRedGroups; ++g) y += red[g * kMseRedEntries + tid];
    publish(y2 + blockIdx.x * kMseRedEntries + tid, y);
  }
  stores_done();
  __syncthreads();
  if (tid == 0) last = arrive(ctl) == gridDim.x - 1u;
  __syncthreads();
  if (!last) return;
  if (tid == 0) publish_u32(ctl, 0u);
  {
    double v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) v[q] = fetch(y2 + q * kOrthThreads + tid);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = q * kOrthThreads + tid;
      Y[(e / kMseRP) * kOrthLd + e % kMseRP] = v[q];
    }
  }
  if (tid < kMseRP) act[tid] = tid < r ? 1 : 0;
  __syncthreads();
  const double u = sizeof(T) == 8 ? 0x1p-53 : 0x1p-24;
  const double tau = (double)r * fmax(u * u, 0x1p-53);
  mse_chol_round<PP>(Y, r, tau, act, gsh, red);
  mse_chol_round<PP>(Y, r, tau, act, gsh, red);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = q * kOrthThreads + tid;
    Q[e] = (T)Y[(e / kMseRP) * kOrthLd + e % kMseRP];
  }
}

// U_row = N_row Q and E_row = N_row - U_row Q^T for every row of the label,
// a group of rows of a wavefront at a time (V in LDS, transposed; Q in
// registers); the first group's loads are issued before V is staged.
// Two wavefronts per SIMD (at most 256 registers): two blocks per CU, so
// that a label's blocks (one per 16 rows) run in one round.
template <typename T, int S, bool FIRST>
__global__ __launch_bounds__(256, 2) void km_update(T* __restrict__ E, int64_t lde,
                                                 const T* __restrict__ X, int64_t ldx,
                                                 const T* __restrict__ cnt,
                                                 const int64_t* __restrict__ rows,
                                                 int64_t nrows, int64_t p,
                                                 T* __restrict__ U, const T* __restrict__ V,
                                                 const T* __restrict__ Q) {
  constexpr int PP = 64 * S;
  constexpr int G = MseGroup<T>::update;
  __shared__ T vt[kMseRP * PP];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t stride = (int64_t)gridDim.x * kMseWaves;
  // u: lane l holds entry l & 7 of the row of U (read out as scalars)
  T e[G][S], xl[FIRST ? G : 1][FIRST ? S : 1], u[FIRST ? 1 : G], c[G];
  int64_t gg[G];
  // branch-free loads, as in km_gram_v; X past column p is not read
  auto load_group = [&](int64_t j0) {
#pragma unroll
    for (int h = 0; h < G; ++h) {
      const int64_t j = j0 + h * stride;
      gg[h] = rows[j < nrows ? j : nrows - 1];
    }
#pragma unroll
    for (int h = 0; h < G; ++h) {
      const int64_t j = j0 + h * stride;
      const bool rv = j < nrows;   // wavefront-uniform
      const int64_t jc = rv ? j : nrows - 1;
      const int64_t g = gg[h];
      if constexpr (FIRST) {
        const T cv = cnt[g];
        c[h] = rv ? cv : T(0);
      } else {
        c[h] = T(0);
        const T uv = U[jc * kMseRP + (lane & 7)];
        u[h] = rv ? uv : T(0);
      }
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int64_t col = lane + 64 * s;
        const T ev = E[g * lde + col];
        e[h][s] = rv ? ev : T(0);
        if constexpr (FIRST) xl[h][s] = (rv && col < p) ? X[g * ldx + col] : T(0);
      }
    }
  };
  // the panels are loaded before the rows (the memory counters complete in
  // issue order), so the rows can be processed while later ones arrive
  constexpr int NST = PP * kMseRP / 256;
  T vv[NST];
#pragma unroll
  for (int k = 0; k < NST; ++k) vv[k] = FIRST ? T(0) : V[k * 256 + threadIdx.x];
  T qq[S][kMseRP];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int t = 0; t < kMseRP; ++t) qq[s][t] = Q[(lane + 64 * s) * kMseRP + t];
  int64_t j0 = (int64_t)blockIdx.x * kMseWaves + wave;
  if (j0 < nrows) load_group(j0);
#pragma unroll
  for (int k = 0; k < NST; ++k) {
    const int q = k * 256 + threadIdx.x;
    vt[(q % kMseRP) * PP + q / kMseRP] = vv[k];
  }
  __syncthreads();
  for (; j0 < nrows; j0 += G * stride) {
#pragma unroll
    for (int h = 0; h < G; ++h) {
      const int64_t j = j0 + h * stride;
      if (j >= nrows) break;   // wavefront-uniform
      T nrow[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int col = lane + 64 * s;
        T l = T(0);
        if constexpr (FIRST) {
          l = (col < p && c[h] > T(0)) ? xl[h][s] / c[h] : T(0);
        } else {
#pragma unroll
          for (int t = 0; t < kMseRP; ++t) l = fma_t(lane_read(u[h], t), vt[t * PP + col], l);
        }
        nrow[s] = e[h][s] + l;
      }
      T w[kMseRP];
#pragma unroll
      for (int t = 0; t < kMseRP; ++t) {
        T d = T(0);
#pragma unroll
        for (int s = 0; s < S; ++s) d = fma_t(nrow[s], qq[s][t], d);
        w[t] = d;
      }
      wave_sum8(w);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int64_t col = lane + 64 * s;
        T l = T(0);
#pragma unroll
        for (int t = 0; t < kMseRP; ++t) l = fma_t(w[t], qq[s][t], l);
        if (col < p) store_wt(E + gg[h] * lde + col, nrow[s] - l);
      }
      // every lane holds w; lanes 0..7 store the row of U (its loads are done)
      T wl = w[0];
#pragma unroll
      for (int t = 1; t < kMseRP; ++t) wl = (lane == t) ? w[t] : wl;
      if (lane < kMseRP) store_wt(U + j * kMseRP + lane, wl);
    }
    if (j0 + G * stride < nrows) load_group(j0 + G * stride);
  }
}

// E = X - sum_i Z_{Omega_i} with Z = D^{-1} X: each labelled row gets cnt
// copies of X_row / cnt subtracted, added up in label order.
template <typename T>
__global__ __launch_bounds__(256) void km_init_e(T* __restrict__ E, int64_t lde,
                                                 const T* __restrict__ X, int64_t ldx,
                                                 const T* __restrict__ cnt, int64_t n,
                                                 int64_t p) {
  const int64_t total = n * lde;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t g = e / lde, col = e % lde;
    T out = T(0);
    if (col < p) {
      const T x = X[g * ldx + col];
      const T c = cnt[g];
      T acc = T(0);
      if (c > T(0)) {
        const T z = x / c;
        for (int u = 0; u < (int)c; ++u) acc += z;
      }
      out = x - acc;
    }
    E[e] = out;
  }
}

// E[idx] += val for the entries of the previous S (R = E + S before the
// sparse step).
template <typename T>
__global__ __launch_bounds__(256) void km_add_s(T* __restrict__ E, int64_t lde, int64_t p,
                                                const int64_t* __restrict__ idx,
                                                const T* __restrict__ val,
                                                const SelPlan* __restrict__ plan) {
  const long long cnt = plan->nnz;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (long long)gridDim.x * 256) {
    const int64_t id = idx[e];
    const int64_t i = id / p, j = id % p;
    E[i * lde + j] += val[e];
  }
}

// Copy of one label's factors without the padding: U (n_i x r), V (p x r).
template <typename T>
__global__ __launch_bounds__(256) void km_copy_factors(const T* __restrict__ U,
                                                       const T* __restrict__ V, int64_t ni,
                                                       int64_t p, int r, T* __restrict__ Uo,
                                                       T* __restrict__ Vo) {
  const int64_t nu = ni * r, nv = p * r;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nu + nv;
       e += (int64_t)gridDim.x * 256) {
    if (e < nu)
      Uo[e] = U[(e / r) * kMseRP + e % r];
    else
      Vo[e - nu] = V[((e - nu) / r) * kMseRP + (e - nu) % r];
  }
}

// E (lde) -> out (ldo), the first p columns.
template <typename T>
__global__ __launch_bounds__(256) void km_copy_e(const T* __restrict__ E, int64_t lde,
                                                 int64_t n, int64_t p, T* __restrict__ out,
                                                 int64_t ldo) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n * p;
       e += (int64_t)gridDim.x * 256)
    out[(e / p) * ldo + e % p] = E[(e / p) * lde + e % p];
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
#define GODEC_MSE_S_SWITCH(S_, ...)                  \
  switch (S_) {                                      \
    case 1: { constexpr int S = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int S = 2; __VA_ARGS__; } break; \
    case 4: { constexpr int S = 4; __VA_ARGS__; } break; \
    case 8: { constexpr int S = 8; __VA_ARGS__; } break; \
    default: break;                                  \
  }

template <typename T>
static void mse_label_t(const Launch& L, const MseLabelArgs& a) {
  GODEC_MSE_S_SWITCH(a.S, {
    // FP64 rows are limited to 256 columns (S <= 4): three 8-wide FP64
    // panels of 8 columns per lane fill the register file
    if constexpr (!(sizeof(T) == 8 && S == 8)) {
      if (a.first)
        hipLaunchKernelGGL((km_gram<T, S, true>), dim3((unsigned)a.nblk), dim3(256), 0,
                           L.stream, (const T*)a.E, a.lde, (const T*)a.X, a.ldx,
                           (const T*)a.cnt, a.rows, a.nrows, a.p, (const T*)a.U,
                           (const T*)a.Vold, (const T*)a.A1, (T*)a.part);
      else
        hipLaunchKernelGGL((km_gram_v<T, S>), dim3((unsigned)a.nblk), dim3(256), 0, L.stream,
                           (const T*)a.E, a.lde, a.rows, a.nrows, a.p, (const T*)a.U,
                           (const T*)a.Vold, (const T*)a.A1, (T*)a.part);
      hipLaunchKernelGGL((km_reduce_orth<T, 64 * S>),
                         dim3(64 * S * kMseRP / kMseRedEntries), dim3(kOrthThreads), 0,
                         L.stream, (const T*)a.part, a.nblk, a.r, a.y2, a.ctl, (T*)a.Vnew);
      // the update writes no partials: a block per kMseWaves groups of rows
      constexpr int RPB = kMseWaves * MseGroup<T>::update;
      int64_t nbu = (a.nrows + RPB - 1) / RPB;
      nbu = nbu < 1 ? 1 : (nbu > (int64_t)L.num_cu * 8 ? (int64_t)L.num_cu * 8 : nbu);
      if (a.first)
        hipLaunchKernelGGL((km_update<T, S, true>), dim3((unsigned)nbu), dim3(256), 0,
                           L.stream, (T*)a.E, a.lde, (const T*)a.X, a.ldx, (const T*)a.cnt,
                           a.rows, a.nrows, a.p, (T*)a.U, (const T*)a.Vold,
                           (const T*)a.Vnew);
      else
        hipLaunchKernelGGL((km_update<T, S, false>), dim3((unsigned)nbu), dim3(256), 0,
                           L.stream, (T*)a.E, a.lde, (const T*)a.X, a.ldx, (const T*)a.cnt,
                           a.rows, a.nrows, a.p, (T*)a.U, (const T*)a.Vold,
                           (const T*)a.Vnew);
    }
  });
}

void launch_mse_label(const Launch& L, bool f64, const MseLabelArgs& a) {
  if (f64) mse_label_t<double>(L, a);
  else mse_label_t<float>(L, a);
}

void launch_mse_init_e(const Launch& L, bool f64, void* E, int64_t lde, const void* X,
                       int64_t ldx, const void* cnt, int64_t n, int64_t p) {
  int64_t g = (n * lde + 255) / 256;
  g = g > (int64_t)L.num_cu * 16 ? (int64_t)L.num_cu * 16 : (g < 1 ? 1 : g);
  if (f64)
    hipLaunchKernelGGL(km_init_e<double>, dim3((unsigned)g), dim3(256), 0, L.stream,
                       (double*)E, lde, (const double*)X, ldx, (const double*)cnt, n, p);
  else
    hipLaunchKernelGGL(km_init_e<float>, dim3((unsigned)g), dim3(256), 0, L.stream,
                       (float*)E, lde, (const float*)X, ldx, (const float*)cnt, n, p);
}

void launch_mse_add_s(const Launch& L, bool f64, void* E, int64_t lde, int64_t p,
                      const int64_t* idx, const void* val, const SelPlan* plan, int64_t kmax) {
  int64_t g = (kmax + 255) / 256;
  g = g > (int64_t)L.num_cu * 4 ? (int64_t)L.num_cu * 4 : (g < 1 ? 1 : g);
  if (f64)
    hipLaunchKernelGGL(km_add_s<double>, dim3((unsigned)g), dim3(256), 0, L.stream,
                       (double*)E, lde, p, idx, (const double*)val, plan);
  else
    hipLaunchKernelGGL(km_add_s<float>, dim3((unsigned)g), dim3(256), 0, L.stream,
                       (float*)E, lde, p, idx, (const float*)val, plan);
}

void launch_mse_copy_factors(const Launch& L, bool f64, const void* U, const void* V,
                             int64_t ni, int64_t p, int r, void* Uo, void* Vo) {
  int64_t g = ((ni + p) * r + 255) / 256;
  g = g > (int64_t)L.num_cu * 4 ? (int64_t)L.num_cu * 4 : (g < 1 ? 1 : g);
  if (f64)
    hipLaunchKernelGGL(km_copy_factors<double>, dim3((unsigned)g), dim3(256), 0, L.stream,
                       (const double*)U, (const double*)V, ni, p, r, (double*)Uo, (double*)Vo);
  else
    hipLaunchKernelGGL(km_copy_factors<float>, dim3((unsigned)g), dim3(256), 0, L.stream,
                       (const float*)U, (const float*)V, ni, p, r, (float*)Uo, (float*)Vo);
}

void launch_mse_copy_e(const Launch& L, bool f64, const void* E, int64_t lde, int64_t n,
                       int64_t p, void* out, int64_t ldo) {
  int64_t g = (n * p + 255) / 256;
  g = g > (int64_t)L.num_cu * 16 ? (int64_t)L.num_cu * 16 : (g < 1 ? 1 : g);
  if (f64)
    hipLaunchKernelGGL(km_copy_e<double>, dim3((unsigned)g), dim3(256), 0, L.stream,
                       (const double*)E, lde, n, p, (double*)out, ldo);
  else
    hipLaunchKernelGGL(km_copy_e<float>, dim3((unsigned)g), dim3(256), 0, L.stream,
                       (const float*)E, lde, n, p, (float*)out, ldo);
}

}  // namespace godec
