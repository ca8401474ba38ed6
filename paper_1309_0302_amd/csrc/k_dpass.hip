// Row-pass products of the differentiable layer's backward: one read of a
// dense m x n matrix D (row stride n, n <= 512 in FP32, <= 128 in FP64)
// forms, for a panel P (n x NY),
//   Y = D P'          (P' column c = P column (c + rot) mod NY), and / or
//   Z = D^T Y[:, :NA] (the first NA columns of Y back through D^T),
// so that A P = D^T (D P) with A = D^T D, or a pair of rank terms D [U W]
// together with A U, costs a single pass over D instead of two or three.
//
// Lane l of a wave owns columns l + 64 s (s < SM) and keeps their rows of P.
// A wave takes G rows at a time: each lane forms its share of y_i = D_i P'
// for the G rows, and the wave adds the G NY values across its lanes by
// recursive halving (at each step a lane passes half of its values to its
// partner and keeps the other half, so every lane ends with one total).  The
// lane that holds a total stores it to Y; the totals feeding Z are read back
// from their lanes and each lane adds D_ij y_i into its columns.  The next G
// rows are loaded while the current ones reduce.  For Z, the four waves' sums
// are added in order through LDS and each block stores its partial; a second
// kernel adds the partials in block order.
#include "godec_internal.h"
#include "k_common.h"

#include <algorithm>

namespace godec {
namespace {

#define GODEC_RANK_SWITCH(rr, ...)                         \
  switch (rr) {                                            \
    case 1: { constexpr int R = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int R = 2; __VA_ARGS__; } break;   \
    case 3: { constexpr int R = 3; __VA_ARGS__; } break;   \
    case 4: { constexpr int R = 4; __VA_ARGS__; } break;   \
    case 5: { constexpr int R = 5; __VA_ARGS__; } break;   \
    case 6: { constexpr int R = 6; __VA_ARGS__; } break;   \
    case 7: { constexpr int R = 7; __VA_ARGS__; } break;   \
    case 8: { constexpr int R = 8; __VA_ARGS__; } break;   \
    default: break;                                        \
  }

constexpr int dp_pow2(int v) { return v <= 1 ? 1 : 2 * dp_pow2((v + 1) / 2); }

// rows per wave step: G NY <= 16 values per halving
template <int NY>
constexpr int dp_rows() { return 16 / NY < 1 ? 1 : 16 / NY > 8 ? 8 : 16 / NY; }

// lane whose halving path keeps value v
template <int VP>
__device__ constexpr int dp_lane_of(int v) {
  int lane = 0, c = VP;
  for (int o = 32; o >= 1; o >>= 1) {
    if (c > 1) {
      c >>= 1;
      if (v & c) lane |= o;
    }
  }
  return lane;
}

// One halving step per lane-distance O (32, 16, .., 1) on CNT live values;
// with one value left the remaining steps add the partner's total.
template <typename T, int VP, int CNT, int O>
__device__ __forceinline__ void dp_halve(T (&a)[VP], int lane) {
  if constexpr (O >= 1) {
    if constexpr (CNT > 1) {
      constexpr int H = CNT / 2;
      const bool up = (lane & O) != 0;
#pragma unroll
      for (int t = 0; t < H; ++t) {
        const T send = up ? a[t] : a[t + H];
        const T keep = up ? a[t + H] : a[t];
        a[t] = keep + __shfl_xor(send, O, 64);
      }
      dp_halve<T, VP, H, O / 2>(a, lane);
    } else {
      a[0] += __shfl_xor(a[0], O, 64);
      dp_halve<T, VP, 1, O / 2>(a, lane);
    }
  }
}

template <typename T, int NY, int NA, int SM, bool WY>
__global__ __launch_bounds__(256) void kd_pass(int m, int n, int rpb, const T* __restrict__ D,
                                               int64_t sD, const T* __restrict__ P,
                                               int64_t ldp, int64_t sP, int rot,
                                               T* __restrict__ Y, int64_t ldy, int64_t sY,
                                               T* __restrict__ part) {
  constexpr int G = dp_rows<NY>();
  constexpr int V = G * NY;
  constexpr int VP = dp_pow2(V);
  constexpr int NZ = NA > 0 ? NA : 1;
  static_assert(VP <= 64, "at most 64 values per halving");
  extern __shared__ unsigned char dp_lds[];
  const int b = blockIdx.y, blk = blockIdx.x, tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const T* Db = D + (int64_t)b * sD;
  const T* Pb = P + (int64_t)b * sP;
  T p[SM][NY], acc[SM][NZ];
#pragma unroll
  for (int s = 0; s < SM; ++s) {
    const int j = lane + 64 * s;
#pragma unroll
    for (int c = 0; c < NY; ++c) p[s][c] = j < n ? Pb[(int64_t)j * ldp + (c + rot) % NY] : T(0);
#pragma unroll
    for (int c = 0; c < NZ; ++c) acc[s][c] = T(0);
  }
  // the value index this lane ends with after the halving
  int base = 0;
  {
    int cnt = VP;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
      if (cnt > 1) {
        cnt >>= 1;
        if (lane & o) base += cnt;
      }
  }
  const int row0 = blk * rpb;
  const int row1 = (m - row0) < rpb ? m : row0 + rpb;
  T d[G][SM], dn[G][SM];
  auto load_rows = [&](int g0, T (&dd)[G][SM]) {
#pragma unroll
    for (int gg = 0; gg < G; ++gg)
#pragma unroll
      for (int s = 0; s < SM; ++s) {
        const int i = g0 + gg, j = lane + 64 * s;
        dd[gg][s] = (i < row1 && j < n) ? Db[(int64_t)i * n + j] : T(0);
      }
  };
  load_rows(row0 + wave * G, d);
  for (int g0 = row0 + wave * G; g0 < row1; g0 += 4 * G) {
    if (g0 + 4 * G < row1) load_rows(g0 + 4 * G, dn);
    T a[VP];
#pragma unroll
    for (int gg = 0; gg < G; ++gg)
#pragma unroll
      for (int c = 0; c < NY; ++c) {
        T t = T(0);
#pragma unroll
        for (int s = 0; s < SM; ++s) t += d[gg][s] * p[s][c];
        a[gg * NY + c] = t;
      }
#pragma unroll
    for (int v = V; v < VP; ++v) a[v] = T(0);
    dp_halve<T, VP, VP, 32>(a, lane);
    if (WY && base < V) {
      const int row = g0 + base / NY;
      if (row < row1) Y[(int64_t)b * sY + (int64_t)row * ldy + base % NY] = a[0];
    }
    if (NA > 0) {
#pragma unroll
      for (int gg = 0; gg < G; ++gg)
#pragma unroll
        for (int c = 0; c < NZ; ++c) {
          const T y = __shfl(a[0], dp_lane_of<VP>(gg * NY + c), 64);
#pragma unroll
          for (int s = 0; s < SM; ++s) acc[s][c] += d[gg][s] * y;
        }
    }
#pragma unroll
    for (int gg = 0; gg < G; ++gg)
#pragma unroll
      for (int s = 0; s < SM; ++s) d[gg][s] = dn[gg][s];
  }
  if (NA == 0) return;
  T* red = reinterpret_cast<T*>(dp_lds);
#pragma unroll
  for (int s = 0; s < SM; ++s) {
    const int j = lane + 64 * s;
    if (j < n)
#pragma unroll
      for (int c = 0; c < NZ; ++c) red[((int64_t)wave * n + j) * NZ + c] = acc[s][c];
  }
  __syncthreads();
  const int nn = n * NZ;
  T* o = part + ((int64_t)b * gridDim.x + blk) * nn;
  for (int e = tid; e < nn; e += 256)
    o[e] = ((red[e] + red[nn + e]) + red[2 * nn + e]) + red[3 * nn + e];
}

// Z[b] = sum over blocks (in order) of the partials; Z n x NA, row stride NA.
template <typename T>
__global__ __launch_bounds__(256) void kd_reduce(int count, int nblk, const T* __restrict__ part,
                                                 T* __restrict__ Z, int64_t sZ) {
  const int b = blockIdx.y;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  const T* pe = part + (int64_t)b * nblk * count + e;
  T s = T(0);
  int k = 0;
  for (; k + 8 <= nblk; k += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = pe[(int64_t)(k + u) * count];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; k < nblk; ++k) s += pe[(int64_t)k * count];
  Z[(int64_t)b * sZ + e] = s;
}

struct DpArgs {
  int nb, m, n, rpb, nblk;
  const void* D;
  int64_t sD;
  const void* P;
  int64_t ldp, sP;
  int rot;
  void* Y;
  int64_t ldy, sY;
  void* part;
};

template <typename T, int NY, int NA, int SM, bool WY>
void dp_launch(const Launch& L, const DpArgs& a) {
  const size_t lds = NA > 0 ? sizeof(T) * 4 * (size_t)a.n * NA : 0;
  hipLaunchKernelGGL((kd_pass<T, NY, NA, SM, WY>), dim3((unsigned)a.nblk, (unsigned)a.nb),
                     dim3(256), lds, L.stream, a.m, a.n, a.rpb, (const T*)a.D, a.sD,
                     (const T*)a.P, a.ldp, a.sP, a.rot, (T*)a.Y, a.ldy, a.sY, (T*)a.part);
}

// FP32 takes SM = 4 (n <= 256) or 8 (n <= 512); FP64 SM = 2 (n <= 128).
template <typename T, int NY, int NA, bool WY>
void dp_sm(const Launch& L, const DpArgs& a) {
  if constexpr (sizeof(T) == 8) {
    dp_launch<T, NY, NA, 2, WY>(L, a);
  } else {
    if (a.n <= 256) dp_launch<T, NY, NA, 4, WY>(L, a);
    else dp_launch<T, NY, NA, 8, WY>(L, a);
  }
}

// kinds: 0 Y = D P (NY = r), 1 Z = A P (NY = NA = r), 2 Y = D [U W] rotated
// (NY = 2r), 3 the pair with Z = A U (NY = 2r, NA = r)
template <typename T>
void dp_dispatch(const Launch& L, const DpArgs& a, int kind, int r) {
  switch (kind) {
    case 0: GODEC_RANK_SWITCH(r, (dp_sm<T, R, 0, true>(L, a))); break;
    case 1: GODEC_RANK_SWITCH(r, (dp_sm<T, R, R, false>(L, a))); break;
    case 2: GODEC_RANK_SWITCH(r, (dp_sm<T, 2 * R, 0, true>(L, a))); break;
    default: GODEC_RANK_SWITCH(r, (dp_sm<T, 2 * R, R, true>(L, a))); break;
  }
}

}  // namespace

bool lk_dpass(const Launch& L, bool f64, int nb, int m, int n, int r, const void* D, bool pair,
              const void* P, int64_t ldp, int64_t sP, void* Y, int64_t ldy, int64_t sY, void* Z,
              void* part, int64_t part_cap) {
  const int na = Z ? r : 0;
  if (r < 1 || r > 8 || n > (f64 ? 128 : 512) || (!Y && !Z) || (pair && !Y)) return false;
  const int rot = pair ? r : 0;
  const size_t ts = f64 ? 8 : 4;
  if (na > 0 && ts * 4 * (size_t)n * na > 65536) return false;
  DpArgs a{};
  a.nb = nb;
  a.m = m;
  a.n = n;
  a.D = D;
  a.sD = (int64_t)m * n;
  a.P = P;
  a.ldp = ldp;
  a.sP = sP;
  a.rot = rot;
  a.Y = Y;
  a.ldy = ldy;
  a.sY = sY;
  a.part = part;
  if (na > 0) {
    // about four blocks per compute unit over the batch, at most 64 per problem
    int nblk = std::max(1, std::min(64, (4 * L.num_cu + nb - 1) / nb));
    int rpb = (m + nblk - 1) / nblk;
    rpb = (rpb + 15) / 16 * 16;
    nblk = (m + rpb - 1) / rpb;
    if ((int64_t)nb * nblk * n * na > part_cap) return false;
    a.rpb = rpb;
    a.nblk = nblk;
  } else {
    a.rpb = 64;
    a.nblk = (m + 63) / 64;
  }
  const int kind = na == 0 ? (pair ? 2 : 0) : (pair ? 3 : 1);
  if (f64) dp_dispatch<double>(L, a, kind, r);
  else dp_dispatch<float>(L, a, kind, r);
  if (na > 0) {
    const int count = n * na;
    const dim3 g((unsigned)((count + 255) / 256), (unsigned)nb);
    if (f64)
      hipLaunchKernelGGL(kd_reduce<double>, g, dim3(256), 0, L.stream, count, a.nblk,
                         (const double*)part, (double*)Z, (int64_t)n * r);
    else
      hipLaunchKernelGGL(kd_reduce<float>, g, dim3(256), 0, L.stream, count, a.nblk,
                         (const float*)part, (float*)Z, (int64_t)n * r);
  }
  return true;
}

}  // namespace godec
