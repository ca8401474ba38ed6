// Panel products of the power chain on the CDNA4 matrix cores.
//
// Both halves of a Gram pass stream the working copy D (mpad x ldd,
// row-major, zero padded to multiples of 64 rows and 128 columns):
//
//   k_mm_a:  W^T = (D Z)^T         (32 x mpad)  A = rows of D, B = Z^T
//   k_mm_b:  Z_out^T = W^T D       (32 x ldd)   A = W^T,      B = D
//
// The panel width is padded to 32 (one MFMA tile); padding columns are zero.
// The contraction index may be permuted freely as long as both operands use
// the same (lane group, slot) -> k assignment.  k_mm_a stages D through
// LDS (coalesced row reads); k_mm_b reads 8-byte column groups of D rows
// directly (lanes cover consecutive columns, so a wave reads whole rows).
//
// Layouts used (v_mfma_f32_32x32x{16_bf16, 2_f32}, lane l, l%32 = index on
// the lanes, l/32 = group g):  A operand row i = l%32; B operand column
// j = l%32; accumulator register v holds C[8(v/4) + 4g + v%4][l%32].
#include <hip/hip_ext.h>

#include "godec_internal.h"
#include "k_common.h"
#include "k_mmb.h"

namespace godec {

// ---------------------------------------------------------------------------
// k_mm_a: Wtpart[ct] = (D[:, tile ct] Z[tile ct, :])^T.
// Block = 4 waves and 128 rows of D; wave w owns the 32-row MFMA tile
// [32w, 32w + 32).  The block walks its KC-column tile in steps of 128
// bytes per row: every step, the 128 x 128-byte slab of D and the 32 x
// 128-byte slab of Z^T are read with coalesced 16-byte loads (eight lanes
// per row), written to LDS (chunk index XOR-swizzled by the row to spread
// banks), and read back in the MFMA operand layout.  The loads of step s+1
// are issued before the products of step s (double-buffered LDS).
// ---------------------------------------------------------------------------
constexpr int kMmaRows = 128;

template <typename TT>
__device__ __forceinline__ void mma_gload(const TT* __restrict__ D, int64_t ldd, int64_t mpad,
                                          const TT* __restrict__ Zt, int64_t rb, int64_t kk,
                                          int lr, int lc, u32x4 (&st)[4], u32x4& sz) {
  constexpr int E = 16 / sizeof(TT);   // elements per 16-byte chunk
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int64_t row = rb + lr + 32 * h;
    st[h] = row < mpad ? *reinterpret_cast<const u32x4*>(D + row * ldd + kk + E * lc)
                       : u32x4{0u, 0u, 0u, 0u};
  }
  sz = *reinterpret_cast<const u32x4*>(Zt + (int64_t)lr * ldd + kk + E * lc);
}

__device__ __forceinline__ void mma_sstore(u32x4* tD, u32x4* tZ, int lr, int lc,
                                           const u32x4 (&st)[4], const u32x4& sz) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int row = lr + 32 * h;
    tD[row * 8 + (lc ^ (row & 7))] = st[h];
  }
  tZ[lr * 8 + (lc ^ (lr & 7))] = sz;
}

__device__ __forceinline__ void mma_store_w(float* __restrict__ Wtpart, int64_t mpad, int64_t r0,
                                            int lane, const f32x16& acc) {
  if (r0 >= mpad) return;
  float* out = Wtpart + ((int64_t)blockIdx.x * 32 + (lane & 31)) * mpad;
#pragma unroll
  for (int v = 0; v < 16; ++v) out[r0 + acc_row(v, lane)] = acc[v];
}

// bf16: a 128-byte step is 64 columns = four 16-wide MFMA slices; lane
// group g takes chunks 4g .. 4g+3 (the K order is the same on both operands).
__global__ __launch_bounds__(256) void k_mm_a_bf16(const uint16_t* __restrict__ D,
                                                   int64_t ldd, int64_t mpad,
                                                   const uint16_t* __restrict__ Zt,
                                                   float* __restrict__ Wtpart,
                                                   int64_t KC) {
  __shared__ u32x4 tD[2][kMmaRows * 8];
  __shared__ u32x4 tZ[2][32 * 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 31, g = lane >> 5;
  const int lr = tid >> 3, lc = tid & 7;
  const int64_t rb = (int64_t)blockIdx.y * kMmaRows;
  const int64_t c0 = (int64_t)blockIdx.x * KC;
  const int64_t c1 = (c0 + KC) < ldd ? (c0 + KC) : ldd;
  const int row = 32 * wave + i;
  u32x4 st[4], sz;
  f32x16 acc = {};
  mma_gload(D, ldd, mpad, Zt, rb, c0, lr, lc, st, sz);
  mma_sstore(tD[0], tZ[0], lr, lc, st, sz);
  __syncthreads();
  int buf = 0;
  for (int64_t kk = c0; kk < c1; kk += 64) {
    const bool more = kk + 64 < c1;
    if (more) mma_gload(D, ldd, mpad, Zt, rb, kk + 64, lr, lc, st, sz);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int ch = 4 * g + s;
      const u32x4 av = tD[buf][row * 8 + (ch ^ (row & 7))];
      const u32x4 bv = tZ[buf][i * 8 + (ch ^ (i & 7))];
      acc = mfma_bf16(as_bf16x8(av), as_bf16x8(bv), acc);
    }
    if (more) mma_sstore(tD[buf ^ 1], tZ[buf ^ 1], lr, lc, st, sz);
    __syncthreads();
    buf ^= 1;
  }
  mma_store_w(Wtpart, mpad, rb + 32 * wave, lane, acc);
}

// f32: a 128-byte step is 32 columns = sixteen 2-wide MFMA slices; slice s
// of lane group g is element s%4 of chunk 2(s/4) + g.
__global__ __launch_bounds__(256) void k_mm_a_f32(const float* __restrict__ D, int64_t ldd,
                                                  int64_t mpad, const float* __restrict__ Zt,
                                                  float* __restrict__ Wtpart, int64_t KC) {
  __shared__ u32x4 tD[2][kMmaRows * 8];
  __shared__ u32x4 tZ[2][32 * 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 31, g = lane >> 5;
  const int lr = tid >> 3, lc = tid & 7;
  const int64_t rb = (int64_t)blockIdx.y * kMmaRows;
  const int64_t c0 = (int64_t)blockIdx.x * KC;
  const int64_t c1 = (c0 + KC) < ldd ? (c0 + KC) : ldd;
  const int row = 32 * wave + i;
  u32x4 st[4], sz;
  // four independent accumulators (one per slot e of a 16-byte chunk), so
  // consecutive MFMAs do not wait on each other; added in a fixed order
  f32x16 acc4[4];
#pragma unroll
  for (int a_ = 0; a_ < 4; ++a_) acc4[a_] = f32x16{};
  mma_gload(D, ldd, mpad, Zt, rb, c0, lr, lc, st, sz);
  mma_sstore(tD[0], tZ[0], lr, lc, st, sz);
  __syncthreads();
  int buf = 0;
  for (int64_t kk = c0; kk < c1; kk += 32) {
    const bool more = kk + 32 < c1;
    if (more) mma_gload(D, ldd, mpad, Zt, rb, kk + 32, lr, lc, st, sz);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ch = 2 * q + g;
      const u32x4 av = tD[buf][row * 8 + (ch ^ (row & 7))];
      const u32x4 bv = tZ[buf][i * 8 + (ch ^ (i & 7))];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        acc4[(4 * q + e) % 4] = mfma_f32(__uint_as_float(av[e]), __uint_as_float(bv[e]),
                                         acc4[(4 * q + e) % 4]);
    }
    if (more) mma_sstore(tD[buf ^ 1], tZ[buf ^ 1], lr, lc, st, sz);
    __syncthreads();
    buf ^= 1;
  }
  f32x16 acc = acc4[0];
#pragma unroll
  for (int a_ = 1; a_ < 4; ++a_) acc += acc4[a_];
  mma_store_w(Wtpart, mpad, rb + 32 * wave, lane, acc);
}

// ---------------------------------------------------------------------------
// k_soft_mm_a_f32 (GreBsmo, Sec. 3.2.1): the soft-thresholding pass of Eq. 12
// fused with the next inner iteration's D V^T (Eq. 13).  Same tiling as
// k_mm_a_f32, but the slab read from HBM is the zero-padded copy Xp of X:
// every 16-byte chunk (four columns of one row) is turned into
//   d = x - S_lambda(x - u_i . v_j)
// in registers (u_i: the thread's four rows of U, kept in registers; v_j:
// rows of V^T read from the panel), written to D, and staged in LDS as the
// A operand of W^T = (D V^T)^T.  Zt holds V^T transposed (the same V), so
// one read of X replaces the soft pass plus one read of D.  Padding rows and
// columns stay zero (U and V^T are zero there).  RP <= 8.
// ---------------------------------------------------------------------------
template <int RP>
__device__ __forceinline__ void soft_load_v(const float* __restrict__ Vt, int64_t col0,
                                            float (&v)[4][RP]) {
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int c = 0; c < RP; ++c) v[e][c] = Vt[(col0 + e) * RP + c];
}

template <int RP>
__device__ __forceinline__ void soft_chunks(u32x4 (&st)[4], const float (&u)[4][RP],
                                            const float (&v)[4][RP], float lam,
                                            float* __restrict__ D, int64_t ldd, int64_t mpad,
                                            int64_t row0, int64_t col0) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int64_t row = row0 + 32 * h;
    float d[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float l = 0.f;
#pragma unroll
      for (int c = 0; c < RP; ++c) l = fma_t(u[h][c], v[e][c], l);
      const float x = __uint_as_float(st[h][e]);
      const float res = x - l;
      const float a = fabsf(res) - lam;
      const float sv = a > 0.f ? copysignf(a, res) : 0.f;
      d[e] = x - sv;
      st[h][e] = __float_as_uint(d[e]);
    }
    if (row < mpad)
      *reinterpret_cast<float4*>(D + row * ldd + col0) = make_float4(d[0], d[1], d[2], d[3]);
  }
}

template <int RP>
__global__ __launch_bounds__(256) void k_soft_mm_a_f32(const float* __restrict__ Xp,
                                                       int64_t ldd, int64_t mpad,
                                                       const float* __restrict__ U,
                                                       const float* __restrict__ Vt,
                                                       float lam, float* __restrict__ D,
                                                       const float* __restrict__ Zt,
                                                       float* __restrict__ Wtpart, int64_t KC) {
  __shared__ u32x4 tD[2][kMmaRows * 8];
  __shared__ u32x4 tZ[2][32 * 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i = lane & 31, g = lane >> 5;
  const int lr = tid >> 3, lc = tid & 7;
  const int64_t rb = (int64_t)blockIdx.y * kMmaRows;
  const int64_t c0 = (int64_t)blockIdx.x * KC;
  const int64_t c1 = (c0 + KC) < ldd ? (c0 + KC) : ldd;
  const int row = 32 * wave + i;
  float u[4][RP], v[4][RP];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int64_t r = rb + lr + 32 * h;
#pragma unroll
    for (int c = 0; c < RP; ++c) u[h][c] = r < mpad ? U[r * RP + c] : 0.f;
  }
  u32x4 st[4], sz;
  f32x16 acc4[4];   // independent accumulators (as k_mm_a_f32)
#pragma unroll
  for (int a_ = 0; a_ < 4; ++a_) acc4[a_] = f32x16{};
  mma_gload(Xp, ldd, mpad, Zt, rb, c0, lr, lc, st, sz);
  soft_load_v<RP>(Vt, c0 + 4 * lc, v);
  soft_chunks<RP>(st, u, v, lam, D, ldd, mpad, rb + lr, c0 + 4 * lc);
  mma_sstore(tD[0], tZ[0], lr, lc, st, sz);
  __syncthreads();
  int buf = 0;
  for (int64_t kk = c0; kk < c1; kk += 32) {
    const bool more = kk + 32 < c1;
    if (more) {
      mma_gload(Xp, ldd, mpad, Zt, rb, kk + 32, lr, lc, st, sz);
      soft_load_v<RP>(Vt, kk + 32 + 4 * lc, v);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ch = 2 * q + g;
      const u32x4 av = tD[buf][row * 8 + (ch ^ (row & 7))];
      const u32x4 bv = tZ[buf][i * 8 + (ch ^ (i & 7))];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        acc4[(4 * q + e) % 4] = mfma_f32(__uint_as_float(av[e]), __uint_as_float(bv[e]),
                                         acc4[(4 * q + e) % 4]);
    }
    if (more) {
      soft_chunks<RP>(st, u, v, lam, D, ldd, mpad, rb + lr, kk + 32 + 4 * lc);
      mma_sstore(tD[buf ^ 1], tZ[buf ^ 1], lr, lc, st, sz);
    }
    __syncthreads();
    buf ^= 1;
  }
  f32x16 acc = acc4[0];
#pragma unroll
  for (int a_ = 1; a_ < 4; ++a_) acc += acc4[a_];
  mma_store_w(Wtpart, mpad, rb + 32 * wave, lane, acc);
}

// ---------------------------------------------------------------------------
// k_mm_b: Zpart[ch] (ldd x zs, row = column of D) = (W^T D[rows of ch, :])^T.
// Block = 4 waves on the same 128-column strip [blockIdx.x*128, +128): lane n
// holds columns 4n .. 4n+3 of the strip, one per 32-column MFMA tile, so a
// wave reads each row as one contiguous run.  The waves split the rows of
// the chunk into four ranges and add their tiles through LDS at the end;
// only the zs = zpart_stride(rp) leading entries of each output row are
// stored (the rest of the 32-wide tile is padding).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mmb_store(const f32x16 (&acc)[4], int lane, int zs,
                                          float* __restrict__ Zpart, int64_t row0) {
  const int n = lane & 31;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float* out = Zpart + (row0 + 4 * n + t) * zs;
#pragma unroll
    for (int v = 0; v < 16; v += 4) {
      const int i0 = acc_row(v, lane);
      if (i0 < zs)
        *reinterpret_cast<float4*>(out + i0) =
            make_float4(acc[t][v], acc[t][v + 1], acc[t][v + 2], acc[t][v + 3]);
    }
  }
}

__global__ __launch_bounds__(256) void k_mm_b_bf16(const uint16_t* __restrict__ D, int64_t ldd,
                                                   int64_t mpad,
                                                   const uint16_t* __restrict__ Wt,
                                                   float* __restrict__ Zpart, int64_t RC,
                                                   int zs) {
  __shared__ float lds[2 * 64 * 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t cw = (int64_t)blockIdx.x * 128;
  const int64_t kc0 = (int64_t)blockIdx.y * RC;
  const int64_t kc1 = (kc0 + RC) < mpad ? (kc0 + RC) : mpad;
  int64_t k0, k1;
  mmb_wave_rows(kc0, kc1, wave, 16, k0, k1);
  f32x16 acc[4] = {};
  mmb_loop_bf16(D, ldd, mpad, Wt, cw, k0, k1, lane, acc);
  mmb_block_reduce(acc, lds, wave, lane);
  if (wave == 0) mmb_store(acc, lane, zs, Zpart, (int64_t)blockIdx.y * ldd + cw);
}

__global__ __launch_bounds__(256) void k_mm_b_f32(const float* __restrict__ D, int64_t ldd,
                                                  int64_t mpad, const float* __restrict__ Wt,
                                                  float* __restrict__ Zpart, int64_t RC,
                                                  int zs) {
  __shared__ float lds[2 * 64 * 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t cw = (int64_t)blockIdx.x * 128;
  const int64_t kc0 = (int64_t)blockIdx.y * RC;
  const int64_t kc1 = (kc0 + RC) < mpad ? (kc0 + RC) : mpad;
  int64_t k0, k1;
  mmb_wave_rows(kc0, kc1, wave, 8, k0, k1);
  f32x16 acc[4] = {};
  mmb_loop_f32(D, ldd, mpad, Wt, cw, k0, k1, lane, acc);
  mmb_block_reduce(acc, lds, wave, lane);
  if (wave == 0) mmb_store(acc, lane, zs, Zpart, (int64_t)blockIdx.y * ldd + cw);
}

// ---------------------------------------------------------------------------
// Panel conversions around the MFMA kernels.
// ---------------------------------------------------------------------------
// Zt (32 x ldd, bf16 or f32) <- Z (ldd x rp, f32), zero rows j >= rp.
template <typename TT>
__global__ __launch_bounds__(256) void k_to_t(const float* __restrict__ Z, int64_t rows, int rp,
                                              TT* __restrict__ Zt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * 32) return;
  const int64_t j = e / rows, c = e % rows;
  const float v = (j < rp) ? Z[c * rp + j] : 0.f;
  if constexpr (sizeof(TT) == 2)
    Zt[e] = f32_to_bf16(v);
  else
    Zt[e] = v;
}

// Wt = sum_ct Wtpart[ct] (32 x mpad) -> TT (bf16 or f32) transposed panel,
// and optionally row-major rows x rp f32 (for B' = D Y).
template <typename TT>
__global__ __launch_bounds__(256) void k_reduce_w(const float* __restrict__ Wtpart, int nct,
                                                  int64_t mpad, int64_t m, int rp,
                                                  TT* __restrict__ Wt, float* __restrict__ Wrow) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= 32 * mpad) return;
  float s = 0.f;
  for (int c = 0; c < nct; ++c) s += Wtpart[(int64_t)c * 32 * mpad + e];
  if (Wt) {
    if constexpr (sizeof(TT) == 2)
      Wt[e] = f32_to_bf16(s);
    else
      Wt[e] = s;
  }
  if (Wrow) {
    const int64_t j = e / mpad, i = e % mpad;
    if (j < rp && i < m) Wrow[i * rp + j] = s;
  }
}

// Zo (ldd x rp, f32) = sum_ch Zpart[ch] (ldd x 32).  One block per 16
// consecutive outputs e = c * rp + j: each of 16 chunk lanes adds every 16th
// chunk (ascending), then the lane sums are added in lane order, so the
// result does not depend on scheduling.  Many short chains instead of one
// long one per output keep enough loads in flight when there are many
// chunks and few outputs (narrow matrices).
constexpr int kRzVals = 16;
constexpr int kRzLanes = 16;
__global__ __launch_bounds__(256) void k_reduce_z(const float* __restrict__ Zpart, int64_t nch,
                                                  int64_t ldd, int rp, float* __restrict__ Zo) {
  __shared__ float red[kRzLanes][kRzVals];
  const int v = threadIdx.x % kRzVals, hl = threadIdx.x / kRzVals;
  const int64_t e = (int64_t)blockIdx.x * kRzVals + v;
  const bool live = e < ldd * rp;
  float s = 0.f;
  if (live) {
    const int zs = zpart_stride(rp);
    const float* p = Zpart + (e / rp) * zs + (e % rp);
    const int64_t step = ldd * zs;
    int64_t h = hl;
    for (; h + 3 * kRzLanes < nch; h += 4 * kRzLanes) {
      const float a0 = p[h * step];
      const float a1 = p[(h + kRzLanes) * step];
      const float a2 = p[(h + 2 * kRzLanes) * step];
      const float a3 = p[(h + 3 * kRzLanes) * step];
      s += a0;
      s += a1;
      s += a2;
      s += a3;
    }
    for (; h < nch; h += kRzLanes) s += p[h * step];
  }
  red[hl][v] = s;
  __syncthreads();
  if (hl == 0 && live) {
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < kRzLanes; ++q) t += red[q][v];
    Zo[e] = t;
  }
}

// ---------------------------------------------------------------------------
// Host side: one Gram pass Zo = D^T (D Z) and the plain product W = D Y.
// ---------------------------------------------------------------------------
static unsigned blocks_for(int64_t work) { return (unsigned)((work + 255) / 256); }

void mfma_to_t(const Launch& L, bool bf16, const void* Z, int64_t ldd, int rp, void* Zt) {
  if (bf16)
    hipLaunchKernelGGL(k_to_t<uint16_t>, dim3(blocks_for(ldd * 32)), dim3(256), 0, L.stream,
                       (const float*)Z, ldd, rp, (uint16_t*)Zt);
  else
    hipLaunchKernelGGL(k_to_t<float>, dim3(blocks_for(ldd * 32)), dim3(256), 0, L.stream,
                       (const float*)Z, ldd, rp, (float*)Zt);
}

// ev_a/ev_b (optional): events that receive the kernel's own start and end
// timestamps (timing mode).
void mfma_mm_a(const Launch& L, bool bf16, const void* D, int64_t ldd, int64_t mpad,
               const void* Zt, float* Wtpart, int64_t KC, hipEvent_t ev_a, hipEvent_t ev_b) {
  dim3 grid((unsigned)((ldd + KC - 1) / KC), (unsigned)((mpad + kMmaRows - 1) / kMmaRows));
  if (bf16)
    hipExtLaunchKernelGGL(k_mm_a_bf16, grid, dim3(256), 0, L.stream, ev_a, ev_b, 0,
                          (const uint16_t*)D, ldd, mpad, (const uint16_t*)Zt, Wtpart, KC);
  else
    hipExtLaunchKernelGGL(k_mm_a_f32, grid, dim3(256), 0, L.stream, ev_a, ev_b, 0,
                          (const float*)D, ldd, mpad, (const float*)Zt, Wtpart, KC);
}

void mfma_reduce_w(const Launch& L, bool bf16, const float* Wtpart, int nct, int64_t mpad,
                   int64_t m, int rp, void* Wt, float* Wrow) {
  const unsigned b = blocks_for(32 * mpad);
  if (bf16)
    hipLaunchKernelGGL(k_reduce_w<uint16_t>, dim3(b), dim3(256), 0, L.stream, Wtpart, nct, mpad,
                       m, rp, (uint16_t*)Wt, Wrow);
  else
    hipLaunchKernelGGL(k_reduce_w<float>, dim3(b), dim3(256), 0, L.stream, Wtpart, nct, mpad, m,
                       rp, (float*)Wt, Wrow);
}

void mfma_mm_b(const Launch& L, bool bf16, const void* D, int64_t ldd, int64_t mpad,
               const void* Wt, float* Zpart, int64_t RC, int64_t nch, int rp, hipEvent_t ev_a,
               hipEvent_t ev_b) {
  dim3 grid((unsigned)(ldd / 128), (unsigned)nch);
  const int zs = zpart_stride(rp);
  if (bf16)
    hipExtLaunchKernelGGL(k_mm_b_bf16, grid, dim3(256), 0, L.stream, ev_a, ev_b, 0,
                          (const uint16_t*)D, ldd, mpad, (const uint16_t*)Wt, Zpart, RC, zs);
  else
    hipExtLaunchKernelGGL(k_mm_b_f32, grid, dim3(256), 0, L.stream, ev_a, ev_b, 0,
                          (const float*)D, ldd, mpad, (const float*)Wt, Zpart, RC, zs);
}

void mfma_reduce_z(const Launch& L, const float* Zpart, int64_t nch, int64_t ldd, int rp,
                   float* Zo) {
  const unsigned b = (unsigned)((ldd * rp + kRzVals - 1) / kRzVals);
  hipLaunchKernelGGL(k_reduce_z, dim3(b), dim3(256), 0, L.stream, Zpart, nch, ldd, rp, Zo);
}

bool mfma_soft_mm_a(const Launch& L, int rp, const float* Xp, int64_t ldd, int64_t mpad,
                    const float* U, const float* Vt, float lam, float* D, const float* Zt,
                    float* Wtpart, int64_t KC) {
  dim3 grid((unsigned)((ldd + KC - 1) / KC), (unsigned)((mpad + kMmaRows - 1) / kMmaRows));
  switch (rp) {
#define GB_SOFT_CASE(R)                                                                      \
  case R:                                                                                    \
    hipLaunchKernelGGL(k_soft_mm_a_f32<R>, grid, dim3(256), 0, L.stream, Xp, ldd, mpad, U, Vt, \
                       lam, D, Zt, Wtpart, KC);                                              \
    return true;
    GB_SOFT_CASE(1)
    GB_SOFT_CASE(2)
    GB_SOFT_CASE(4)
    GB_SOFT_CASE(8)
#undef GB_SOFT_CASE
    default:
      return false;
  }
}

}  // namespace godec
