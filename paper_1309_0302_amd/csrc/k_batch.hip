// Batched GoDec: many independent FP32 problems X_i (m_i x n_i, n_i small),
// every phase of Algorithm 1 in one launch over all of them.
//
// Streaming phases walk a flat list of work items, each a problem and a
// range of its rows; the problems' r x r work runs one workgroup per problem
// (k_small.hip).  Panels are kBatchRP = 8 columns wide for every problem;
// columns at or past a problem's rank stay zero.
//
// Gram pass (Algorithm 1's products with L~ and L~^T, Sec. 3.1.3): because
// n_i is small, one work item holds a 16-row slab of D in LDS together with
// the whole n x 8 panel Z, forms W = D_slab Z and immediately accumulates
// D_slab^T W, so each pass reads D once (the single-problem path reads it
// twice, since its panel is too long for LDS).
//
// Sparse step (Eq. 4): a level-0 histogram pass over every problem, a
// collection pass of the entries at or above each problem's bucket, and the
// remaining radix digits resolved over the candidates; ties at the threshold
// are taken by row-major index, smallest first, and exact zeros are never
// selected.
#include "godec_internal.h"
#include "k_common.h"

#include <algorithm>

namespace godec {

constexpr int RP8 = kBatchRP;

__device__ __forceinline__ const float* bpanel(const BProb& b, int which) {
  return which == 0 ? b.P0 : (which == 1 ? b.P1 : b.VL);
}

// Residual entry with a fixed multiply-add order (selection, compaction and
// the residual getter all use it).
__device__ __forceinline__ float bresid(float x, const float* u, const float* v) {
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < RP8; ++c) s = fmaf(u[c], v[c], s);
  return x - s;
}

__device__ __forceinline__ uint32_t fkey(float r) { return __float_as_uint(r) & 0x7fffffffu; }

// ---------------------------------------------------------------------------
// Chain kernels.
// ---------------------------------------------------------------------------

// P0 <- A1 (columns at or past r_eff zero).
__global__ __launch_bounds__(256) void kb_copy_a1(const BProb* __restrict__ probs) {
  const BProb& b = probs[blockIdx.y];
  const int reff = b.st->r_eff;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= b.n * RP8) return;
  const int64_t j = e / RP8;
  const int c = (int)(e % RP8);
  b.P0[e] = (c < reff && c < b.r) ? (float)b.A1[j * b.r + c] : 0.f;
}

// Gram pass (MODE 0): zslots[item] = D_rows^T (D_rows Z); apply (MODE 1):
// Bp[rows] = D_rows Z and the FP64 Gram of those Bp rows into gslots[item].
//
// On the matrix cores, v_mfma_f32_16x16x4f32 (lane l: A row l%16 and B
// column l%16 at k = l/16; accumulator register v holds C[4(l/16)+v][l%16]).
// Per 16-row slab of D (in LDS):
//   (a) W = D_slab Z (16 x 8): the 4 waves split the contraction over n in
//       16-wide steps; a lane reads 4 consecutive k with one 16-byte load and
//       feeds them to 4 MFMAs (same k order on both operands); the 4 partial
//       W go through LDS.
//   (b) Zout^T += W^T D_slab (8 x n): wave w owns column tiles w, w+4, ...
//       of 16 columns, whose accumulators live across the whole work item.
// The next slab is loaded into registers while the current one is used.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void kb_pass(const BProb* __restrict__ probs,
                                               const BItem* __restrict__ items, int in,
                                               float* __restrict__ zslots,
                                               double* __restrict__ gslots) {
  constexpr int LDT = kBatchMaxN + 4;          // LDS row stride of the D slab
  constexpr int PF = kBatchSub * (kBatchMaxN / 4) / 256;   // prefetch float4 per thread
  constexpr int MAXT = kBatchMaxN / 16 / 4;    // column tiles per wave
  __shared__ float zt[RP8][kBatchMaxN + 4];    // Z^T (zero past n); padded rows: no bank conflicts
  __shared__ float dt[kBatchSub * LDT];        // D slab (zero past ldd)
  __shared__ float wp[4][kBatchSub][RP8];      // per-wave partial W
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kg = lane >> 4;
  const BItem it = items[blockIdx.x];
  const BProb& b = probs[it.prob];
  const int n = (int)b.n;
  const int64_t ldd = b.ldd;
  const int n16 = (n + 15) & ~15;
  const int q4 = (int)(ldd / 4);
  const float* Z = bpanel(b, in);
  // Z^T over the columns the products read (j < n16): one row of Z (two
  // 16-byte loads) per thread
  static_assert(RP8 == 8, "the panel rows are two float4");
  for (int j = tid; j < n16; j += 256) {
    float4 z0 = make_float4(0.f, 0.f, 0.f, 0.f), z1 = z0;
    if (j < n) {
      z0 = *reinterpret_cast<const float4*>(Z + (int64_t)j * RP8);
      z1 = *reinterpret_cast<const float4*>(Z + (int64_t)j * RP8 + 4);
    }
    zt[0][j] = z0.x; zt[1][j] = z0.y; zt[2][j] = z0.z; zt[3][j] = z0.w;
    zt[4][j] = z1.x; zt[5][j] = z1.y; zt[6][j] = z1.z; zt[7][j] = z1.w;
  }
  // columns [ldd, n16) of the slab are never loaded: zero them once
  for (int e = tid; e < kBatchSub * 16; e += 256) {
    const int row = e / 16, c = (int)ldd + e % 16;
    if (c < n16) dt[row * LDT + c] = 0.f;
  }
  f32x4 acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  double g = 0.0;                              // MODE 1: Gram entry tid < 64
  const int ga = tid / RP8, gb = tid % RP8;
  float4 pf[PF];
  // thread's float4 number u of a slab: e = tid + 256 u, row e / q4 and
  // column group e % q4; e / q4 = (e Rq) >> 20 with Rq = ceil(2^20 / q4), exact
  // for e < 2^11 and q4 <= 2^7 (the rounding adds less than 2^-9, below the
  // 1/q4 gap).  Recomputed where used rather than kept in registers.
  static_assert(kBatchSub * (kBatchMaxN / 4) <= 2048 && kBatchMaxN / 4 <= 128, "range of Rq");
  const uint32_t Rq = ((1u << 20) + (uint32_t)q4 - 1u) / (uint32_t)q4;
  auto slab_pos = [&](int u, int& row, int& off) {
    const int e = tid + 256 * u;
    row = (int)(((uint32_t)e * Rq) >> 20);
    off = 4 * (e - row * q4);
  };
  auto prefetch = [&](int64_t i0, int nr) {
    const float* base = b.D + i0 * ldd;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      int row, off;
      slab_pos(u, row, off);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (row < nr) v = *reinterpret_cast<const float4*>(base + (int64_t)row * ldd + off);
      pf[u] = v;
    }
  };
  int nr = (it.i1 - it.i0) < kBatchSub ? (int)(it.i1 - it.i0) : kBatchSub;
  prefetch(it.i0, nr);
  for (int64_t i0 = it.i0; i0 < it.i1; i0 += kBatchSub) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      int row, off;
      slab_pos(u, row, off);
      if (row < kBatchSub) *reinterpret_cast<float4*>(&dt[row * LDT + off]) = pf[u];
    }
    __syncthreads();
    const int cur_nr = nr;
    const int64_t nx = i0 + kBatchSub;
    if (nx < it.i1) {
      nr = (it.i1 - nx) < kBatchSub ? (int)(it.i1 - nx) : kBatchSub;
      prefetch(nx, nr);
    }
    // (a) partial W of this wave's k steps
    f32x4 wa = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 16 * wave; k0 < n16; k0 += 64) {
      const float4 av = *reinterpret_cast<const float4*>(&dt[li * LDT + k0 + 4 * kg]);
      float4 bv = make_float4(0.f, 0.f, 0.f, 0.f);
      if (li < RP8) bv = *reinterpret_cast<const float4*>(&zt[li][k0 + 4 * kg]);
      wa = mfma16(av.x, bv.x, wa);
      wa = mfma16(av.y, bv.y, wa);
      wa = mfma16(av.z, bv.z, wa);
      wa = mfma16(av.w, bv.w, wa);
    }
    if (li < RP8) {
#pragma unroll
      for (int v = 0; v < 4; ++v) wp[wave][4 * kg + v][li] = wa[v];
    }
    __syncthreads();
    if constexpr (MODE == 0) {
      // (b) this lane's W^T operand: W[4 kg + s][li] for s = 0..3 (li < 8)
      float wt[4];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        const int i = 4 * kg + s2;
        wt[s2] = (li < RP8 && i < cur_nr)
                     ? (wp[0][i][li] + wp[1][i][li]) + (wp[2][i][li] + wp[3][i][li])
                     : 0.f;
      }
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        const int j0 = 16 * (wave + 4 * t);
        if (j0 < n16) {
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2) {
            const int i = 4 * kg + s2;
            acc[t] = mfma16(wt[s2], dt[i * LDT + j0 + li], acc[t]);
          }
        }
      }
    } else {
      if (tid < cur_nr * RP8) {
        const int i = tid / RP8, c = tid % RP8;
        b.Bp[(i0 + i) * RP8 + c] = (wp[0][i][c] + wp[1][i][c]) + (wp[2][i][c] + wp[3][i][c]);
      }
      if (tid < RP8 * RP8) {
        for (int i = 0; i < cur_nr; ++i) {
          const float wa_ = (wp[0][i][ga] + wp[1][i][ga]) + (wp[2][i][ga] + wp[3][i][ga]);
          const float wb_ = (wp[0][i][gb] + wp[1][i][gb]) + (wp[2][i][gb] + wp[3][i][gb]);
          g = fma((double)wa_, (double)wb_, g);
        }
      }
    }
  }
  if constexpr (MODE == 0) {
    // lane holds Zout^T[4 kg + v][j0 + li]; rows 0..7 are the panel columns
    if (kg < 2) {
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        const int j = 16 * (wave + 4 * t) + li;
        if (j < n) {
#pragma unroll
          for (int v = 0; v < 4; ++v) zslots[it.zoff + (int64_t)j * RP8 + 4 * kg + v] = acc[t][v];
        }
      }
    }
  } else {
    if (tid < RP8 * RP8) gslots[(int64_t)blockIdx.x * RP8 * RP8 + tid] = g;
  }
}

// P1 = sum of the problem's Gram-pass partials, in item order.
__global__ __launch_bounds__(256) void kb_reduce_slots(const BProb* __restrict__ probs,
                                                       const BItem* __restrict__ items,
                                                       const float* __restrict__ zslots) {
  const BProb& b = probs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= b.n * RP8) return;
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  int it = 0;
  for (; it + 7 < b.nitems; it += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += zslots[items[b.item0 + it + u].zoff + e];
  }
  for (; it < b.nitems; ++it) a[0] += zslots[items[b.item0 + it].zoff + e];
  b.P1[e] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// U_L = B' K' (m x 8).
__global__ __launch_bounds__(256) void kb_apply_k(const BProb* __restrict__ probs) {
  const BProb& b = probs[blockIdx.y];
  __shared__ float ks[RP8 * RP8];
  if (threadIdx.x < RP8 * RP8) ks[threadIdx.x] = b.Kp[threadIdx.x];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= b.m * RP8) return;
  const int64_t i = e / RP8;
  const int c = (int)(e % RP8);
  float s = 0.f;
#pragma unroll
  for (int l = 0; l < RP8; ++l) s = fmaf(b.Bp[i * RP8 + l], ks[l * RP8 + c], s);
  b.UL[e] = s;
}

// ---------------------------------------------------------------------------
// Full-data passes of the sparse step.  Threads own columns (their V_L rows
// in registers); a block covers `rg` rows at once when the row is short.
// ---------------------------------------------------------------------------
struct ColMap {
  int lanes;   // threads per row (multiple of 64, >= n unless two columns each)
  int rg;      // rows processed together
  int cpt;     // columns per thread (1 or 2)
};

__device__ __forceinline__ ColMap colmap(int n) {
  ColMap cm;
  const int r64 = ((n + 63) / 64) * 64;
  if (r64 <= 256) {
    cm.lanes = r64;
    cm.rg = 256 / r64;
    cm.cpt = 1;
  } else {
    cm.lanes = 256;
    cm.rg = 1;
    cm.cpt = 2;
  }
  return cm;
}

// Candidate segment of wave w of a work item of R rows: the wave's thread
// map covers ceil(R / rg) rows of 64 * cpt positions, so it cannot write more.
__device__ __forceinline__ int64_t wave_seg_cap(int R, const ColMap& cm) {
  return (int64_t)((R + cm.rg - 1) / cm.rg) * 64 * cm.cpt;
}

// KIND 0 (problems in BS_HIST): level-0 histogram, sum of R^2, NaN check.
// KIND 1 (BS_COLLECT): collect the entries at or above the bucket.
// KIND 2 (BS_CARRY): sum of R^2 and NaN check; histogram and collect the
// entries whose level-0 digit lies in the carried window.
// The item's U_L rows are staged in LDS; each wave appends to its own
// candidate segment with a wave-uniform fill counter (no atomics).  The
// problem's fields are read once into registers, and the row loop is
// compiled for one or two columns per thread (a block-uniform choice).
struct SelArgs {
  const float* X;
  int64_t ldx, n, i0, segw;
  int32_t* cand_idx;
  float* cand_val;
  float* cand_x;
  uint32_t klo;
  bool add_s2;
};

template <int KIND, int CPT>
__device__ __forceinline__ void sel_rows(const SelArgs& A, const ColMap& cm, int R, int rsub,
                                         int col0, const float* us, const float (&v)[2][RP8],
                                         unsigned int* lh, unsigned int& fill, double& s2,
                                         int& bad) {
  const int rows_w = (R + cm.rg - 1) / cm.rg;   // same trip count for every thread
  const int n = (int)A.n;
  constexpr int G = 8;                           // rows whose X loads are in flight together
  for (int t0 = 0; t0 < rows_w; t0 += G) {
    float x[G][CPT];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int ir = rsub + cm.rg * (t0 + g);
      const bool rok = rsub < cm.rg && t0 + g < rows_w && ir < R;
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int j = col0 + 256 * u;
        x[g][u] = (rok && j < n) ? A.X[(A.i0 + ir) * A.ldx + j] : 0.f;
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (t0 + g >= rows_w) break;               // uniform
      const int ir = rsub + cm.rg * (t0 + g);
      const bool rok = rsub < cm.rg && ir < R;
      float uu[RP8];
      {
        const int ro = rok ? ir : 0;
        const float4 u0 = *reinterpret_cast<const float4*>(&us[ro * RP8]);
        const float4 u1 = *reinterpret_cast<const float4*>(&us[ro * RP8 + 4]);
        uu[0] = u0.x; uu[1] = u0.y; uu[2] = u0.z; uu[3] = u0.w;
        uu[4] = u1.x; uu[5] = u1.y; uu[6] = u1.z; uu[7] = u1.w;
      }
      const int64_t i = A.i0 + ir;
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int j = col0 + 256 * u;
        const bool ok = rok && j < n;
        const float r = bresid(x[g][u], uu, v[u]);
        const uint32_t key = fkey(r);
        if (KIND == 0) {
          if (ok) {
            if (A.add_s2) s2 += (double)r * (double)r;
            atomicAdd(&lh[key >> (31 - kHistBits0)], 1u);
            if (!isfinite(x[g][u])) bad = 1;
          }
        } else {
          const bool take = ok && key >= A.klo;
          if (KIND == 2 && ok) {
            s2 += (double)r * (double)r;
            if (!isfinite(x[g][u])) bad = 1;
            if (take) atomicAdd(&lh[key >> (31 - kHistBits0)], 1u);
          }
          const unsigned long long mask = __ballot(take);
          if (mask) {
            const unsigned int lo = (unsigned int)mask, hi = (unsigned int)(mask >> 32);
            const unsigned int rank = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
            if (take) {
              const int64_t pos = A.segw + fill + rank;
              A.cand_idx[pos] = (int32_t)(i * n + j);
              A.cand_val[pos] = r;
              A.cand_x[pos] = x[g][u];
            }
            fill += (unsigned int)__popcll(mask);
          }
        }
      }
    }
  }
}

// LDS: the histogram, then the item's U_L rows (dynamic size: kHistBins
// words plus the most rows of a work item times 8 floats).
template <int KIND>
__global__ __launch_bounds__(256) void kb_sel_pass(const BProb* __restrict__ probs,
                                                   const BItem* __restrict__ items,
                                                   unsigned int* __restrict__ seg_count,
                                                   double* __restrict__ s2slot) {
  extern __shared__ __align__(16) unsigned char sel_lds[];
  unsigned int* lh = reinterpret_cast<unsigned int*>(sel_lds);
  float* us = reinterpret_cast<float*>(sel_lds + sizeof(unsigned int) * kHistBins);
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const BItem it = items[blockIdx.x];
  const BProb& b = probs[it.prob];
  BSel* sel = b.sel;
  const int want = KIND == 0 ? BS_HIST : (KIND == 1 ? BS_COLLECT : BS_CARRY);
  // k == 0 (BS_NONE) problems take the histogram pass for the objective alone
  if (sel->mode != want && !(KIND == 0 && sel->mode == BS_NONE)) return;
  const int n = (int)b.n;
  const ColMap cm = colmap(n);
  const int rsub = tid / cm.lanes;
  const int col0 = tid % cm.lanes;
  SelArgs A;
  A.X = b.X;
  A.ldx = b.ldx;
  A.n = b.n;
  A.i0 = it.i0;
  A.cand_idx = b.cand_idx;
  A.cand_val = b.cand_val;
  A.cand_x = b.cand_x;
  A.add_s2 = KIND == 2 || (KIND == 0 && !sel->s2_done);
  uint32_t klo = 1u;
  if (KIND == 1) {
    const int pb = sel->pbits;
    klo = (uint32_t)(sel->prefix << (31 - pb));
  } else if (KIND == 2) {
    klo = (uint32_t)sel->carry_dlo << (31 - kHistBits0);
  }
  A.klo = klo < 1u ? 1u : klo;
  if (KIND != 1)
    for (int e = tid; e < kHistBins; e += 256) lh[e] = 0u;
  const int R = (int)(it.i1 - it.i0);
  const float* ULb = b.UL + it.i0 * RP8;
  for (int e = tid; e < R * RP8; e += 256) us[e] = ULb[e];
  __syncthreads();
  float v[2][RP8];
  const float* VLb = b.VL;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int j = col0 + 256 * u;
#pragma unroll
    for (int c = 0; c < RP8; ++c) v[u][c] = (u < cm.cpt && j < n) ? VLb[(int64_t)j * RP8 + c] : 0.f;
  }
  A.segw = it.i0 * b.rowcap + (int64_t)wave * wave_seg_cap(R, cm);
  unsigned int fill = 0u;                        // wave-uniform
  double s2 = 0.0;
  int bad = 0;
  if (cm.cpt == 1)
    sel_rows<KIND, 1>(A, cm, R, rsub, col0, us, v, lh, fill, s2, bad);
  else
    sel_rows<KIND, 2>(A, cm, R, rsub, col0, us, v, lh, fill, s2, bad);
  if (KIND != 0 && lane == 0) seg_count[(int64_t)blockIdx.x * 4 + wave] = fill;
  if (KIND != 1) {
    __syncthreads();
    for (int e = tid; e < kHistBins; e += 256)
      if (lh[e]) atomicAdd(&b.hist[e], lh[e]);
    s2 = wave_sum(s2);
    if (lane == 0) red[wave] = s2;
    if (bad) atomicOr(&sel->nonfinite, 1);
    __syncthreads();
    // per-item partial of sum R^2 (one pass per problem and iteration writes
    // it); kb_ties adds the problem's items in order
    if (tid == 0 && A.add_s2) s2slot[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
  }
}

// Reset of the per-problem selection state (one workgroup per problem).
__global__ __launch_bounds__(256) void kb_sel_reset(const BProb* __restrict__ probs) {
  const BProb& b = probs[blockIdx.x];
  for (int e = threadIdx.x; e < kHistBins; e += 256) b.hist[e] = 0u;
  if (threadIdx.x == 0) {
    BSel* s = b.sel;
    s->prefix = 0; s->k_rem = b.k; s->count_above = 0; s->ncand = 0; s->nabove = 0;
    s->nties = 0; s->nnz = 0; s->pbits = 0; s->s2_done = 0;
    s->mode = b.k > 0 ? (s->carry_valid ? BS_CARRY : BS_HIST) : BS_NONE;
    s->sum_r2 = 0.0; s->sum_sel2 = 0.0; s->threshold = 0.0;
  }
}

// Digit selection over a histogram of `bins` counts (one workgroup per
// problem): the digit holding the k_rem-th largest key, by a suffix scan.
// level 0 follows the full-data histogram (BS_HIST), level -1 the carried
// window (BS_CARRY), later levels the candidates' histograms (BS_REFINE).
// A carried window is accepted when the k-th key's digit lies inside it (all
// keys at or above that digit were collected); otherwise the problem falls
// back to the full histogram pass.
__global__ __launch_bounds__(256) void kb_sel_plan(const BProb* __restrict__ probs, int level) {
  __shared__ unsigned long long h[kHistBins];
  __shared__ unsigned long long part[256];
  __shared__ int sel_t;
  const BProb& b = probs[blockIdx.x];
  BSel* s = b.sel;
  const int tid = threadIdx.x;
  const int want = level < 0 ? BS_CARRY : (level == 0 ? BS_HIST : BS_REFINE);
  if (s->mode != want) return;
  const int pbits = s->pbits;
  const int dbits = level <= 0 ? kHistBits0 : (31 - pbits < kHistBits ? 31 - pbits : kHistBits);
  const int bins = 1 << dbits;
  const int per = (bins + 255) / 256;
  for (int e = tid; e < bins; e += 256) {
    h[e] = b.hist[e];
    b.hist[e] = 0u;
  }
  __syncthreads();
  unsigned long long acc = 0;
  for (int u = 0; u < per; ++u) {
    const int d = bins - 1 - (tid * per + u);
    if (d >= 0) acc += h[d];
  }
  part[tid] = acc;
  if (tid == 0) sel_t = -1;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const unsigned long long add = tid >= off ? part[tid - off] : 0ull;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  const long long k_rem = s->k_rem;
  const unsigned long long before = tid > 0 ? part[tid - 1] : 0ull;
  if (before < (unsigned long long)k_rem && part[tid] >= (unsigned long long)k_rem) sel_t = tid;
  __syncthreads();
  if (tid != 0) return;
  int dsel = -1;
  unsigned long long cum = 0;
  if (sel_t >= 0) {
    cum = sel_t > 0 ? part[sel_t - 1] : 0ull;
    for (int u = 0; u < per; ++u) {
      const int d = bins - 1 - (sel_t * per + u);
      if (d < 0) break;
      if (cum + h[d] >= (unsigned long long)k_rem) { dsel = d; break; }
      cum += h[d];
    }
  }
  if (level < 0) {
    if (dsel < 0 || dsel < s->carry_dlo) {
      // window missed the k-th key: full histogram pass (R^2 already summed)
      s->s2_done = 1;
      s->mode = BS_HIST;
      return;
    }
    s->count_above = (long long)cum;
    s->k_rem = k_rem - (long long)cum;
    s->prefix = (unsigned long long)dsel;
    s->pbits = dbits;
    s->mode = BS_REFINE;
    return;
  }
  if (dsel < 0) {
    // fewer nonzero keys than k_rem: settle on digit 0 (zeros are excluded
    // from the candidates)
    dsel = 0;
    cum = part[255] - h[0];
  }
  s->count_above += (long long)cum;
  s->k_rem = k_rem - (long long)cum;
  s->prefix = (s->prefix << dbits) | (unsigned long long)dsel;
  s->pbits = pbits + dbits;
  if (level == 0) s->mode = BS_COLLECT;
  else s->mode = s->pbits == 31 ? BS_FINAL : BS_REFINE;
}

// After the collection pass: move to candidate refinement.
__global__ __launch_bounds__(64) void kb_sel_to_refine(const BProb* __restrict__ probs,
                                                       int nprob) {
  const int p = blockIdx.x * 64 + threadIdx.x;
  if (p >= nprob) return;
  BSel* s = probs[p].sel;
  if (s->mode == BS_COLLECT) s->mode = s->pbits == 31 ? BS_FINAL : BS_REFINE;
}

// Histogram of the next digit over the candidates inside the bucket.  The
// blocks of a problem take its work items' candidate segments in turn.
__global__ __launch_bounds__(256) void kb_cand_hist(const BProb* __restrict__ probs,
                                                    const BItem* __restrict__ items,
                                                    const unsigned int* __restrict__ seg_count) {
  __shared__ unsigned int lh[1 << kHistBits];
  const BProb& b = probs[blockIdx.y];
  const BSel* s = b.sel;
  if (s->mode != BS_REFINE) return;
  const int pbits = s->pbits;
  const int dbits = 31 - pbits < kHistBits ? 31 - pbits : kHistBits;
  const unsigned long long prefix = s->prefix;
  for (int e = threadIdx.x; e < (1 << dbits); e += 256) lh[e] = 0u;
  __syncthreads();
  const ColMap cm = colmap((int)b.n);
  for (int sg = blockIdx.x; sg < b.nitems * 4; sg += gridDim.x) {
    const int item = b.item0 + sg / 4, w = sg % 4;
    const BItem itm = items[item];
    const int64_t c0 = itm.i0 * b.rowcap + (int64_t)w * wave_seg_cap((int)(itm.i1 - itm.i0), cm);
    const int64_t c1 = c0 + seg_count[(int64_t)item * 4 + w];
    for (int64_t c = c0 + threadIdx.x; c < c1; c += 256) {
      const uint32_t key = fkey(b.cand_val[c]);
      if ((key >> (31 - pbits)) == prefix)
        atomicAdd(&lh[(key >> (31 - pbits - dbits)) & ((1u << dbits) - 1)], 1u);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < (1 << dbits); e += 256)
    if (lh[e]) atomicAdd(&b.hist[e], lh[e]);
}

// S lists of the problems in BS_FINAL: the candidates above the threshold
// key (at most count_above) and the tied ones (their candidate positions).
// Each block counts its segments' entries first, reserves its output ranges
// with one atomic per kind, and then writes them wave by wave in segment
// order (a second read of the candidate values).
__global__ __launch_bounds__(256) void kb_compact(const BProb* __restrict__ probs,
                                                  const BItem* __restrict__ items,
                                                  const unsigned int* __restrict__ seg_count,
                                                  int cur, double* __restrict__ cslot) {
  __shared__ double red[4];
  __shared__ unsigned long long wcnt[2][4];
  __shared__ unsigned long long wbase[2][4];
  const BProb& b = probs[blockIdx.y];
  BSel* s = b.sel;
  if (s->mode != BS_FINAL) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t tkey = (uint32_t)s->prefix;
  const long long kcap = s->count_above;
  const double rn = 1.0 / (double)b.n;
  const ColMap cm = colmap((int)b.n);
  const int nseg = b.nitems * 4;
  const int item0 = b.item0;
  const int64_t rowcap = b.rowcap;
  const float* cval = b.cand_val;
  const int32_t* cidx = b.cand_idx;
  const float* cxv = b.cand_x;
  auto seg_range = [&](int sg, int64_t& c0, int64_t& c1) {
    const int item = item0 + sg / 4, w = sg % 4;
    const BItem itm = items[item];
    c0 = itm.i0 * rowcap + (int64_t)w * wave_seg_cap((int)(itm.i1 - itm.i0), cm);
    c1 = c0 + seg_count[(int64_t)item * 4 + w];
  };
  // counts of this block's segments, per wave
  unsigned long long na = 0ull, nt = 0ull;   // wave-uniform
  for (int sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
    int64_t c0, c1;
    seg_range(sg, c0, c1);
    for (int64_t cb = c0; cb < c1; cb += 256) {
      const int64_t c = cb + tid;
      const bool valid = c < c1;
      const uint32_t key = fkey(valid ? cval[c] : 0.f);
      na += (unsigned long long)__popcll(__ballot(valid && key > tkey));
      nt += (unsigned long long)__popcll(__ballot(valid && key == tkey && tkey > 0));
    }
  }
  if (lane == 0) {
    wcnt[0][wave] = na;
    wcnt[1][wave] = nt;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int kind = 0; kind < 2; ++kind) {
      const unsigned long long tot = wcnt[kind][0] + wcnt[kind][1] + wcnt[kind][2] + wcnt[kind][3];
      unsigned long long base = 0ull;
      if (tot) base = atomicAdd(kind == 0 ? &s->nabove : &s->nties, tot);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        wbase[kind][w] = base;
        base += wcnt[kind][w];
      }
    }
  }
  __syncthreads();
  unsigned long long pa = wbase[0][wave], pt = wbase[1][wave];   // wave-uniform
  int64_t* sidx = b.s_idx[cur];
  float* sval = b.s_val[cur];
  float* sx = b.s_x[cur];
  int32_t* tie = b.tie_idx;
  double s2 = 0.0;
  for (int sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
    int64_t c0, c1;
    seg_range(sg, c0, c1);
    for (int64_t cb = c0; cb < c1; cb += 256) {
      const int64_t c = cb + tid;
      const bool valid = c < c1;
      const float v = valid ? cval[c] : 0.f;
      const uint32_t key = fkey(v);
      const bool above = valid && key > tkey;
      const bool istie = valid && key == tkey && tkey > 0;
      const unsigned long long ma = __ballot(above);
      if (ma) {
        const unsigned int rank = __builtin_amdgcn_mbcnt_hi(
            (unsigned int)(ma >> 32), __builtin_amdgcn_mbcnt_lo((unsigned int)ma, 0u));
        if (above) {
          const unsigned long long pos = pa + rank;
          if ((long long)pos < kcap) {
            const int32_t li = cidx[c];
            const float xv = cxv[c];
            sidx[pos] = (int64_t)li;
            sval[pos] = v;
            sx[pos] = xv;
            s2 += (double)v * (double)v;
            // the working copy: D = X - S on the new support (its old
            // support was restored before the selection)
            int64_t i, j;
            divmod_nn((int64_t)li, b.n, rn, i, j);
            b.D[i * b.ldd + j] = xv - v;
          }
        }
        pa += (unsigned long long)__popcll(ma);
      }
      const unsigned long long mt = __ballot(istie);
      if (mt) {
        const unsigned int rank = __builtin_amdgcn_mbcnt_hi(
            (unsigned int)(mt >> 32), __builtin_amdgcn_mbcnt_lo((unsigned int)mt, 0u));
        if (istie) tie[pt + rank] = (int32_t)c;
        pt += (unsigned long long)__popcll(mt);
      }
    }
  }
  s2 = wave_sum(s2);
  if (lane == 0) red[wave] = s2;
  __syncthreads();
  // per-block partial of sum S^2; kb_ties adds the problem's blocks in order
  if (tid == 0)
    cslot[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Ties: keep the k_rem smallest linear indices among the candidates equal to
// the threshold (bitonic sort in LDS when they fit, else a radix select on
// the index).  One workgroup per problem.  Also sets nnz, the threshold and
// the objective.
__global__ __launch_bounds__(1024) void kb_ties(const BProb* __restrict__ probs, int cur,
                                                const double* __restrict__ s2slot,
                                                const double* __restrict__ cslot, int cblocks) {
  constexpr int NS = 4096;
  __shared__ unsigned long long sk[NS];     // linear indices
  __shared__ int sp[NS];                    // their tie-list slots
  __shared__ unsigned int cnt[256];
  __shared__ unsigned long long sh_pref;
  __shared__ long long sh_need;
  __shared__ unsigned int wpos;
  __shared__ double red[20];
  const BProb& b = probs[blockIdx.x];
  BSel* s = b.sel;
  const int tid = threadIdx.x;
  // the objective's sums from their partials, in item / block order
  const double r2 = block_sum_fixed(s2slot + b.item0, b.nitems, red);
  const double sel_above =
      block_sum_fixed(cslot + (int64_t)blockIdx.x * cblocks, cblocks, red);
  if (tid == 0) s->sum_r2 = r2;
  if (s->mode == BS_NONE) {
    if (tid == 0) {
      s->carry_valid = 0;
      s->nnz = 0;
      s->nnz_list[cur] = 0;
      s->threshold = 0.0;
      s->sum_sel2 = 0.0;
      s->rel_err_sq = s->norm_x2 > 0.0 ? r2 / s->norm_x2 : 0.0;
    }
    return;
  }
  if (s->mode != BS_FINAL) return;
  const uint32_t tkey = (uint32_t)s->prefix;
  const long long nabove = s->count_above;
  const long long nties = (long long)s->nties;
  long long take = tkey > 0 ? s->k_rem : 0;
  if (take > nties) take = nties;
  const float tval = __uint_as_float(tkey);
  if (take == nties) {
    for (long long e = tid; e < take; e += blockDim.x) {
      const long long c = b.tie_idx[e];
      b.s_idx[cur][nabove + e] = (int64_t)b.cand_idx[c];
      b.s_val[cur][nabove + e] = b.cand_val[c];
      b.s_x[cur][nabove + e] = b.cand_x[c];
    }
  } else if (nties <= NS) {
    for (int e = tid; e < NS; e += blockDim.x) {
      if (e < nties) {
        const long long c = b.tie_idx[e];
        sk[e] = (unsigned long long)b.cand_idx[c];
        sp[e] = (int)e;
      } else {
        sk[e] = ~0ull;
        sp[e] = -1;
      }
    }
    __syncthreads();
    for (int size = 2; size <= NS; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int e = tid; e < NS; e += blockDim.x) {
          const int o = e ^ stride;
          if (o > e) {
            const bool up = (e & size) == 0;
            const unsigned long long a = sk[e], c = sk[o];
            if ((a > c) == up) {
              sk[e] = c; sk[o] = a;
              const int t = sp[e]; sp[e] = sp[o]; sp[o] = t;
            }
          }
        }
        __syncthreads();
      }
    for (long long e = tid; e < take; e += blockDim.x) {
      const long long c = b.tie_idx[sp[e]];
      b.s_idx[cur][nabove + e] = (int64_t)b.cand_idx[c];
      b.s_val[cur][nabove + e] = b.cand_val[c];
      b.s_x[cur][nabove + e] = b.cand_x[c];
    }
  } else {
    // radix select of the take-th smallest linear index, 8 bits at a time
    if (tid == 0) { sh_pref = 0; sh_need = take; }
    __syncthreads();
    for (int shift = 56; shift >= 0; shift -= 8) {
      if (tid < 256) cnt[tid] = 0u;
      __syncthreads();
      const unsigned long long pref = sh_pref;
      for (long long e = tid; e < nties; e += blockDim.x) {
        const unsigned long long x = (unsigned long long)b.cand_idx[b.tie_idx[e]];
        if (shift == 56 || (x >> (shift + 8)) == pref) atomicAdd(&cnt[(x >> shift) & 255], 1u);
      }
      __syncthreads();
      if (tid == 0) {
        const long long need = sh_need;
        unsigned long long cum = 0;
        int d = 0;
        for (; d < 256; ++d) {
          if ((long long)(cum + cnt[d]) >= need) break;
          cum += cnt[d];
        }
        sh_need = need - (long long)cum;
        sh_pref = (pref << 8) | (unsigned long long)d;
      }
      __syncthreads();
    }
    const unsigned long long lim = sh_pref;
    if (tid == 0) wpos = 0u;
    __syncthreads();
    for (long long e = tid; e < nties; e += blockDim.x) {
      const long long c = b.tie_idx[e];
      const unsigned long long x = (unsigned long long)b.cand_idx[c];
      if (x <= lim) {
        const unsigned int p = atomicAdd(&wpos, 1u);
        b.s_idx[cur][nabove + p] = (int64_t)x;
        b.s_val[cur][nabove + p] = b.cand_val[c];
        b.s_x[cur][nabove + p] = b.cand_x[c];
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    // next iteration: histogram and collect from two level-0 digits (a
    // quarter octave) below this threshold's digit
    const int d0 = (int)(tkey >> (31 - kHistBits0));
    s->carry_dlo = d0 > 2 ? d0 - 2 : 0;
    s->carry_valid = tkey > 0 ? 1 : 0;
    s->nnz = nabove + take;
    s->nnz_list[cur] = nabove + take;
    s->threshold = (double)tval;
    s->sum_sel2 = sel_above + (double)take * (double)tval * (double)tval;
    s->rel_err_sq = s->norm_x2 > 0.0 ? (r2 - s->sum_sel2) / s->norm_x2 : 0.0;
  }
}

// D <- X on the old support (restore) or X - S on the new one.
__global__ __launch_bounds__(256) void kb_update_d(const BProb* __restrict__ probs,
                                                   const int* __restrict__ iter, int list,
                                                   int restore) {
  const BProb& b = probs[blockIdx.y];
  if (restore && *iter == 0) return;
  const long long nnz = b.sel->nnz_list[list];
  // restore: the whole old list; otherwise the new list's tie entries (the
  // entries above the threshold were written by kb_compact)
  const long long e_begin = restore ? 0 : b.sel->count_above;
  const int64_t n = b.n;
  const double rn = 1.0 / (double)n;
  const int64_t* __restrict__ sidx = b.s_idx[list];
  const float* __restrict__ sx = b.s_x[list];
  const float* __restrict__ sv = b.s_val[list];
  float* __restrict__ D = b.D;
  const int64_t ldd = b.ldd;
  // U entries per thread and round, all loads in flight before the stores
  constexpr int U = 4;
  const long long step = (long long)gridDim.x * 256;
  for (long long e0 = e_begin + (long long)blockIdx.x * 256 + threadIdx.x; e0 < nnz;
       e0 += U * step) {
    int64_t idx[U];
    float x[U], v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long e = e0 + u * step;
      const bool ok = e < nnz;
      idx[u] = ok ? sidx[e] : -1;
      x[u] = ok ? sx[e] : 0.f;
      v[u] = (ok && !restore) ? sv[e] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (idx[u] < 0) continue;
      int64_t i, j;
      divmod_nn(idx[u], n, rn, i, j);
      D[i * ldd + j] = restore ? x[u] : x[u] - v[u];
    }
  }
}

// D = X (rows of the item), ||X||_F^2 and the NaN/Inf check.
__global__ __launch_bounds__(256) void kb_init_d(const BProb* __restrict__ probs,
                                                 const BItem* __restrict__ items,
                                                 double* __restrict__ nslot) {
  __shared__ double red[4];
  const BItem it = items[blockIdx.x];
  const BProb& b = probs[it.prob];
  const int tid = threadIdx.x;
  double s2 = 0.0;
  int bad = 0;
  const int64_t rows = it.i1 - it.i0;
  for (int64_t e = tid; e < rows * b.ldd; e += 256) {
    const int64_t i = it.i0 + e / b.ldd, j = e % b.ldd;
    float x = 0.f;
    if (j < b.n) {
      x = b.X[i * b.ldx + j];
      s2 += (double)x * (double)x;
      if (!isfinite(x)) bad = 1;
    }
    b.D[i * b.ldd + j] = x;
  }
  s2 = wave_sum(s2);
  if ((tid & 63) == 0) red[tid >> 6] = s2;
  if (bad) atomicOr(&b.sel->nonfinite, 1);
  __syncthreads();
  if (tid == 0) nslot[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// ||X||_F^2 of each problem from its items' partials, in item order (one
// workgroup per problem).
__global__ __launch_bounds__(256) void kb_norm_sum(const BProb* __restrict__ probs,
                                                   const double* __restrict__ nslot) {
  __shared__ double red[8];
  const BProb& b = probs[blockIdx.x];
  const double s = block_sum_fixed(nslot + b.item0, b.nitems, red);
  if (threadIdx.x == 0) b.sel->norm_x2 = s;
}

// Residual R = X - U_L V_L^T of one problem (getter).
__global__ __launch_bounds__(256) void kb_residual(const BProb* __restrict__ prob, float* R,
                                                   int64_t ldr) {
  const BProb& b = *prob;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= b.m * b.n) return;
  const int64_t i = e / b.n, j = e % b.n;
  float u[RP8], v[RP8];
#pragma unroll
  for (int c = 0; c < RP8; ++c) { u[c] = b.UL[i * RP8 + c]; v[c] = b.VL[j * RP8 + c]; }
  R[i * ldr + j] = bresid(b.X[i * b.ldx + j], u, v);
}

// Snapshot of every problem's current S list (entries in selection order)
// and its length: problem blockIdx.y, list `list`.
__global__ __launch_bounds__(256) void kb_copy_lists(const BProb* __restrict__ probs, int list,
                                                     int64_t* __restrict__ idx_out,
                                                     float* __restrict__ val_out,
                                                     int64_t kstride,
                                                     int64_t* __restrict__ nnz_out) {
  const BProb& P = probs[blockIdx.y];
  const int64_t nnz = P.sel->nnz_list[list];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e == 0) nnz_out[blockIdx.y] = nnz;
  if (e >= nnz) return;
  idx_out[(int64_t)blockIdx.y * kstride + e] = P.s_idx[list][e];
  val_out[(int64_t)blockIdx.y * kstride + e] = P.s_val[list][e];
}

__global__ void kb_iter_inc(int* iter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *iter += 1;
}

}  // namespace godec

namespace godec {

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
void bl_copy_a1(const Launch& L, const BatchArgs& a, int64_t max_n) {
  dim3 grid((unsigned)((max_n * kBatchRP + 255) / 256), (unsigned)a.nprob);
  hipLaunchKernelGGL(kb_copy_a1, grid, dim3(256), 0, L.stream, a.probs);
}

void bl_pass(const Launch& L, const BatchArgs& a, int in, int mode) {
  if (mode == 0)
    hipLaunchKernelGGL(kb_pass<0>, dim3((unsigned)a.nitems), dim3(256), 0, L.stream, a.probs,
                       a.items, in, a.zslots, a.gslots);
  else
    hipLaunchKernelGGL(kb_pass<1>, dim3((unsigned)a.nitems), dim3(256), 0, L.stream, a.probs,
                       a.items, in, a.zslots, a.gslots);
}

void bl_reduce_slots(const Launch& L, const BatchArgs& a, int64_t max_n) {
  dim3 grid((unsigned)((max_n * kBatchRP + 255) / 256), (unsigned)a.nprob);
  hipLaunchKernelGGL(kb_reduce_slots, grid, dim3(256), 0, L.stream, a.probs, a.items, a.zslots);
}

void bl_apply_k(const Launch& L, const BatchArgs& a, int64_t max_m) {
  dim3 grid((unsigned)((max_m * kBatchRP + 255) / 256), (unsigned)a.nprob);
  hipLaunchKernelGGL(kb_apply_k, grid, dim3(256), 0, L.stream, a.probs);
}

// Sparse step into S list `cur`, then the D update (restore list cur ^ 1,
// write list cur).
void bl_select(const Launch& L, const BatchArgs& a, int cur, int64_t max_k) {
  const unsigned np = (unsigned)a.nprob;
  const size_t lds = sizeof(unsigned int) * kHistBins +
                     sizeof(float) * RP8 * (size_t)std::min(a.rows_per_item, kBatchMaxRows);
  hipLaunchKernelGGL(kb_sel_reset, dim3(np), dim3(256), 0, L.stream, a.probs);
  hipLaunchKernelGGL(kb_sel_pass<2>, dim3((unsigned)a.nitems), dim3(256), lds, L.stream, a.probs,
                     a.items, a.seg_count, a.dslots);
  hipLaunchKernelGGL(kb_sel_plan, dim3(np), dim3(256), 0, L.stream, a.probs, -1);
  hipLaunchKernelGGL(kb_sel_pass<0>, dim3((unsigned)a.nitems), dim3(256), lds, L.stream, a.probs,
                     a.items, a.seg_count, a.dslots);
  hipLaunchKernelGGL(kb_sel_plan, dim3(np), dim3(256), 0, L.stream, a.probs, 0);
  hipLaunchKernelGGL(kb_sel_pass<1>, dim3((unsigned)a.nitems), dim3(256), lds, L.stream, a.probs,
                     a.items, a.seg_count, a.dslots);
  hipLaunchKernelGGL(kb_sel_to_refine, dim3((np + 63) / 64), dim3(64), 0, L.stream, a.probs,
                     a.nprob);
  // blocks per problem over its candidate segments
  const unsigned cb = (unsigned)std::max(1, std::min(64, a.max_items));
  (void)max_k;
  for (int level = 1; level <= 2; ++level) {
    hipLaunchKernelGGL(kb_cand_hist, dim3(cb, np), dim3(256), 0, L.stream, a.probs, a.items,
                       a.seg_count);
    hipLaunchKernelGGL(kb_sel_plan, dim3(np), dim3(256), 0, L.stream, a.probs, level);
  }
  double* cslot = a.dslots + 2 * (int64_t)a.items_cap;
  hipLaunchKernelGGL(kb_compact, dim3(cb, np), dim3(256), 0, L.stream, a.probs, a.items,
                     a.seg_count, cur, cslot);
  hipLaunchKernelGGL(kb_ties, dim3(np), dim3(1024), 0, L.stream, a.probs, cur,
                     (const double*)a.dslots, (const double*)cslot, (int)cb);
}

void bl_restore_d(const Launch& L, const BatchArgs& a, int cur, int64_t max_k) {
  const unsigned g = (unsigned)std::min<int64_t>(256, std::max<int64_t>(1, (max_k + 255) / 256));
  hipLaunchKernelGGL(kb_update_d, dim3(g, (unsigned)a.nprob), dim3(256), 0, L.stream, a.probs,
                     a.iter, cur ^ 1, 1);
}

void bl_update_d(const Launch& L, const BatchArgs& a, int cur, int64_t max_k) {
  (void)max_k;
  // the tie slice of the new list only: a few entries per problem
  hipLaunchKernelGGL(kb_update_d, dim3(1, (unsigned)a.nprob), dim3(256), 0, L.stream, a.probs,
                     a.iter, cur, 0);
  hipLaunchKernelGGL(kb_iter_inc, dim3(1), dim3(64), 0, L.stream, a.iter);
}

void bl_init(const Launch& L, const BatchArgs& a) {
  double* nslot = a.dslots + a.items_cap;
  hipLaunchKernelGGL(kb_init_d, dim3((unsigned)a.nitems), dim3(256), 0, L.stream, a.probs,
                     a.items, nslot);
  hipLaunchKernelGGL(kb_norm_sum, dim3((unsigned)a.nprob), dim3(256), 0, L.stream, a.probs,
                     (const double*)nslot);
}

void bl_residual(const Launch& L, const BProb* prob_dev, int64_t m, int64_t n, float* R,
                 int64_t ldr) {
  const unsigned g = (unsigned)((m * n + 255) / 256);
  hipLaunchKernelGGL(kb_residual, dim3(g), dim3(256), 0, L.stream, prob_dev, R, ldr);
}

// U_L (m x 8) and V_L (n x 8) of every problem into dense m x r and n x r
// panels (problem b at U + b sU, V + b sV).
__global__ __launch_bounds__(256) void kb_copy_factors(const BProb* __restrict__ probs,
                                                       float* __restrict__ U, int64_t sU,
                                                       float* __restrict__ V, int64_t sV) {
  const BProb& b = probs[blockIdx.y];
  const int r = b.r;
  const int64_t nu = b.m * r, nv = b.n * r;
  const float* UL = b.UL;
  const float* VL = b.VL;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nu + nv;
       e += (int64_t)gridDim.x * 256) {
    if (e < nu) {
      U[(int64_t)blockIdx.y * sU + e] = UL[(e / r) * RP8 + e % r];
    } else {
      const int64_t f = e - nu;
      V[(int64_t)blockIdx.y * sV + f] = VL[(f / r) * RP8 + f % r];
    }
  }
}

void bl_copy_factors(const Launch& L, const BProb* probs_dev, int nprob, int64_t max_elems,
                     float* U, int64_t sU, float* V, int64_t sV) {
  const unsigned g = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (max_elems + 255) / 256));
  hipLaunchKernelGGL(kb_copy_factors, dim3(g, (unsigned)nprob), dim3(256), 0, L.stream, probs_dev,
                     U, sU, V, sV);
}

// out[2i] = problem i's non-finite flag, out[2i + 1] = its current rank
__global__ __launch_bounds__(256) void kb_gather_state(const BProb* __restrict__ probs, int nprob,
                                                       int* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nprob) return;
  out[2 * i] = probs[i].sel->nonfinite;
  out[2 * i + 1] = probs[i].st->r_eff;
}

void bl_gather_state(const Launch& L, const BProb* probs_dev, int nprob, int* out) {
  hipLaunchKernelGGL(kb_gather_state, dim3((unsigned)((nprob + 255) / 256)), dim3(256), 0,
                     L.stream, probs_dev, nprob, out);
}

void bl_copy_lists(const Launch& L, const BProb* probs_dev, int nprob, int list, int64_t kmax,
                   int64_t* idx_out, float* val_out, int64_t kstride, int64_t* nnz_out) {
  const dim3 g((unsigned)((std::max<int64_t>(kmax, 1) + 255) / 256), (unsigned)nprob);
  hipLaunchKernelGGL(kb_copy_lists, g, dim3(256), 0, L.stream, probs_dev, list, idx_out, val_out,
                     kstride, nnz_out);
}

}  // namespace godec
