// Sparse step of Algorithm 1: S_t = P_Omega(X - L_t) with Omega the nonzero
// subset of the k largest |X - L_t| (Eq. 4).  Ties are broken by row-major
// linear index, smallest first.
//
// The residual R = X - U_L V_L^T is recomputed on the fly from the factors
// (2r multiply-adds per entry) and never stored.  The k-th largest |R| is
// found by a most-significant-digit radix select on the IEEE bits of |R|
// (monotone in |R|): a full pass histograms the top 12 bits; when the
// entries at or above the bucket holding the k-th key fit in the candidate
// buffer, a second pass collects them and the remaining digits are resolved
// over the candidates only; otherwise further full passes histogram the
// next digits.  Degenerate inputs (more exact ties at the threshold than the
// candidate buffer holds) fall back to an index-ordered scan.
#include "godec_internal.h"
#include "k_common.h"

namespace godec {

template <typename T> struct KeyBits;
template <> struct KeyBits<float> { static constexpr int value = 31; };
template <> struct KeyBits<double> { static constexpr int value = 63; };

__device__ __forceinline__ float key_to_val(unsigned long long k, float*) { return __uint_as_float((uint32_t)k); }
__device__ __forceinline__ double key_to_val(unsigned long long k, double*) { return __longlong_as_double((long long)k); }

// Residual entry with a fixed multiply-add order (shared by selection and
// godec_get_residual so both see the same bits).
template <typename T, int RP>
__device__ __forceinline__ T resid(T x, const T* __restrict__ u, const T (&v)[RP]) {
  T s = T(0);
#pragma unroll
  for (int c = 0; c < RP; ++c) s = fma_t(u[c], v[c], s);
  return x - s;
}

constexpr int kRowsPerTile = 32;
constexpr int kCandBuf = 2048;

__device__ __forceinline__ int digit_bits(int pbits, int kbits) {
  if (pbits == 0) return kHistBits0;
  const int rem = kbits - pbits;
  return rem < kHistBits ? rem : kHistBits;
}

// ---------------------------------------------------------------------------
// Full-data pass.  Mode comes from the plan: pass_index == 0 is always the
// level-0 histogram (plus sum R^2); later passes histogram the next digit
// inside the bucket (SEL_HIST), collect every entry at or above the bucket
// (SEL_COLLECT), or collect the entries strictly above the resolved
// threshold (SEL_TIES).  Any other mode returns at once.
// ---------------------------------------------------------------------------
template <typename T, int RP>
__global__ __launch_bounds__(256) void k_sel_pass(const T* __restrict__ X, int64_t ldx,
                                                  const T* __restrict__ UL,
                                                  const T* __restrict__ VL,
                                                  int64_t m, int64_t n,
                                                  SelPlan* __restrict__ plan,
                                                  unsigned long long* __restrict__ hist,
                                                  int64_t* __restrict__ cand_idx,
                                                  T* __restrict__ cand_val,
                                                  int pass_index) {
  constexpr int KB = KeyBits<T>::value;
  __shared__ unsigned int lh[kHistBins];
  __shared__ T us[kRowsPerTile * RP];
  __shared__ int64_t bidx[kCandBuf];
  __shared__ T bval[kCandBuf];
  __shared__ int bcount;
  __shared__ unsigned long long gbase;
  __shared__ double red[8];

  int mode = SEL_HIST;
  unsigned long long prefix = 0;
  int pbits = 0;
  if (pass_index > 0) {
    mode = plan->mode;
    if (mode != SEL_HIST && mode != SEL_COLLECT && mode != SEL_TIES) return;
    prefix = plan->prefix;
    pbits = plan->pbits;
  }
  const int dbits = digit_bits(pbits, KB);
  const bool do_hist = (mode == SEL_HIST);
  const bool do_coll = (mode == SEL_COLLECT || mode == SEL_TIES);
  const int tid = threadIdx.x;
  if (do_hist)
    for (int e = tid; e < kHistBins; e += 256) lh[e] = 0u;
  if (tid == 0) bcount = 0;
  __syncthreads();

  const int64_t ctiles = (n + 255) / 256;
  const int64_t rtiles = (m + kRowsPerTile - 1) / kRowsPerTile;
  const int64_t ntiles = ctiles * rtiles;
  double s2 = 0.0;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t ct = tile % ctiles, rt = tile / ctiles;
    const int64_t j = ct * 256 + tid;
    const int64_t i0 = rt * kRowsPerTile;
    const int nr = (m - i0) < kRowsPerTile ? (int)(m - i0) : kRowsPerTile;
    __syncthreads();
    for (int e = tid; e < kRowsPerTile * RP; e += 256)
      us[e] = (e < nr * RP) ? UL[i0 * RP + e] : T(0);
    __syncthreads();
    T v[RP];
#pragma unroll
    for (int c = 0; c < RP; ++c) v[c] = (j < n) ? VL[j * RP + c] : T(0);
    for (int ii = 0; ii < nr; ++ii) {
      if (do_coll && (ii & 3) == 0) {
        // flush the block buffer when another 4 rows could overflow it; the
        // count is read between two barriers so every thread sees the same
        // value and takes the same branch
        __syncthreads();
        const int bc = bcount;
        __syncthreads();
        if (bc > kCandBuf - 4 * 256) {
          if (tid == 0) {
            gbase = atomicAdd((unsigned long long*)&plan->ncand, (unsigned long long)bcount);
          }
          __syncthreads();
          const long long cap = plan->cap;
          for (int e = tid; e < bcount; e += 256) {
            const long long pos = (long long)gbase + e;
            if (pos < cap) { cand_idx[pos] = bidx[e]; cand_val[pos] = bval[e]; }
          }
          __syncthreads();
          if (tid == 0) bcount = 0;
          __syncthreads();
        }
      }
      if (j >= n) continue;
      const int64_t i = i0 + ii;
      const T r = resid<T, RP>(X[i * ldx + j], us + ii * RP, v);
      const unsigned long long key = abs_key(r);
      if (pass_index == 0) {
        s2 += (double)r * (double)r;
        atomicAdd(&lh[key >> (KB - kHistBits0)], 1u);
      } else if (do_hist) {
        if ((key >> (KB - pbits)) == prefix)
          atomicAdd(&lh[(key >> (KB - pbits - dbits)) & ((1ull << dbits) - 1)], 1u);
      } else {
        bool take;
        if (mode == SEL_COLLECT)
          take = key > 0 && (key >> (KB - pbits)) >= prefix;
        else
          take = key > prefix;   // SEL_TIES: prefix holds the full threshold key
        if (take) {
          const int slot = atomicAdd(&bcount, 1);
          bidx[slot] = i * n + j;
          bval[slot] = r;
        }
      }
    }
  }
  __syncthreads();
  if (do_coll && bcount > 0) {
    if (tid == 0)
      gbase = atomicAdd((unsigned long long*)&plan->ncand, (unsigned long long)bcount);
    __syncthreads();
    const long long cap = plan->cap;
    for (int e = tid; e < bcount; e += 256) {
      const long long pos = (long long)gbase + e;
      if (pos < cap) { cand_idx[pos] = bidx[e]; cand_val[pos] = bval[e]; }
    }
  }
  if (do_hist) {
    const int bins = 1 << dbits;
    for (int e = tid; e < bins; e += 256)
      if (lh[e]) atomicAdd(&hist[e], (unsigned long long)lh[e]);
  }
  if (pass_index == 0) {
    s2 = wave_sum(s2);
    if ((tid & 63) == 0) red[tid >> 6] = s2;
    __syncthreads();
    if (tid == 0) atomicAdd(&plan->sum_r2, red[0] + red[1] + red[2] + red[3]);
  }
}

// Histogram of the next digit over the candidates inside the bucket.
template <typename T>
__global__ __launch_bounds__(256) void k_cand_hist(SelPlan* __restrict__ plan,
                                                   const T* __restrict__ cand_val,
                                                   unsigned long long* __restrict__ hist) {
  constexpr int KB = KeyBits<T>::value;
  __shared__ unsigned int lh[kHistBins];
  if (plan->mode != SEL_REFINE) return;
  const unsigned long long prefix = plan->prefix;
  const int pbits = plan->pbits;
  const int dbits = digit_bits(pbits, KB);
  const long long nc = plan->ncand < plan->cap ? plan->ncand : plan->cap;
  for (int e = threadIdx.x; e < (1 << dbits); e += 256) lh[e] = 0u;
  __syncthreads();
  for (long long c = (long long)blockIdx.x * 256 + threadIdx.x; c < nc;
       c += (long long)gridDim.x * 256) {
    const unsigned long long key = abs_key(cand_val[c]);
    if ((key >> (KB - pbits)) == prefix)
      atomicAdd(&lh[(key >> (KB - pbits - dbits)) & ((1ull << dbits) - 1)], 1u);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < (1 << dbits); e += 256)
    if (lh[e]) atomicAdd(&hist[e], (unsigned long long)lh[e]);
}

// Advance the plan.  One block.  stage 0 follows a full-data pass (which
// histogrammed in SEL_HIST or collected in SEL_COLLECT); stage 1 follows a
// candidate histogram (SEL_REFINE).  In any other combination the preceding
// kernel did nothing and neither does this one.
template <typename T>
__global__ __launch_bounds__(256) void k_sel_plan(SelPlan* __restrict__ plan,
                                                  unsigned long long* __restrict__ hist,
                                                  int stage) {
  constexpr int KB = KeyBits<T>::value;
  __shared__ unsigned long long part[256];
  const int tid = threadIdx.x;
  const int mode = plan->mode;
  if (stage == 0 && mode == SEL_COLLECT) {
    if (tid == 0) {
      if (plan->ncand > plan->cap) plan->overflow = 1;
      plan->mode = (plan->pbits == KB) ? SEL_FINAL : SEL_REFINE;
    }
    return;
  }
  if (!((stage == 0 && mode == SEL_HIST) || (stage == 1 && mode == SEL_REFINE))) return;
  const int pbits = plan->pbits;
  const int dbits = digit_bits(pbits, KB);
  const int bins = 1 << dbits;
  const int per = (bins + 255) / 256;
  // thread t owns the digits [bins - (t+1)*per, bins - t*per): top first
  unsigned long long s = 0;
  for (int u = 0; u < per; ++u) {
    const int d = bins - 1 - (tid * per + u);
    if (d >= 0) s += hist[d];
  }
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    const long long k_rem = plan->k_rem;
    unsigned long long cum = 0;
    int dsel = -1;
    for (int t = 0; t < 256 && dsel < 0; ++t) {
      if (cum + part[t] >= (unsigned long long)k_rem) {
        for (int u = 0; u < per; ++u) {
          const int d = bins - 1 - (t * per + u);
          if (d < 0) break;
          if (cum + hist[d] >= (unsigned long long)k_rem) { dsel = d; break; }
          cum += hist[d];
        }
      } else {
        cum += part[t];
      }
    }
    if (dsel < 0) {
      // fewer keys than k_rem in the bucket: only when the remaining keys
      // are zeros (excluded from the candidates); settle on digit 0
      dsel = 0;
      cum -= hist[0];
    }
    plan->count_above += (long long)cum;
    plan->k_rem = k_rem - (long long)cum;
    plan->prefix = (plan->prefix << dbits) | (unsigned long long)dsel;
    plan->pbits = pbits + dbits;
    plan->bucket_count = (long long)hist[dsel];
    int next;
    if (mode == SEL_HIST) {
      if (plan->count_above + plan->bucket_count <= plan->cap) {
        next = SEL_COLLECT;
        plan->ncand = 0;
      } else if (plan->pbits == KB) {
        next = SEL_TIES;
        plan->ncand = 0;
        plan->slow = 1;
      } else {
        next = SEL_HIST;
        plan->slow = 1;
      }
    } else {
      next = (plan->pbits == KB) ? SEL_FINAL : SEL_REFINE;
    }
    plan->mode = next;
  }
  __syncthreads();
  for (int e = tid; e < bins; e += 256) hist[e] = 0ull;
}

// FINAL: write S from the candidates.  Entries above the threshold key go
// straight to S; entries equal to it go to the tie list.
template <typename T>
__global__ __launch_bounds__(256) void k_sel_compact(SelPlan* __restrict__ plan,
                                                     const int64_t* __restrict__ cand_idx,
                                                     const T* __restrict__ cand_val,
                                                     int64_t* __restrict__ s_idx,
                                                     T* __restrict__ s_val,
                                                     int64_t* __restrict__ tie_idx,
                                                     unsigned long long* __restrict__ counters) {
  __shared__ double red[4];
  if (plan->mode != SEL_FINAL) return;
  const unsigned long long tkey = plan->prefix;
  const long long nc = plan->ncand < plan->cap ? plan->ncand : plan->cap;
  const unsigned long long kcap = (unsigned long long)(plan->count_above + plan->k_rem);
  double s2 = 0.0;
  for (long long c = (long long)blockIdx.x * 256 + threadIdx.x; c < nc;
       c += (long long)gridDim.x * 256) {
    const T v = cand_val[c];
    const unsigned long long key = abs_key(v);
    if (key > tkey) {
      const unsigned long long pos = atomicAdd(&counters[0], 1ull);
      if (pos < kcap) {
        s_idx[pos] = cand_idx[c];
        s_val[pos] = v;
        s2 += (double)v * (double)v;
      }
    } else if (key == tkey && tkey > 0) {
      const unsigned long long pos = atomicAdd(&counters[1], 1ull);
      if (pos < (unsigned long long)plan->cap) tie_idx[pos] = cand_idx[c];
    }
  }
  s2 = wave_sum(s2);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s2;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&plan->sum_sel2, red[0] + red[1] + red[2] + red[3]);
}

// Resolve ties: keep the k_rem smallest linear indices among the entries
// equal to the threshold key (one block; bitonic sort in LDS when they fit,
// otherwise repeated minimum extraction by a radix select on the index).
template <typename T>
__global__ __launch_bounds__(1024) void k_sel_ties(SelPlan* __restrict__ plan,
                                                   int64_t* __restrict__ s_idx,
                                                   T* __restrict__ s_val,
                                                   int64_t* __restrict__ tie_idx,
                                                   unsigned long long* __restrict__ counters) {
  constexpr int KB = KeyBits<T>::value;
  constexpr int NS = 4096;
  __shared__ int64_t sk[NS];
  __shared__ unsigned long long cnt[256];
  __shared__ unsigned long long sh_pref;
  __shared__ long long sh_need;
  const int tid = threadIdx.x;
  if (plan->mode != SEL_FINAL) return;
  const unsigned long long tkey = plan->prefix;
  long long nabove = (long long)counters[0];
  if (nabove > plan->count_above) nabove = plan->count_above;
  long long nties = (long long)counters[1];
  if (nties > plan->cap) nties = plan->cap;
  long long take = (tkey > 0) ? plan->k_rem : 0;
  if (take > nties) take = nties;
  const T tval = key_to_val(tkey, (T*)nullptr);
  if (take == nties) {
    for (long long e = tid; e < take; e += blockDim.x) {
      s_idx[nabove + e] = tie_idx[e];
      s_val[nabove + e] = T(0);   // sign restored below
    }
  } else if (nties <= NS) {
    for (int e = tid; e < NS; e += blockDim.x) sk[e] = (e < nties) ? tie_idx[e] : INT64_MAX;
    __syncthreads();
    for (int size = 2; size <= NS; size <<= 1)
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int e = tid; e < NS; e += blockDim.x) {
          const int o = e ^ stride;
          if (o > e) {
            const bool up = (e & size) == 0;
            const int64_t a = sk[e], b = sk[o];
            if ((a > b) == up) { sk[e] = b; sk[o] = a; }
          }
        }
        __syncthreads();
      }
    for (long long e = tid; e < take; e += blockDim.x) {
      s_idx[nabove + e] = sk[e];
      s_val[nabove + e] = T(0);
    }
  } else {
    // radix select of the take-th smallest index (8 bits at a time)
    if (tid == 0) { sh_pref = 0; sh_need = take; }
    __syncthreads();
    for (int shift = 56; shift >= 0; shift -= 8) {
      if (tid < 256) cnt[tid] = 0;
      __syncthreads();
      const unsigned long long pref = sh_pref;
      for (long long e = tid; e < nties; e += blockDim.x) {
        const unsigned long long x = (unsigned long long)tie_idx[e];
        if (shift == 56 || (x >> (shift + 8)) == pref)
          atomicAdd(&cnt[(x >> shift) & 255], 1ull);
      }
      __syncthreads();
      if (tid == 0) {
        long long need = sh_need;
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
    const unsigned long long lim = sh_pref;   // the take-th smallest index
    __shared__ unsigned long long wpos;
    if (tid == 0) wpos = 0;
    __syncthreads();
    for (long long e = tid; e < nties; e += blockDim.x) {
      const unsigned long long x = (unsigned long long)tie_idx[e];
      if (x <= lim) {
        const unsigned long long p = atomicAdd(&wpos, 1ull);
        s_idx[nabove + p] = (int64_t)x;
        s_val[nabove + p] = T(0);
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    plan->nnz = nabove + take;
    plan->threshold = (double)tval;
    plan->sum_sel2 += (double)take * (double)tval * (double)tval;
  }
  (void)KB;
}

// TIES mode: candidates hold the entries above the threshold; the tied
// entries are taken in index order by one block scanning all of X.
template <typename T, int RP>
__global__ __launch_bounds__(256) void k_sel_ties_stream(const T* __restrict__ X, int64_t ldx,
                                                         const T* __restrict__ UL,
                                                         const T* __restrict__ VL,
                                                         int64_t m, int64_t n,
                                                         SelPlan* __restrict__ plan,
                                                         const int64_t* __restrict__ cand_idx,
                                                         const T* __restrict__ cand_val,
                                                         int64_t* __restrict__ s_idx,
                                                         T* __restrict__ s_val) {
  __shared__ T us[RP];
  __shared__ long long taken;
  __shared__ int flags[256];
  if (plan->mode != SEL_TIES) return;
  const int tid = threadIdx.x;
  const unsigned long long tkey = plan->prefix;
  long long nabove = plan->ncand < plan->cap ? plan->ncand : plan->cap;
  if (nabove > plan->count_above) nabove = plan->count_above;
  double s2 = 0.0;
  for (long long c = tid; c < nabove; c += 256) {
    s_idx[c] = cand_idx[c];
    s_val[c] = cand_val[c];
    s2 += (double)cand_val[c] * (double)cand_val[c];
  }
  const long long need = (tkey > 0) ? plan->k_rem : 0;
  if (tid == 0) taken = 0;
  __syncthreads();
  for (int64_t i = 0; i < m && taken < need; ++i) {
    __syncthreads();
    if (tid < RP) us[tid] = UL[i * RP + tid];
    __syncthreads();
    for (int64_t j0 = 0; j0 < n && taken < need; j0 += 256) {
      const int64_t j = j0 + tid;
      int hit = 0;
      if (j < n) {
        T v[RP];
#pragma unroll
        for (int c = 0; c < RP; ++c) v[c] = VL[j * RP + c];
        const T r = resid<T, RP>(X[i * ldx + j], us, v);
        hit = abs_key(r) == tkey;
      }
      flags[tid] = hit;
      __syncthreads();
      if (tid == 0) {
        long long t = taken;
        for (int e = 0; e < 256 && t < need; ++e)
          if (flags[e]) { s_idx[nabove + t] = i * n + j0 + e; s_val[nabove + t] = T(0); ++t; }
        taken = t;
      }
      __syncthreads();
    }
  }
  s2 = wave_sum(s2);
  __shared__ double red[4];
  if ((tid & 63) == 0) red[tid >> 6] = s2;
  __syncthreads();
  if (tid == 0) {
    const T tval = key_to_val(tkey, (T*)nullptr);
    plan->nnz = nabove + taken;
    plan->threshold = (double)tval;
    plan->sum_sel2 = red[0] + red[1] + red[2] + red[3] + (double)taken * (double)tval * (double)tval;
    plan->mode = SEL_DONE;
  }
}

// Restore the sign of tied entries: their stored value is the residual,
// recomputed here from X and the factors (same arithmetic as selection).
template <typename T, int RP>
__global__ __launch_bounds__(256) void k_fix_tie_values(const T* __restrict__ X, int64_t ldx,
                                                        const T* __restrict__ UL,
                                                        const T* __restrict__ VL, int64_t n,
                                                        const SelPlan* __restrict__ plan,
                                                        const unsigned long long* __restrict__ counters,
                                                        int64_t* __restrict__ s_idx,
                                                        T* __restrict__ s_val) {
  const long long start = (long long)counters[0];
  const long long nnz = plan->nnz;
  for (long long e = start + (long long)blockIdx.x * 256 + threadIdx.x; e < nnz;
       e += (long long)gridDim.x * 256) {
    if (s_val[e] != T(0)) continue;
    const int64_t idx = s_idx[e];
    const int64_t i = idx / n, j = idx % n;
    T u[RP], v[RP];
#pragma unroll
    for (int c = 0; c < RP; ++c) { u[c] = UL[i * RP + c]; v[c] = VL[j * RP + c]; }
    s_val[e] = resid<T, RP>(X[i * ldx + j], u, v);
  }
}

template <typename T>
__global__ void k_sel_reset(SelPlan* plan, unsigned long long* hist,
                            unsigned long long* counters, long long k, long long cap) {
  constexpr int KB = KeyBits<T>::value;
  for (int e = threadIdx.x; e < kHistBins; e += blockDim.x) hist[e] = 0ull;
  if (threadIdx.x == 0) {
    plan->prefix = 0; plan->k_rem = k; plan->count_above = 0; plan->bucket_count = 0;
    plan->ncand = 0; plan->cap = cap; plan->nnz = 0; plan->pbits = 0; plan->kbits = KB;
    plan->mode = (k > 0) ? SEL_HIST : SEL_FINAL; plan->slow = 0; plan->overflow = 0;
    plan->sum_r2 = 0.0; plan->sum_sel2 = 0.0; plan->threshold = 0.0;
    counters[0] = 0; counters[1] = 0;
  }
}

// ---------------------------------------------------------------------------
// Dense helpers.
// ---------------------------------------------------------------------------
template <typename T, int RP>
__global__ __launch_bounds__(256) void k_residual(const T* __restrict__ X, int64_t ldx,
                                                  const T* __restrict__ UL,
                                                  const T* __restrict__ VL, int64_t m,
                                                  int64_t n, T* __restrict__ R, int64_t ldr,
                                                  int dense_l) {
  __shared__ T us[kRowsPerTile * RP];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * kRowsPerTile;
  const int nr = (m - i0) < kRowsPerTile ? (int)(m - i0) : kRowsPerTile;
  for (int e = threadIdx.x; e < kRowsPerTile * RP; e += 256)
    us[e] = (e < nr * RP) ? UL[i0 * RP + e] : T(0);
  __syncthreads();
  if (j >= n) return;
  T v[RP];
#pragma unroll
  for (int c = 0; c < RP; ++c) v[c] = VL[j * RP + c];
  for (int ii = 0; ii < nr; ++ii) {
    const int64_t i = i0 + ii;
    if (dense_l) {
      R[i * ldr + j] = T(0) - resid<T, RP>(T(0), us + ii * RP, v);
    } else {
      R[i * ldr + j] = resid<T, RP>(X[i * ldx + j], us + ii * RP, v);
    }
  }
}

template <typename TD, typename TX>
__device__ __forceinline__ TD to_store(TX x);
template <> __device__ __forceinline__ double to_store<double, double>(double x) { return x; }
template <> __device__ __forceinline__ float to_store<float, float>(float x) { return x; }
template <> __device__ __forceinline__ uint16_t to_store<uint16_t, float>(float x) { return f32_to_bf16(x); }

template <typename TD, typename TX>
__global__ __launch_bounds__(256) void k_init_d(TD* __restrict__ D, int64_t ldd,
                                                const TX* __restrict__ X, int64_t ldx,
                                                int64_t m, int64_t n) {
  const int64_t total = m * ldd;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / ldd, j = e % ldd;
    D[e] = (j < n) ? to_store<TD, TX>(X[i * ldx + j]) : TD(0);
  }
}

template <typename TD, typename TX>
__global__ __launch_bounds__(256) void k_update_d(TD* __restrict__ D, int64_t ldd,
                                                  const TX* __restrict__ X, int64_t ldx,
                                                  int64_t n, const int64_t* __restrict__ idx,
                                                  const TX* __restrict__ val,
                                                  const SelPlan* __restrict__ plan) {
  const long long cnt = plan->nnz;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (long long)gridDim.x * 256) {
    const int64_t id = idx[e];
    const int64_t i = id / n, j = id % n;
    const TX x = X[i * ldx + j];
    D[i * ldd + j] = to_store<TD, TX>(val ? (TX)(x - val[e]) : x);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_norm_check(const T* __restrict__ X, int64_t ldx,
                                                    int64_t m, int64_t n, double* out2,
                                                    int* nonfinite) {
  __shared__ double red[4];
  double s = 0.0;
  int bad = 0;
  const int64_t total = m * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const T x = X[(e / n) * ldx + (e % n)];
    if (!isfinite(x)) bad = 1;
    s += (double)x * (double)x;
  }
  if (bad) atomicOr(nonfinite, 1);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out2, red[0] + red[1] + red[2] + red[3]);
}

// Ordered output of S: set bits of a bitmap over the linear indices, scan
// the per-word popcounts, and scatter each entry to its rank.
__global__ void k_bitmap_set(const int64_t* __restrict__ idx, const SelPlan* __restrict__ plan,
                             uint32_t* __restrict__ bitmap) {
  const long long cnt = plan->nnz;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (long long)gridDim.x * 256) {
    const int64_t id = idx[e];
    atomicOr(&bitmap[id >> 5], 1u << (id & 31));
  }
}

// Block-local exclusive scan of word popcounts (1024 words per block).
__global__ __launch_bounds__(1024) void k_bitmap_scan1(const uint32_t* __restrict__ bitmap,
                                                       int64_t nwords, uint32_t* __restrict__ wpre,
                                                       uint32_t* __restrict__ bsum) {
  __shared__ uint32_t s[1024];
  const int64_t w = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const uint32_t c = (w < nwords) ? __popc(bitmap[w]) : 0u;
  s[threadIdx.x] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (w < nwords) wpre[w] = s[threadIdx.x] - c;
  if (threadIdx.x == 1023) bsum[blockIdx.x] = s[1023];
}

// Exclusive scan of the block sums (one block, sequential chunks).
__global__ __launch_bounds__(1024) void k_bitmap_scan2(uint32_t* __restrict__ bsum, int64_t nb,
                                                       unsigned long long* __restrict__ boff) {
  __shared__ unsigned long long s[1024];
  __shared__ unsigned long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    const int64_t b = b0 + threadIdx.x;
    const unsigned long long c = (b < nb) ? bsum[b] : 0ull;
    s[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const unsigned long long t = threadIdx.x >= off ? s[threadIdx.x - off] : 0ull;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (b < nb) boff[b] = carry + s[threadIdx.x] - c;
    __syncthreads();
    if (threadIdx.x == 1023) carry += s[1023];
    __syncthreads();
  }
}

template <typename T>
__global__ void k_bitmap_scatter(const int64_t* __restrict__ idx, const T* __restrict__ val,
                                 const SelPlan* __restrict__ plan,
                                 const uint32_t* __restrict__ bitmap,
                                 const uint32_t* __restrict__ wpre,
                                 const unsigned long long* __restrict__ boff,
                                 int64_t* __restrict__ out_idx, T* __restrict__ out_val) {
  const long long cnt = plan->nnz;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (long long)gridDim.x * 256) {
    const int64_t id = idx[e];
    const int64_t w = id >> 5;
    const uint32_t below = bitmap[w] & ((1u << (id & 31)) - 1u);
    const unsigned long long pos = boff[w >> 10] + wpre[w] + (unsigned)__popc(below);
    out_idx[pos] = id;
    out_val[pos] = val[e];
  }
}

__global__ void k_fill_zero(uint32_t* p, int64_t nwords) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nwords;
       e += (int64_t)gridDim.x * 256)
    p[e] = 0u;
}

// ---------------------------------------------------------------------------
// Host launchers.
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

static unsigned grid_for(int64_t work, int num_cu, int per_cu) {
  int64_t g = (work + 255) / 256;
  const int64_t lim = (int64_t)num_cu * per_cu;
  if (g > lim) g = lim;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <typename T>
static void select_t(const Launch& L, int rp, const SelectArgs& a) {
  constexpr int KB = KeyBits<T>::value;
  const int levels = 1 + (KB - kHistBits0 + kHistBits - 1) / kHistBits;
  const int64_t ctiles = (a.n + 255) / 256;
  const int64_t rtiles = (a.m + kRowsPerTile - 1) / kRowsPerTile;
  int64_t g = ctiles * rtiles;
  if (g > (int64_t)L.num_cu * 4) g = (int64_t)L.num_cu * 4;
  const unsigned pass_grid = (unsigned)g;
  hipLaunchKernelGGL(k_sel_reset<T>, dim3(1), dim3(256), 0, L.stream, a.plan, a.hist,
                     a.counters, (long long)a.k, (long long)a.cap);
  GODEC_RP_SWITCH(rp, {
    for (int pass = 0; pass <= levels; ++pass) {
      if (pass == 0 && a.ev_a) (void)hipEventRecord(a.ev_a, L.stream);
      hipLaunchKernelGGL((k_sel_pass<T, RP>), dim3(pass_grid), dim3(256), 0, L.stream,
                         (const T*)a.X, a.ldx, (const T*)a.UL, (const T*)a.VL, a.m, a.n,
                         a.plan, a.hist, a.cand_idx, (T*)a.cand_val, pass);
      if (pass == 0 && a.ev_b) (void)hipEventRecord(a.ev_b, L.stream);
      hipLaunchKernelGGL(k_sel_plan<T>, dim3(1), dim3(256), 0, L.stream, a.plan, a.hist, 0);
    }
  });
  const unsigned cg = grid_for(a.cap, L.num_cu, 4);
  for (int round = 0; round < levels - 1; ++round) {
    hipLaunchKernelGGL(k_cand_hist<T>, dim3(cg), dim3(256), 0, L.stream, a.plan,
                       (const T*)a.cand_val, a.hist);
    hipLaunchKernelGGL(k_sel_plan<T>, dim3(1), dim3(256), 0, L.stream, a.plan, a.hist, 1);
  }
  GODEC_RP_SWITCH(rp, {
    hipLaunchKernelGGL((k_sel_ties_stream<T, RP>), dim3(1), dim3(256), 0, L.stream,
                       (const T*)a.X, a.ldx, (const T*)a.UL, (const T*)a.VL, a.m, a.n, a.plan,
                       a.cand_idx, (const T*)a.cand_val, a.s_idx, (T*)a.s_val);
  });
  hipLaunchKernelGGL(k_sel_compact<T>, dim3(cg), dim3(256), 0, L.stream, a.plan, a.cand_idx,
                     (const T*)a.cand_val, a.s_idx, (T*)a.s_val, a.tie_idx, a.counters);
  hipLaunchKernelGGL(k_sel_ties<T>, dim3(1), dim3(1024), 0, L.stream, a.plan, a.s_idx,
                     (T*)a.s_val, a.tie_idx, a.counters);
  GODEC_RP_SWITCH(rp, {
    hipLaunchKernelGGL((k_fix_tie_values<T, RP>), dim3(grid_for(a.k, L.num_cu, 2)), dim3(256),
                       0, L.stream, (const T*)a.X, a.ldx, (const T*)a.UL, (const T*)a.VL, a.n,
                       a.plan, a.counters, a.s_idx, (T*)a.s_val);
  });
}

void launch_select(const Launch& L, bool f64, int rp, const SelectArgs& a) {
  if (f64) select_t<double>(L, rp, a);
  else select_t<float>(L, rp, a);
}

void launch_residual(const Launch& L, bool f64, int rp, const void* X, int64_t ldx,
                     const void* UL, const void* VL, int64_t m, int64_t n, void* R,
                     int64_t ldr, int dense_l) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)((m + kRowsPerTile - 1) / kRowsPerTile));
  GODEC_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((k_residual<double, RP>), grid, dim3(256), 0, L.stream,
                         (const double*)X, ldx, (const double*)UL, (const double*)VL, m, n,
                         (double*)R, ldr, dense_l);
    else
      hipLaunchKernelGGL((k_residual<float, RP>), grid, dim3(256), 0, L.stream,
                         (const float*)X, ldx, (const float*)UL, (const float*)VL, m, n,
                         (float*)R, ldr, dense_l);
  });
}

void launch_init_d(const Launch& L, DType td, bool xf64, void* D, int64_t ldd,
                   const void* X, int64_t ldx, int64_t m, int64_t n) {
  dim3 grid(grid_for(m * ldd, L.num_cu, 16));
  if (td == F64)
    hipLaunchKernelGGL((k_init_d<double, double>), grid, dim3(256), 0, L.stream, (double*)D,
                       ldd, (const double*)X, ldx, m, n);
  else if (td == F32)
    hipLaunchKernelGGL((k_init_d<float, float>), grid, dim3(256), 0, L.stream, (float*)D, ldd,
                       (const float*)X, ldx, m, n);
  else
    hipLaunchKernelGGL((k_init_d<uint16_t, float>), grid, dim3(256), 0, L.stream,
                       (uint16_t*)D, ldd, (const float*)X, ldx, m, n);
  (void)xf64;
}

void launch_update_d(const Launch& L, DType td, bool xf64, void* D, int64_t ldd,
                     const void* X, int64_t ldx, int64_t n, const int64_t* idx,
                     const void* val, const SelPlan* plan, int64_t kmax) {
  const unsigned g = grid_for(kmax, L.num_cu, 4);
  if (td == F64)
    hipLaunchKernelGGL((k_update_d<double, double>), dim3(g), dim3(256), 0, L.stream,
                       (double*)D, ldd, (const double*)X, ldx, n, idx, (const double*)val, plan);
  else if (td == F32)
    hipLaunchKernelGGL((k_update_d<float, float>), dim3(g), dim3(256), 0, L.stream, (float*)D,
                       ldd, (const float*)X, ldx, n, idx, (const float*)val, plan);
  else
    hipLaunchKernelGGL((k_update_d<uint16_t, float>), dim3(g), dim3(256), 0, L.stream,
                       (uint16_t*)D, ldd, (const float*)X, ldx, n, idx, (const float*)val, plan);
  (void)xf64;
}

void launch_norm_check(const Launch& L, bool f64, const void* X, int64_t ldx, int64_t m,
                       int64_t n, double* out2, int* nonfinite) {
  const unsigned g = grid_for(m * n, L.num_cu, 8);
  if (f64)
    hipLaunchKernelGGL(k_norm_check<double>, dim3(g), dim3(256), 0, L.stream,
                       (const double*)X, ldx, m, n, out2, nonfinite);
  else
    hipLaunchKernelGGL(k_norm_check<float>, dim3(g), dim3(256), 0, L.stream, (const float*)X,
                       ldx, m, n, out2, nonfinite);
}

void launch_sort_s(const Launch& L, bool f64, const int64_t* idx, const void* val,
                   const SelPlan* plan, int64_t mn, int64_t kmax, uint32_t* bitmap,
                   uint32_t* wpre, uint32_t* bsum, unsigned long long* boff,
                   int64_t* out_idx, void* out_val) {
  const int64_t nwords = (mn + 31) / 32;
  const int64_t nb = (nwords + 1023) / 1024;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(nwords, L.num_cu, 8)), dim3(256), 0, L.stream,
                     bitmap, nwords);
  const unsigned g = grid_for(kmax, L.num_cu, 4);
  hipLaunchKernelGGL(k_bitmap_set, dim3(g), dim3(256), 0, L.stream, idx, plan, bitmap);
  hipLaunchKernelGGL(k_bitmap_scan1, dim3((unsigned)nb), dim3(1024), 0, L.stream, bitmap,
                     nwords, wpre, bsum);
  hipLaunchKernelGGL(k_bitmap_scan2, dim3(1), dim3(1024), 0, L.stream, bsum, nb, boff);
  if (f64)
    hipLaunchKernelGGL(k_bitmap_scatter<double>, dim3(g), dim3(256), 0, L.stream, idx,
                       (const double*)val, plan, bitmap, wpre, boff, out_idx, (double*)out_val);
  else
    hipLaunchKernelGGL(k_bitmap_scatter<float>, dim3(g), dim3(256), 0, L.stream, idx,
                       (const float*)val, plan, bitmap, wpre, boff, out_idx, (float*)out_val);
}

}  // namespace godec
