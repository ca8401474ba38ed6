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
//
// FP32 residuals are evaluated on the matrix cores in aligned 16 x 16 tiles
// (res_tile); every FP32 consumer (selection passes, tie scan, tie values,
// the dense residual and L) computes an entry inside the same aligned tile,
// so all of them see the same bits.  FP64 residuals use the FMA chain resid().
#include "godec_internal.h"
#include "k_common.h"

#include <algorithm>

namespace godec {

template <typename T> struct KeyBits;
template <> struct KeyBits<float> { static constexpr int value = 31; using key_t = uint32_t; };
template <> struct KeyBits<double> { static constexpr int value = 63; using key_t = uint64_t; };

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

// ---------------------------------------------------------------------------
// FP32 residual tiles: L = U_L V_L^T over rows [r0, r0 + 16) and columns
// [c0, c0 + 16) (r0, c0 multiples of 16) by one wavefront with
// v_mfma_f32_16x16x4f32 evaluating the transposed tile V_L U_L^T, k-steps of
// four rank columns in ascending order.  Lane l supplies
// V_L[c0 + l%16][4s + l/16] (A operand) and U_L[r0 + l%16][4s + l/16]
// (B operand), zero past m, n or RP, and receives L at row r0 + l%16 and
// columns c0 + res_col(v, l), v < 4: four consecutive columns of one row, so
// that a lane reads its four X entries with one 16-byte load.
// ---------------------------------------------------------------------------
typedef float f32x4_t __attribute__((ext_vector_type(4)));

template <int RP>
struct ResK { static constexpr int KS = (RP + 3) / 4; };

__device__ __forceinline__ int res_col(int v, int lane) { return 4 * (lane >> 4) + v; }

// The loaders read a clamped in-bounds address on every lane and zero the
// padding afterwards, so no load sits behind a lane-dependent branch (m, n
// and RP are at least 1).
template <int RP>
__device__ __forceinline__ void res_load_u(const float* __restrict__ UL, int64_t m, int64_t r0,
                                           int lane, float (&a)[ResK<RP>::KS]) {
  const int64_t row = r0 + (lane & 15);
  const int64_t rowc = row < m ? row : m - 1;
  const int g = lane >> 4;
#pragma unroll
  for (int s = 0; s < ResK<RP>::KS; ++s) {
    const int k = 4 * s + g;
    const int kc = k < RP ? k : RP - 1;
    const float u = UL[rowc * RP + kc];
    a[s] = (k < RP && row < m) ? u : 0.f;
  }
}

// V operand from V_L^T (RP x ldv).
template <int RP>
__device__ __forceinline__ void res_load_vt(const float* __restrict__ VLt, int64_t ldv,
                                            int64_t n, int64_t c0, int lane,
                                            float (&b)[ResK<RP>::KS]) {
  const int64_t col = c0 + (lane & 15);
  const int64_t colc = col < n ? col : n - 1;
  const int g = lane >> 4;
#pragma unroll
  for (int s = 0; s < ResK<RP>::KS; ++s) {
    const int k = 4 * s + g;
    const int kc = k < RP ? k : RP - 1;
    const float v = VLt[kc * ldv + colc];
    b[s] = (k < RP && col < n) ? v : 0.f;
  }
}

// V operand from V_L (n x RP, row-major): the same values.
template <int RP>
__device__ __forceinline__ void res_load_v(const float* __restrict__ VL, int64_t n, int64_t c0,
                                           int lane, float (&b)[ResK<RP>::KS]) {
  const int64_t col = c0 + (lane & 15);
  const int64_t colc = col < n ? col : n - 1;
  const int g = lane >> 4;
#pragma unroll
  for (int s = 0; s < ResK<RP>::KS; ++s) {
    const int k = 4 * s + g;
    const int kc = k < RP ? k : RP - 1;
    const float v = VL[colc * RP + kc];
    b[s] = (k < RP && col < n) ? v : 0.f;
  }
}

// u: the U_L operand (res_load_u), v: the V_L operand (res_load_vt or
// res_load_v).
template <int RP>
__device__ __forceinline__ f32x4_t res_tile(const float (&u)[ResK<RP>::KS],
                                            const float (&v)[ResK<RP>::KS]) {
  f32x4_t acc = {};
#pragma unroll
  for (int s = 0; s < ResK<RP>::KS; ++s)
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(v[s], u[s], acc, 0, 0, 0);
  return acc;
}

__device__ __forceinline__ float res_pick(const f32x4_t& L, int v) {
  float out = L[0];
  out = (v == 1) ? L[1] : out;
  out = (v == 2) ? L[2] : out;
  out = (v == 3) ? L[3] : out;
  return out;
}

constexpr int kRowsPerTile = 64;
// per-wave candidate staging (entries), sized to keep the pass under 64 KB LDS
template <typename T>
constexpr int wave_buf() { return sizeof(T) == 8 ? 256 : 512; }
constexpr int kHistRep = kHistReplicas;

__device__ __forceinline__ int digit_bits(int pbits, int kbits) {
  if (pbits == 0) return kHistBits0;
  const int rem = kbits - pbits;
  return rem < kHistBits ? rem : kHistBits;
}

template <typename T, int RP>
constexpr int sel_cpt() {
  if (sizeof(T) == 8) return RP <= 8 ? 4 : (RP <= 16 ? 2 : 1);
  return RP <= 24 ? 4 : 2;
}

// Candidate output of a collecting pass.  Wave w of block b owns the
// segment number b * kSelWaves + w, entries [seg * seg_cap, (seg + 1) *
// seg_cap) of the candidate arrays.  Its fill is wave-uniform (kept in a
// scalar register and advanced by ballot counts), so appending needs no
// atomics.  Appended entries first go to the wave's ring of kSegRing slots
// in LDS; whenever 64 are pending they leave as one fully populated store
// per array (lane l writes logical position flushed + l).  Positions at or
// beyond a full segment go to the spill region [cap, 2 * cap) through the
// global counter plan->ncand.  Whenever the total fits in cap, every entry
// is kept.  Each wave publishes its segment fill in seg_count[seg] at the
// end of the pass (seg_close writes out the last pending entries first).
constexpr int kSelWaves = 4;   // waves per block of the full-data passes
constexpr int kSegRing = 128;  // ring slots per wave (at most 63 pending + 64 new)

template <typename T>
struct SegSink {
  int64_t* idx;             // candidate arrays (2 * cap entries)
  T* val;
  T* xv;
  long long base;           // first entry of the wave's segment
  unsigned int cap;         // segment capacity
  unsigned int fill;        // wave-uniform fill (logical positions handed out)
  unsigned long long* sp_cnt;  // spill fill counter
  long long sp_cap;         // spill capacity (= cap; the spill starts at cap)
  int64_t* ring_i;          // this wave's LDS ring
  T* ring_v;
  T* ring_x;
  unsigned int flushed;     // wave-uniform: logical positions already stored
};

// Store the ring entry of logical position e (lanes with act).
template <typename T>
__device__ __forceinline__ void seg_emit(SegSink<T>& s, bool act, unsigned int e) {
  if (!act) return;
  const unsigned int slot = e & (kSegRing - 1);
  const int64_t i = s.ring_i[slot];
  const T v = s.ring_v[slot], x = s.ring_x[slot];
  long long pos;
  if (e < s.cap) {
    pos = s.base + e;
  } else {
    const unsigned long long q = atomicAdd(s.sp_cnt, 1ull);
    pos = (long long)q < s.sp_cap ? s.sp_cap + (long long)q : -1;
  }
  if (pos >= 0) {
    s.idx[pos] = i;
    s.val[pos] = v;
    s.xv[pos] = x;
  }
}

// Called by every lane of the wave (uniform control flow); lanes with
// `take` append (idx, r, x).  Positions follow lane order within the wave.
template <typename T>
__device__ __forceinline__ void seg_push(SegSink<T>& s, bool take, int64_t idx, T r, T x) {
  const unsigned long long mask = __ballot(take);
  if (mask == 0ull) return;
  const unsigned int lo = (unsigned int)mask, hi = (unsigned int)(mask >> 32);
  const unsigned int rank = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
  if (take) {
    const unsigned int slot = (s.fill + rank) & (kSegRing - 1);
    s.ring_i[slot] = idx;
    s.ring_v[slot] = r;
    s.ring_x[slot] = x;
  }
  // the fill is wave-uniform: keep it in a scalar register
  s.fill = __builtin_amdgcn_readfirstlane(s.fill + (unsigned int)__popcll(mask));
  if (s.fill - s.flushed >= 64u) {
    // the ring's writes above precede these reads (LDS is in order within a
    // wave; the barrier keeps the compiler from moving them across)
    __builtin_amdgcn_wave_barrier();
    const unsigned int e = s.flushed + (threadIdx.x & 63);
    if (s.flushed + 64u <= s.cap) {
      // wave-uniform common case: the 64 entries stay in the segment (no
      // atomic whose returned value would hold up the loads in flight)
      const unsigned int slot = e & (kSegRing - 1);
      const long long pos = s.base + e;
      s.idx[pos] = s.ring_i[slot];
      s.val[pos] = s.ring_v[slot];
      s.xv[pos] = s.ring_x[slot];
    } else {
      seg_emit(s, true, e);
    }
    s.flushed = __builtin_amdgcn_readfirstlane(s.flushed + 64u);
    __builtin_amdgcn_wave_barrier();
  }
}

// End of a collecting pass: store the entries still in the ring.
template <typename T>
__device__ __forceinline__ void seg_close(SegSink<T>& s) {
  __builtin_amdgcn_wave_barrier();
  const unsigned int l = threadIdx.x & 63;
  seg_emit(s, l < s.fill - s.flushed, s.flushed + l);
  s.flushed = s.fill;
}

// Candidate segments: the nseg wave segments, then the spill region cut
// into chunks of kSpillChunk entries, so that data whose candidates crowd a
// few waves (clustered outliers) spreads its spill over many readers.
constexpr long long kSpillChunk = 1024;
__device__ __forceinline__ int seg_total(const SelPlan* plan) {
  const long long sp = plan->ncand < plan->cap ? plan->ncand : plan->cap;
  return plan->nseg + (int)((sp + kSpillChunk - 1) / kSpillChunk);
}
// Range of candidate segment sg < seg_total(plan).
__device__ __forceinline__ void seg_range(const SelPlan* plan, const unsigned int* seg_count,
                                          int sg, long long& base, long long& cnt) {
  const int nseg = plan->nseg;
  const long long cap = plan->cap;
  if (sg < nseg) {
    base = (long long)sg * (cap / nseg);
    cnt = (long long)seg_count[sg];
  } else {
    const long long sp = plan->ncand < cap ? plan->ncand : cap;
    const long long o = (long long)(sg - nseg) * kSpillChunk;
    base = cap + o;
    const long long left = sp - o;
    cnt = left < 0 ? 0 : (left < kSpillChunk ? left : kSpillChunk);
  }
}

// ---------------------------------------------------------------------------
// Full-data pass.  A block handles tiles of kRowsPerTile rows x 256*CPT
// columns; each thread owns CPT consecutive columns (their V_L rows live in
// registers, read from V_L^T with coalesced loads) and reads the U_L row
// from LDS as a broadcast.  What a pass does with each residual key is set
// by three switches, resolved outside the row loop:
//   HIST  histogram (key >> shift) & mask over the keys in [klo, klo + kspan)
//   TAKE  append every key >= kmin (kmin >= 1, so zeros are never taken)
//   S2    sum R^2 over all entries
// Uses: level-0 histogram (HIST over every key, with S2, in pass 0), deeper
// digits (HIST inside the bucket), collection (TAKE from the bucket low
// key, or from the threshold key + 1 when ties are resolved by index), and
// the carried-window pass 0 (HIST + TAKE + S2 over the window).
// ---------------------------------------------------------------------------
template <typename T>
struct PassKeys {
  typename KeyBits<T>::key_t klo, kspan, kmin, mask;
  int shift;
};

template <typename T, int RP, int CPT, bool HIST, bool TAKE, bool S2, bool FULL, bool VEC>
__device__ __forceinline__ void sel_tile(const T* __restrict__ X, int64_t ldx, int64_t n,
                                         int64_t i0, int nr, int64_t j0, const T* us,
                                         const T (&v)[CPT][RP], unsigned int* lh,
                                         const PassKeys<T>& pk, SegSink<T>& sink,
                                         double& s2) {
  using K = typename KeyBits<T>::key_t;
  // rows whose X loads are in flight together (fewer when collecting, to
  // leave registers for the append)
  constexpr int G = TAKE ? 2 : 4;
  T xa[G][CPT], xb[G][CPT];
  auto load_group = [&](T (&xx)[G][CPT], int gi) {
#pragma unroll
    for (int a = 0; a < G; ++a) {
      const int64_t i = i0 + gi + a;
      const bool rok = gi + a < nr;
      if constexpr (VEC && CPT == 4 && sizeof(T) == 4) {
        if (rok) {
          const float4 q = *reinterpret_cast<const float4*>(X + i * ldx + j0);
          xx[a][0] = q.x; xx[a][1] = q.y; xx[a][2] = q.z; xx[a][3] = q.w;
        } else {
#pragma unroll
          for (int t = 0; t < CPT; ++t) xx[a][t] = T(0);
        }
      } else {
#pragma unroll
        for (int t = 0; t < CPT; ++t)
          xx[a][t] = (rok && (FULL || j0 + t < n)) ? X[i * ldx + j0 + t] : T(0);
      }
    }
  };
  load_group(xa, 0);
  for (int gi = 0; gi < nr; gi += G) {
    if (gi + G < nr) load_group(xb, gi + G);
#pragma unroll
    for (int a = 0; a < G; ++a) {
      const int ii = gi + a;
      const bool rok = ii < nr;
      T u[RP];
#pragma unroll
      for (int c = 0; c < RP; ++c) u[c] = us[(rok ? ii : 0) * RP + c];
#pragma unroll
      for (int t = 0; t < CPT; ++t) {
        const bool ok = rok && (FULL || j0 + t < n);
        T acc = T(0);
#pragma unroll
        for (int c = 0; c < RP; ++c) acc = fma_t(u[c], v[t][c], acc);
        const T r = xa[a][t] - acc;
        const K key = (K)abs_key(r);
        if constexpr (S2) {
          if (ok) s2 += (double)r * (double)r;
        }
        if constexpr (HIST) {
          if (ok && (K)(key - pk.klo) < pk.kspan) atomicAdd(&lh[(key >> pk.shift) & pk.mask], 1u);
        }
        if constexpr (TAKE) seg_push(sink, ok && key >= pk.kmin, (i0 + ii) * n + j0 + t, r, xa[a][t]);
      }
    }
#pragma unroll
    for (int a = 0; a < G; ++a)
#pragma unroll
      for (int t = 0; t < CPT; ++t) xa[a][t] = xb[a][t];
  }
}

// FP32 full-data pass on the matrix cores.  The matrix is cut into column
// strips of 4 * 16 * WT columns (wave w owns the WT 16-column tiles
// [16 WT w, 16 WT (w + 1)) of a strip) and 16-row bands; work unit = one
// (strip, band) pair, in strip-major order, and block b takes the units
// [W b / G, W (b + 1) / G) of the W units (G blocks).  A wave keeps the V_L
// operand of its WT tiles in registers while it walks down the bands of a
// strip, so per band it loads only the U_L operand and the band's X entries
// (all WT tiles issued before the first is used).  The candidates a wave
// appends lie in one 16 WT-column strip, in band order (local for the later
// scattered updates of D).  Bands wholly inside the matrix (and a 16-byte
// aligned X) take a path without bounds checks; in the carried-window pass
// (HIST and TAKE together, whose key windows coincide) one comparison serves
// both.
template <int RP> struct ResStrip {
  // four tiles per wave keep the pass within 128 registers (four waves per
  // SIMD at four blocks per CU)
  static constexpr int WT = 4;               // tiles per wave
  static constexpr int COLS = 4 * 16 * WT;   // columns per strip
};

template <int RP, bool HIST, bool TAKE, bool S2, bool FULL>
__device__ __forceinline__ void sel_band_mfma(const float* __restrict__ X, int64_t ldx,
                                              int64_t m, int64_t n, int64_t r0, int64_t cw,
                                              int nt, const float (&a)[ResK<RP>::KS],
                                              const float (&b)[ResStrip<RP>::WT][ResK<RP>::KS],
                                              unsigned int* lh, const PassKeys<float>& pk,
                                              SegSink<float>& sink, double& s2, bool vec_ok) {
  using K = uint32_t;
  constexpr int WT = ResStrip<RP>::WT;
  const int lane = threadIdx.x & 63;
  const int64_t row = r0 + (lane & 15);
  const bool rowok = FULL || row < m;
  const int cg = res_col(0, lane);
  const float* xrow = X + (rowok ? row : 0) * ldx;
  const int ntt = FULL ? WT : nt;
  float x[WT][4];
#pragma unroll
  for (int t = 0; t < WT; ++t) {
    if (t < ntt) {
      const int64_t col = cw + 16 * t + cg;
      if (FULL) {
        const float4 q = *reinterpret_cast<const float4*>(xrow + col);
        x[t][0] = q.x; x[t][1] = q.y; x[t][2] = q.z; x[t][3] = q.w;
      } else if (vec_ok && rowok && col + 3 < n) {
        const float4 q = *reinterpret_cast<const float4*>(xrow + col);
        x[t][0] = q.x; x[t][1] = q.y; x[t][2] = q.z; x[t][3] = q.w;
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float xv = xrow[col + v < n ? col + v : n - 1];
          x[t][v] = (rowok && col + v < n) ? xv : 0.f;
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < WT; ++t) {
    if (t < ntt) {
      const int64_t col0 = cw + 16 * t + cg;
      const f32x4_t L = res_tile<RP>(a, b[t]);
      double t2 = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool ok = FULL || (rowok && col0 + v < n);
        const float r = x[t][v] - L[v];
        const K key = (K)abs_key(r);
        if constexpr (S2) {
          if (ok) t2 = fma((double)r, (double)r, t2);
        }
        if constexpr (HIST && TAKE) {
          const bool c = ok && key >= pk.kmin;
          if (c) atomicAdd(&lh[(key >> pk.shift) & pk.mask], 1u);
          seg_push(sink, c, row * n + col0 + v, r, x[t][v]);
        } else {
          if constexpr (HIST) {
            if (ok && (K)(key - pk.klo) < pk.kspan)
              atomicAdd(&lh[(key >> pk.shift) & pk.mask], 1u);
          }
          if constexpr (TAKE)
            seg_push(sink, ok && key >= pk.kmin, row * n + col0 + v, r, x[t][v]);
        }
      }
      if constexpr (S2) s2 += t2;
    }
  }
}

template <int RP, bool HIST, bool TAKE, bool S2>
__device__ __forceinline__ void sel_pass_mfma(const float* __restrict__ X, int64_t ldx,
                                              const float* __restrict__ UL,
                                              const float* __restrict__ VLt, int64_t ldv,
                                              int64_t m, int64_t n, unsigned int* lh,
                                              const PassKeys<float>& pk, SegSink<float>& sink,
                                              double& s2, bool vec_ok) {
  constexpr int KS = ResK<RP>::KS;
  constexpr int WT = ResStrip<RP>::WT;
  constexpr int SC = 16 * WT;   // columns per wave
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform (SGPR)
  const int64_t nstrip = (n + ResStrip<RP>::COLS - 1) / ResStrip<RP>::COLS;
  const int64_t nband = (m + 15) / 16;
  const int64_t units = nstrip * nband;
  const int64_t u0 = units * blockIdx.x / gridDim.x;
  const int64_t u1 = units * (blockIdx.x + 1) / gridDim.x;
  float b[WT][KS];
  int64_t have = -1;   // strip whose V_L operand b holds
  for (int64_t u = u0; u < u1; ++u) {
    const int64_t st = u / nband, band = u - st * nband;
    const int64_t cw = st * ResStrip<RP>::COLS + (int64_t)SC * wave;
    if (cw >= n) continue;   // wave-uniform
    if (st != have) {
#pragma unroll
      for (int t = 0; t < WT; ++t) res_load_vt<RP>(VLt, ldv, n, cw + 16 * t, lane, b[t]);
      have = st;
    }
    const int64_t r0 = band * 16;
    float a[KS];
    res_load_u<RP>(UL, m, r0, lane, a);
    const int nt = (int)(((n - cw) + 15) / 16 < WT ? ((n - cw) + 15) / 16 : WT);
    const bool full = vec_ok && r0 + 16 <= m && cw + SC <= n;   // wave-uniform
    if (full)
      sel_band_mfma<RP, HIST, TAKE, S2, true>(X, ldx, m, n, r0, cw, nt, a, b, lh, pk, sink, s2,
                                              vec_ok);
    else
      sel_band_mfma<RP, HIST, TAKE, S2, false>(X, ldx, m, n, r0, cw, nt, a, b, lh, pk, sink,
                                               s2, vec_ok);
  }
}

template <typename T, int RP, bool HIST, bool TAKE, bool S2>
__device__ __forceinline__ void sel_pass_body(const T* __restrict__ X, int64_t ldx,
                                              const T* __restrict__ UL,
                                              const T* __restrict__ VLt, int64_t ldv,
                                              int64_t m, int64_t n, unsigned int* lh, T* us,
                                              const PassKeys<T>& pk, SegSink<T>& sink,
                                              bool vec_ok, double& s2) {
  if constexpr (sizeof(T) == 4) {
    sel_pass_mfma<RP, HIST, TAKE, S2>(X, ldx, UL, VLt, ldv, m, n, lh, pk, sink, s2, vec_ok);
  } else {
  constexpr int CPT = sel_cpt<T, RP>();
  constexpr int TW = 256 * CPT;
  const int tid = threadIdx.x;
  const int64_t ctiles = (n + TW - 1) / TW;
  const int64_t rtiles = (m + kRowsPerTile - 1) / kRowsPerTile;
  const int64_t ntiles = ctiles * rtiles;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t ct = tile % ctiles, rt = tile / ctiles;
    const int64_t j0 = ct * TW + (int64_t)tid * CPT;
    const int64_t i0 = rt * kRowsPerTile;
    const int nr = (m - i0) < kRowsPerTile ? (int)(m - i0) : kRowsPerTile;
    __syncthreads();
    for (int e = tid; e < kRowsPerTile * RP; e += 256)
      us[e] = (e < nr * RP) ? UL[i0 * RP + e] : T(0);
    __syncthreads();
    // V_L^T (RP x ldv): lanes read consecutive columns of each row
    T v[CPT][RP];
#pragma unroll
    for (int c = 0; c < RP; ++c)
#pragma unroll
      for (int t = 0; t < CPT; ++t) v[t][c] = (j0 + t < n) ? VLt[c * ldv + j0 + t] : T(0);
    const bool full = (ct + 1) * TW <= n;   // block-uniform
    if (full && vec_ok)
      sel_tile<T, RP, CPT, HIST, TAKE, S2, true, true>(X, ldx, n, i0, nr, j0, us, v, lh, pk,
                                                       sink, s2);
    else if (full)
      sel_tile<T, RP, CPT, HIST, TAKE, S2, true, false>(X, ldx, n, i0, nr, j0, us, v, lh, pk,
                                                        sink, s2);
    else
      sel_tile<T, RP, CPT, HIST, TAKE, S2, false, false>(X, ldx, n, i0, nr, j0, us, v, lh, pk,
                                                         sink, s2);
  }
  }
}

// Key switches of the level-0 histogram over every key.
template <typename T>
__device__ __forceinline__ PassKeys<T> keys_level0() {
  using K = typename KeyBits<T>::key_t;
  constexpr int KB = KeyBits<T>::value;
  PassKeys<T> pk;
  pk.klo = 0;
  pk.kspan = (K)(K(1) << KB);
  pk.kmin = 1;
  pk.shift = KB - kHistBits0;
  pk.mask = (K)(kHistBins - 1);
  return pk;
}

// Common prologue of the two full-pass kernels.
#define GODEC_SEL_SHARED                                                      \
  constexpr int KB = KeyBits<T>::value;                                       \
  using K = typename KeyBits<T>::key_t;                                       \
  __shared__ unsigned int lh[kHistBins];                                      \
  __shared__ T us[kRowsPerTile * RP];                                         \
  __shared__ double red[4];                                                   \
  const int tid = threadIdx.x;                                                \
  const int lane = tid & 63;                                                  \
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);                  \
  (void)KB; (void)red;                                                        \
  const long long ccap = plan->cap;                                           \
  const unsigned int seg_cap = (unsigned int)(ccap / ((long long)gridDim.x * kSelWaves)); \
  const int seg = (int)blockIdx.x * kSelWaves + wave;                         \
  __shared__ int64_t ring_i[kSelWaves * kSegRing];                            \
  __shared__ T ring_v[kSelWaves * kSegRing], ring_x[kSelWaves * kSegRing];    \
  SegSink<T> sink{cand_idx, cand_val, cand_x, (long long)seg * seg_cap, seg_cap, 0u, \
                  (unsigned long long*)&plan->ncand, ccap, ring_i + wave * kSegRing, \
                  ring_v + wave * kSegRing, ring_x + wave * kSegRing, 0u};

// Closing of a collecting pass: publish the wave's segment fill.
#define GODEC_SEL_SEG_CLOSE                                                   \
  seg_close(sink);                                                            \
  if (lane == 0) seg_count[seg] = sink.fill < seg_cap ? sink.fill : seg_cap;

// Pass 0: the carried-window pass (steady state) or the full level-0
// histogram (first iteration); both also sum R^2.  With r16, the blocks
// first restore bf16(X) at the previous S's entries of that copy (scattered
// 2-byte stores that overlap the pass).
template <typename T, int RP>
__global__ __launch_bounds__(256) void k_sel_pass0(const T* __restrict__ X, int64_t ldx,
                                                   const T* __restrict__ UL,
                                                   const T* __restrict__ VLt, int64_t ldv,
                                                   int64_t m, int64_t n,
                                                   SelPlan* __restrict__ plan,
                                                   unsigned long long* __restrict__ hist,
                                                   int64_t* __restrict__ cand_idx,
                                                   T* __restrict__ cand_val,
                                                   T* __restrict__ cand_x,
                                                   unsigned int* __restrict__ seg_count,
                                                   double* __restrict__ s2part,
                                                   uint16_t* __restrict__ r16, int64_t ldd16,
                                                   const int64_t* __restrict__ ridx,
                                                   const float* __restrict__ rx,
                                                   const SelPlan* __restrict__ rplan) {
  GODEC_SEL_SHARED
  if (r16 != nullptr) {
    // eight entries per thread in flight at once (one round trip per batch)
    constexpr int B = 8;
    const long long cnt = rplan->nnz;
    const double rn = 1.0 / (double)n;
    const long long stride = (long long)gridDim.x * 256;
    for (long long e0 = (long long)blockIdx.x * 256 + tid; e0 < cnt; e0 += B * stride) {
      int64_t id[B];
      float xv[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const long long e = e0 + b * stride;
        id[b] = e < cnt ? ridx[e] : -1;
        xv[b] = e < cnt ? rx[e] : 0.f;
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (id[b] < 0) continue;
        int64_t i, j;
        divmod_nn(id[b], n, rn, i, j);
        r16[i * ldd16 + j] = f32_to_bf16(xv[b]);
      }
    }
  }
  if (plan->mode != SEL_HIST) {
    // k == 0 (S_t = 0): only the objective, sum R^2 over every entry
    const bool vec_ok0 = (ldx % 4 == 0) && ((((uintptr_t)X) & 15) == 0);
    PassKeys<T> pk0 = keys_level0<T>();
    double s20 = 0.0;
    sel_pass_body<T, RP, false, false, true>(X, ldx, UL, VLt, ldv, m, n, lh, us, pk0, sink,
                                             vec_ok0, s20);
    s20 = wave_sum(s20);
    if (lane == 0) red[wave] = s20;
    __syncthreads();
    if (tid == 0) s2part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    return;
  }
  const int carry = plan->carry_used;
  PassKeys<T> pk = keys_level0<T>();
  if (carry) {
    // histogram and collect the window [dlo-th level-0 digit, top)
    const K lo = (K)plan->carry_dlo << (KB - kHistBits0);
    pk.klo = lo > 0 ? lo : K(1);
    pk.kspan = (K)((K(1) << KB) - pk.klo);
    pk.kmin = pk.klo;
  }
  for (int e = tid; e < kHistBins; e += 256) lh[e] = 0u;
  const bool vec_ok = (ldx % 4 == 0) && ((((uintptr_t)X) & 15) == 0);
  __syncthreads();
  double s2 = 0.0;
  if (carry)
    sel_pass_body<T, RP, true, true, true>(X, ldx, UL, VLt, ldv, m, n, lh, us, pk, sink,
                                           vec_ok, s2);
  else
    sel_pass_body<T, RP, true, false, true>(X, ldx, UL, VLt, ldv, m, n, lh, us, pk, sink,
                                            vec_ok, s2);
  __syncthreads();
  if (carry) { GODEC_SEL_SEG_CLOSE }
  unsigned long long* hrep = hist + (int64_t)(blockIdx.x % kHistRep) * kHistBins;
  for (int e = tid; e < kHistBins; e += 256)
    if (lh[e]) atomicAdd(&hrep[e], (unsigned long long)lh[e]);
  s2 = wave_sum(s2);
  if (lane == 0) red[wave] = s2;
  __syncthreads();
  // per-block partial; k_sel_plan adds them in block order
  if (tid == 0) s2part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Later passes (first iteration and fall-backs): the level-0 histogram
// again (after a missed carry), deeper digits, collection from the bucket,
// or collection above a resolved threshold whose ties overflow the buffer.
// Advance the plan.  One block.  stage 0 follows a full-data pass (which
// histogrammed in SEL_HIST or collected in SEL_COLLECT); stage 1 follows a
// candidate histogram (SEL_REFINE).  In any other combination the preceding
// kernel did nothing and neither does this one.  The digit holding the
// k_rem-th largest key is found with a block-wide suffix scan.
//
// sel_plan_core runs either as the kernel k_sel_plan (COH = false) or in
// the last block to finish the pass or candidate histogram it follows
// (COH = true): then the histogram, which the pass's blocks added to with
// device-scope atomics, and the spill counter are read with device-scope
// loads, and the bins are counted in 32 bits in the pass's own LDS (the
// host uses this form only when m n < 2^32).
template <bool COH>
__device__ __forceinline__ unsigned long long hist_load(const unsigned long long* p) {
  if constexpr (COH)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}
template <bool COH>
__device__ __forceinline__ long long ncand_load(const SelPlan* plan) {
  if constexpr (COH)
    return __hip_atomic_load(&plan->ncand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return plan->ncand;
}

template <typename T, typename HT, bool COH>
__device__ void sel_plan_core(SelPlan* __restrict__ plan, unsigned long long* __restrict__ hist,
                              int stage, HT* h, unsigned long long* part, int* sel_t) {
  constexpr int KB = KeyBits<T>::value;
  const int tid = threadIdx.x;
  const int mode = plan->mode;
  if (stage == 0 && (mode == SEL_COLLECT || mode == SEL_TIES)) {
    if (tid == 0) {
      if (ncand_load<COH>(plan) > plan->cap) plan->overflow = 1;
      if (mode == SEL_TIES) plan->mode = SEL_TSCAN;
      else plan->mode = (plan->pbits == KB) ? SEL_FINAL : SEL_REFINE;
    }
    return;
  }
  if (!((stage == 0 && mode == SEL_HIST) || (stage == 1 && mode == SEL_REFINE))) return;
  const int pbits = plan->pbits;
  const int dbits = digit_bits(pbits, KB);
  const int bins = 1 << dbits;
  const int per = (bins + 255) / 256;
  // sum the replicas in replica order (and clear them for the next
  // histogram); every load of a batch is issued before the first add: all
  // of the thread's bins at once in the kernel, UB bins at a time in the
  // last block of a pass (whose register budget is the pass's)
  constexpr int MAXPER = (kHistBins + 255) / 256;
  constexpr int UB = COH ? 2 : MAXPER;
  for (int u0 = 0; u0 < MAXPER; u0 += UB) {
    unsigned long long v[UB][kHistRep];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int e = tid + 256 * (u0 + u);
#pragma unroll
      for (int r = 0; r < kHistRep; ++r)
        v[u][r] = e < bins ? hist_load<COH>(hist + r * kHistBins + e) : 0ull;
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int e = tid + 256 * (u0 + u);
      if (e < bins) {
        unsigned long long acc = 0;
#pragma unroll
        for (int r = 0; r < kHistRep; ++r) {
          acc += v[u][r];
          hist[r * kHistBins + e] = 0ull;
        }
        h[e] = (HT)acc;
      }
    }
  }
  __syncthreads();
  // thread t owns digits [bins - (t+1)*per, bins - t*per): top digits first
  unsigned long long s = 0;
  for (int u = 0; u < per; ++u) {
    const int d = bins - 1 - (tid * per + u);
    if (d >= 0) s += h[d];
  }
  part[tid] = s;
  if (tid == 0) *sel_t = -1;
  __syncthreads();
  // inclusive scan of part[] (Hillis-Steele)
  for (int off = 1; off < 256; off <<= 1) {
    const unsigned long long add = tid >= off ? part[tid - off] : 0ull;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  const long long k_rem = plan->k_rem;
  const unsigned long long before = tid > 0 ? part[tid - 1] : 0ull;
  if (before < (unsigned long long)k_rem && part[tid] >= (unsigned long long)k_rem) *sel_t = tid;
  __syncthreads();
  if (tid == 0) {
    int dsel = -1;
    unsigned long long cum = 0;
    if (*sel_t >= 0) {
      cum = *sel_t > 0 ? part[*sel_t - 1] : 0ull;
      for (int u = 0; u < per; ++u) {
        const int d = bins - 1 - (*sel_t * per + u);
        if (d < 0) break;
        if (cum + h[d] >= (unsigned long long)k_rem) { dsel = d; break; }
        cum += h[d];
      }
    }
    if (stage == 0 && pbits == 0 && plan->carry_used == 1) {
      // pass 0 histogrammed and collected only digits >= carry_dlo: accept
      // when the k-th key lies there and every candidate was kept;
      // otherwise fall back to the full level-0 histogram in the next pass
      if (dsel < 0 || ncand_load<COH>(plan) > plan->cap) {
        plan->carry_used = 0;
        plan->ncand = 0;
        plan->slow = 1;
        plan->mode = SEL_HIST;   // prefix 0, pbits 0, k_rem = k unchanged
        return;
      }
      plan->carry_used = 2;
      plan->count_above += (long long)cum;
      plan->k_rem = k_rem - (long long)cum;
      plan->prefix = (unsigned long long)dsel;
      plan->pbits = dbits;
      plan->bucket_count = (long long)h[dsel];
      plan->mode = (plan->pbits == KB) ? SEL_FINAL : SEL_REFINE;
      return;
    }
    if (dsel < 0) {
      // fewer keys than k_rem in the bucket: only when the remaining keys
      // are zeros (excluded from the candidates); settle on digit 0
      dsel = 0;
      cum = part[255] - h[0];
    }
    plan->count_above += (long long)cum;
    plan->k_rem = k_rem - (long long)cum;
    plan->prefix = (plan->prefix << dbits) | (unsigned long long)dsel;
    plan->pbits = pbits + dbits;
    plan->bucket_count = (long long)h[dsel];
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
}

template <typename T>
__global__ __launch_bounds__(256) void k_sel_plan(SelPlan* __restrict__ plan,
                                                  unsigned long long* __restrict__ hist,
                                                  int stage, const double* __restrict__ s2part,
                                                  int ns2) {
  __shared__ unsigned long long h[kHistBins];
  __shared__ unsigned long long part[256];
  __shared__ int sel_t;
  __shared__ double red[8];
  if (s2part) {
    // right after pass 0: its per-block sums of R^2, added in block order
    const double s = block_sum_fixed(s2part, ns2, red);
    if (threadIdx.x == 0) plan->sum_r2 = s;
  }
  sel_plan_core<T, unsigned long long, false>(plan, hist, stage, h, part, &sel_t);
}

// End of a pass or candidate histogram that plans in its last block: every
// block waits for its histogram atomics and stores to complete and signals
// arrival; the last one resets the counter and advances the plan in the
// LDS the pass no longer needs (h: kHistBins 32-bit bins, part: 256 u64).
template <typename T>
__device__ __forceinline__ void plan_in_last_block(SelPlan* __restrict__ plan,
                                                   unsigned long long* __restrict__ hist,
                                                   int stage, unsigned int* h,
                                                   unsigned long long* part, int* flags) {
  stores_done();
  __syncthreads();
  if (threadIdx.x == 0) flags[0] = arrive(&plan->arrivals) == gridDim.x - 1u;
  __syncthreads();
  if (!flags[0]) return;
  if (threadIdx.x == 0) publish_u32(&plan->arrivals, 0u);
  sel_plan_core<T, unsigned int, true>(plan, hist, stage, h, part, flags + 1);
}

template <typename T, int RP>
__global__ __launch_bounds__(256) void k_sel_passN(const T* __restrict__ X, int64_t ldx,
                                                   const T* __restrict__ UL,
                                                   const T* __restrict__ VLt, int64_t ldv,
                                                   int64_t m, int64_t n,
                                                   SelPlan* __restrict__ plan,
                                                   unsigned long long* __restrict__ hist,
                                                   int64_t* __restrict__ cand_idx,
                                                   T* __restrict__ cand_val,
                                                   T* __restrict__ cand_x,
                                                   unsigned int* __restrict__ seg_count,
                                                   int fuse_plan) {
  const int mode = plan->mode;
  if (mode != SEL_HIST && mode != SEL_COLLECT && mode != SEL_TIES) return;
  GODEC_SEL_SHARED
  __shared__ int pl_flags[2];
  const unsigned long long prefix = plan->prefix;
  const int pbits = plan->pbits;
  const int dbits = digit_bits(pbits, KB);
  const bool do_hist = (mode == SEL_HIST);
  PassKeys<T> pk = keys_level0<T>();
  if (pbits > 0) {
    pk.klo = (K)(prefix << (KB - pbits));
    pk.kspan = (K)(K(1) << (KB - pbits));
    pk.shift = KB - pbits - dbits;
    pk.mask = (K)((K(1) << dbits) - 1);
    pk.kmin = pk.klo > 0 ? pk.klo : K(1);
  }
  if (mode == SEL_TIES) pk.kmin = (K)prefix + 1;   // prefix is the full threshold key
  if (do_hist)
    for (int e = tid; e < kHistBins; e += 256) lh[e] = 0u;
  const bool vec_ok = (ldx % 4 == 0) && ((((uintptr_t)X) & 15) == 0);
  __syncthreads();
  double s2 = 0.0;
  if (do_hist)
    sel_pass_body<T, RP, true, false, false>(X, ldx, UL, VLt, ldv, m, n, lh, us, pk, sink,
                                             vec_ok, s2);
  else
    sel_pass_body<T, RP, false, true, false>(X, ldx, UL, VLt, ldv, m, n, lh, us, pk, sink,
                                             vec_ok, s2);
  __syncthreads();
  if (!do_hist) { GODEC_SEL_SEG_CLOSE }
  if (do_hist) {
    const int bins = 1 << dbits;
    unsigned long long* hrep = hist + (int64_t)(blockIdx.x % kHistRep) * kHistBins;
    for (int e = tid; e < bins; e += 256)
      if (lh[e]) atomicAdd(&hrep[e], (unsigned long long)lh[e]);
  }
  // the plan step in the last block (its LDS: lh for the bins, the index
  // ring for the scan)
  if (fuse_plan)
    plan_in_last_block<T>(plan, hist, 0, lh, reinterpret_cast<unsigned long long*>(ring_i),
                          pl_flags);
}

// Histogram of the next digit over the candidates inside the bucket.
template <typename T>
__global__ __launch_bounds__(256) void k_cand_hist(SelPlan* __restrict__ plan,
                                                   const T* __restrict__ cand_val,
                                                   const unsigned int* __restrict__ seg_count,
                                                   unsigned long long* __restrict__ hist) {
  constexpr int KB = KeyBits<T>::value;
  __shared__ unsigned int lh[kHistBins];
  if (plan->mode != SEL_REFINE) return;
  const unsigned long long prefix = plan->prefix;
  const int pbits = plan->pbits;
  const int dbits = digit_bits(pbits, KB);
  for (int e = threadIdx.x; e < (1 << dbits); e += 256) lh[e] = 0u;
  __syncthreads();
  const int ntot = seg_total(plan);
  for (int sg = blockIdx.x; sg < ntot; sg += gridDim.x) {
    long long base, cnt;
    seg_range(plan, seg_count, sg, base, cnt);
    for (long long c = base + threadIdx.x; c < base + cnt; c += 256) {
      const unsigned long long key = abs_key(cand_val[c]);
      if ((key >> (KB - pbits)) == prefix)
        atomicAdd(&lh[(key >> (KB - pbits - dbits)) & ((1ull << dbits) - 1)], 1u);
    }
  }
  __syncthreads();
  unsigned long long* hrep = hist + (int64_t)(blockIdx.x % kHistRep) * kHistBins;
  for (int e = threadIdx.x; e < (1 << dbits); e += 256)
    if (lh[e]) atomicAdd(&hrep[e], (unsigned long long)lh[e]);
}

// FINAL: write S from the candidates.  Entries above the threshold key go
// straight to S; entries equal to it go to the tie list.  Wave w of block b
// takes the candidate segments 4 b + w, 4 b + w + 4 gridDim.x, ...: the
// waves count their entries, the block reserves its output range with one
// atomic per list, and each wave then writes its entries in order (ballots
// only, no block barrier), 256 candidates per step.
template <typename T>
__global__ __launch_bounds__(256) void k_sel_compact(SelPlan* __restrict__ plan,
                                                     const int64_t* __restrict__ cand_idx,
                                                     const T* __restrict__ cand_val,
                                                     const T* __restrict__ cand_x,
                                                     const unsigned int* __restrict__ seg_count,
                                                     int64_t* __restrict__ s_idx,
                                                     T* __restrict__ s_val,
                                                     T* __restrict__ s_x,
                                                     int64_t* __restrict__ tie_idx,
                                                     unsigned long long* __restrict__ counters,
                                                     double* __restrict__ s2sel,
                                                     T* __restrict__ dwn,
                                                     uint16_t* __restrict__ dw16,
                                                     int64_t lddw, int64_t ncols) {
  __shared__ double red[4];
  __shared__ unsigned int wa[4], wt[4];
  __shared__ unsigned long long base_a, base_t;
  if (plan->mode != SEL_FINAL) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const unsigned long long tkey = plan->prefix;
  const unsigned long long kcap = (unsigned long long)(plan->count_above + plan->k_rem);
  const long long dkeep = plan->count_above;
  const double rcols = 1.0 / (double)(ncols > 0 ? ncols : 1);
  const unsigned long long tcap = (unsigned long long)plan->cap;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int ntot = seg_total(plan);
  const int wstride = 4 * (int)gridDim.x;
  const int w0 = 4 * (int)blockIdx.x + wave;
  // phase 1: per-wave counts, one reservation per block and list
  unsigned int na = 0, nt = 0;
  for (int sg = w0; sg < ntot; sg += wstride) {
    long long c0, cnt;
    seg_range(plan, seg_count, sg, c0, cnt);
    for (long long c = c0 + lane; c < c0 + cnt; c += 64) {
      const unsigned long long key = abs_key(cand_val[c]);
      na += key > tkey;
      nt += (key == tkey && tkey > 0);
    }
  }
  na = wave_sum(na);
  nt = wave_sum(nt);
  if (lane == 0) { wa[wave] = na; wt[wave] = nt; }
  __syncthreads();
  if (tid == 0) {
    const unsigned int ta = wa[0] + wa[1] + wa[2] + wa[3];
    const unsigned int tt = wt[0] + wt[1] + wt[2] + wt[3];
    base_a = ta ? atomicAdd(&counters[0], (unsigned long long)ta) : 0ull;
    base_t = tt ? atomicAdd(&counters[1], (unsigned long long)tt) : 0ull;
  }
  __syncthreads();
  unsigned long long ba = base_a, bt = base_t;
  for (int w = 0; w < wave; ++w) { ba += wa[w]; bt += wt[w]; }
  // phase 2: each wave writes its segments in order, four loads in flight
  double s2 = 0.0;
  for (int sg = w0; sg < ntot; sg += wstride) {
    long long c0, cnt;
    seg_range(plan, seg_count, sg, c0, cnt);
    const long long c1 = c0 + cnt;
    for (long long cb = c0; cb < c1; cb += 256) {
      T v[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const long long c = cb + 64 * h + lane;
        v[h] = c < c1 ? cand_val[c] : T(0);
      }
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const long long c = cb + 64 * h + lane;
        const bool valid = c < c1;
        const unsigned long long key = abs_key(v[h]);
        const bool above = valid && key > tkey;
        const bool tie = valid && key == tkey && tkey > 0;
        const unsigned long long ma = __ballot(above), mt = __ballot(tie);
        if (above) {
          const unsigned long long pos = ba + __popcll(ma & below);
          if (pos < kcap) {
            const int64_t id = cand_idx[c];
            const T xv = cand_x[c];
            s_idx[pos] = id;
            s_val[pos] = v[h];
            s_x[pos] = xv;
            s2 += (double)v[h] * (double)v[h];
            // D = X - S at the entries surely kept (the tie list may
            // replace positions from count_above on)
            if ((dwn != nullptr || dw16 != nullptr) && (long long)pos < dkeep) {
              int64_t i, j;
              divmod_nn(id, ncols, rcols, i, j);
              const T dv = (T)(xv - v[h]);
              if (dwn) dwn[i * lddw + j] = dv;
              if constexpr (sizeof(T) == 4)
                if (dw16) dw16[i * lddw + j] = f32_to_bf16(dv);
            }
          }
        }
        if (tie) {
          const unsigned long long pos = bt + __popcll(mt & below);
          if (pos < tcap) tie_idx[pos] = cand_idx[c];
        }
        ba += __popcll(ma);
        bt += __popcll(mt);
      }
    }
  }
  s2 = wave_sum(s2);
  if (lane == 0) red[wave] = s2;
  __syncthreads();
  // per-block partial; k_sel_ties adds them in block order
  if (tid == 0) s2sel[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Resolve ties: keep the k_rem smallest linear indices among the entries
// equal to the threshold key (one block; bitonic sort in LDS when they fit,
// otherwise repeated minimum extraction by a radix select on the index).
// The next iteration histograms and collects from kCarryWindow level-0
// digits below this threshold (1/8 octave for f32 keys, which have 16 digits
// per octave; 1 octave for f64 keys).
template <typename T>
__device__ __forceinline__ void carry_update(SelCarry* carry, unsigned long long tkey) {
  constexpr int KB = KeyBits<T>::value;
  constexpr int W = sizeof(T) == 4 ? 2 : 2;
  const int d = (int)(tkey >> (KB - kHistBits0)) - W;
  carry->dlo = d > 0 ? d : 0;
  carry->valid = 1;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_sel_ties(SelPlan* __restrict__ plan,
                                                   int64_t* __restrict__ s_idx,
                                                   T* __restrict__ s_val,
                                                   int64_t* __restrict__ tie_idx,
                                                   unsigned long long* __restrict__ counters,
                                                   SelCarry* __restrict__ carry,
                                                   const double* __restrict__ s2sel, int nsel) {
  constexpr int KB = KeyBits<T>::value;
  constexpr int NS = 4096;
  __shared__ int64_t sk[NS];
  __shared__ unsigned long long cnt[256];
  __shared__ unsigned long long sh_pref;
  __shared__ long long sh_need;
  __shared__ double red[20];
  const int tid = threadIdx.x;
  if (plan->mode != SEL_FINAL) return;
  // sum of S_t^2 over the entries above the threshold: the compaction's
  // per-block partials in block order
  const double sel_above = block_sum_fixed(s2sel, nsel, red);
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
    plan->sum_sel2 = sel_above + (double)take * (double)tval * (double)tval;
    carry_update<T>(carry, tkey);
  }
}

// After a TIES collection the candidates hold the entries above the
// threshold; the tied entries are taken in index order by one block
// scanning all of X.
// FP32 form of the index-ordered tie scan: bands of 16 rows; the hits of
// each band are counted per row, the rows that fit are taken whole and the
// first row that does not fit is taken in column order by one wavefront
// (the four lanes holding that row of a tile hold its columns 4g .. 4g+3,
// g = lane / 16, so column order is lane-group order, then register order).
// Returns the number of tied entries written at s_idx[base ..].
template <int RP>
__device__ long long ties_scan_mfma(const float* __restrict__ X, int64_t ldx,
                                    const float* __restrict__ UL,
                                    const float* __restrict__ VLt, int64_t ldv, int64_t m,
                                    int64_t n, uint32_t tkey, long long need, long long base,
                                    int64_t* __restrict__ s_idx, float* __restrict__ s_val) {
  constexpr int KS = ResK<RP>::KS;
  __shared__ unsigned int rowcnt[16];
  __shared__ unsigned int wpos, full_cnt, cut_q;
  __shared__ int cut_row;
  __shared__ long long done;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) done = 0;
  __syncthreads();
  for (int64_t r0 = 0; r0 < m; r0 += 16) {
    if (done >= need) break;
    if (tid < 16) rowcnt[tid] = 0u;
    if (tid == 0) wpos = 0u;
    __syncthreads();
    float a[KS];
    res_load_u<RP>(UL, m, r0, lane, a);
    const int lr = lane & 15;
    const int64_t row = r0 + lr;
    // hits per row of the band
    for (int64_t c0 = 16 * wave; c0 < n; c0 += 64) {
      float b[KS];
      res_load_vt<RP>(VLt, ldv, n, c0, lane, b);
      const f32x4_t L = res_tile<RP>(a, b);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t col = c0 + res_col(v, lane);
        if (col < n && row < m && (uint32_t)abs_key(X[row * ldx + col] - L[v]) == tkey)
          atomicAdd(&rowcnt[lr], 1u);
      }
    }
    __syncthreads();
    if (tid == 0) {
      const long long rem = need - done;
      long long acc = 0;
      int cut = 16;
      long long q = 0;
      for (int rr = 0; rr < 16; ++rr) {
        if (acc + (long long)rowcnt[rr] > rem) { cut = rr; q = rem - acc; break; }
        acc += rowcnt[rr];
      }
      cut_row = cut;
      cut_q = (unsigned int)q;
      full_cnt = (unsigned int)acc;
    }
    __syncthreads();
    const int cut = cut_row;
    const long long at = base + done;
    // rows before the cut: every hit (order within S does not matter)
    if (full_cnt > 0u) {
      for (int64_t c0 = 16 * wave; c0 < n; c0 += 64) {
        float b[KS];
        res_load_vt<RP>(VLt, ldv, n, c0, lane, b);
        const f32x4_t L = res_tile<RP>(a, b);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t col = c0 + res_col(v, lane);
          if (lr < cut && col < n && row < m &&
              (uint32_t)abs_key(X[row * ldx + col] - L[v]) == tkey) {
            const unsigned int p = atomicAdd(&wpos, 1u);
            s_idx[at + p] = row * n + col;
            s_val[at + p] = 0.f;
          }
        }
      }
    }
    // the cut row: its first cut_q hits in column order (lanes cut + 16 g
    // hold its columns 4g .. 4g+3 of a tile)
    if (cut < 16 && wave == 0) {
      const unsigned int q = cut_q;
      const int64_t crow = r0 + cut;
      unsigned int got = 0;
      for (int64_t c0 = 0; c0 < n && got < q; c0 += 16) {
        float b[KS];
        res_load_vt<RP>(VLt, ldv, n, c0, lane, b);
        const f32x4_t L = res_tile<RP>(a, b);
        unsigned int hits = 0u;   // bit v: column c0 + 4g + v is a hit
        if (lr == cut && crow < m) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t col = c0 + res_col(v, lane);
            if (col < n && (uint32_t)abs_key(X[crow * ldx + col] - L[v]) == tkey)
              hits |= 1u << v;
          }
        }
        // hits of the lanes cut + 16 g' for g' < g come first
        unsigned int before = 0u, total = 0u;
#pragma unroll
        for (int g2 = 0; g2 < 4; ++g2) {
          const unsigned int h = (unsigned int)__popc(__shfl(hits, cut + 16 * g2, 64));
          if (g2 < (lane >> 4)) before += h;
          total += h;
        }
        if (lr == cut) {
          unsigned int rank = before;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if ((hits >> v) & 1u) {
              if (got + rank < q) {
                s_idx[at + full_cnt + got + rank] = crow * n + c0 + res_col(v, lane);
                s_val[at + full_cnt + got + rank] = 0.f;
              }
              ++rank;
            }
          }
        }
        got = (got + total < q) ? got + total : q;
      }
    }
    __syncthreads();
    if (tid == 0) done += (long long)full_cnt + (cut < 16 ? (long long)cut_q : 0ll);
    __syncthreads();
  }
  return done;
}

template <typename T, int RP>
__global__ __launch_bounds__(256) void k_sel_ties_stream(const T* __restrict__ X, int64_t ldx,
                                                         const T* __restrict__ UL,
                                                         const T* __restrict__ VL,
                                                         const T* __restrict__ VLt, int64_t ldv,
                                                         int64_t m, int64_t n,
                                                         SelPlan* __restrict__ plan,
                                                         const int64_t* __restrict__ cand_idx,
                                                         const T* __restrict__ cand_val,
                                                         const T* __restrict__ cand_x,
                                                         const unsigned int* __restrict__ seg_count,
                                                         int64_t* __restrict__ s_idx,
                                                         T* __restrict__ s_val,
                                                         T* __restrict__ s_x,
                                                         SelCarry* __restrict__ carry) {
  __shared__ T us[RP];
  __shared__ long long taken;
  __shared__ int flags[256];
  if (plan->mode != SEL_TSCAN) return;
  const int tid = threadIdx.x;
  const unsigned long long tkey = plan->prefix;
  // the candidates are exactly the entries above the threshold
  // (count_above of them, all kept since count_above <= cap)
  const long long nabove = plan->count_above;
  double s2 = 0.0;
  long long out = 0;
  const int ntot = seg_total(plan);
  for (int sg = 0; sg < ntot; ++sg) {
    long long base, cnt;
    seg_range(plan, seg_count, sg, base, cnt);
    for (long long e = tid; e < cnt; e += 256) {
      const long long c = base + e;
      if (out + e < nabove) {
        s_idx[out + e] = cand_idx[c];
        s_val[out + e] = cand_val[c];
        s_x[out + e] = cand_x[c];
        s2 += (double)cand_val[c] * (double)cand_val[c];
      }
    }
    out += cnt;
  }
  const long long need = (tkey > 0) ? plan->k_rem : 0;
  if (tid == 0) taken = 0;
  __syncthreads();
  if constexpr (sizeof(T) == 4) {
    const long long got = ties_scan_mfma<RP>(X, ldx, UL, VLt, ldv, m, n, (uint32_t)tkey, need,
                                             nabove, s_idx, s_val);
    if (tid == 0) taken = got;
    __syncthreads();
  } else {
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
    carry_update<T>(carry, tkey);
  }
}

// Restore the sign of tied entries: their stored value is the residual,
// recomputed here from X and the factors (same arithmetic as selection).
// FP32: one wavefront per entry, which evaluates the entry's aligned tile.
template <typename T, int RP>
__global__ __launch_bounds__(256) void k_fix_tie_values(const T* __restrict__ X, int64_t ldx,
                                                        const T* __restrict__ UL,
                                                        const T* __restrict__ VL,
                                                        const T* __restrict__ VLt, int64_t ldv,
                                                        int64_t m, int64_t n,
                                                        const SelPlan* __restrict__ plan,
                                                        const unsigned long long* __restrict__ counters,
                                                        int64_t* __restrict__ s_idx,
                                                        T* __restrict__ s_val,
                                                        T* __restrict__ s_x,
                                                        T* __restrict__ dwn,
                                                        uint16_t* __restrict__ dw16,
                                                        int64_t lddw) {
  // the entries the compaction did not write: the ties (from where the tie
  // list starts), or every entry after a threshold scan (counters[0] = 0)
  long long start = (long long)counters[0];
  if (start > plan->count_above) start = plan->count_above;
  const long long nnz = plan->nnz;
  const bool dupd = dwn != nullptr || dw16 != nullptr;
  // D = X - S at entry (i, j) of the working copies
  auto put_d = [&](int64_t i, int64_t j, T x, T v) {
    const T dv = (T)(x - v);
    if (dwn) dwn[i * lddw + j] = dv;
    if constexpr (sizeof(T) == 4)
      if (dw16) dw16[i * lddw + j] = f32_to_bf16(dv);
  };
  if constexpr (sizeof(T) == 4) {
    constexpr int KS = ResK<RP>::KS;
    const int lane = threadIdx.x & 63;
    const long long nw = (long long)gridDim.x * (blockDim.x >> 6);
    for (long long e = start + (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
         e < nnz; e += nw) {
      const int64_t idx = s_idx[e];
      const int64_t i = idx / n, j = idx % n;
      if (s_val[e] != 0.f) {   // the whole wavefront reads the same entry
        if (dupd && lane == 0) put_d(i, j, s_x[e], s_val[e]);
        continue;
      }
      const int64_t r0 = i - i % 16, c0 = j - j % 16;
      float a[KS], b[KS];
      res_load_u<RP>(UL, m, r0, lane, a);
      res_load_vt<RP>(VLt, ldv, n, c0, lane, b);
      const f32x4_t L = res_tile<RP>(a, b);
      const int li = (int)(i - r0), lj = (int)(j - c0);
      if (lane == li + 16 * (lj >> 2)) {
        const float x = X[i * ldx + j];
        const float sv = x - res_pick(L, lj & 3);
        s_val[e] = sv;
        s_x[e] = x;
        if (dupd) put_d(i, j, x, sv);
      }
    }
    return;
  }
  for (long long e = start + (long long)blockIdx.x * 256 + threadIdx.x; e < nnz;
       e += (long long)gridDim.x * 256) {
    const int64_t idx = s_idx[e];
    const int64_t i = idx / n, j = idx % n;
    if (s_val[e] != T(0)) {
      if (dupd) put_d(i, j, s_x[e], s_val[e]);
      continue;
    }
    T u[RP], v[RP];
#pragma unroll
    for (int c = 0; c < RP; ++c) { u[c] = UL[i * RP + c]; v[c] = VL[j * RP + c]; }
    const T x = X[i * ldx + j];
    const T sv = resid<T, RP>(x, u, v);
    s_val[e] = sv;
    s_x[e] = x;
    if (dupd) put_d(i, j, x, sv);
  }
}

template <typename T>
__global__ void k_sel_reset(SelPlan* plan, unsigned long long* hist,
                            unsigned long long* counters, unsigned int* seg_count, long long k,
                            long long cap, int nseg, const SelCarry* carry) {
  constexpr int KB = KeyBits<T>::value;
  for (int e = threadIdx.x; e < kHistRep * kHistBins; e += blockDim.x) hist[e] = 0ull;
  // empty segments, so that consumers see no candidates when no collecting
  // pass runs (k == 0 goes straight to SEL_FINAL)
  for (int e = threadIdx.x; e < nseg; e += blockDim.x) seg_count[e] = 0u;
  if (threadIdx.x == 0) {
    plan->prefix = 0; plan->k_rem = k; plan->count_above = 0; plan->bucket_count = 0;
    plan->ncand = 0; plan->cap = cap; plan->nnz = 0; plan->pbits = 0; plan->kbits = KB;
    plan->mode = (k > 0) ? SEL_HIST : SEL_FINAL; plan->slow = 0; plan->overflow = 0;
    plan->nseg = nseg;
    plan->sum_r2 = 0.0; plan->sum_sel2 = 0.0; plan->threshold = 0.0;
    plan->carry_used = carry->valid ? 1 : 0;
    plan->carry_dlo = carry->dlo;
    plan->arrivals = 0u;
    counters[0] = 0; counters[1] = 0;
  }
}

// VLt (rp x ldv) <- VL (ldv x rp), both in the residual type.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_panel(const T* __restrict__ VL, int64_t rows,
                                                         int rp, T* __restrict__ VLt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * rp) return;
  const int64_t c = e / rows, j = e % rows;
  VLt[e] = VL[j * rp + c];
}

// ---------------------------------------------------------------------------
// Dense helpers.
// ---------------------------------------------------------------------------
// FP32 dense residual (or L) by aligned tiles: block (x, y) covers rows
// [16 y, 16 y + 16) and columns [64 x, 64 x + 64), one tile per wavefront.
template <int RP>
__global__ __launch_bounds__(256) void k_residual_f32(const float* __restrict__ X, int64_t ldx,
                                                      const float* __restrict__ UL,
                                                      const float* __restrict__ VL, int64_t m,
                                                      int64_t n, float* __restrict__ R,
                                                      int64_t ldr, int dense_l) {
  constexpr int KS = ResK<RP>::KS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.y * 16;
  const int64_t c0 = (int64_t)blockIdx.x * 64 + 16 * wave;
  float a[KS], b[KS];
  res_load_u<RP>(UL, m, r0, lane, a);
  res_load_v<RP>(VL, n, c0, lane, b);
  const f32x4_t L = res_tile<RP>(a, b);
  const int64_t row = r0 + (lane & 15);
  if (row >= m) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t col = c0 + res_col(v, lane);
    if (col >= n) continue;
    R[row * ldr + col] = dense_l ? 0.f - (0.f - L[v]) : X[row * ldx + col] - L[v];
  }
}

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
                                                int64_t m, int64_t n, int64_t mpad) {
  const int64_t total = mpad * ldd;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / ldd, j = e % ldd;
    D[e] = (i < m && j < n) ? to_store<TD, TX>(X[i * ldx + j]) : TD(0);
  }
}

template <typename TD, typename TX>
__global__ __launch_bounds__(256) void k_update_d(TD* __restrict__ D, int64_t ldd, int64_t n,
                                                  const int64_t* __restrict__ idx,
                                                  const TX* __restrict__ val,
                                                  const TX* __restrict__ xv,
                                                  const SelPlan* __restrict__ plan) {
  const long long cnt = plan->nnz;
  const double rn = 1.0 / (double)n;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < cnt;
       e += (long long)gridDim.x * 256) {
    const int64_t id = idx[e];
    int64_t i, j;
    divmod_nn(id, n, rn, i, j);
    const TX x = xv[e];
    D[i * ldd + j] = to_store<TD, TX>(val ? (TX)(x - val[e]) : x);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_norm_check(const T* __restrict__ X, int64_t ldx,
                                                    int64_t m, int64_t n, double* part,
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
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// out = the sum of part[0 .. n) in a fixed order (one block).
__global__ __launch_bounds__(256) void k_sum_fixed(const double* __restrict__ part, int64_t n,
                                                   double* __restrict__ out) {
  __shared__ double red[8];
  const double s = block_sum_fixed(part, n, red);
  if (threadIdx.x == 0) *out = s;
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

// Blocks of the full-data passes (one candidate segment each).
// FP32 passes (matrix-core tiles, four blocks per CU fit) take up to four
// blocks per CU; FP64 passes two.
template <typename T>
static int64_t sel_grid(int rp, int64_t m, int64_t n, int num_cu) {
  int64_t g = 1;
  if (sizeof(T) == 4) {
    int64_t cols = 512;
    GODEC_RP_SWITCH(rp, { cols = ResStrip<RP>::COLS; });
    g = ((n + cols - 1) / cols) * ((m + 15) / 16);
    g = std::min<int64_t>(g, (int64_t)num_cu * 4);
  } else {
    GODEC_RP_SWITCH(rp, {
      constexpr int TW = 256 * sel_cpt<T, RP>();
      g = ((n + TW - 1) / TW) * ((m + kRowsPerTile - 1) / kRowsPerTile);
    });
    g = std::min<int64_t>(g, (int64_t)num_cu * 2);
  }
  return std::max<int64_t>(1, std::min<int64_t>(g, kMaxSeg / kSelWaves));
}

template <typename T>
static void select_t(const Launch& L, int rp, const SelectArgs& a) {
  constexpr int KB = KeyBits<T>::value;
  const int levels = 1 + (KB - kHistBits0 + kHistBits - 1) / kHistBits;
  const int64_t g = sel_grid<T>(rp, a.m, a.n, L.num_cu);
  const int nseg = (int)g * kSelWaves;
  // the passes after pass 0 advance the plan in their last block (32-bit
  // bin counts: m n < 2^32), so a pass with nothing to do costs one launch;
  // otherwise, and after pass 0 and the candidate histograms, k_sel_plan
  const bool fuse = (uint64_t)a.m * (uint64_t)a.n < (1ull << 32);
  hipLaunchKernelGGL(k_sel_reset<T>, dim3(1), dim3(256), 0, L.stream, a.plan, a.hist,
                     a.counters, a.seg_count, (long long)a.k, (long long)a.cap, nseg, a.carry);
  GODEC_RP_SWITCH(rp, {
    // pass 0 (carried window or full level 0), one spare pass for the
    // fall-back level-0 histogram, then one per deeper level and the collection
    for (int pass = 0; pass <= levels + 1; ++pass) {
      if (pass == 0) {
        if (a.ev_a) (void)hipEventRecord(a.ev_a, L.stream);
        hipLaunchKernelGGL((k_sel_pass0<T, RP>), dim3((unsigned)g), dim3(256), 0, L.stream,
                           (const T*)a.X, a.ldx, (const T*)a.UL, (const T*)a.VLt, a.ldv, a.m,
                           a.n, a.plan, a.hist, a.cand_idx, (T*)a.cand_val, (T*)a.cand_x,
                           a.seg_count, a.s2part, sizeof(T) == 4 ? a.r16 : nullptr, a.ldd16,
                           a.ridx, a.rx, a.rplan);
        if (a.ev_b) (void)hipEventRecord(a.ev_b, L.stream);
      } else {
        hipLaunchKernelGGL((k_sel_passN<T, RP>), dim3((unsigned)g), dim3(256), 0, L.stream,
                           (const T*)a.X, a.ldx, (const T*)a.UL, (const T*)a.VLt, a.ldv, a.m,
                           a.n, a.plan, a.hist, a.cand_idx, (T*)a.cand_val, (T*)a.cand_x,
                           a.seg_count, fuse ? 1 : 0);
      }
      if (pass == 0 || !fuse)
        hipLaunchKernelGGL(k_sel_plan<T>, dim3(1), dim3(256), 0, L.stream, a.plan, a.hist, 0,
                           pass == 0 ? (const double*)a.s2part : nullptr, (int)g);
    }
  });
  const unsigned cg = (unsigned)(g + 1);   // segments are taken round-robin by blocks
  for (int round = 0; round < levels - 1; ++round) {
    hipLaunchKernelGGL(k_cand_hist<T>, dim3(cg), dim3(256), 0, L.stream, a.plan,
                       (const T*)a.cand_val, (const unsigned int*)a.seg_count, a.hist);
    hipLaunchKernelGGL(k_sel_plan<T>, dim3(1), dim3(256), 0, L.stream, a.plan, a.hist, 1,
                       (const double*)nullptr, 0);
  }
  GODEC_RP_SWITCH(rp, {
    hipLaunchKernelGGL((k_sel_ties_stream<T, RP>), dim3(1), dim3(256), 0, L.stream,
                       (const T*)a.X, a.ldx, (const T*)a.UL, (const T*)a.VL, (const T*)a.VLt,
                       a.ldv, a.m, a.n, a.plan,
                       a.cand_idx, (const T*)a.cand_val, (const T*)a.cand_x,
                       (const unsigned int*)a.seg_count, a.s_idx, (T*)a.s_val, (T*)a.s_x,
                       a.carry);
  });
  hipLaunchKernelGGL(k_sel_compact<T>, dim3(cg), dim3(256), 0, L.stream, a.plan, a.cand_idx,
                     (const T*)a.cand_val, (const T*)a.cand_x, (const unsigned int*)a.seg_count,
                     a.s_idx, (T*)a.s_val, (T*)a.s_x, a.tie_idx, a.counters,
                     a.s2part + kSelParts, (T*)a.dwn, sizeof(T) == 4 ? a.dw16 : nullptr,
                     a.lddw, a.n);
  hipLaunchKernelGGL(k_sel_ties<T>, dim3(1), dim3(1024), 0, L.stream, a.plan, a.s_idx,
                     (T*)a.s_val, a.tie_idx, a.counters, a.carry,
                     (const double*)(a.s2part + kSelParts), (int)cg);
  GODEC_RP_SWITCH(rp, {
    hipLaunchKernelGGL((k_fix_tie_values<T, RP>), dim3(grid_for(a.k, L.num_cu, 2)), dim3(256),
                       0, L.stream, (const T*)a.X, a.ldx, (const T*)a.UL, (const T*)a.VL,
                       (const T*)a.VLt, a.ldv, a.m, a.n, a.plan, a.counters, a.s_idx,
                       (T*)a.s_val, (T*)a.s_x, (T*)a.dwn,
                       sizeof(T) == 4 ? a.dw16 : nullptr, a.lddw);
  });
}

void launch_transpose_panel(const Launch& L, bool f64, const void* VL, int64_t rows, int rp,
                            void* VLt) {
  const unsigned b = (unsigned)((rows * rp + 255) / 256);
  if (f64)
    hipLaunchKernelGGL(k_transpose_panel<double>, dim3(b), dim3(256), 0, L.stream,
                       (const double*)VL, rows, rp, (double*)VLt);
  else
    hipLaunchKernelGGL(k_transpose_panel<float>, dim3(b), dim3(256), 0, L.stream,
                       (const float*)VL, rows, rp, (float*)VLt);
}

void launch_select(const Launch& L, bool f64, int rp, const SelectArgs& a) {
  if (f64) select_t<double>(L, rp, a);
  else select_t<float>(L, rp, a);
}

void launch_residual(const Launch& L, bool f64, int rp, const void* X, int64_t ldx,
                     const void* UL, const void* VL, int64_t m, int64_t n, void* R,
                     int64_t ldr, int dense_l) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)((m + kRowsPerTile - 1) / kRowsPerTile));
  dim3 grid16((unsigned)((n + 63) / 64), (unsigned)((m + 15) / 16));
  GODEC_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((k_residual<double, RP>), grid, dim3(256), 0, L.stream,
                         (const double*)X, ldx, (const double*)UL, (const double*)VL, m, n,
                         (double*)R, ldr, dense_l);
    else
      hipLaunchKernelGGL((k_residual_f32<RP>), grid16, dim3(256), 0, L.stream,
                         (const float*)X, ldx, (const float*)UL, (const float*)VL, m, n,
                         (float*)R, ldr, dense_l);
  });
}

void launch_init_d(const Launch& L, DType td, bool xf64, void* D, int64_t ldd,
                   const void* X, int64_t ldx, int64_t m, int64_t n, int64_t mpad) {
  dim3 grid(grid_for(mpad * ldd, L.num_cu, 16));
  if (td == F64)
    hipLaunchKernelGGL((k_init_d<double, double>), grid, dim3(256), 0, L.stream, (double*)D,
                       ldd, (const double*)X, ldx, m, n, mpad);
  else if (td == F32)
    hipLaunchKernelGGL((k_init_d<float, float>), grid, dim3(256), 0, L.stream, (float*)D, ldd,
                       (const float*)X, ldx, m, n, mpad);
  else
    hipLaunchKernelGGL((k_init_d<uint16_t, float>), grid, dim3(256), 0, L.stream,
                       (uint16_t*)D, ldd, (const float*)X, ldx, m, n, mpad);
  (void)xf64;
}

void launch_update_d(const Launch& L, DType td, void* D, int64_t ldd, int64_t n,
                     const int64_t* idx, const void* val, const void* xv, const SelPlan* plan,
                     int64_t kmax) {
  const unsigned g = grid_for(kmax, L.num_cu, 4);
  if (td == F64)
    hipLaunchKernelGGL((k_update_d<double, double>), dim3(g), dim3(256), 0, L.stream,
                       (double*)D, ldd, n, idx, (const double*)val, (const double*)xv, plan);
  else if (td == F32)
    hipLaunchKernelGGL((k_update_d<float, float>), dim3(g), dim3(256), 0, L.stream, (float*)D,
                       ldd, n, idx, (const float*)val, (const float*)xv, plan);
  else
    hipLaunchKernelGGL((k_update_d<uint16_t, float>), dim3(g), dim3(256), 0, L.stream,
                       (uint16_t*)D, ldd, n, idx, (const float*)val, (const float*)xv, plan);
}

void launch_norm_check(const Launch& L, bool f64, const void* X, int64_t ldx, int64_t m,
                       int64_t n, double* out2, int* nonfinite, double* part) {
  const unsigned g = std::min<unsigned>(grid_for(m * n, L.num_cu, 8), (unsigned)kNormParts);
  if (f64)
    hipLaunchKernelGGL(k_norm_check<double>, dim3(g), dim3(256), 0, L.stream,
                       (const double*)X, ldx, m, n, part, nonfinite);
  else
    hipLaunchKernelGGL(k_norm_check<float>, dim3(g), dim3(256), 0, L.stream, (const float*)X,
                       ldx, m, n, part, nonfinite);
  hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, L.stream, (const double*)part,
                     (int64_t)g, out2);
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
