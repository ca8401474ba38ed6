// libgodec host side: the C ABI of include/godec.h.
//
// One iteration of Algorithm 1 (Sec. 3.1.3) is enqueued as:
//   subspace chain  p = 2q+1 passes  Z <- orth(D^T (D Z)), Z_0 = A1,
//                   keeping Y2 = (D^T D)^p A1 = Q2 R2 (R2 in FP64),
//   B chain         q passes Y <- orth(D^T (D Y)), Y_0 = Q2, tracking T,
//                   then B' = D Y_q, so B = L~ Q2 = B' T,
//   core            rank check on R2, eigen-decomposition of B^T B,
//                   U_L = B' T K with K = V S^{(1-p)/p} V^T, V_L = Q2,
//   sparse step     fused residual / radix select / compaction of S_t,
//   D update        D <- X on supp(S_{t-1}), D <- X - S_t on supp(S_t).
// Everything runs on the caller's stream with no host synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/godec.h"
#include "godec_internal.h"
#include "k_mmb.h"
#include "host_common.h"

using namespace godec;
using namespace godec_host;

namespace godec_host {
thread_local std::string g_last_error;
}  // namespace godec_host

struct godec_ctx {
  // problem
  int64_t m, n, ldx, ldd, mpad, k;
  int r, rp, q, p;
  uint64_t seed;
  godec_dtype dtype;
  int prec, refine_iters;
  double rank_tol;
  const void* X;
  hipStream_t stream;
  int num_cu;
  int lstep = 0;                      // 1: projection form of the L update
  bool warm = false;                  // chains start from the previous Q2
  // redraw_a1: iteration t draws A1 from seed + t.  The draws of
  // kA1Chunk consecutive iterations are made together into slot s, a pinned
  // host buffer a1_pin[s] and its device copy in a1_dev (a1_t0[s] = first
  // iteration held, a1_cnt[s] = count).  The host-to-device copy of a slot
  // runs on a1_stream (a1_up[s] recorded after it); each iteration's draw
  // then goes from the device slot to A1 on the caller's stream (a1_rd[s]
  // recorded after the last such copy out of slot s).
  bool redraw = false;
  double* a1_dev = nullptr;
  double* a1_pin[2] = {nullptr, nullptr};
  hipStream_t a1_stream = nullptr;
  hipEvent_t a1_up[2] = {nullptr, nullptr};
  hipEvent_t a1_rd[2] = {nullptr, nullptr};
  bool a1_used[2] = {false, false};
  bool a1_waited[2] = {false, false};   // the caller's stream waits on a1_up[s]
  int64_t a1_t0[2] = {-1, -1};
  int a1_cnt[2] = {0, 0};
  int a1_next = 0;
  static constexpr int kA1Chunk = 4;
  const int64_t* support = nullptr;   // completion: fixed support of S
  int64_t support_nnz = 0;
  int64_t* row_ptr = nullptr;         // completion: m x (ncb + 1) run starts (see init)
  bool completion = false;
  bool f64;            // panel / residual type is double
  size_t ta;           // sizeof panel type
  // workspace
  void* D = nullptr;       // native-precision working copy
  void* D16 = nullptr;     // bf16 working copy (BF16_REFINE)
  double* A1 = nullptr;    // n x r FP64
  void *P0, *P1, *VL, *VLt, *W, *Zpart, *Bp, *UL, *Kp;
  void *Zt, *Wt;             // 32-row transposed panels for the matrix cores
  float *Wtpart, *Zpart32;   // partial sums of the two MFMA halves
  double* Gpart;
  GramCtl* gram_ctl;
  SmallState* st;
  SelPlan* plan[2];
  unsigned long long* hist;
  unsigned long long* counters;
  int64_t* cand_idx;
  void* cand_val;
  void* cand_x;
  unsigned int* seg_count;
  int64_t cap;
  int64_t* tie_idx;
  SelCarry* carry;
  int64_t* s_idx[2];
  void* s_val[2];
  void* s_x[2];
  uint32_t *bitmap, *wpre, *bsum;
  unsigned long long* boff;
  double* norm_x2;
  int* nonfinite;
  double* s2part;          // fixed-order partial sums (selection, norm check)
  // schedule
  int64_t nchunks, rows_per_chunk;
  int64_t kc_a, nct_a, rc_b, nch_b;   // MFMA tiling
  // state
  int64_t iters_done = 0;
  // BF16_REFINE: the FP32 working copy D is only read by the refinement
  // iterations; it is rebuilt from X and S when one starts and kept in step
  // from then on.  NATIVE: always in step.
  bool d_native_valid = true;
  int cur = 0;
  std::vector<double> a1_host;
  // tracing
  bool prof = false;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  // graph replay (godec_set_graphs): one executable graph per steady
  // iteration shape, recorded on a private stream, launched on `stream`
  bool graphs = false;
  hipStream_t cap_stream = nullptr;
  struct GraphEntry { int key; hipGraphExec_t exec; };
  std::vector<GraphEntry> gcache;
};

PanelPlan godec_host::plan_sizes(int64_t m, int64_t n, int64_t k, int num_cu) {
  PanelPlan s;
  s.ldd = (n + 127) / 128 * 128;
  s.mpad = (m + 63) / 64 * 64;
  // k_mm_a: 1152-column tiles (the fastest of 640 ... 2048 in steps of 64
  // columns on 10000 x 10000, for the BF16 and the FP32 panels alike);
  // k_mm_b: 128-column strips x row chunks.
  // k_mm_b's registers allow two 4-wave blocks per CU; the chunk count keeps
  // strips x chunks within one round of 2 * num_cu resident blocks, so no
  // block of a pass waits for a second round.
  s.kc_a = 1152;
  // Narrow matrices: with 128-row blocks one column tile can leave CUs idle,
  // so the tile narrows (512, then 256 columns) until the pass has at least
  // 1.5 blocks per CU (25 344 x 500: 198 -> 396 blocks, measured 5% faster).
  const int64_t rblocks = (s.mpad + 127) / 128;
  for (int64_t kc : {512, 256}) {
    if (2 * rblocks * ((s.ldd + s.kc_a - 1) / s.kc_a) >= 3LL * num_cu) break;
    s.kc_a = kc;
  }
  s.nct_a = (s.ldd + s.kc_a - 1) / s.kc_a;
  const int64_t strips = s.ldd / 128;
  int64_t nch = std::max<int64_t>(1, (2LL * num_cu) / strips);
  nch = std::min<int64_t>(nch, std::max<int64_t>(1, s.mpad / 256));
  s.rc_b = ((s.mpad + nch - 1) / nch + 63) / 64 * 64;
  s.nch_b = (s.mpad + s.rc_b - 1) / s.rc_b;
  const int64_t ctiles = (s.ldd + 1023) / 1024;
  int64_t want = std::max<int64_t>(1, (4LL * num_cu + ctiles - 1) / ctiles);
  want = std::min<int64_t>(want, std::max<int64_t>(1, (m + 63) / 64));
  s.rpc = (m + want - 1) / want;
  s.rpc = (s.rpc + 15) / 16 * 16;
  s.nchunks = (m + s.rpc - 1) / s.rpc;
  s.cap = std::min<int64_t>(m * n, 2 * k + (1 << 20));
  // few Gram partials: the one-block r x r kernels sum them serially
  return s;
}

namespace {

// Carve every buffer; returns the total size.  ctx may be a measuring dummy.
size_t carve(godec_ctx* c, void* base) {
  Carver cv{(char*)base};
  const int64_t m = c->m, ldd = c->ldd, rp = c->rp;
  const size_t ta = c->ta;
  const size_t dsz = c->f64 ? 8 : 4;
  const int64_t mpad = c->mpad;
  c->D = cv.take((size_t)mpad * ldd * dsz);
  c->D16 = (c->prec == GODEC_PREC_BF16_REFINE) ? cv.take((size_t)mpad * ldd * 2) : nullptr;
  if (!c->f64) {
    c->Zt = cv.take((size_t)32 * ldd * 4);
    c->Wt = cv.take((size_t)32 * mpad * 4);
    c->Wtpart = (float*)cv.take((size_t)c->nct_a * 32 * mpad * 4);
    c->Zpart32 = (float*)cv.take((size_t)c->nch_b * ldd * zpart_stride(c->rp) * 4);
  } else {
    c->Zt = c->Wt = nullptr;
    c->Wtpart = c->Zpart32 = nullptr;
  }
  c->A1 = (double*)cv.take((size_t)c->n * c->r * 8);
  // redraw_a1: two device slots of kA1Chunk draws each
  c->a1_dev = c->redraw
                  ? (double*)cv.take((size_t)2 * godec_ctx::kA1Chunk * c->n * c->r * 8)
                  : nullptr;
  c->P0 = cv.take((size_t)ldd * rp * ta);
  c->P1 = cv.take((size_t)ldd * rp * ta);
  c->VL = cv.take((size_t)ldd * rp * ta);
  c->VLt = cv.take((size_t)ldd * rp * ta);
  c->W = cv.take((size_t)m * rp * ta);
  c->Zpart = c->f64 ? cv.take((size_t)c->nchunks * ldd * rp * ta) : nullptr;
  c->Bp = cv.take((size_t)m * rp * ta);
  c->UL = cv.take((size_t)m * rp * ta);
  c->Kp = cv.take((size_t)rp * rp * ta);
  c->Gpart = (double*)cv.take((size_t)kGramSlots * rp * rp * 8);
  c->gram_ctl = (GramCtl*)cv.take(sizeof(GramCtl));
  c->st = (SmallState*)cv.take(sizeof(SmallState));
  c->plan[0] = (SelPlan*)cv.take(sizeof(SelPlan));
  c->plan[1] = (SelPlan*)cv.take(sizeof(SelPlan));
  c->hist = (unsigned long long*)cv.take((size_t)kHistReplicas * kHistBins * 8);
  c->counters = (unsigned long long*)cv.take(64);
  c->cand_idx = (int64_t*)cv.take((size_t)c->cap * 2 * 8);
  c->cand_val = cv.take((size_t)c->cap * 2 * ta);
  c->cand_x = cv.take((size_t)c->cap * 2 * ta);
  c->seg_count = (unsigned int*)cv.take((size_t)kMaxSeg * 4);
  c->tie_idx = (int64_t*)cv.take((size_t)c->cap * 8);
  c->carry = (SelCarry*)cv.take(sizeof(SelCarry));
  const int64_t kk = std::max<int64_t>(c->k, 1);
  for (int b = 0; b < 2; ++b) {
    c->s_idx[b] = (int64_t*)cv.take((size_t)kk * 8);
    c->s_val[b] = cv.take((size_t)kk * ta);
    c->s_x[b] = cv.take((size_t)kk * ta);
  }
  const int64_t nwords = (m * c->n + 31) / 32;
  const int64_t nb = (nwords + 1023) / 1024;
  c->bitmap = (uint32_t*)cv.take((size_t)nwords * 4);
  c->wpre = (uint32_t*)cv.take((size_t)nwords * 4);
  c->bsum = (uint32_t*)cv.take((size_t)nb * 4);
  c->boff = (unsigned long long*)cv.take((size_t)nb * 8);
  c->norm_x2 = (double*)cv.take(8);
  c->nonfinite = (int*)cv.take(8);
  c->s2part = (double*)cv.take((size_t)std::max(2 * kSelParts, kNormParts) * 8);
  // completion: start of each (row, 256-column block) run of the support
  c->row_ptr = c->completion
                   ? (int64_t*)cv.take((size_t)m * ((c->n + 255) / 256 + 1) * 8)
                   : nullptr;
  return align_up(cv.off, 256);
}

godec_status validate(int64_t m, int64_t n, int32_t r, int64_t k, int32_t q,
                      godec_dtype dtype, const godec_opts* o) {
  if (m < 1 || n < 1) return fail(GODEC_E_INVAL, "m and n must be >= 1");
  if (r < 1 || r > std::min<int64_t>(m, n)) return fail(GODEC_E_INVAL, "need 1 <= r <= min(m, n)");
  if (r > GODEC_MAX_RANK) return fail(GODEC_E_UNSUPPORTED, "r exceeds GODEC_MAX_RANK");
  if (k < 0 || k > m * n) return fail(GODEC_E_INVAL, "need 0 <= k <= m*n");
  if (q < 0 || q > 16) return fail(GODEC_E_INVAL, "need 0 <= q <= 16");
  if (dtype != GODEC_F64 && dtype != GODEC_F32) return fail(GODEC_E_INVAL, "bad dtype");
  if (o) {
    if (o->size != sizeof(godec_opts)) return fail(GODEC_E_INVAL, "opts.size mismatch");
    if (o->prec != GODEC_PREC_NATIVE && o->prec != GODEC_PREC_BF16_REFINE)
      return fail(GODEC_E_INVAL, "bad opts.prec");
    if (o->prec == GODEC_PREC_BF16_REFINE && dtype != GODEC_F32)
      return fail(GODEC_E_INVAL, "BF16_REFINE needs an FP32 X");
    if (o->refine_iters < 0) return fail(GODEC_E_INVAL, "refine_iters < 0");
    if (o->lstep != 0 && o->lstep != 1) return fail(GODEC_E_INVAL, "opts.lstep must be 0 or 1");
    if (o->warm_start != 0 && o->warm_start != 1)
      return fail(GODEC_E_INVAL, "opts.warm_start must be 0 or 1");
    if (o->redraw_a1 != 0 && o->redraw_a1 != 1)
      return fail(GODEC_E_INVAL, "opts.redraw_a1 must be 0 or 1");
    if (o->redraw_a1 && o->warm_start)
      return fail(GODEC_E_INVAL, "redraw_a1 and warm_start exclude each other");
    if (o->redraw_a1 && o->a1_host)
      return fail(GODEC_E_INVAL, "redraw_a1 draws every A1 itself: a1_host must be NULL");
    if (o->support_dev != nullptr || o->support_nnz != 0) {
      if (o->support_nnz < 0 || o->support_nnz > m * n)
        return fail(GODEC_E_INVAL, "need 0 <= support_nnz <= m*n");
      if (o->support_nnz > 0 && o->support_dev == nullptr)
        return fail(GODEC_E_INVAL, "support_dev is NULL");
      if (o->support_nnz != k) return fail(GODEC_E_INVAL, "completion needs k == support_nnz");
    }
  }
  return GODEC_OK;
}

void fill_ctx_params(godec_ctx* c, int64_t m, int64_t n, int32_t r, int64_t k,
                     int32_t q, godec_dtype dtype, const godec_opts* o, int num_cu) {
  c->m = m; c->n = n; c->r = r; c->k = k; c->q = q; c->p = 2 * q + 1;
  c->dtype = dtype;
  c->prec = o ? o->prec : GODEC_PREC_NATIVE;
  c->refine_iters = o ? o->refine_iters : 1;
  c->rank_tol = (o && o->rank_tol > 0) ? o->rank_tol : (double)r * std::ldexp(1.0, -52);
  c->rp = round_rp(r);
  c->f64 = dtype == GODEC_F64;
  c->ta = c->f64 ? 8 : 4;
  c->num_cu = num_cu;
  PanelPlan s = plan_sizes(m, n, k, num_cu);
  c->ldd = s.ldd; c->mpad = s.mpad; c->nchunks = s.nchunks; c->rows_per_chunk = s.rpc;
  c->cap = s.cap;
  c->kc_a = s.kc_a; c->nct_a = s.nct_a; c->rc_b = s.rc_b; c->nch_b = s.nch_b;
  c->completion = o && (o->support_dev != nullptr || o->support_nnz != 0);
  c->redraw = o && o->redraw_a1;
}

// Counter-based SplitMix64 (Steele, Lea, Flood 2014): output i of the stream
// seeded with `seed` is mix(seed + (i + 1) * golden_gamma).
uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform53(uint64_t seed, uint64_t i) {
  return ((double)(splitmix64(seed, i) >> 11) + 0.5) * std::ldexp(1.0, -53);
}

// Box-Muller pair j -> Gaussians 2j (cos) and 2j+1 (sin).
double gaussian(uint64_t seed, uint64_t j) {
  const uint64_t pair = j / 2;
  const double u1 = uniform53(seed, 2 * pair);
  const double u2 = uniform53(seed, 2 * pair + 1);
  const double rad = std::sqrt(-2.0 * std::log(u1));
  const double ang = (2.0 * M_PI) * u2;
  return rad * ((j % 2 == 0) ? std::cos(ang) : std::sin(ang));
}

// Gaussians j0 .. j1-1 of the stream of `seed` into out[0 .. j1-j0): the
// same values as gaussian(seed, j), with each Box-Muller pair's logarithm
// and square root taken once for both of its members.
void gaussians(uint64_t seed, uint64_t j0, uint64_t j1, double* out) {
  uint64_t j = j0;
  if (j < j1 && (j & 1)) {
    out[0] = gaussian(seed, j);
    ++j;
  }
  for (; j + 1 < j1; j += 2) {
    const double u1 = uniform53(seed, j);
    const double u2 = uniform53(seed, j + 1);
    const double rad = std::sqrt(-2.0 * std::log(u1));
    const double ang = (2.0 * M_PI) * u2;
    out[j - j0] = rad * std::cos(ang);
    out[j + 1 - j0] = rad * std::sin(ang);
  }
  if (j < j1) out[j - j0] = gaussian(seed, j);
}

// count draws of n x r entries, draw d from seed0 + d into out + d n r,
// split over up to 16 threads in contiguous ranges of the joint index.
void draw_many(uint64_t seed0, int count, int64_t n, int32_t r, double* out) {
  const uint64_t per = (uint64_t)n * (uint64_t)r;
  const uint64_t total = per * (uint64_t)count;
  unsigned nth = 1;
  if (total >= (1u << 16))
    nth = std::max(1u, std::min<unsigned>(16u, std::thread::hardware_concurrency()));
  auto work = [&](unsigned w) {
    uint64_t g = total * w / nth;
    const uint64_t g1 = total * (w + 1) / nth;
    while (g < g1) {
      const uint64_t d = g / per, j = g % per;
      const uint64_t e = std::min(g1 - g, per - j);
      gaussians(seed0 + d, j, j + e, out + g);
      g += e;
    }
  };
  std::vector<std::thread> th;
  for (unsigned w = 1; w < nth; ++w) {
    // a thread that cannot be started leaves its share to this one
    try {
      th.emplace_back(work, w);
    } catch (...) {
      work(w);
    }
  }
  work(0);
  for (auto& t : th) t.join();
}

Launch launch_of(const godec_ctx* c) { return Launch{c->stream, c->num_cu}; }

// Kernel classes timed by godec_profile.
enum ProfClass { PC_APPLY = 0, PC_APPLY_T, PC_APPLY_BF16, PC_APPLY_T_BF16, PC_SEL_PASS,
                 PC_COUNT };
const char* kProfNames[PC_COUNT] = {"mm_a(D*Z)", "mm_b(W^T*D)", "mm_a_bf16(D*Z)",
                                    "mm_b_bf16(W^T*D)", "select_pass(hist)"};
const double kProfElemBytes[PC_COUNT] = {0, 0, 2, 2, 0};   // 0: element size of X

hipEvent_t prof_event(godec_ctx* c) {
  if (c->pool_used == c->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->pool.push_back(e);
  }
  return c->pool[c->pool_used++];
}

// Pair of events timing one launch (no-op unless profiling).  With
// ext = true the launch itself stamps the events with the kernel's start and
// end (extended launch); otherwise they are recorded on the stream around it.
struct ProfScope {
  godec_ctx* c;
  int cls;
  bool ext;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(godec_ctx* ctx, int k, bool ext_launch = false) : c(ctx), cls(k), ext(ext_launch) {
    if (!c->prof) return;
    a = prof_event(c);
    b = prof_event(c);
    if (!a || !b) a = b = nullptr;
    if (a && !ext) (void)hipEventRecord(a, c->stream);
  }
  ~ProfScope() {
    if (!c->prof || !a) return;
    if (!ext) (void)hipEventRecord(b, c->stream);
    c->recs.push_back({cls, a, b});
  }
};

// W^T panel of D Y on the matrix cores (f32 / bf16 storage).  zt_ready:
// c->Zt already holds Y^T in the type of td (written by the preceding
// Cholesky QR step).
void mfma_apply(godec_ctx* c, DType td, const void* Dsrc, const void* in, bool zt_ready,
                void* Wt_out, float* Wrow_out) {
  const Launch L = launch_of(c);
  const bool b16 = td == BF16;
  if (!zt_ready) mfma_to_t(L, b16, in, c->ldd, c->rp, c->Zt);
  {
    ProfScope ps(c, b16 ? PC_APPLY_BF16 : PC_APPLY, true);
    mfma_mm_a(L, b16, Dsrc, c->ldd, c->mpad, c->Zt, c->Wtpart, c->kc_a, ps.a, ps.b);
  }
  mfma_reduce_w(L, b16, c->Wtpart, (int)c->nct_a, c->mpad, c->m, c->rp, Wt_out, Wrow_out);
}

// One Gram pass: out = D^T (D in), through W and the chunk partials.  With
// defer_sum (matrix-core passes only) the chunk partials are left in
// c->Zpart32 for the Gram step to add up (gram_chol).
void gram_pass(godec_ctx* c, DType td, const void* Dsrc, const void* in, bool zt_ready,
               void* out, bool defer_sum = false) {
  const Launch L = launch_of(c);
  if (td != F64) {
    const bool b16 = td == BF16;
    mfma_apply(c, td, Dsrc, in, zt_ready, c->Wt, nullptr);
    {
      ProfScope ps(c, b16 ? PC_APPLY_T_BF16 : PC_APPLY_T, true);
      mfma_mm_b(L, b16, Dsrc, c->ldd, c->mpad, c->Wt, c->Zpart32, c->rc_b, c->nch_b, c->rp, ps.a,
                ps.b);
    }
    if (!defer_sum) mfma_reduce_z(L, c->Zpart32, c->nch_b, c->ldd, c->rp, (float*)out);
    return;
  }
  {
    ProfScope ps(c, PC_APPLY);
    launch_apply(L, td, c->rp, Dsrc, c->ldd, c->m, in, c->W);
  }
  {
    ProfScope ps(c, PC_APPLY_T);
    launch_apply_t(L, td, c->rp, Dsrc, c->ldd, c->m, c->W, c->Zpart, c->rows_per_chunk,
                   c->nchunks);
  }
  launch_reduce_chunks(L, c->f64, c->rp, c->Zpart, c->nchunks, c->ldd, out);
}

// Orthonormalise `in` (ldd x RP) into `out` by one Cholesky QR step,
// accumulating its R factor into acc (reset when reset != 0).  next_td:
// type of the matrix-core pass that reads `out` next (its transpose is
// written to c->Zt), or F64 when none does.
void chol_qr(godec_ctx* c, const void* in, void* out, double* acc, int reset, DType next_td,
             bool from_parts = false) {
  const Launch L = launch_of(c);
  launch_gram_tree(L, c->f64, c->rp, in, c->ldd, c->Gpart, c->gram_ctl, 1, c->st, acc, reset,
                   acc == c->st->R2 ? 1 : 0, from_parts ? c->Zpart32 : nullptr,
                   from_parts ? (int)c->nch_b : 0);
  const bool zt = !c->f64 && next_td != F64;
  launch_apply_rinv(L, c->f64, c->rp, in, c->ldd, c->st, out, next_td, zt ? c->Zt : nullptr,
                    c->ldd);
}

// A Gram pass and one Cholesky QR step: out = orth(D^T (D in)) via tmp, its
// R factor folded into acc.  For matrix-core passes the Gram kernel adds up
// the pass's row-chunk partials itself (and stores tmp).
void gram_chol(godec_ctx* c, DType td, const void* Dsrc, const void* in, bool zt_ready,
               void* tmp, void* out, double* acc, int reset, DType next_td) {
  const bool parts = td != F64 && c->nch_b <= kGramMaxChunks;
  gram_pass(c, td, Dsrc, in, zt_ready, tmp, parts);
  chol_qr(c, tmp, out, acc, reset, next_td, parts);
}

godec_status run_iteration(godec_ctx* c, int64_t t, int64_t total) {
  const Launch L = launch_of(c);
  const DType native = c->f64 ? F64 : F32;
  const bool mixed = c->prec == GODEC_PREC_BF16_REFINE;
  const bool refine = mixed && total > 0 && t >= total - c->refine_iters;
  // ---- subspace chain: Q2 = orth((D^T D)^p A1), R2 tracked ----
  if (c->warm && c->iters_done > 0)
    HIP_TRY(hipMemcpyAsync(c->P0, c->VL, (size_t)c->ldd * c->rp * c->ta, hipMemcpyDeviceToDevice,
                           c->stream));   // Q2 of the last iteration (zero past r_eff)
  else
    launch_copy_panel(L, c->f64, c->rp, c->A1, c->n, c->ldd, c->r, c->st, c->P0);
  const int64_t kk = std::max<int64_t>(c->k, 1);
  if (refine && !c->d_native_valid) {
    // D = X - S_{t-1} in FP32 for the refinement passes
    launch_init_d(L, F32, false, c->D, c->ldd, c->X, c->ldx, c->m, c->n, c->mpad);
    if (c->iters_done > 0)
      launch_update_d(L, F32, c->D, c->ldd, c->n, c->s_idx[c->cur], c->s_val[c->cur],
                      c->s_x[c->cur], c->plan[c->cur], kk);
    c->d_native_valid = true;
  }
  // type of chain pass j (the refinement redoes the last one in FP32)
  auto chain_td = [&](int j) {
    return (mixed && !(refine && j == c->p - 1)) ? BF16 : native;
  };
  const bool low_b = mixed && !refine;
  const DType tdb = low_b ? BF16 : native;
  const void* Db = low_b ? c->D16 : c->D;
  const void* in = c->P0;
  bool zt = false;
  for (int j = 0; j < c->p; ++j) {
    const DType td = chain_td(j);
    const bool more = j + 1 < c->p;
    gram_chol(c, td, td == BF16 ? c->D16 : c->D, in, zt, c->P1, c->P0, c->st->R2, j == 0,
              more ? chain_td(j + 1) : F64);
    zt = more;
    in = c->P0;
  }
  // second Cholesky QR round on Q2 (restores orthonormality to working
  // precision); its R factor joins R2.  Its transpose feeds the B chain.
  chol_qr(c, c->P0, c->VL, c->st->R2, 0, tdb);
  if (c->lstep == 1) {
    // projection form: L = D Q2 Q2^T, i.e. U_L = D Q2 and V_L = Q2
    if (c->f64)
      launch_apply(L, tdb, c->rp, Db, c->ldd, c->m, c->VL, c->UL);
    else
      mfma_apply(c, tdb, Db, c->VL, true, nullptr, (float*)c->UL);
  } else {
  // ---- B chain: (D^T D)^q Q2 = Y_q T, then B' = D Y_q ----
  in = c->VL;
  for (int j = 0; j < c->q; ++j) {
    gram_chol(c, tdb, Db, in, true, c->P1, c->P0, c->st->T, j == 0, tdb);
    in = c->P0;
  }
  if (c->f64)
    launch_apply(L, tdb, c->rp, Db, c->ldd, c->m, in, c->Bp);
  else
    mfma_apply(c, tdb, Db, in, true, nullptr, (float*)c->Bp);
  // ---- core ----
  launch_gram_tree(L, c->f64, c->rp, c->Bp, c->m, c->Gpart, c->gram_ctl, 0, c->st, nullptr, 0,
                   0);
  launch_core(L, c->f64, c->rp, c->Gpart + (size_t)kGramFinal * c->rp * c->rp, 1, c->st, c->p,
              c->rank_tol, c->q == 0 ? 1 : 0, c->Kp);
  launch_apply_small(L, c->f64, c->rp, c->Bp, c->m, c->Kp, c->UL);
  }
  // ---- sparse step ----
  const int prev = c->cur;
  const int nxt = c->cur ^ 1;
  launch_transpose_panel(L, c->f64, c->VL, c->ldd, c->rp, c->VLt);
  SelectArgs a;
  a.X = c->X; a.ldx = c->ldx; a.UL = c->UL; a.VL = c->VL; a.m = c->m; a.n = c->n; a.k = c->k;
  a.VLt = c->VLt; a.ldv = c->ldd;
  a.plan = c->plan[nxt]; a.hist = c->hist; a.counters = c->counters;
  a.cand_idx = c->cand_idx; a.cand_val = c->cand_val; a.cand_x = c->cand_x; a.cap = c->cap;
  a.seg_count = c->seg_count;
  a.s_idx = c->s_idx[nxt]; a.s_val = c->s_val[nxt]; a.s_x = c->s_x[nxt];
  a.tie_idx = c->tie_idx;
  a.carry = c->carry;
  a.s2part = c->s2part;
  // the bf16 copy's old support is restored inside pass 0 (after the chain
  // has read it, before the new support is written below)
  const bool restore_in_pass = mixed && !c->completion && !c->f64 && c->iters_done > 0;
  if (restore_in_pass) {
    a.r16 = (uint16_t*)c->D16;
    a.ldd16 = c->ldd;
    a.ridx = c->s_idx[prev];
    a.rx = (const float*)c->s_x[prev];
    a.rplan = c->plan[prev];
  }
  if (c->prof) {
    a.ev_a = prof_event(c);
    a.ev_b = prof_event(c);
    if (a.ev_a && a.ev_b) c->recs.push_back({PC_SEL_PASS, a.ev_a, a.ev_b});
  }
  // ---- D update, old support: X is restored there before the selection
  // (the chain has finished reading D and the selection reads X), so that
  // the compaction can write X - S on the new support as it takes it ----
  const bool upd_native = c->d_native_valid;
  // a fixed support is rewritten in place: no restore of the old one
  if (c->iters_done > 0 && !c->completion) {
    if (upd_native)
      launch_update_d(L, native, c->D, c->ldd, c->n, c->s_idx[prev], nullptr, c->s_x[prev],
                      c->plan[prev], kk);
    if (mixed && !restore_in_pass)
      launch_update_d(L, BF16, c->D16, c->ldd, c->n, c->s_idx[prev], nullptr, c->s_x[prev],
                      c->plan[prev], kk);
  }
  const bool fused_d = !c->completion;
  if (fused_d) {
    a.dwn = upd_native ? c->D : nullptr;
    a.dw16 = mixed ? (uint16_t*)c->D16 : nullptr;
    a.lddw = c->ldd;
  }
  if (c->completion)
    launch_fixed_support(L, c->f64, c->rp, c->X, c->ldx, c->UL, c->VL, c->m, c->n, c->support,
                         c->row_ptr, c->support_nnz, c->s_idx[nxt], c->s_val[nxt],
                         c->s_x[nxt], c->plan[nxt], (double*)c->hist);
  else
    launch_select(L, c->f64, c->rp, a);
  // ---- D update, new support: X - S (written inside the selection; on a
  // fixed support here) ----
  if (!fused_d) {
    if (upd_native)
      launch_update_d(L, native, c->D, c->ldd, c->n, c->s_idx[nxt], c->s_val[nxt],
                      c->s_x[nxt], c->plan[nxt], kk);
    if (mixed)
      launch_update_d(L, BF16, c->D16, c->ldd, c->n, c->s_idx[nxt], c->s_val[nxt],
                      c->s_x[nxt], c->plan[nxt], kk);
  }
  c->cur = nxt;
  c->iters_done += 1;
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

}  // namespace

extern "C" {

void godec_opts_default(godec_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->size = sizeof(godec_opts);
  o->prec = GODEC_PREC_NATIVE;
  o->refine_iters = 1;
  o->rank_tol = 0.0;
  o->a1_host = nullptr;
  o->stream = nullptr;
}

godec_status godec_draw_a1(uint64_t seed, int64_t n, int32_t r, double* a1_host) {
  if (n < 1 || r < 1 || !a1_host) return fail(GODEC_E_INVAL, "bad arguments");
  // entry j depends on (seed, j) only, so the result does not depend on
  // how the range is split over threads
  draw_many(seed, 1, n, r, a1_host);
  return GODEC_OK;
}

}  // extern "C" (reopened below)

int godec_host::device_cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
    return 256;
  return cu;
}

extern "C" {

godec_status godec_workspace_size(int64_t m, int64_t n, int32_t r, int64_t k, int32_t q,
                                  godec_dtype dtype, const godec_opts* opts, size_t* bytes) {
  if (!bytes) return fail(GODEC_E_INVAL, "bytes is NULL");
  godec_status s = validate(m, n, r, k, q, dtype, opts);
  if (s != GODEC_OK) return s;
  godec_ctx tmp;
  // size with the largest chunk count any device would use (256 CUs)
  fill_ctx_params(&tmp, m, n, r, k, q, dtype, opts, 256);
  *bytes = carve(&tmp, nullptr);
  return GODEC_OK;
}

static godec_status fill_a1_slot(godec_ctx* c, int s, int64_t t0, int cnt);

godec_status godec_init(godec_ctx** out, const void* X_dev, godec_dtype dtype, int64_t m,
                        int64_t n, int64_t ldx, int32_t r, int64_t k, int32_t q, uint64_t seed,
                        void* ws, size_t ws_bytes, const godec_opts* opts) {
  if (!out) return fail(GODEC_E_INVAL, "out is NULL");
  *out = nullptr;
  godec_status s = validate(m, n, r, k, q, dtype, opts);
  if (s != GODEC_OK) return s;
  if (!X_dev || !ws) return fail(GODEC_E_INVAL, "X or workspace is NULL");
  if (ldx < n) return fail(GODEC_E_INVAL, "ldx < n");
  if (((uintptr_t)ws) % 256 != 0) return fail(GODEC_E_INVAL, "workspace not 256-byte aligned");
  if (((uintptr_t)X_dev) % (dtype == GODEC_F64 ? 8 : 4) != 0)
    return fail(GODEC_E_INVAL, "X not aligned to its element size");
  godec_ctx* c = new godec_ctx();
  fill_ctx_params(c, m, n, r, k, q, dtype, opts, 256);
  c->ldx = ldx;
  c->seed = seed;
  c->X = X_dev;
  c->lstep = opts ? opts->lstep : 0;
  c->warm = opts && opts->warm_start;
  c->stream = opts ? (hipStream_t)opts->stream : nullptr;
  const size_t need = carve(c, nullptr);
  if (ws_bytes < need) {
    delete c;
    return fail(GODEC_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  c->num_cu = device_cu_count();
  carve(c, ws);
  if (opts && (opts->support_dev != nullptr || opts->support_nnz != 0)) {
    // the fixed support must be strictly ascending and inside the matrix
    if (fixed_support_scratch_doubles() > (int64_t)kHistReplicas * kHistBins) {
      delete c;
      return fail(GODEC_E_UNSUPPORTED, "completion scratch exceeds the histogram buffer");
    }
    c->completion = true;
    c->support = opts->support_dev;
    c->support_nnz = opts->support_nnz;
    // one copy of the support to the host, on the context's stream: it is
    // checked, then turned into the run starts below
    std::vector<int64_t> h((size_t)c->support_nnz);
    if (!h.empty()) {
      hipError_t e = hipMemcpyAsync(h.data(), c->support, sizeof(int64_t) * h.size(),
                                    hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) {
        delete c;
        return fail(GODEC_E_DEVICE, hipGetErrorString(e));
      }
      for (size_t q = 0; q < h.size(); ++q)
        if (h[q] < 0 || h[q] >= m * n || (q > 0 && h[q] <= h[q - 1])) {
          delete c;
          return fail(GODEC_E_INVAL, "support must be strictly ascending in [0, m*n)");
        }
    }
    // run starts of the sorted support: entry (i, cb) is the first support
    // entry at or after (row i, column 256 cb); entry (i, ncb) is the first
    // entry of row i + 1 (blocked CSR, ncb = ceil(n / 256))
    const int64_t ncb = (n + 255) / 256;
    std::vector<int64_t> rp((size_t)(m * (ncb + 1)), 0);
    size_t pos = 0;
    for (int64_t i = 0; i < m; ++i)
      for (int64_t cb = 0; cb <= ncb; ++cb) {
        const int64_t key = cb < ncb ? i * n + cb * 256 : (i + 1) * n;
        while (pos < h.size() && h[pos] < key) ++pos;
        rp[(size_t)(i * (ncb + 1) + cb)] = (int64_t)pos;
      }
    // the host table must outlive the copy: wait for it before returning
    hipError_t e = hipMemcpyAsync(c->row_ptr, rp.data(), sizeof(int64_t) * rp.size(),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      delete c;
      return fail(GODEC_E_DEVICE, hipGetErrorString(e));
    }
  }
  c->a1_host.resize((size_t)n * r);
  if (opts && opts->a1_host)
    std::memcpy(c->a1_host.data(), opts->a1_host, sizeof(double) * n * r);
  else
    godec_draw_a1(seed, n, r, c->a1_host.data());
  const Launch L = launch_of(c);
  auto cleanup = [&](godec_status st, const std::string& msg) {
    godec_destroy(c);   // also frees the pinned staging slots
    return fail(st, msg);
  };
  hipError_t e = hipMemcpyAsync(c->A1, c->a1_host.data(), sizeof(double) * n * r,
                                hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return cleanup(GODEC_E_DEVICE, hipGetErrorString(e));
  if (c->redraw) {
    // both staging slots, the side stream, and the draws of iterations
    // 1 .. kA1Chunk in slot 0
    const size_t slot = sizeof(double) * (size_t)n * r * godec_ctx::kA1Chunk;
    e = hipStreamCreateWithFlags(&c->a1_stream, hipStreamNonBlocking);
    for (int q = 0; q < 2 && e == hipSuccess; ++q) {
      e = hipHostMalloc((void**)&c->a1_pin[q], slot, hipHostMallocDefault);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&c->a1_up[q], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&c->a1_rd[q], hipEventDisableTiming);
    }
    if (e != hipSuccess) return cleanup(GODEC_E_DEVICE, hipGetErrorString(e));
    godec_status st = fill_a1_slot(c, 0, 1, godec_ctx::kA1Chunk);
    if (st != GODEC_OK) {
      godec_destroy(c);
      return st;
    }
    c->a1_next = 1;
  }
  if (c->D16) {
    launch_init_d(L, BF16, false, c->D16, c->ldd, X_dev, ldx, m, n, c->mpad);
    c->d_native_valid = false;
  } else {
    launch_init_d(L, c->f64 ? F64 : F32, c->f64, c->D, c->ldd, X_dev, ldx, m, n, c->mpad);
  }
  launch_small_init(L, c->st, r);
  // zero the small scalars, plans and the (unused) panel padding
  e = hipMemsetAsync(c->norm_x2, 0, 8, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->nonfinite, 0, 8, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->plan[0], 0, sizeof(SelPlan), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->plan[1], 0, sizeof(SelPlan), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->carry, 0, sizeof(SelCarry), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->gram_ctl, 0, sizeof(GramCtl), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->VL, 0, (size_t)c->ldd * c->rp * c->ta, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->UL, 0, (size_t)c->m * c->rp * c->ta, c->stream);
  if (e != hipSuccess) return cleanup(GODEC_E_DEVICE, hipGetErrorString(e));
  launch_norm_check(L, c->f64, X_dev, ldx, m, n, c->norm_x2, c->nonfinite, c->s2part);
  e = hipGetLastError();
  if (e != hipSuccess) return cleanup(GODEC_E_DEVICE, hipGetErrorString(e));
  int bad = 0;
  e = hipMemcpyAsync(&bad, c->nonfinite, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return cleanup(GODEC_E_DEVICE, hipGetErrorString(e));
  if (bad) return cleanup(GODEC_E_NUMERIC, "X contains NaN or Inf");
  *out = c;
  return GODEC_OK;
}

// Record one iteration on the capture stream (run_iteration advances the
// host state as it records) and instantiate it.
godec_status capture_iteration(godec_ctx* c, int64_t t, int64_t total, hipGraphExec_t* out) {
  hipStream_t user = c->stream;
  c->stream = c->cap_stream;
  hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    c->stream = user;
    return fail(GODEC_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  }
  godec_status s = run_iteration(c, t, total);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(c->cap_stream, &g);
  c->stream = user;
  if (s != GODEC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(GODEC_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(GODEC_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  return GODEC_OK;
}

// redraw_a1: fill slot s with the draws of iterations t0 .. t0 + cnt - 1
// and queue their host-to-device copy on the side stream.  The draws are
// made on the host while the device works through the iterations queued
// before.
static godec_status fill_a1_slot(godec_ctx* c, int s, int64_t t0, int cnt) {
  const size_t one = (size_t)c->n * c->r;
  // the slot's last upload has left the host buffer
  if (c->a1_used[s]) HIP_TRY(hipEventSynchronize(c->a1_up[s]));
  c->a1_t0[s] = -1;
  draw_many(c->seed + (uint64_t)t0, cnt, c->n, c->r, c->a1_pin[s]);
  c->a1_t0[s] = t0;
  c->a1_cnt[s] = cnt;
  // the device slot is overwritten after the last copy out of it
  if (c->a1_used[s]) HIP_TRY(hipStreamWaitEvent(c->a1_stream, c->a1_rd[s], 0));
  HIP_TRY(hipMemcpyAsync(c->a1_dev + (size_t)s * godec_ctx::kA1Chunk * one, c->a1_pin[s],
                         sizeof(double) * one * cnt, hipMemcpyHostToDevice, c->a1_stream));
  HIP_TRY(hipEventRecord(c->a1_up[s], c->a1_stream));
  c->a1_used[s] = true;
  c->a1_waited[s] = false;
  return GODEC_OK;
}

// redraw_a1: queue the copy of iteration t's A1 (from seed + t) into the
// device A1 ahead of the iteration, on the caller's stream and outside any
// recorded graph.  When no slot holds it, the draws of iterations t ..
// t + kA1Chunk - 1 (not past the solve's end) go to the other slot first.
// (godec_init sets up both slots and fills slot 0 with iterations
// 1 .. kA1Chunk.)
static godec_status stage_a1(godec_ctx* c, int64_t t, int64_t total) {
  const size_t one = (size_t)c->n * c->r;
  int s = -1;
  for (int q = 0; q < 2; ++q)
    if (c->a1_t0[q] >= 0 && t >= c->a1_t0[q] && t < c->a1_t0[q] + c->a1_cnt[q]) s = q;
  if (s < 0) {
    s = c->a1_next;
    c->a1_next ^= 1;
    const int cnt =
        (int)std::max<int64_t>(1, std::min<int64_t>(godec_ctx::kA1Chunk, total - t));
    godec_status st = fill_a1_slot(c, s, t, cnt);
    if (st != GODEC_OK) return st;
  }
  // one wait per fill of the slot; the slot's iterations are staged in
  // order, so the copy of its last iteration is the last read of it
  if (!c->a1_waited[s]) {
    HIP_TRY(hipStreamWaitEvent(c->stream, c->a1_up[s], 0));
    c->a1_waited[s] = true;
  }
  HIP_TRY(hipMemcpyAsync(c->A1,
                         c->a1_dev + ((size_t)s * godec_ctx::kA1Chunk + (t - c->a1_t0[s])) * one,
                         sizeof(double) * one, hipMemcpyDeviceToDevice, c->stream));
  if (t == c->a1_t0[s] + c->a1_cnt[s] - 1) HIP_TRY(hipEventRecord(c->a1_rd[s], c->stream));
  return GODEC_OK;
}

godec_status godec_step(godec_ctx* c, int32_t iters, int32_t total_iters) {
  if (!c) return fail(GODEC_E_INVAL, "ctx is NULL");
  if (iters < 0) return fail(GODEC_E_INVAL, "iters < 0");
  int64_t total = total_iters > 0 ? total_iters : c->iters_done + iters;
  const bool mixed = c->prec == GODEC_PREC_BF16_REFINE;
  for (int32_t i = 0; i < iters; ++i) {
    const int64_t t = c->iters_done;
    const bool refine = mixed && total > 0 && t >= total - c->refine_iters;
    // iteration 0 uses the draw of godec_init (seed + 0); the copy of a
    // later draw is queued ahead of the iteration, outside any graph
    if (c->redraw && t > 0) {
      godec_status s = stage_a1(c, t, total);
      if (s != GODEC_OK) return s;
    }
    // the first iteration, the refinement iterations (which rebuild the FP32
    // copy of D once) and traced iterations run eagerly; every other
    // iteration's launches depend only on the S-list parity and on whether
    // the FP32 copy of D is kept in step
    if (!c->graphs || c->prof || t == 0 || refine) {
      godec_status s = run_iteration(c, t, total);
      if (s != GODEC_OK) return s;
      continue;
    }
    const int key = c->cur | (c->d_native_valid ? 2 : 0);
    hipGraphExec_t exec = nullptr;
    for (const auto& ge : c->gcache)
      if (ge.key == key) exec = ge.exec;
    if (!exec) {
      godec_status s = capture_iteration(c, t, total, &exec);
      if (s != GODEC_OK) return s;
      c->gcache.push_back({key, exec});
    } else {
      // the host state a recorded iteration advances
      c->cur ^= 1;
      c->iters_done += 1;
    }
    HIP_TRY(hipGraphLaunch(exec, c->stream));
  }
  return GODEC_OK;
}

godec_status godec_set_graphs(godec_ctx* c, int32_t enable) {
  if (!c) return fail(GODEC_E_INVAL, "ctx is NULL");
  if (enable && !c->cap_stream)
    HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  c->graphs = enable != 0;
  return GODEC_OK;
}

godec_status godec_get_factors(godec_ctx* c, void* UL_dev, void* VL_dev) {
  if (!c || !UL_dev || !VL_dev) return fail(GODEC_E_INVAL, "NULL argument");
  const Launch L = launch_of(c);
  launch_cast_panel(L, c->f64, c->rp, c->UL, c->m, c->r, UL_dev);
  launch_cast_panel(L, c->f64, c->rp, c->VL, c->n, c->r, VL_dev);
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

godec_status godec_get_L_dense(godec_ctx* c, void* L_dev, int64_t ldl) {
  if (!c || !L_dev || ldl < c->n) return fail(GODEC_E_INVAL, "bad argument");
  launch_residual(launch_of(c), c->f64, c->rp, c->X, c->ldx, c->UL, c->VL, c->m, c->n, L_dev,
                  ldl, 1);
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

godec_status godec_get_residual(godec_ctx* c, void* R_dev, int64_t ldr) {
  if (!c || !R_dev || ldr < c->n) return fail(GODEC_E_INVAL, "bad argument");
  launch_residual(launch_of(c), c->f64, c->rp, c->X, c->ldx, c->UL, c->VL, c->m, c->n, R_dev,
                  ldr, 0);
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

godec_status godec_get_S(godec_ctx* c, int64_t* idx_dev, void* val_dev, int64_t* nnz_host) {
  if (!c || !nnz_host) return fail(GODEC_E_INVAL, "NULL argument");
  if (c->iters_done == 0) {
    *nnz_host = 0;
    return GODEC_OK;
  }
  if (!idx_dev || !val_dev) return fail(GODEC_E_INVAL, "NULL output buffer");
  const Launch L = launch_of(c);
  launch_sort_s(L, c->f64, c->s_idx[c->cur], c->s_val[c->cur], c->plan[c->cur], c->m * c->n,
                std::max<int64_t>(c->k, 1), c->bitmap, c->wpre, c->bsum, c->boff, idx_dev,
                val_dev);
  SelPlan hp;
  HIP_TRY(hipMemcpyAsync(&hp, c->plan[c->cur], sizeof(SelPlan), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *nnz_host = hp.nnz;
  return GODEC_OK;
}

godec_status godec_get_A1(godec_ctx* c, double* a1_host) {
  if (!c || !a1_host) return fail(GODEC_E_INVAL, "NULL argument");
  // redraw_a1: the A1 of the last iteration run (of iteration 0 before any)
  const int64_t t = c->iters_done > 0 ? c->iters_done - 1 : 0;
  if (c->redraw && t > 0) return godec_draw_a1(c->seed + (uint64_t)t, c->n, c->r, a1_host);
  std::memcpy(a1_host, c->a1_host.data(), sizeof(double) * c->n * c->r);
  return GODEC_OK;
}

godec_status godec_get_info(godec_ctx* c, godec_info* info) {
  if (!c || !info) return fail(GODEC_E_INVAL, "NULL argument");
  SelPlan hp;
  std::memset(&hp, 0, sizeof(hp));
  double nx2 = 0.0;
  int r_eff = c->r, flags = 0;
  HIP_TRY(hipMemcpyAsync(&nx2, c->norm_x2, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&r_eff, &c->st->r_eff, 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(&flags, &c->st->flags, 4, hipMemcpyDeviceToHost, c->stream));
  if (c->iters_done > 0)
    HIP_TRY(hipMemcpyAsync(&hp, c->plan[c->cur], sizeof(SelPlan), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  info->iters = c->iters_done;
  info->nnz = hp.nnz;
  info->rank_eff = r_eff;
  info->flags = (flags & 1) | (flags & 2) | (hp.slow ? 4 : 0) | (hp.overflow ? 8 : 0);
  info->sum_r2 = hp.sum_r2;
  info->norm_x2 = nx2;
  // with a fixed support the error off the support is summed directly (the
  // difference of the two sums would lose it to cancellation)
  const double off = c->completion ? hp.sum_obs2 : hp.sum_r2 - hp.sum_sel2;
  info->rel_err_sq = nx2 > 0 ? off / nx2 : 0.0;
  if (info->rel_err_sq < 0) info->rel_err_sq = 0.0;
  info->threshold = hp.threshold;
  if (flags & 1) return fail(GODEC_E_NUMERIC, "non-finite value in the r x r core");
  return GODEC_OK;
}

godec_status godec_destroy(godec_ctx* c) {
  if (c) {
    if (!c->gcache.empty()) (void)hipStreamSynchronize(c->stream);
    for (const auto& ge : c->gcache) (void)hipGraphExecDestroy(ge.exec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    if (c->a1_stream) (void)hipStreamSynchronize(c->a1_stream);
    for (int s = 0; s < 2; ++s) {
      if (c->a1_up[s]) (void)hipEventDestroy(c->a1_up[s]);
      if (c->a1_rd[s]) (void)hipEventDestroy(c->a1_rd[s]);
      if (c->a1_pin[s]) (void)hipHostFree(c->a1_pin[s]);
    }
    if (c->a1_stream) (void)hipStreamDestroy(c->a1_stream);
    delete c;
  }
  return GODEC_OK;
}

godec_status godec_profile(godec_ctx* c, int32_t enable) {
  if (!c) return fail(GODEC_E_INVAL, "ctx is NULL");
  if (enable) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->recs.clear();
    c->pool_used = 0;
  }
  c->prof = enable != 0;
  return GODEC_OK;
}

godec_status godec_profile_read(godec_ctx* c, godec_kernel_stat* out, int32_t cap,
                                int32_t* count) {
  if (!c || !count) return fail(GODEC_E_INVAL, "NULL argument");
  HIP_TRY(hipStreamSynchronize(c->stream));
  double ms[PC_COUNT] = {0};
  int64_t n[PC_COUNT] = {0};
  for (const auto& r : c->recs) {
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.cls] += t;
    n[r.cls] += 1;
  }
  const double ds = c->f64 ? 8.0 : 4.0;
  const double mn = (double)c->m * (double)c->n;
  int32_t k = 0;
  for (int cls = 0; cls < PC_COUNT; ++cls) {
    if (n[cls] == 0) continue;
    if (out && k < cap) {
      godec_kernel_stat& st = out[k];
      std::memset(&st, 0, sizeof(st));
      std::snprintf(st.name, sizeof(st.name), "%s", kProfNames[cls]);
      st.launches = n[cls];
      st.total_ms = ms[cls];
      // one streaming read of the m x n operand per launch
      st.bytes_per_launch = mn * (kProfElemBytes[cls] > 0 ? kProfElemBytes[cls] : ds);
    }
    ++k;
  }
  *count = k;
  return GODEC_OK;
}

const char* godec_last_error(void) { return g_last_error.c_str(); }

godec_status godec_solve(const void* X_dev, godec_dtype dtype, int64_t m, int64_t n, int64_t ldx,
                         int32_t r, int64_t k, int32_t q, uint64_t seed, int32_t iters, void* ws,
                         size_t ws_bytes, const godec_opts* opts, void* UL_dev, void* VL_dev,
                         int64_t* S_idx_dev, void* S_val_dev, godec_info* info) {
  godec_ctx* c = nullptr;
  godec_status s = godec_init(&c, X_dev, dtype, m, n, ldx, r, k, q, seed, ws, ws_bytes, opts);
  if (s != GODEC_OK) return s;
  s = godec_step(c, iters, iters);
  if (s == GODEC_OK && UL_dev && VL_dev) s = godec_get_factors(c, UL_dev, VL_dev);
  int64_t nnz = 0;
  if (s == GODEC_OK && S_idx_dev && S_val_dev) s = godec_get_S(c, S_idx_dev, S_val_dev, &nnz);
  if (s == GODEC_OK && info) s = godec_get_info(c, info);
  if (s == GODEC_OK) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) s = fail(GODEC_E_DEVICE, hipGetErrorString(e));
  }
  godec_destroy(c);
  return s;
}

godec_status godec_solve_tol(const void* X_dev, godec_dtype dtype, int64_t m, int64_t n,
                             int64_t ldx, int32_t r, int64_t k, int32_t q, uint64_t seed,
                             int32_t max_iters, double eps, void* ws, size_t ws_bytes,
                             const godec_opts* opts, void* UL_dev, void* VL_dev,
                             int64_t* S_idx_dev, void* S_val_dev, godec_info* info) {
  if (max_iters < 1) return fail(GODEC_E_INVAL, "max_iters < 1");
  if (!(eps >= 0.0)) return fail(GODEC_E_INVAL, "eps must be >= 0");
  godec_ctx* c = nullptr;
  godec_status s = godec_init(&c, X_dev, dtype, m, n, ldx, r, k, q, seed, ws, ws_bytes, opts);
  if (s != GODEC_OK) return s;
  const int32_t nref =
      c->prec == GODEC_PREC_BF16_REFINE ? std::min<int32_t>(c->refine_iters, max_iters) : 0;
  const int32_t budget = max_iters - nref;
  int32_t done = 0;
  godec_info cur;
  // the loop test of Algorithm 1 after each iteration (the FP32 refinement
  // iterations, when asked for, follow the last tested one)
  while (s == GODEC_OK && done < budget) {
    s = godec_step(c, 1, max_iters);
    if (s != GODEC_OK) break;
    ++done;
    s = godec_get_info(c, &cur);
    if (s == GODEC_OK && cur.rel_err_sq <= eps) break;
  }
  if (s == GODEC_OK && nref > 0) s = godec_step(c, nref, done + nref);
  if (s == GODEC_OK && UL_dev && VL_dev) s = godec_get_factors(c, UL_dev, VL_dev);
  int64_t nnz = 0;
  if (s == GODEC_OK && S_idx_dev && S_val_dev) s = godec_get_S(c, S_idx_dev, S_val_dev, &nnz);
  if (s == GODEC_OK && info) s = godec_get_info(c, info);
  if (s == GODEC_OK) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) s = fail(GODEC_E_DEVICE, hipGetErrorString(e));
  }
  godec_destroy(c);
  return s;
}

const char* godec_version(void) {
  return "libgodec 0.1 (gfx950; GoDec by bilateral random projection)";
}

}  // extern "C"
