// libgodec host side of the batched form (include/godec.h, godec_batch_*).
//
// One iteration of Algorithm 1 (Sec. 3.1.3) for every problem of the batch:
//   copy A1 -> P0;  p = 2q+1 Gram passes, each followed by a per-problem
//   Cholesky QR step (R folded into R2);  a second Cholesky QR round into
//   V_L = Q2;  q more Gram passes tracking T;  B' = D Y_q with the FP64 Gram
//   of B';  the per-problem core (K' = T K);  U_L = B' K';  the sparse step
//   into S list t mod 2;  the D update.
// The launches of one iteration are captured once (for each parity of t)
// into a HIP graph; godec_batch_step replays it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/godec.h"
#include "godec_internal.h"
#include "host_common.h"

using namespace godec;
using namespace godec_host;

namespace {

constexpr int64_t kMinRowsPerItem = 64;
const int kTuneRows[] = {64, 128, 256, 512, kBatchMaxRows};

struct HostProb {
  int64_t m, n, ldx, ldd, k;
  int r;
  uint64_t seed;
  const float* X;
  std::vector<double> a1;
};

}  // namespace

struct godec_batch {
  int count = 0, q = 0, p = 1;
  double rank_tol = 0.0;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  std::vector<HostProb> hp;
  std::vector<BProb> tab;      // host copy of the device table
  std::vector<BItem> items;    // host copy of the work items (source of async copies)
  BProb* dprobs = nullptr;
  BItem* ditems = nullptr;
  int64_t items_cap = 0;
  int nitems = 0;
  int rows_per_item = 0;
  float* zslots = nullptr;
  double* gslots = nullptr;
  unsigned int* seg_count = nullptr;
  double* dslots = nullptr;            // fixed-order partial sums
  int max_items = 1;
  int* iter = nullptr;
  int* state = nullptr;        // 2 ints per problem: non-finite flag, current rank
  int64_t max_m = 0, max_n = 0, max_k = 0;
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int64_t iters_done = 0;
};

namespace {

godec_status validate_batch(const godec_problem* probs, int32_t count, int32_t q,
                            const godec_opts* opts) {
  if (!probs || count < 1) return fail(GODEC_E_INVAL, "probs is NULL or count < 1");
  if (q < 0) return fail(GODEC_E_INVAL, "q < 0");
  if (opts && opts->size != sizeof(godec_opts)) return fail(GODEC_E_INVAL, "opts->size mismatch");
  if (opts && opts->prec != GODEC_PREC_NATIVE)
    return fail(GODEC_E_UNSUPPORTED, "the batched form runs FP32 only (prec NATIVE)");
  if (opts && (opts->support_dev || opts->support_nnz))
    return fail(GODEC_E_UNSUPPORTED, "the batched form has no fixed-support (completion) form");
  if (opts && opts->lstep != 0)
    return fail(GODEC_E_UNSUPPORTED, "the batched form runs the root-form L update");
  if (opts && opts->warm_start != 0)
    return fail(GODEC_E_UNSUPPORTED, "the batched form starts every chain from A1");
  if (opts && opts->redraw_a1 != 0)
    return fail(GODEC_E_UNSUPPORTED, "the batched form draws A1 once per problem");
  for (int i = 0; i < count; ++i) {
    const godec_problem& P = probs[i];
    const std::string at = " (problem " + std::to_string(i) + ")";
    if (P.m < 1 || P.n < 1) return fail(GODEC_E_INVAL, "m, n must be >= 1" + at);
    if (P.ldx < P.n) return fail(GODEC_E_INVAL, "ldx < n" + at);
    if (P.r < 1 || P.r > std::min(P.m, P.n)) return fail(GODEC_E_INVAL, "r out of range" + at);
    if (P.k < 0 || P.k > P.m * P.n) return fail(GODEC_E_INVAL, "k out of range" + at);
    if (P.r > kBatchRP) return fail(GODEC_E_UNSUPPORTED, "r > 8" + at);
    if (P.n > kBatchMaxN) return fail(GODEC_E_UNSUPPORTED, "n > 512" + at);
  }
  return GODEC_OK;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Carve the workspace (base == nullptr only measures).  Fills b->tab's
// pointers and the shared arrays.
size_t carve_batch(godec_batch* b, void* base) {
  Carver cv{(char*)base};
  b->dprobs = (BProb*)cv.take(sizeof(BProb) * b->count);
  int64_t items = 0, zfl = 0;
  for (const HostProb& h : b->hp) {
    const int64_t it = ceil_div(h.m, kMinRowsPerItem);
    items += it;
    zfl += it * h.n * kBatchRP;
  }
  b->items_cap = items;
  b->ditems = (BItem*)cv.take(sizeof(BItem) * items);
  b->zslots = (float*)cv.take(sizeof(float) * zfl);
  b->gslots = (double*)cv.take(sizeof(double) * items * kBatchRP * kBatchRP);
  b->seg_count = (unsigned int*)cv.take(sizeof(unsigned int) * items * 4);
  b->dslots = (double*)cv.take(sizeof(double) * (2 * items + 64 * (int64_t)b->count));
  b->iter = (int*)cv.take(sizeof(int));
  b->state = (int*)cv.take(sizeof(int) * 2 * b->count);
  b->tab.assign(b->count, BProb{});
  for (int i = 0; i < b->count; ++i) {
    const HostProb& h = b->hp[i];
    BProb& t = b->tab[i];
    t.m = h.m; t.n = h.n; t.ldx = h.ldx; t.ldd = h.ldd; t.k = h.k; t.r = h.r;
    // rank check tolerance: the MATLAB rank() default for the r x r matrix
    t.rank_tol = b->rank_tol > 0.0 ? b->rank_tol : (double)h.r * 0x1p-52;
    t.X = h.X;
    t.D = (float*)cv.take(sizeof(float) * h.m * h.ldd);
    t.P0 = (float*)cv.take(sizeof(float) * h.n * kBatchRP);
    t.P1 = (float*)cv.take(sizeof(float) * h.n * kBatchRP);
    t.VL = (float*)cv.take(sizeof(float) * h.n * kBatchRP);
    t.Bp = (float*)cv.take(sizeof(float) * h.m * kBatchRP);
    t.UL = (float*)cv.take(sizeof(float) * h.m * kBatchRP);
    t.Kp = (float*)cv.take(sizeof(float) * kBatchRP * kBatchRP);
    t.A1 = (const double*)cv.take(sizeof(double) * h.n * h.r);
    t.st = (SmallState*)cv.take(sizeof(SmallState));
    t.sel = (BSel*)cv.take(sizeof(BSel));
    t.hist = (unsigned int*)cv.take(sizeof(unsigned int) * kHistBins);
    // candidate slots: every (row, thread column) position of the selection
    // pass's thread map (at least n per row), plus 3 rows of slack for a last
    // work item whose row count is not a multiple of the rows per block step
    const int64_t r64 = (h.n + 63) / 64 * 64;
    t.rowcap = r64 <= 256 ? 256 / (256 / r64) : 512;
    const int64_t cap = (h.m + 3) * t.rowcap;
    t.cand_idx = (int32_t*)cv.take(sizeof(int32_t) * cap);
    t.cand_val = (float*)cv.take(sizeof(float) * cap);
    t.cand_x = (float*)cv.take(sizeof(float) * cap);
    t.tie_idx = (int32_t*)cv.take(sizeof(int32_t) * cap);
    const int64_t kk = std::max<int64_t>(h.k, 1);
    for (int l = 0; l < 2; ++l) {
      t.s_idx[l] = (int64_t*)cv.take(sizeof(int64_t) * kk);
      t.s_val[l] = (float*)cv.take(sizeof(float) * kk);
      t.s_x[l] = (float*)cv.take(sizeof(float) * kk);
    }
  }
  return cv.off;
}

void fill_host(godec_batch* b, const godec_problem* probs, int32_t count, int32_t q,
               const godec_opts* opts) {
  b->count = count;
  b->q = q;
  b->p = 2 * q + 1;
  b->hp.resize(count);
  b->max_m = b->max_n = b->max_k = 0;
  for (int i = 0; i < count; ++i) {
    HostProb& h = b->hp[i];
    h.m = probs[i].m; h.n = probs[i].n; h.ldx = probs[i].ldx; h.k = probs[i].k;
    h.r = probs[i].r; h.seed = probs[i].seed; h.X = (const float*)probs[i].X_dev;
    h.ldd = ceil_div(h.n, 4) * 4;
    b->max_m = std::max(b->max_m, h.m);
    b->max_n = std::max(b->max_n, h.n);
    b->max_k = std::max(b->max_k, h.k);
  }
  b->rank_tol = 0.0;
  if (opts && opts->rank_tol > 0.0) b->rank_tol = opts->rank_tol;
}

BatchArgs args_of(const godec_batch* b) {
  BatchArgs a;
  a.probs = b->dprobs;
  a.nprob = b->count;
  a.items = b->ditems;
  a.nitems = b->nitems;
  a.zslots = b->zslots;
  a.gslots = b->gslots;
  a.seg_count = b->seg_count;
  a.dslots = b->dslots;
  a.items_cap = b->items_cap;
  a.max_items = b->max_items;
  a.iter = b->iter;
  a.q = b->q;
  a.p = b->p;
  a.rows_per_item = b->rows_per_item;
  return a;
}

// Work items of `rows` rows (problem-major), their partial-slot offsets, and
// each problem's first item and item count; uploads items and table.
godec_status set_items(godec_batch* b, int64_t rows) {
  HIP_TRY(hipStreamSynchronize(b->stream));   // earlier copies from b->items are done
  std::vector<BItem>& items = b->items;
  items.clear();
  b->max_items = 1;
  int64_t zoff = 0;
  for (int i = 0; i < b->count; ++i) {
    const HostProb& h = b->hp[i];
    b->tab[i].item0 = (int32_t)items.size();
    for (int64_t i0 = 0; i0 < h.m; i0 += rows) {
      BItem it;
      it.prob = i;
      it.pad = 0;
      it.i0 = i0;
      it.i1 = std::min(h.m, i0 + rows);
      it.zoff = zoff;
      zoff += h.n * kBatchRP;
      items.push_back(it);
    }
    b->tab[i].nitems = (int32_t)(items.size() - b->tab[i].item0);
    b->max_items = std::max(b->max_items, (int)b->tab[i].nitems);
  }
  if ((int64_t)items.size() > b->items_cap) return fail(GODEC_E_STATE, "work item overflow");
  b->nitems = (int)items.size();
  b->rows_per_item = (int)rows;
  HIP_TRY(hipMemcpyAsync(b->ditems, items.data(), sizeof(BItem) * items.size(),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->dprobs, b->tab.data(), sizeof(BProb) * b->count,
                         hipMemcpyHostToDevice, b->stream));
  return GODEC_OK;
}

void enqueue_iteration(godec_batch* b, int cur) {
  const Launch L{b->stream, b->num_cu};
  const BatchArgs a = args_of(b);
  bl_copy_a1(L, a, b->max_n);
  for (int j = 0; j < b->p; ++j) {
    bl_pass(L, a, 0, 0);
    bl_reduce_slots(L, a, b->max_n);
    bl_chol(L, a, 0, 1, 0, 0, j == 0);
  }
  bl_chol(L, a, 0, 0, 2, 0, 0);   // second round: P0 -> V_L, R joins R2
  int in = 2;
  for (int j = 0; j < b->q; ++j) {
    bl_pass(L, a, in, 0);
    bl_reduce_slots(L, a, b->max_n);
    bl_chol(L, a, 0, 1, 0, 1, j == 0);
    in = 0;
  }
  bl_pass(L, a, in, 1);
  bl_restore_d(L, a, cur, b->max_k);   // the last read of D in this iteration is done
  bl_core(L, a, b->q == 0 ? 1 : 0);
  bl_apply_k(L, a, b->max_m);
  bl_select(L, a, cur, b->max_k);
  bl_update_d(L, a, cur, b->max_k);
}

// Time the Gram pass for each candidate row count; keep the fastest.
// Tuned rows per work item, kept for the life of the process per device and
// batch shape (q and every problem's m, n): later batches of the same shape
// (a layer's forward on each call, say) skip the timing runs.
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, int64_t> g_tune_cache;

std::vector<int64_t> tune_key(const godec_batch* b) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::vector<int64_t> key{dev, b->q, b->count};
  for (const HostProb& h : b->hp) {
    key.push_back(h.m);
    key.push_back(h.n);
  }
  return key;
}

godec_status autotune(godec_batch* b) {
  const std::vector<int64_t> key = tune_key(b);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) return set_items(b, it->second);
  }
  const Launch L{b->stream, b->num_cu};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = 1e30f;
  int64_t best_rows = kMinRowsPerItem;
  for (int rows : kTuneRows) {
    if (rows > std::max<int64_t>(b->max_m, kMinRowsPerItem) && rows != kMinRowsPerItem) break;
    godec_status s = set_items(b, rows);
    if (s != GODEC_OK) return s;
    const BatchArgs a = args_of(b);
    bl_pass(L, a, 0, 0);   // warm-up
    HIP_TRY(hipEventRecord(e0, b->stream));
    for (int rep = 0; rep < 3; ++rep) {
      bl_pass(L, a, 0, 0);
      bl_reduce_slots(L, a, b->max_n);
    }
    HIP_TRY(hipEventRecord(e1, b->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) {
      best = ms;
      best_rows = rows;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best_rows;
  }
  return set_items(b, best_rows);
}

godec_status capture(godec_batch* b) {
  for (int cur = 0; cur < 2; ++cur) {
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    enqueue_iteration(b, cur);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess) return fail(GODEC_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    b->graph[cur] = g;
    HIP_TRY(hipGraphInstantiate(&b->exec[cur], g, nullptr, nullptr, 0));
  }
  return GODEC_OK;
}

void release(godec_batch* b) {
  for (int cur = 0; cur < 2; ++cur) {
    if (b->exec[cur]) (void)hipGraphExecDestroy(b->exec[cur]);
    if (b->graph[cur]) (void)hipGraphDestroy(b->graph[cur]);
  }
  delete b;
}

godec_status check_index(godec_batch* b, int32_t i) {
  if (!b) return fail(GODEC_E_INVAL, "batch is NULL");
  if (i < 0 || i >= b->count) return fail(GODEC_E_INVAL, "problem index out of range");
  return GODEC_OK;
}

}  // namespace

namespace godec_host {

godec_status batch_snapshot_S(godec_batch* b, int64_t* idx_dev, float* val_dev, int64_t kstride,
                              int64_t* nnz_dev) {
  if (!b || b->iters_done == 0) return fail(GODEC_E_STATE, "no iteration has run");
  const Launch L{b->stream, b->num_cu};
  bl_copy_lists(L, b->dprobs, b->count, (int)((b->iters_done - 1) & 1), b->max_k, idx_dev, val_dev,
                kstride, nnz_dev);
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

godec_status batch_factors(godec_batch* b, float* U_dev, int64_t sU, float* V_dev, int64_t sV) {
  if (!b || !U_dev || !V_dev) return fail(GODEC_E_INVAL, "NULL argument");
  int64_t most = 0;
  for (const HostProb& h : b->hp) most = std::max<int64_t>(most, (h.m + h.n) * h.r);
  const Launch L{b->stream, b->num_cu};
  bl_copy_factors(L, b->dprobs, b->count, most, U_dev, sU, V_dev, sV);
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

godec_status batch_ranks(godec_batch* b, int* rank_host) {
  if (!b || !rank_host) return fail(GODEC_E_INVAL, "NULL argument");
  const Launch L{b->stream, b->num_cu};
  bl_gather_state(L, b->dprobs, b->count, b->state);
  std::vector<int> st(2 * (size_t)b->count);
  HIP_TRY(hipMemcpyAsync(st.data(), b->state, sizeof(int) * st.size(), hipMemcpyDeviceToHost,
                         b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  HIP_TRY(hipGetLastError());
  for (int i = 0; i < b->count; ++i) rank_host[i] = st[2 * i + 1];
  return GODEC_OK;
}

}  // namespace godec_host

extern "C" {

godec_status godec_batch_workspace_size(const godec_problem* probs, int32_t count, int32_t q,
                                        const godec_opts* opts, size_t* bytes) {
  if (!bytes) return fail(GODEC_E_INVAL, "bytes is NULL");
  godec_status s = validate_batch(probs, count, q, opts);
  if (s != GODEC_OK) return s;
  godec_batch tmp;
  fill_host(&tmp, probs, count, q, opts);
  *bytes = carve_batch(&tmp, nullptr);
  return GODEC_OK;
}

godec_status godec_batch_init(godec_batch** out, const godec_problem* probs, int32_t count,
                              int32_t q, void* workspace_dev, size_t workspace_bytes,
                              const godec_opts* opts) {
  if (!out) return fail(GODEC_E_INVAL, "out is NULL");
  *out = nullptr;
  godec_status s = validate_batch(probs, count, q, opts);
  if (s != GODEC_OK) return s;
  if (!opts || !opts->stream)
    return fail(GODEC_E_INVAL, "the batched form needs a non-default stream (opts->stream)");
  for (int i = 0; i < count; ++i)
    if (!probs[i].X_dev) return fail(GODEC_E_INVAL, "X_dev is NULL");
  if (!workspace_dev || ((uintptr_t)workspace_dev & 255))
    return fail(GODEC_E_INVAL, "workspace must be non-NULL and 256-byte aligned");
  godec_batch* b = new godec_batch;
  fill_host(b, probs, count, q, opts);
  b->stream = (hipStream_t)opts->stream;
  b->num_cu = device_cu_count();
  const size_t need = carve_batch(b, nullptr);
  if (workspace_bytes < need) {
    delete b;
    return fail(GODEC_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  carve_batch(b, workspace_dev);
  auto bail = [&](godec_status st) {
    release(b);
    return st;
  };
  // A1 per problem (host draw), zeroed selection state
  for (int i = 0; i < count; ++i) {
    HostProb& h = b->hp[i];
    h.a1.resize((size_t)h.n * h.r);
    godec_draw_a1(h.seed, h.n, h.r, h.a1.data());
    hipError_t e = hipMemcpyAsync((void*)b->tab[i].A1, h.a1.data(), sizeof(double) * h.a1.size(),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->tab[i].sel, 0, sizeof(BSel), b->stream);
    if (e != hipSuccess) return bail(fail(GODEC_E_DEVICE, hipGetErrorString(e)));
  }
  if (hipMemsetAsync(b->iter, 0, sizeof(int), b->stream) != hipSuccess)
    return bail(fail(GODEC_E_DEVICE, "memset"));
  s = set_items(b, kMinRowsPerItem);
  if (s != GODEC_OK) return bail(s);
  const Launch L{b->stream, b->num_cu};
  BatchArgs a = args_of(b);
  bl_init(L, a);
  bl_small_init(L, a);
  bl_copy_a1(L, a, b->max_n);
  bl_gather_state(L, b->dprobs, count, b->state);
  std::vector<int> st(2 * (size_t)count);
  if (hipMemcpyAsync(st.data(), b->state, sizeof(int) * st.size(), hipMemcpyDeviceToHost,
                     b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess || hipGetLastError() != hipSuccess)
    return bail(fail(GODEC_E_DEVICE, "batch init kernels failed"));
  for (int i = 0; i < count; ++i)
    if (st[2 * i])
      return bail(fail(GODEC_E_NUMERIC, "X of problem " + std::to_string(i) + " has NaN/Inf"));
  s = autotune(b);
  if (s != GODEC_OK) return bail(s);
  s = capture(b);
  if (s != GODEC_OK) return bail(s);
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bail(fail(GODEC_E_DEVICE, "sync"));
  *out = b;
  return GODEC_OK;
}

godec_status godec_batch_step(godec_batch* b, int32_t iters) {
  if (!b) return fail(GODEC_E_INVAL, "batch is NULL");
  if (iters < 0) return fail(GODEC_E_INVAL, "iters < 0");
  for (int t = 0; t < iters; ++t) {
    HIP_TRY(hipGraphLaunch(b->exec[b->iters_done & 1], b->stream));
    ++b->iters_done;
  }
  return GODEC_OK;
}

godec_status godec_batch_step_eager(godec_batch* b, int32_t iters) {
  if (!b) return fail(GODEC_E_INVAL, "batch is NULL");
  if (iters < 0) return fail(GODEC_E_INVAL, "iters < 0");
  for (int t = 0; t < iters; ++t) {
    enqueue_iteration(b, (int)(b->iters_done & 1));
    ++b->iters_done;
  }
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

godec_status godec_batch_get_factors(godec_batch* b, int32_t i, void* UL_dev, void* VL_dev) {
  godec_status s = check_index(b, i);
  if (s != GODEC_OK) return s;
  if (!UL_dev || !VL_dev) return fail(GODEC_E_INVAL, "NULL output");
  const HostProb& h = b->hp[i];
  const size_t w = sizeof(float) * h.r;
  HIP_TRY(hipMemcpy2DAsync(UL_dev, w, b->tab[i].UL, sizeof(float) * kBatchRP, w, h.m,
                           hipMemcpyDeviceToDevice, b->stream));
  HIP_TRY(hipMemcpy2DAsync(VL_dev, w, b->tab[i].VL, sizeof(float) * kBatchRP, w, h.n,
                           hipMemcpyDeviceToDevice, b->stream));
  return GODEC_OK;
}

godec_status godec_batch_get_S(godec_batch* b, int32_t i, int64_t* idx_dev, void* val_dev,
                               int64_t* nnz_host) {
  godec_status s = check_index(b, i);
  if (s != GODEC_OK) return s;
  if (!idx_dev || !val_dev || !nnz_host) return fail(GODEC_E_INVAL, "NULL output");
  *nnz_host = 0;
  if (b->iters_done == 0) return GODEC_OK;
  const int list = (int)((b->iters_done - 1) & 1);
  BSel hs;
  HIP_TRY(hipMemcpyAsync(&hs, b->tab[i].sel, sizeof(BSel), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  const int64_t nnz = hs.nnz_list[list];
  std::vector<int64_t> idx(nnz);
  std::vector<float> val(nnz);
  if (nnz > 0) {
    HIP_TRY(hipMemcpy(idx.data(), b->tab[i].s_idx[list], sizeof(int64_t) * nnz, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(val.data(), b->tab[i].s_val[list], sizeof(float) * nnz, hipMemcpyDeviceToHost));
  }
  std::vector<int64_t> order(nnz);
  for (int64_t e = 0; e < nnz; ++e) order[e] = e;
  std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return idx[x] < idx[y]; });
  std::vector<int64_t> si(nnz);
  std::vector<float> sv(nnz);
  for (int64_t e = 0; e < nnz; ++e) { si[e] = idx[order[e]]; sv[e] = val[order[e]]; }
  if (nnz > 0) {
    HIP_TRY(hipMemcpy(idx_dev, si.data(), sizeof(int64_t) * nnz, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(val_dev, sv.data(), sizeof(float) * nnz, hipMemcpyHostToDevice));
  }
  *nnz_host = nnz;
  return GODEC_OK;
}

godec_status godec_batch_get_residual(godec_batch* b, int32_t i, void* R_dev, int64_t ldr) {
  godec_status s = check_index(b, i);
  if (s != GODEC_OK) return s;
  if (!R_dev || ldr < b->hp[i].n) return fail(GODEC_E_INVAL, "bad residual output");
  const Launch L{b->stream, b->num_cu};
  bl_residual(L, b->dprobs + i, b->hp[i].m, b->hp[i].n, (float*)R_dev, ldr);
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

godec_status godec_batch_get_A1(godec_batch* b, int32_t i, double* a1_host) {
  godec_status s = check_index(b, i);
  if (s != GODEC_OK) return s;
  if (!a1_host) return fail(GODEC_E_INVAL, "a1_host is NULL");
  std::memcpy(a1_host, b->hp[i].a1.data(), sizeof(double) * b->hp[i].a1.size());
  return GODEC_OK;
}

godec_status godec_batch_get_info(godec_batch* b, int32_t i, godec_info* info) {
  godec_status s = check_index(b, i);
  if (s != GODEC_OK) return s;
  if (!info) return fail(GODEC_E_INVAL, "info is NULL");
  BSel hs;
  int r_eff = 0, flags = 0;
  HIP_TRY(hipMemcpyAsync(&hs, b->tab[i].sel, sizeof(BSel), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipMemcpyAsync(&r_eff, &b->tab[i].st->r_eff, 4, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipMemcpyAsync(&flags, &b->tab[i].st->flags, 4, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  std::memset(info, 0, sizeof(*info));
  info->iters = b->iters_done;
  info->nnz = b->iters_done > 0 ? hs.nnz_list[(b->iters_done - 1) & 1] : 0;
  info->rank_eff = r_eff;
  info->flags = (flags & 3) | (hs.nonfinite ? 1 : 0);
  info->rel_err_sq = hs.rel_err_sq;
  info->threshold = hs.threshold;
  info->sum_r2 = hs.sum_r2;
  info->norm_x2 = hs.norm_x2;
  return GODEC_OK;
}

godec_status godec_batch_tuning(godec_batch* b, int32_t* rows_per_item, int32_t* items) {
  if (!b) return fail(GODEC_E_INVAL, "batch is NULL");
  if (rows_per_item) *rows_per_item = b->rows_per_item;
  if (items) *items = b->nitems;
  return GODEC_OK;
}

godec_status godec_batch_destroy(godec_batch* b) {
  if (!b) return fail(GODEC_E_INVAL, "batch is NULL");
  release(b);
  return GODEC_OK;
}

}  // extern "C"
