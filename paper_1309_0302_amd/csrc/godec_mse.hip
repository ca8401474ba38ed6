// libgodec host side of MSE training (Sec. 4.2.1, Algorithm 4): the
// godec_mse_* entry points of include/godec.h.
//
// One iteration enqueues, for every label i in index order, the three
// launches of the label update (k_mse.hip), then the sparse step:
//   E += S_{t-1}              (E now holds R = X - sum_j L^j)
//   radix select of the K largest |R| over E (the selection of the GoDec
//     path, with zero low-rank factors, so each residual is E itself)
//   E = 0 on the new support  (E = R - S_t)
// All work is on the caller's stream; the random matrices A1 of a chunk of
// iterations are drawn on the host (godec_draw_a1, several threads) into a
// pinned staging buffer and copied ahead of the chunk's launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/godec.h"
#include "godec_internal.h"
#include "host_common.h"

using namespace godec;
using namespace godec_host;

namespace {

constexpr int kRP = 8;           // padded rank of every label
constexpr int kChunk = 4;        // iterations whose A1 draws are staged together
constexpr int kMaxBlk = 256;     // blocks of a label's Y2 row pass (km_reduce_orth adds <= 256)

}  // namespace

struct godec_mse {
  int64_t n, p, ldx, lde, pp, K;
  int k, S;
  bool f64;
  size_t ta;
  uint64_t seed;
  hipStream_t stream;
  int num_cu;
  const void* X;
  std::vector<int32_t> ranks;
  std::vector<int64_t> lptr;
  // workspace
  void* E = nullptr;
  void* cnt = nullptr;
  int64_t* rows = nullptr;
  void* U = nullptr;               // sum n_i x 8
  void* V = nullptr;               // k x 2 x pp x 8
  void* A1dev = nullptr;           // 2 x kChunk x k x pp x 8
  void* part = nullptr;            // kMaxBlk x pp x 8
  double* y2 = nullptr;            // pp x 8: Y2 of the label being updated (FP64)
  unsigned int* ctl = nullptr;     // arrival counter of the Y2 reduction
  void *UL0, *VL0, *VLt0;          // zero factors for the selection
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
  double* s2part;
  uint32_t *bitmap, *wpre, *bsum;
  unsigned long long* boff;
  double* norm_x2;
  int* nonfinite;
  // state
  std::vector<int> vcur;
  std::vector<char> inited;
  int cur = 0;
  int64_t iters_done = 0;
  // staging of the A1 draws
  void* host_a1[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_used[2] = {false, false};
  int slot = 0;
};

namespace {

size_t slot_elems(const godec_mse* m) { return (size_t)kChunk * m->k * m->pp * kRP; }

size_t carve_mse(godec_mse* m, void* base) {
  Carver cv{(char*)base};
  const size_t ta = m->ta;
  const int64_t n = m->n, pp = m->pp;
  const int64_t tot = m->lptr.empty() ? 0 : m->lptr.back();
  m->E = cv.take((size_t)n * m->lde * ta);
  m->cnt = cv.take((size_t)n * ta);
  m->rows = (int64_t*)cv.take((size_t)std::max<int64_t>(tot, 1) * 8);
  m->U = cv.take((size_t)std::max<int64_t>(tot, 1) * kRP * ta);
  m->V = cv.take((size_t)m->k * 2 * pp * kRP * ta);
  m->A1dev = cv.take(2 * slot_elems(m) * ta);
  m->part = cv.take((size_t)kMaxBlk * pp * kRP * ta);
  m->y2 = (double*)cv.take((size_t)pp * kRP * 8);
  m->ctl = (unsigned int*)cv.take(256);
  m->UL0 = cv.take((size_t)n * ta);
  m->VL0 = cv.take((size_t)pp * ta);
  m->VLt0 = cv.take((size_t)pp * ta);
  m->plan[0] = (SelPlan*)cv.take(sizeof(SelPlan));
  m->plan[1] = (SelPlan*)cv.take(sizeof(SelPlan));
  m->hist = (unsigned long long*)cv.take((size_t)kHistReplicas * kHistBins * 8);
  m->counters = (unsigned long long*)cv.take(64);
  m->cap = std::min<int64_t>(n * m->p, 2 * m->K + (1 << 20));
  m->cand_idx = (int64_t*)cv.take((size_t)m->cap * 2 * 8);
  m->cand_val = cv.take((size_t)m->cap * 2 * ta);
  m->cand_x = cv.take((size_t)m->cap * 2 * ta);
  m->seg_count = (unsigned int*)cv.take((size_t)kMaxSeg * 4);
  m->tie_idx = (int64_t*)cv.take((size_t)m->cap * 8);
  m->carry = (SelCarry*)cv.take(sizeof(SelCarry));
  const int64_t kk = std::max<int64_t>(m->K, 1);
  for (int b = 0; b < 2; ++b) {
    m->s_idx[b] = (int64_t*)cv.take((size_t)kk * 8);
    m->s_val[b] = cv.take((size_t)kk * ta);
    m->s_x[b] = cv.take((size_t)kk * ta);
  }
  m->s2part = (double*)cv.take((size_t)std::max(2 * kSelParts, kNormParts) * 8);
  const int64_t nwords = (n * m->p + 31) / 32;
  const int64_t nb = (nwords + 1023) / 1024;
  m->bitmap = (uint32_t*)cv.take((size_t)nwords * 4);
  m->wpre = (uint32_t*)cv.take((size_t)nwords * 4);
  m->bsum = (uint32_t*)cv.take((size_t)nb * 4);
  m->boff = (unsigned long long*)cv.take((size_t)nb * 8);
  m->norm_x2 = (double*)cv.take(8);
  m->nonfinite = (int*)cv.take(8);
  return align_up(cv.off, 256);
}

godec_status validate_mse(int64_t n, int64_t p, int32_t k, const int32_t* ranks,
                          const int64_t* lptr, int64_t K, godec_dtype dtype) {
  if (n < 1 || p < 1) return fail(GODEC_E_INVAL, "need n, p >= 1");
  if (k < 1) return fail(GODEC_E_INVAL, "need at least one label");
  if (!ranks || !lptr) return fail(GODEC_E_INVAL, "ranks or label_ptr is NULL");
  if (dtype != GODEC_F64 && dtype != GODEC_F32) return fail(GODEC_E_INVAL, "bad dtype");
  if (K < 0 || K > n * p) return fail(GODEC_E_INVAL, "need 0 <= K <= n*p");
  if (p > (dtype == GODEC_F64 ? 256 : 512))
    return fail(GODEC_E_UNSUPPORTED, "p exceeds 512 (FP32) or 256 (FP64)");
  if (lptr[0] != 0) return fail(GODEC_E_INVAL, "label_ptr[0] must be 0");
  for (int i = 0; i < k; ++i) {
    if (ranks[i] < 1) return fail(GODEC_E_INVAL, "ranks must be >= 1");
    if (ranks[i] > kRP) return fail(GODEC_E_UNSUPPORTED, "ranks above 8 are not supported");
    if (lptr[i + 1] < lptr[i]) return fail(GODEC_E_INVAL, "label_ptr must not decrease");
    if (lptr[i + 1] - lptr[i] > n) return fail(GODEC_E_INVAL, "a label has more rows than X");
  }
  return GODEC_OK;
}

void fill_params(godec_mse* m, int64_t n, int64_t p, int32_t k, const int32_t* ranks,
                 const int64_t* lptr, int64_t K, godec_dtype dtype) {
  m->n = n;
  m->p = p;
  m->k = k;
  m->K = K;
  m->f64 = dtype == GODEC_F64;
  m->ta = m->f64 ? 8 : 4;
  m->S = p <= 64 ? 1 : (p <= 128 ? 2 : (p <= 256 ? 4 : 8));
  m->pp = 64 * m->S;
  m->lde = m->pp;
  m->ranks.assign(ranks, ranks + k);
  m->lptr.assign(lptr, lptr + k + 1);
}

// Draw the A1 matrices of iterations [t0, t0 + count) into host slot s
// (padded to pp x 8 in the working type), several labels per thread.
void draw_chunk(godec_mse* m, int s, int64_t t0, int count) {
  const int k = m->k;
  const int64_t pp = m->pp, p = m->p;
  const int jobs = count * k;
  unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nth = std::min<unsigned>(nth, (unsigned)jobs);
  auto work = [&](unsigned w) {
    std::vector<double> a;
    for (int job = (int)w; job < jobs; job += (int)nth) {
      const int tt = job / k, i = job % k;
      const int r = m->ranks[(size_t)i];
      a.resize((size_t)p * r);
      godec_draw_a1(m->seed + (uint64_t)(t0 + tt) * (uint64_t)k + (uint64_t)i, p, r, a.data());
      const size_t base = ((size_t)tt * k + i) * pp * kRP;
      for (int64_t c = 0; c < pp; ++c)
        for (int t = 0; t < kRP; ++t) {
          const double v = (c < p && t < r) ? a[(size_t)c * r + t] : 0.0;
          if (m->f64)
            ((double*)m->host_a1[s])[base + c * kRP + t] = v;
          else
            ((float*)m->host_a1[s])[base + c * kRP + t] = (float)v;
        }
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

void run_iteration(godec_mse* m, const char* a1_base) {
  const Launch L{m->stream, m->num_cu};
  const size_t vsz = (size_t)m->pp * kRP * m->ta;
  for (int i = 0; i < m->k; ++i) {
    const int64_t ni = m->lptr[i + 1] - m->lptr[i];
    if (ni == 0) continue;
    MseLabelArgs a;
    a.E = m->E;
    a.lde = m->lde;
    a.X = m->X;
    a.ldx = m->ldx;
    a.cnt = m->cnt;
    a.rows = m->rows + m->lptr[i];
    a.nrows = ni;
    a.p = m->p;
    a.S = m->S;
    a.first = m->inited[i] ? 0 : 1;
    a.r = m->ranks[i];
    // one group of rows per wavefront of the Y2 pass: 32 FP32 or 16 FP64
    // rows per block
    const int64_t rpb = m->f64 ? 16 : 32;
    a.nblk = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxBlk, (ni + rpb - 1) / rpb));
    a.U = (char*)m->U + (size_t)m->lptr[i] * kRP * m->ta;
    const int vc = m->vcur[i];
    a.Vold = (const char*)m->V + ((size_t)i * 2 + vc) * vsz;
    a.Vnew = (char*)m->V + ((size_t)i * 2 + (vc ^ 1)) * vsz;
    a.A1 = a1_base + (size_t)i * vsz;
    a.part = m->part;
    a.y2 = m->y2;
    a.ctl = m->ctl;
    launch_mse_label(L, m->f64, a);
    m->vcur[i] = vc ^ 1;
    m->inited[i] = 1;
  }
  // sparse step: R = E + S_{t-1}, S_t = top-K of R, E = R - S_t
  const int64_t kk = std::max<int64_t>(m->K, 1);
  if (m->iters_done > 0)
    launch_mse_add_s(L, m->f64, m->E, m->lde, m->p, m->s_idx[m->cur], m->s_val[m->cur],
                     m->plan[m->cur], kk);
  const int nxt = m->cur ^ 1;
  SelectArgs s;
  s.X = m->E; s.ldx = m->lde; s.UL = m->UL0; s.VL = m->VL0; s.VLt = m->VLt0; s.ldv = m->pp;
  s.m = m->n; s.n = m->p; s.k = m->K;
  s.plan = m->plan[nxt]; s.hist = m->hist; s.counters = m->counters;
  s.cand_idx = m->cand_idx; s.cand_val = m->cand_val; s.cand_x = m->cand_x; s.cap = m->cap;
  s.seg_count = m->seg_count;
  s.s_idx = m->s_idx[nxt]; s.s_val = m->s_val[nxt]; s.s_x = m->s_x[nxt];
  s.tie_idx = m->tie_idx;
  s.carry = m->carry;
  s.s2part = m->s2part;
  launch_select(L, m->f64, 1, s);
  // the selected entries leave E: x - val = R - R = 0 there
  launch_update_d(L, m->f64 ? F64 : F32, m->E, m->lde, m->p, m->s_idx[nxt], m->s_val[nxt],
                  m->s_x[nxt], m->plan[nxt], kk);
  m->cur = nxt;
  m->iters_done += 1;
}

}  // namespace

extern "C" {

godec_status godec_mse_workspace_size(int64_t n, int64_t p, int32_t k, const int32_t* ranks,
                                      const int64_t* lptr, int64_t K, godec_dtype dtype,
                                      size_t* bytes) {
  if (!bytes) return fail(GODEC_E_INVAL, "bytes is NULL");
  godec_status s = validate_mse(n, p, k, ranks, lptr, K, dtype);
  if (s != GODEC_OK) return s;
  godec_mse tmp;
  fill_params(&tmp, n, p, k, ranks, lptr, K, dtype);
  *bytes = carve_mse(&tmp, nullptr);
  return GODEC_OK;
}

godec_status godec_mse_init(godec_mse** out, const void* X_dev, godec_dtype dtype, int64_t n,
                            int64_t p, int64_t ldx, int32_t k, const int32_t* ranks,
                            const int64_t* lptr, const int64_t* lrows, int64_t K,
                            uint64_t seed, void* ws, size_t ws_bytes, void* stream) {
  if (!out) return fail(GODEC_E_INVAL, "out is NULL");
  *out = nullptr;
  godec_status s = validate_mse(n, p, k, ranks, lptr, K, dtype);
  if (s != GODEC_OK) return s;
  if (!X_dev || !ws) return fail(GODEC_E_INVAL, "X or workspace is NULL");
  if (ldx < p) return fail(GODEC_E_INVAL, "ldx < p");
  if (((uintptr_t)ws) % 256 != 0) return fail(GODEC_E_INVAL, "workspace not 256-byte aligned");
  const int64_t tot = lptr[k];
  if (tot > 0 && !lrows) return fail(GODEC_E_INVAL, "label_rows is NULL");
  // every row list strictly ascending inside [0, n); the label count of
  // each sample for the initialisation
  std::vector<double> cnt((size_t)n, 0.0);
  for (int i = 0; i < k; ++i)
    for (int64_t e = lptr[i]; e < lptr[i + 1]; ++e) {
      const int64_t g = lrows[e];
      if (g < 0 || g >= n || (e > lptr[i] && g <= lrows[e - 1]))
        return fail(GODEC_E_INVAL, "each label's rows must be strictly ascending in [0, n)");
      cnt[(size_t)g] += 1.0;
    }
  godec_mse* m = new godec_mse();
  fill_params(m, n, p, k, ranks, lptr, K, dtype);
  m->ldx = ldx;
  m->seed = seed;
  m->X = X_dev;
  m->stream = (hipStream_t)stream;
  m->num_cu = device_cu_count();
  const size_t need = carve_mse(m, nullptr);
  if (ws_bytes < need) {
    delete m;
    return fail(GODEC_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  carve_mse(m, ws);
  m->vcur.assign((size_t)k, 0);
  m->inited.assign((size_t)k, 0);
  auto bail = [&](godec_status st, const std::string& msg) {
    for (int b = 0; b < 2; ++b) {
      if (m->host_a1[b]) (void)hipHostFree(m->host_a1[b]);
      if (m->ev[b]) (void)hipEventDestroy(m->ev[b]);
    }
    delete m;
    return fail(st, msg);
  };
  for (int b = 0; b < 2; ++b) {
    if (hipHostMalloc(&m->host_a1[b], slot_elems(m) * m->ta, hipHostMallocDefault) != hipSuccess)
      return bail(GODEC_E_DEVICE, "pinned staging buffer");
    if (hipEventCreateWithFlags(&m->ev[b], hipEventDisableTiming) != hipSuccess)
      return bail(GODEC_E_DEVICE, "event");
  }
  const Launch L{m->stream, m->num_cu};
  std::vector<float> cnt32;
  const void* cnt_src = cnt.data();
  if (!m->f64) {
    cnt32.assign(cnt.begin(), cnt.end());
    cnt_src = cnt32.data();
  }
  hipError_t e = hipMemcpyAsync(m->cnt, cnt_src, (size_t)n * m->ta, hipMemcpyHostToDevice,
                                m->stream);
  if (e == hipSuccess && tot > 0)
    e = hipMemcpyAsync(m->rows, lrows, (size_t)tot * 8, hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess)
    e = hipMemsetAsync(m->V, 0, (size_t)k * 2 * m->pp * kRP * m->ta, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->UL0, 0, (size_t)n * m->ta, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->VL0, 0, (size_t)m->pp * m->ta, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->VLt0, 0, (size_t)m->pp * m->ta, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->plan[0], 0, sizeof(SelPlan), m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->plan[1], 0, sizeof(SelPlan), m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->carry, 0, sizeof(SelCarry), m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->nonfinite, 0, 8, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->ctl, 0, 256, m->stream);
  if (e != hipSuccess) return bail(GODEC_E_DEVICE, hipGetErrorString(e));
  launch_mse_init_e(L, m->f64, m->E, m->lde, X_dev, ldx, m->cnt, n, p);
  launch_norm_check(L, m->f64, X_dev, ldx, n, p, m->norm_x2, m->nonfinite, m->s2part);
  int bad = 0;
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(&bad, m->nonfinite, sizeof(int), hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return bail(GODEC_E_DEVICE, hipGetErrorString(e));
  if (bad) return bail(GODEC_E_NUMERIC, "X contains NaN or Inf");
  *out = m;
  return GODEC_OK;
}

godec_status godec_mse_step(godec_mse* m, int32_t iters) {
  if (!m) return fail(GODEC_E_INVAL, "handle is NULL");
  if (iters < 0) return fail(GODEC_E_INVAL, "iters < 0");
  while (iters > 0) {
    const int c = std::min(iters, kChunk);
    const int s = m->slot;
    // the slot's previous chunk has finished reading both copies
    if (m->ev_used[s]) HIP_TRY(hipEventSynchronize(m->ev[s]));
    draw_chunk(m, s, m->iters_done, c);
    char* dev = (char*)m->A1dev + (size_t)s * slot_elems(m) * m->ta;
    HIP_TRY(hipMemcpyAsync(dev, m->host_a1[s], (size_t)c * m->k * m->pp * kRP * m->ta,
                           hipMemcpyHostToDevice, m->stream));
    for (int tt = 0; tt < c; ++tt)
      run_iteration(m, dev + (size_t)tt * m->k * m->pp * kRP * m->ta);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(m->ev[s], m->stream));
    m->ev_used[s] = true;
    m->slot ^= 1;
    iters -= c;
  }
  return GODEC_OK;
}

godec_status godec_mse_get_factors(godec_mse* m, int32_t i, void* U_dev, void* V_dev) {
  if (!m || !U_dev || !V_dev) return fail(GODEC_E_INVAL, "NULL argument");
  if (i < 0 || i >= m->k) return fail(GODEC_E_INVAL, "label out of range");
  if (!m->inited[i] && m->lptr[i + 1] > m->lptr[i])
    return fail(GODEC_E_STATE, "no iteration has run");
  const int64_t ni = m->lptr[i + 1] - m->lptr[i];
  const size_t vsz = (size_t)m->pp * kRP * m->ta;
  const Launch L{m->stream, m->num_cu};
  launch_mse_copy_factors(L, m->f64, (const char*)m->U + (size_t)m->lptr[i] * kRP * m->ta,
                          (const char*)m->V + ((size_t)i * 2 + m->vcur[i]) * vsz, ni, m->p,
                          m->ranks[i], U_dev, V_dev);
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

godec_status godec_mse_get_S(godec_mse* m, int64_t* idx_dev, void* val_dev, int64_t* nnz) {
  if (!m || !nnz) return fail(GODEC_E_INVAL, "NULL argument");
  if (m->iters_done == 0) {
    *nnz = 0;
    return GODEC_OK;
  }
  if (!idx_dev || !val_dev) return fail(GODEC_E_INVAL, "NULL output buffer");
  const Launch L{m->stream, m->num_cu};
  launch_sort_s(L, m->f64, m->s_idx[m->cur], m->s_val[m->cur], m->plan[m->cur], m->n * m->p,
                std::max<int64_t>(m->K, 1), m->bitmap, m->wpre, m->bsum, m->boff, idx_dev,
                val_dev);
  SelPlan hp;
  HIP_TRY(hipMemcpyAsync(&hp, m->plan[m->cur], sizeof(SelPlan), hipMemcpyDeviceToHost,
                         m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  *nnz = hp.nnz;
  return GODEC_OK;
}

godec_status godec_mse_get_residual(godec_mse* m, void* E_dev, int64_t ldo) {
  if (!m || !E_dev || ldo < m->p) return fail(GODEC_E_INVAL, "bad argument");
  const Launch L{m->stream, m->num_cu};
  launch_mse_copy_e(L, m->f64, m->E, m->lde, m->n, m->p, E_dev, ldo);
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

godec_status godec_mse_get_info(godec_mse* m, godec_mse_info* info) {
  if (!m || !info) return fail(GODEC_E_INVAL, "NULL argument");
  SelPlan hp;
  std::memset(&hp, 0, sizeof(hp));
  double nx2 = 0.0;
  HIP_TRY(hipMemcpyAsync(&nx2, m->norm_x2, 8, hipMemcpyDeviceToHost, m->stream));
  if (m->iters_done > 0)
    HIP_TRY(hipMemcpyAsync(&hp, m->plan[m->cur], sizeof(SelPlan), hipMemcpyDeviceToHost,
                           m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  info->iters = m->iters_done;
  info->nnz = hp.nnz;
  info->sum_r2 = hp.sum_r2;
  info->norm_x2 = nx2;
  const double off = hp.sum_r2 - hp.sum_sel2;
  info->rel_err_sq = nx2 > 0 ? std::max(off, 0.0) / nx2 : 0.0;
  info->threshold = hp.threshold;
  return GODEC_OK;
}

godec_status godec_mse_destroy(godec_mse* m) {
  if (m) {
    (void)hipStreamSynchronize(m->stream);
    for (int b = 0; b < 2; ++b) {
      if (m->host_a1[b]) (void)hipHostFree(m->host_a1[b]);
      if (m->ev[b]) (void)hipEventDestroy(m->ev[b]);
    }
    delete m;
  }
  return GODEC_OK;
}

}  // extern "C"
