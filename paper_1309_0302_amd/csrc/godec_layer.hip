// libgodec host side of the differentiable GoDec layer (godec_layer_*).
//
// Forward: every problem of the batch runs T iterations of Algorithm 1
// (Sec. 3.1.3), and the support and values of S_t are checkpointed after each
// iteration.  FP32 problems within the batched form's limits (n <= 512,
// r <= 8) run as one batched decomposition (graph-replayed iterations, one
// snapshot launch per iteration); the others run one single-problem context
// per batch member.
//
// Backward: with the supports frozen, S_t = M_t * (X - L_t) and
// L_t = f(X - S_{t-1}); for t = T .. 1 the library rebuilds D_t = X - S_{t-1}
// from X and the checkpoint, recomputes the forward panels of f at D_t, and
// applies the adjoint of f (k_layer.hip states f and its factorisation) to
// L^bar_t.  The result D^bar_t is kept as low-rank factors U V^T; it is added
// to X^bar, and its values on M_{t-1} become L^bar_{t-1} and leave X^bar,
// since S_{t-1} = M_{t-1} * (X - L_{t-1}) and D_t = X - S_{t-1}.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/godec.h"
#include "godec_internal.h"
#include "host_common.h"

using namespace godec;
using namespace godec_host;

struct godec_layer {
  int nb = 0;
  int64_t m = 0, n = 0, k = 0;
  int r = 0, q = 0, p = 1, T = 0, w = 0;
  bool f64 = false;
  size_t ts = 4;
  hipStream_t stream = nullptr;
  int num_cu = 256;
  const void* X = nullptr;
  bool use_batch = false;  // forward through the batched form
  size_t sub_ws = 0;       // workspace of one context, or of the whole batch
  // Checkpoints of S_t, t = 1..T: slot (t - 1) * nb + b, capacity max(k, 1).
  int64_t* ck_idx = nullptr;
  void* ck_val = nullptr;
  int64_t* ck_nnz = nullptr;
  std::vector<int64_t> ck_nnz_host;
  double* A1 = nullptr;  // nb x n x r
  std::vector<double> a1_host;
  // Backward buffers.  Chains with several members are stored member-major
  // (member j of every problem contiguous) so that one batched launch covers
  // all problems with a single stride.
  void *D = nullptr, *Lbar = nullptr;
  void* Z = nullptr;     // (p + 1) x nb panels n x r: orthonormalised A^j A1
  double* Rc = nullptr;  // (p + 2) x nb r x r: accumulated Cholesky factors
  void* Qs = nullptr;    // (q + 1) x nb panels n x r: A^i Q (member 0 is Q)
  void* Ca = nullptr;  // nb x r x r: C^a
  double *Vv = nullptr, *F = nullptr;
  void *Wm2 = nullptr, *B = nullptr, *LQ = nullptr, *Bbar = nullptr;
  void *Vn = nullptr, *LtB = nullptr, *Qbar = nullptr, *Cur = nullptr, *Tn = nullptr;
  void *Uf = nullptr, *Vf = nullptr;  // nb x m x w, nb x n x w
  void* vals = nullptr;               // nb x max(k, 1)
  uint32_t* bits = nullptr;           // nb x words: support bitmap of one M_t
  int64_t words = 0;
  void* part = nullptr;               // split-K partial products
  int64_t part_cap = 0;
  int* flag = nullptr;
};

namespace {

inline void* at(void* p, size_t ts, int64_t off) { return (char*)p + ts * off; }

// Carve the workspace (base == nullptr only measures).  The forward's own
// workspace comes first: nb single-problem workspaces of ctx_ws bytes, or one
// batch workspace of ctx_ws bytes.
size_t carve_layer(godec_layer* l, void* base, size_t ctx_ws, std::vector<void*>* ctx_ptr) {
  Carver cv{(char*)base};
  const int nb = l->nb, r = l->r, p = l->p, q = l->q;
  const int64_t m = l->m, n = l->n, kk = std::max<int64_t>(l->k, 1);
  const int64_t mn = m * n, nr = n * r, mr = m * r, E = (int64_t)r * r;
  const size_t ts = l->ts;
  l->w = r + 2 * r * (p + q);
  if (ctx_ptr) ctx_ptr->clear();
  for (int b = 0; b < (l->use_batch ? 1 : nb); ++b) {
    void* w = cv.take(ctx_ws);
    if (ctx_ptr) ctx_ptr->push_back(w);
  }
  l->ck_idx = (int64_t*)cv.take(sizeof(int64_t) * l->T * nb * kk);
  l->ck_val = cv.take(ts * l->T * nb * kk);
  l->ck_nnz = (int64_t*)cv.take(sizeof(int64_t) * l->T * nb);
  l->A1 = (double*)cv.take(sizeof(double) * nb * nr);
  l->D = cv.take(ts * nb * mn);
  l->Lbar = cv.take(ts * nb * mn);
  l->Z = cv.take(ts * (p + 1) * nb * nr);
  l->Rc = (double*)cv.take(sizeof(double) * (p + 2) * nb * E);
  l->Qs = cv.take(ts * (q + 1) * nb * nr);
  l->Ca = cv.take(ts * nb * E);
  l->Vv = (double*)cv.take(sizeof(double) * nb * E);
  l->F = (double*)cv.take(sizeof(double) * nb * E);
  void** mpan[] = {&l->Wm2, &l->B, &l->LQ, &l->Bbar};
  for (void** s : mpan) *s = cv.take(ts * nb * mr);
  void** npan[] = {&l->Vn, &l->LtB, &l->Qbar, &l->Cur, &l->Tn};
  for (void** s : npan) *s = cv.take(ts * nb * nr);
  l->Uf = cv.take(ts * nb * m * l->w);
  l->Vf = cv.take(ts * nb * n * l->w);
  l->vals = cv.take(ts * nb * kk);
  l->words = (mn + 31) / 32;
  l->bits = (uint32_t*)cv.take(sizeof(uint32_t) * nb * l->words);
  // Largest split-K product: n x r or r x r outputs, at most 64 chunks.
  l->part_cap = (int64_t)nb * 64 * std::max<int64_t>(nr, E);
  l->part = cv.take(ts * l->part_cap);
  l->flag = (int*)cv.take(sizeof(int) * 4);
  return cv.off;
}

// Batched panel algebra of one layer (all problems per launch).
struct Ops {
  godec_layer* l;
  Launch L;
  // C = alpha op(A) op(B) + beta C with per-problem strides sA, sB, sC.
  void gemm(int M, int N, int K, const void* A, int64_t lda, int64_t sA, int ta, const void* B,
            int64_t ldb, int64_t sB, int tb, double alpha, double beta, void* C, int64_t ldc,
            int64_t sC) {
    lk_gemm(L, l->f64, l->nb, M, N, K, A, lda, sA, ta, B, ldb, sB, tb, alpha, beta, C, ldc, sC,
            l->part, l->part_cap);
  }
  // out (m x r, row stride ldo, problem stride so) = D P, P n x r
  void dmul(const void* P, void* out, int64_t ldo = 0, int64_t so = 0) {
    const int64_t m = l->m, n = l->n;
    const int r = l->r;
    if (!ldo) {
      ldo = r;
      so = m * r;
    }
    if (lk_dpass(L, l->f64, l->nb, (int)m, (int)n, r, l->D, false, P, r, n * r, out, ldo, so,
                 nullptr, l->part, l->part_cap))
      return;
    gemm((int)m, r, (int)n, l->D, n, m * n, 0, P, r, n * r, 0, 1.0, 0.0, out, ldo, so);
  }
  // out (n x r) = D^T W, W m x r
  void dtmul(const void* W, void* out) {
    const int64_t m = l->m, n = l->n;
    const int r = l->r;
    gemm((int)n, r, (int)m, l->D, n, m * n, 1, W, r, m * r, 0, 1.0, 0.0, out, r, n * r);
  }
  // out = A P = D^T (D P)
  void amul(const void* P, void* out) {
    if (lk_dpass(L, l->f64, l->nb, (int)l->m, (int)l->n, l->r, l->D, false, P, l->r,
                 l->n * l->r, nullptr, 0, 0, out, l->part, l->part_cap))
      return;
    dmul(P, l->Wm2);
    dtmul(l->Wm2, out);
  }
  // columns [c0, c0 + r) of the rows x w factor O <- P0, and
  // [c0 + r, c0 + 2r) <- P1 when given
  void put(const void* P0, const void* P1, int64_t rows, void* O, int c0) {
    lk_put_cols(L, l->f64, l->nb, P0, P1, rows * l->r, l->r, O, rows * l->w, l->w, c0, rows);
  }
};

// Factors U (m x w), V (n x w) with D^bar = U V^T for the current D and L^bar.
void vjp_step(godec_layer* l, Ops& o) {
  const int r = l->r, p = l->p, q = l->q, nb = l->nb;
  const int64_t m = l->m, n = l->n, nr = n * r, E = (int64_t)r * r;
  const size_t ts = l->ts;
  const bool f64 = l->f64;
  const Launch& L = o.L;
  auto Zj = [&](int j) { return at(l->Z, ts, (int64_t)j * nb * nr); };
  auto Rcj = [&](int j) { return l->Rc + (int64_t)j * nb * E; };
  auto Qsi = [&](int i) { return at(l->Qs, ts, (int64_t)i * nb * nr); };
  void* Q = Qsi(0);

  // ---- forward panels of f at D ----
  // Z_0 = A1, Rc_0 = I; A Z_{j-1} = Z_j R_j, Rc_j = R_j Rc_{j-1}; so
  // A^j A1 = Z_j Rc_j.  A second Cholesky QR of Z_p gives Q, Rtot = Rc_{p+1}.
  lf_chain_init(L, f64, nb, (int)n, r, l->A1, Zj(0), Rcj(0));
  for (int j = 1; j <= p; ++j) {
    o.amul(Zj(j - 1), l->Vn);
    lf_cholqr(L, f64, nb, (int)n, r, l->Vn, Rcj(j - 1), Rcj(j), Zj(j), l->flag);
  }
  lf_cholqr(L, f64, nb, (int)n, r, Zj(p), Rcj(p), Rcj(p + 1), Q, l->flag);
  for (int i = 1; i <= q; ++i) o.amul(Qsi(i - 1), Qsi(i));
  // B = D A^q Q, C = B^T B, C^a with a = -(p - 1) / (2p)
  o.dmul(Qsi(q), l->B);
  lf_gram_eig(L, f64, nb, (int)m, r, l->B, -(double)(p - 1) / (2.0 * p), l->Ca, l->Vv, l->F,
              l->flag);

  // ---- adjoint of L = B C^a Q^T ----
  if (!lk_dpass(L, f64, nb, (int)m, (int)n, r, l->Lbar, false, Q, r, nr, l->LQ, r, m * r, nullptr,
                l->part, l->part_cap))
    o.gemm((int)m, r, (int)n, l->Lbar, n, m * n, 0, Q, r, nr, 0, 1.0, 0.0, l->LQ, r, m * r);
  o.gemm((int)n, r, (int)m, l->Lbar, n, m * n, 1, l->B, r, m * r, 0, 1.0, 0.0, l->LtB, r, nr);
  // B^bar = L^bar Q C^a + B S2 (S2 from C^a bar = B^T L^bar Q), stored also as
  // the first rank term: B = D (A^q Q) gives B^bar (A^q Q)^T.
  const int64_t w = l->w;
  lf_bbar(L, f64, nb, (int)m, r, l->B, l->LQ, l->Ca, l->Vv, l->F, l->Bbar, l->Uf, (int)w);
  int col = 0;
  o.put(Qsi(q), nullptr, n, l->Vf, col);
  col += r;
  // dA = dD^T D + D^T dD turns <G, dA> with G = U W^T into D^bar terms
  // (D U) W^T + (D W) U^T.  A pair takes columns [col, col + 2r) of both
  // factors: V holds (W, U) (written before the call) and U gets (D U, D W),
  // which is D times V's block with its halves swapped; with AU given the
  // same pass over D also forms AU = A U.
  auto add_term = [&](const void* U, void* AU) {
    if (!lk_dpass(L, f64, nb, (int)m, (int)n, r, l->D, true, at(l->Vf, ts, col), w, n * w,
                  at(l->Uf, ts, col), w, m * w, AU, l->part, l->part_cap)) {
      if (!lk_dmul_rot(L, f64, nb, (int)m, 2 * r, (int)n, l->D, n, m * n, at(l->Vf, ts, col), w,
                       n * w, r, at(l->Uf, ts, col), w, m * w)) {
        o.gemm((int)m, r, (int)n, l->D, n, m * n, 0, at(l->Vf, ts, col + r), w, n * w, 0, 1.0,
               0.0, at(l->Uf, ts, col), w, m * w);
        o.gemm((int)m, r, (int)n, l->D, n, m * n, 0, at(l->Vf, ts, col), w, n * w, 0, 1.0, 0.0,
               at(l->Uf, ts, col + r), w, m * w);
      }
      if (AU) o.amul(U, AU);
    }
    col += 2 * r;
  };
  // A^q inside B: terms (A^i D^T B^bar, A^{q-1-i} Q); Q^bar += A^q D^T B^bar
  void* cur = l->Cur;
  void* spare = l->Tn;
  o.dtmul(l->Bbar, cur);
  for (int i = 0; i < q; ++i) {
    o.put(Qsi(q - 1 - i), cur, n, l->Vf, col);
    add_term(cur, spare);
    std::swap(cur, spare);
  }
  // Q^bar = L^bar^T B C^a + A^q D^T B^bar.  Q = orth(Y), Y = A^p A1 = Q Rtot;
  // f depends on the range of Q only, so Y^bar = (I - Q Q^T) Q^bar Rtot^{-T}.
  lf_qbar(L, f64, nb, (int)n, r, l->LtB, l->Ca, cur, Q, l->Qbar);
  // Terms of A^p: (A^i Y^bar, A^{p-1-i} A1).  With A^j A1 = Z_j Rc_j they are
  // (A^i Ybar0) (Z_j Rc_j Rtot^{-1})^T, Ybar0 = (I - Q Q^T) Q^bar, which keeps
  // every factor well scaled.
  cur = l->Qbar;
  spare = l->Vn;
  for (int i = 0; i < p; ++i) {
    const int j = p - 1 - i;
    lf_pterm(L, f64, nb, (int)n, r, Zj(j), Rcj(j), Rcj(p + 1), cur, l->Vf, (int)w, col);
    const bool more = i + 1 < p;
    add_term(cur, more ? spare : nullptr);
    if (more) std::swap(cur, spare);
  }
}

godec_status validate_layer(int32_t batch, int64_t m, int64_t n, int32_t r, int64_t k, int32_t q,
                            int32_t T, godec_dtype dtype) {
  if (batch < 1 || m < 1 || n < 1 || T < 1)
    return fail(GODEC_E_INVAL, "batch, m, n and T must be >= 1");
  if (r < 1 || r > std::min<int64_t>(m, n)) return fail(GODEC_E_INVAL, "r out of range");
  if (r > kLayerMaxRank) return fail(GODEC_E_UNSUPPORTED, "the layer supports r <= 8");
  if (k < 0 || k > m * n) return fail(GODEC_E_INVAL, "k out of range");
  if (q < 0) return fail(GODEC_E_INVAL, "q < 0");
  if (dtype != GODEC_F64 && dtype != GODEC_F32) return fail(GODEC_E_INVAL, "bad dtype");
  if (m > INT32_MAX || n > INT32_MAX) return fail(GODEC_E_UNSUPPORTED, "m or n too large");
  return GODEC_OK;
}

void fill_layer(godec_layer* l, int32_t batch, int64_t m, int64_t n, int32_t r, int64_t k,
                int32_t q, int32_t T, godec_dtype dtype) {
  l->nb = batch;
  l->m = m;
  l->n = n;
  l->r = r;
  l->k = k;
  l->q = q;
  l->p = 2 * q + 1;
  l->T = T;
  l->f64 = dtype == GODEC_F64;
  l->ts = l->f64 ? 8 : 4;
  l->use_batch = !l->f64 && n <= kBatchMaxN && r <= kBatchRP;
}

std::vector<godec_problem> layer_problems(const godec_layer* l, const void* X_dev, uint64_t seed) {
  std::vector<godec_problem> pr(l->nb);
  for (int b = 0; b < l->nb; ++b) {
    godec_problem& g = pr[b];
    std::memset(&g, 0, sizeof(g));
    g.X_dev = X_dev ? (const char*)X_dev + l->ts * b * l->m * l->n : nullptr;
    g.m = l->m;
    g.n = l->n;
    g.ldx = l->n;
    g.r = l->r;
    g.k = l->k;
    g.seed = seed + (uint64_t)b;
  }
  return pr;
}

// Bytes of the forward's own workspace (per context, or for the batch).
godec_status sub_workspace(godec_layer* l, size_t* bytes) {
  if (!l->use_batch)
    return godec_workspace_size(l->m, l->n, l->r, l->k, l->q, l->f64 ? GODEC_F64 : GODEC_F32,
                                nullptr, bytes);
  const std::vector<godec_problem> pr = layer_problems(l, nullptr, 0);
  return godec_batch_workspace_size(pr.data(), l->nb, l->q, nullptr, bytes);
}


godec_status rank_error(int b) {
  return fail(GODEC_E_UNSUPPORTED, "problem " + std::to_string(b) +
                                       " lost rank in the forward pass; the layer's gradient "
                                       "needs a full-rank sketch");
}

// Forward through one single-problem context per batch member.
godec_status forward_single(godec_layer* l, const void* X_dev, uint64_t seed,
                            const std::vector<void*>& ws, const godec_opts& o, void* L_dev) {
  const int nb = l->nb, T = l->T;
  const int64_t m = l->m, n = l->n, mn = m * n, kk = std::max<int64_t>(l->k, 1);
  const size_t ts = l->ts;
  const godec_dtype dt = l->f64 ? GODEC_F64 : GODEC_F32;
  std::vector<godec_ctx*> ctx(nb, nullptr);
  auto done = [&](godec_status st) {
    for (godec_ctx* c : ctx)
      if (c) godec_destroy(c);
    return st;
  };
  godec_status s;
  for (int b = 0; b < nb; ++b) {
    s = godec_init(&ctx[b], at(const_cast<void*>(X_dev), ts, b * mn), dt, m, n, n, l->r, l->k,
                   l->q, seed + (uint64_t)b, ws[b], l->sub_ws, &o);
    if (s != GODEC_OK) return done(s);
  }
  for (int t = 0; t < T; ++t) {
    for (int b = 0; b < nb; ++b) {
      s = godec_step(ctx[b], 1, 0);
      if (s != GODEC_OK) return done(s);
    }
    for (int b = 0; b < nb; ++b) {
      const int64_t slot = (int64_t)t * nb + b;
      int64_t nnz = 0;
      s = godec_get_S(ctx[b], l->ck_idx + slot * kk, at(l->ck_val, ts, slot * kk), &nnz);
      if (s != GODEC_OK) return done(s);
      l->ck_nnz_host[slot] = nnz;
    }
  }
  for (int b = 0; b < nb; ++b) {
    godec_info info;
    s = godec_get_info(ctx[b], &info);
    if (s != GODEC_OK) return done(s);
    if (info.rank_eff != l->r) return done(rank_error(b));
    s = godec_get_A1(ctx[b], l->a1_host.data() + (size_t)b * n * l->r);
    if (s != GODEC_OK) return done(s);
    if (L_dev) {
      s = godec_get_L_dense(ctx[b], at(L_dev, ts, b * mn), n);
      if (s != GODEC_OK) return done(s);
    }
  }
  hipError_t e = hipMemcpyAsync(l->ck_nnz, l->ck_nnz_host.data(),
                                sizeof(int64_t) * l->ck_nnz_host.size(), hipMemcpyHostToDevice,
                                l->stream);
  if (e != hipSuccess) return done(fail(GODEC_E_DEVICE, hipGetErrorString(e)));
  return done(GODEC_OK);
}

// Forward through one batched decomposition of all members (FP32).  The
// batch runs on a stream of its own (its iterations are graph replays, which
// need a capturable stream) after the caller's stream has drained.
godec_status forward_batched(godec_layer* l, const void* X_dev, uint64_t seed, void* ws,
                             const godec_opts& o, void* L_dev) {
  const int nb = l->nb, T = l->T, r = l->r;
  const int64_t m = l->m, n = l->n, mn = m * n, kk = std::max<int64_t>(l->k, 1);
  HIP_TRY(hipStreamSynchronize(l->stream));
  hipStream_t bs = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
  godec_batch* gb = nullptr;
  auto done = [&](godec_status st) {
    if (gb) godec_batch_destroy(gb);
    (void)hipStreamSynchronize(bs);
    (void)hipStreamDestroy(bs);
    return st;
  };
  godec_opts bo = o;
  bo.stream = bs;
  const std::vector<godec_problem> pr = layer_problems(l, X_dev, seed);
  godec_status s = godec_batch_init(&gb, pr.data(), nb, l->q, ws, l->sub_ws, &bo);
  if (s != GODEC_OK) return done(s);
  for (int t = 0; t < T; ++t) {
    s = godec_batch_step(gb, 1);
    if (s != GODEC_OK) return done(s);
    const int64_t slot = (int64_t)t * nb;
    s = batch_snapshot_S(gb, l->ck_idx + slot * kk, (float*)l->ck_val + slot * kk, kk,
                         l->ck_nnz + slot);
    if (s != GODEC_OK) return done(s);
  }
  hipError_t e = hipMemcpyAsync(l->ck_nnz_host.data(), l->ck_nnz,
                                sizeof(int64_t) * l->ck_nnz_host.size(), hipMemcpyDeviceToHost, bs);
  if (e != hipSuccess) return done(fail(GODEC_E_DEVICE, hipGetErrorString(e)));
  std::vector<int> rank(nb);
  s = batch_ranks(gb, rank.data());   // synchronises bs
  if (s != GODEC_OK) return done(s);
  for (int b = 0; b < nb; ++b) {
    if (rank[b] != r) return done(rank_error(b));
    s = godec_batch_get_A1(gb, b, l->a1_host.data() + (size_t)b * n * r);
    if (s != GODEC_OK) return done(s);
  }
  if (L_dev) {
    s = batch_factors(gb, (float*)l->Uf, m * r, (float*)l->Vf, n * r);
    if (s != GODEC_OK) return done(s);
    const Launch L{bs, l->num_cu};
    lk_uvt_update(L, false, nb, (int)m, (int)n, r, l->Uf, m * r, l->Vf, n * r, L_dev, n, mn, 0,
                  nullptr, 0, nullptr, 0);
  }
  e = hipStreamSynchronize(bs);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return done(fail(GODEC_E_DEVICE, hipGetErrorString(e)));
  return done(GODEC_OK);
}

}  // namespace

extern "C" {

godec_status godec_layer_workspace_size(int32_t batch, int64_t m, int64_t n, int32_t r, int64_t k,
                                        int32_t q, int32_t T, godec_dtype dtype, size_t* bytes) {
  if (!bytes) return fail(GODEC_E_INVAL, "bytes is NULL");
  godec_status s = validate_layer(batch, m, n, r, k, q, T, dtype);
  if (s != GODEC_OK) return s;
  godec_layer tmp;
  fill_layer(&tmp, batch, m, n, r, k, q, T, dtype);
  size_t sub = 0;
  s = sub_workspace(&tmp, &sub);
  if (s != GODEC_OK) return s;
  *bytes = carve_layer(&tmp, nullptr, sub, nullptr);
  return GODEC_OK;
}

godec_status godec_layer_forward(godec_layer** out, const void* X_dev, godec_dtype dtype,
                                 int32_t batch, int64_t m, int64_t n, int32_t r, int64_t k,
                                 int32_t q, int32_t T, uint64_t seed, void* workspace_dev,
                                 size_t workspace_bytes, const godec_opts* opts, void* L_dev,
                                 void* S_dev) {
  if (!out) return fail(GODEC_E_INVAL, "out is NULL");
  *out = nullptr;
  godec_status s = validate_layer(batch, m, n, r, k, q, T, dtype);
  if (s != GODEC_OK) return s;
  if (!X_dev || !workspace_dev || ((uintptr_t)workspace_dev & 255))
    return fail(GODEC_E_INVAL, "X or workspace is NULL, or the workspace is not 256-byte aligned");
  if (opts && opts->size != sizeof(godec_opts)) return fail(GODEC_E_INVAL, "opts->size mismatch");
  if (opts && opts->prec != GODEC_PREC_NATIVE)
    return fail(GODEC_E_UNSUPPORTED, "the layer computes in the dtype of X (prec NATIVE)");
  if (opts && opts->a1_host)
    return fail(GODEC_E_UNSUPPORTED, "the layer draws A1 from the seed");
  if (opts && (opts->support_dev || opts->support_nnz))
    return fail(GODEC_E_UNSUPPORTED, "the layer has no fixed-support (completion) form");
  if (opts && opts->lstep != 0)
    return fail(GODEC_E_UNSUPPORTED, "the layer differentiates the root-form L update");
  if (opts && opts->warm_start != 0)
    return fail(GODEC_E_UNSUPPORTED, "the layer starts every chain from A1");
  if (opts && opts->redraw_a1 != 0)
    return fail(GODEC_E_UNSUPPORTED, "the layer draws A1 once per problem");
  godec_layer* l = new godec_layer;
  fill_layer(l, batch, m, n, r, k, q, T, dtype);
  s = sub_workspace(l, &l->sub_ws);
  if (s != GODEC_OK) {
    delete l;
    return s;
  }
  l->X = X_dev;
  l->stream = opts ? (hipStream_t)opts->stream : nullptr;
  l->num_cu = device_cu_count();
  if (workspace_bytes < carve_layer(l, nullptr, l->sub_ws, nullptr)) {
    delete l;
    return fail(GODEC_E_NOMEM, "workspace too small");
  }
  std::vector<void*> ws;
  carve_layer(l, workspace_dev, l->sub_ws, &ws);
  godec_opts o;
  godec_opts_default(&o);
  if (opts) o.rank_tol = opts->rank_tol;
  o.stream = l->stream;
  l->ck_nnz_host.assign((size_t)T * batch, 0);
  l->a1_host.resize((size_t)batch * n * r);
  s = l->use_batch ? forward_batched(l, X_dev, seed, ws[0], o, L_dev)
                   : forward_single(l, X_dev, seed, ws, o, L_dev);
  if (s != GODEC_OK) {
    delete l;
    return s;
  }
  const int64_t mn = m * n, kk = std::max<int64_t>(k, 1);
  hipError_t e = hipMemcpyAsync(l->A1, l->a1_host.data(), sizeof(double) * l->a1_host.size(),
                                hipMemcpyHostToDevice, l->stream);
  if (e != hipSuccess) {
    delete l;
    return fail(GODEC_E_DEVICE, hipGetErrorString(e));
  }
  if (S_dev) {
    const Launch L{l->stream, l->num_cu};
    const int64_t slot = (int64_t)(T - 1) * batch;
    lk_fill(L, l->f64, batch, S_dev, mn, mn, 0.0);
    lk_scatter(L, l->f64, batch, S_dev, mn, l->ck_idx + slot * kk, at(l->ck_val, l->ts, slot * kk),
               kk, kk, l->ck_nnz + slot, 0, 1.0);
  }
  e = hipStreamSynchronize(l->stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    delete l;
    return fail(GODEC_E_DEVICE, hipGetErrorString(e));
  }
  *out = l;
  return GODEC_OK;
}

godec_status godec_layer_backward(godec_layer* l, const void* dL_dev, const void* dS_dev,
                                  void* dX_dev) {
  if (!l) return fail(GODEC_E_INVAL, "layer is NULL");
  if (!dL_dev || !dS_dev || !dX_dev) return fail(GODEC_E_INVAL, "NULL argument");
  const Launch L{l->stream, l->num_cu};
  const bool f64 = l->f64;
  const int nb = l->nb;
  const int64_t m = l->m, n = l->n, mn = m * n, kk = std::max<int64_t>(l->k, 1);
  const size_t ts = l->ts;
  Ops o{l, L};
  lk_fill(L, false, 1, l->flag, 4, 4, 0.0);
  auto idx_of = [&](int t) { return l->ck_idx + (int64_t)(t - 1) * nb * kk; };
  auto val_of = [&](int t) { return at(l->ck_val, ts, (int64_t)(t - 1) * nb * kk); };
  auto nnz_of = [&](int t) { return l->ck_nnz + (int64_t)(t - 1) * nb; };
  // S_T = M_T * (X - L_T): X^bar = M_T * dS, L^bar_T = dL - M_T * dS
  lk_gather(L, f64, nb, dS_dev, mn, idx_of(l->T), kk, kk, nnz_of(l->T), l->vals);
  lk_fill(L, f64, nb, dX_dev, mn, mn, 0.0);
  lk_scatter(L, f64, nb, dX_dev, mn, idx_of(l->T), l->vals, kk, kk, nnz_of(l->T), 0, 1.0);
  lk_copy(L, f64, nb, dL_dev, l->Lbar, mn, mn);
  lk_scatter(L, f64, nb, l->Lbar, mn, idx_of(l->T), l->vals, kk, kk, nnz_of(l->T), 1, -1.0);
  for (int t = l->T; t >= 1; --t) {
    // D_t = X - S_{t-1}, and the bitmap of M_{t-1}
    lk_rebuild_d(L, f64, nb, l->X, l->D, mn, t >= 2 ? l->bits : nullptr, l->words);
    if (t >= 2)
      lk_sub_mark(L, f64, nb, l->D, mn, idx_of(t - 1), val_of(t - 1), kk, kk, nnz_of(t - 1),
                  l->bits, l->words);
    vjp_step(l, o);
    // X^bar += D^bar = U V^T.  For t >= 2, S_{t-1} = M_{t-1} * (X - L_{t-1})
    // with S^bar_{t-1} = -D^bar: on M_{t-1} the two contributions to X^bar
    // cancel and D^bar becomes L^bar_{t-1}, which is zero off M_{t-1}.
    if (t >= 2) {
      lk_uvt_update(L, f64, nb, (int)m, (int)n, l->w, l->Uf, m * l->w, l->Vf, n * l->w, dX_dev, n,
                    mn, 1, l->bits, l->words, l->Lbar, mn);
    } else {
      lk_uvt_update(L, f64, nb, (int)m, (int)n, l->w, l->Uf, m * l->w, l->Vf, n * l->w, dX_dev, n,
                    mn, 1, nullptr, 0, nullptr, 0);
    }
  }
  int hflag[4] = {0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(hflag, l->flag, sizeof(hflag), hipMemcpyDeviceToHost, l->stream));
  HIP_TRY(hipStreamSynchronize(l->stream));
  HIP_TRY(hipGetLastError());
  if (hflag[0])
    return fail(GODEC_E_NUMERIC, "a non-positive pivot or eigenvalue in the backward pass");
  return GODEC_OK;
}

godec_status godec_layer_get_mask(godec_layer* l, int32_t b, int32_t t, int64_t* idx_host,
                                  int64_t* nnz_host) {
  if (!l || !nnz_host) return fail(GODEC_E_INVAL, "NULL argument");
  if (b < 0 || b >= l->nb || t < 1 || t > l->T) return fail(GODEC_E_INVAL, "index out of range");
  const int64_t kk = std::max<int64_t>(l->k, 1);
  const int64_t slot = (int64_t)(t - 1) * l->nb + b;
  const int64_t nnz = l->ck_nnz_host[slot];
  *nnz_host = nnz;
  if (idx_host && nnz > 0) {
    HIP_TRY(hipMemcpy(idx_host, l->ck_idx + slot * kk, sizeof(int64_t) * nnz,
                      hipMemcpyDeviceToHost));
    std::sort(idx_host, idx_host + nnz);
  }
  return GODEC_OK;
}

godec_status godec_layer_get_A1(godec_layer* l, int32_t b, double* a1_host) {
  if (!l || !a1_host || b < 0 || b >= l->nb) return fail(GODEC_E_INVAL, "bad argument");
  std::memcpy(a1_host, l->a1_host.data() + (size_t)b * l->n * l->r,
              sizeof(double) * l->n * l->r);
  return GODEC_OK;
}

godec_status godec_layer_destroy(godec_layer* l) {
  if (!l) return fail(GODEC_E_INVAL, "layer is NULL");
  delete l;
  return GODEC_OK;
}

}  // extern "C"
