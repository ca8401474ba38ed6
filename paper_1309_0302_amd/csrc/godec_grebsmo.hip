// libgodec host side of GreBsmo (Sec. 3.2.1, Algorithm 2): the
// godec_grebsmo_* entry points of include/godec.h.
//
// A rank stage is enqueued as:
//   greedy step     P = orth((R^T R)^power Omega_s) by power Gram passes over
//                   R = X - U V - S (X itself before the first stage), each
//                   followed by a Cholesky QR step; its columns are appended
//                   to V^T (Eq. 14, random-projection form);
//   K inner steps   W = D V^T,  U = orth(W) (two Cholesky QR rounds),
//                   V^T = D^T U,  then the soft pass D <- X - S_lambda(X - U V)
//                   (Eq. 12-13), which also writes R on the stage's last step.
// Everything runs on the caller's stream; only solve with tau > 0 and the
// info query synchronise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/godec.h"
#include "godec_internal.h"
#include "host_common.h"

using namespace godec;
using namespace godec_host;

struct godec_grebsmo {
  int64_t m, n, ldx;
  int r, rp, dr, power;
  double lambda;
  bool f64;
  size_t ta;
  const void* X;
  hipStream_t stream;
  int num_cu;
  PanelPlan pl;
  // workspace
  void *D, *R;                 // mpad x ldd, zero padded
  float* Xp;                   // FP32: X zero padded to mpad x ldd (fused soft pass)
  double* Om;                  // stage-ordered Gaussian blocks (n x cnt_s each)
  void *Vt, *U, *W, *P0, *P1;  // panels (ldd or mpad rows x RP)
  void* Zpart;                 // FP64 row-chunk partials of D^T U
  void *Zt, *Wt;               // transposed panels for the matrix cores (FP32)
  float *Wtpart, *Zpart32;
  double* Gpart;
  GramCtl* gram_ctl;
  SmallState* st;
  double* part;                // partial triples of the soft pass
  double* stats;               // [0] sum e^2, [1] sum |s|, [2] nnz, [3] ||X||^2
  int* nonfinite;
  double* nrm_part;            // partial sums of the norm check
  // state
  int rank = 0;
  int stages = 0;
  int64_t inner = 0;
  bool w_ready = false;        // Wtpart holds D V^T of the current D and V
};

namespace {

Launch launch_of(const godec_grebsmo* g) { return Launch{g->stream, g->num_cu}; }

void fill_params(godec_grebsmo* g, int64_t m, int64_t n, int r, godec_dtype dtype, int num_cu) {
  g->m = m;
  g->n = n;
  g->r = r;
  g->rp = round_rp(r);
  g->f64 = dtype == GODEC_F64;
  g->ta = g->f64 ? 8 : 4;
  g->pl = plan_sizes(m, n, 0, num_cu);
}

size_t carve(godec_grebsmo* g, void* base) {
  Carver cv{(char*)base};
  const int64_t ldd = g->pl.ldd, mpad = g->pl.mpad, rp = g->rp;
  const size_t ta = g->ta;
  g->D = cv.take((size_t)mpad * ldd * ta);
  g->R = cv.take((size_t)mpad * ldd * ta);
  g->Om = (double*)cv.take((size_t)g->n * g->r * 8);
  g->Vt = cv.take((size_t)ldd * rp * ta);
  g->P0 = cv.take((size_t)ldd * rp * ta);
  g->P1 = cv.take((size_t)ldd * rp * ta);
  g->U = cv.take((size_t)mpad * rp * ta);
  g->W = cv.take((size_t)mpad * rp * ta);
  if (g->f64) {
    g->Zpart = cv.take((size_t)g->pl.nchunks * ldd * rp * ta);
    g->Xp = nullptr;
    g->Zt = g->Wt = nullptr;
    g->Wtpart = g->Zpart32 = nullptr;
  } else {
    g->Zpart = nullptr;
    g->Xp = (float*)cv.take((size_t)mpad * ldd * 4);
    g->Zt = cv.take((size_t)32 * ldd * 4);
    g->Wt = cv.take((size_t)32 * mpad * 4);
    g->Wtpart = (float*)cv.take((size_t)g->pl.nct_a * 32 * mpad * 4);
    g->Zpart32 = (float*)cv.take((size_t)g->pl.nch_b * ldd * 32 * 4);
  }
  g->Gpart = (double*)cv.take((size_t)kGramSlots * rp * rp * 8);
  g->gram_ctl = (GramCtl*)cv.take(sizeof(GramCtl));
  g->st = (SmallState*)cv.take(sizeof(SmallState));
  g->part = (double*)cv.take((size_t)gb_soft_blocks(g->m, g->n) * 3 * 8);
  g->stats = (double*)cv.take(4 * 8);
  g->nonfinite = (int*)cv.take(8);
  g->nrm_part = (double*)cv.take((size_t)kNormParts * 8);
  return align_up(cv.off, 256);
}

godec_status validate(int64_t m, int64_t n, int32_t r, godec_dtype dtype) {
  if (m < 1 || n < 1) return fail(GODEC_E_INVAL, "m and n must be >= 1");
  if (r < 1) return fail(GODEC_E_INVAL, "r must be >= 1");
  if (r > GODEC_MAX_RANK) return fail(GODEC_E_UNSUPPORTED, "r above GODEC_MAX_RANK");
  if ((int64_t)r > std::min(m, n)) return fail(GODEC_E_INVAL, "r > min(m, n)");
  if (dtype != GODEC_F64 && dtype != GODEC_F32) return fail(GODEC_E_INVAL, "bad dtype");
  return GODEC_OK;
}

// P0 <- orth(src^T (src P0)), one Cholesky QR step (R factor discarded).
void gram_orth(godec_grebsmo* g, const void* src) {
  const Launch L = launch_of(g);
  const int64_t ldd = g->pl.ldd, mpad = g->pl.mpad;
  if (g->f64) {
    launch_apply(L, F64, g->rp, src, ldd, g->m, g->P0, g->W);
    launch_apply_t(L, F64, g->rp, src, ldd, g->m, g->W, g->Zpart, g->pl.rpc, g->pl.nchunks);
    launch_reduce_chunks(L, true, g->rp, g->Zpart, g->pl.nchunks, ldd, g->P1);
  } else {
    mfma_to_t(L, false, g->P0, ldd, g->rp, g->Zt);
    mfma_mm_a(L, false, src, ldd, mpad, g->Zt, g->Wtpart, g->pl.kc_a);
    mfma_reduce_w(L, false, g->Wtpart, (int)g->pl.nct_a, mpad, g->m, g->rp, g->Wt, nullptr);
    mfma_mm_b(L, false, src, ldd, mpad, g->Wt, g->Zpart32, g->pl.rc_b, g->pl.nch_b, g->rp);
    mfma_reduce_z(L, g->Zpart32, g->pl.nch_b, ldd, g->rp, (float*)g->P1);
  }
  launch_gram_tree(L, g->f64, g->rp, g->P1, ldd, g->Gpart, g->gram_ctl, 1, g->st, nullptr, 0, 0);
  launch_apply_rinv(L, g->f64, g->rp, g->P1, ldd, g->st, g->P0, F64, nullptr, 0);
}

// Greedy step of stage g->stages: append orth((R^T R)^power Omega_s) to V^T.
void greedy_step(godec_grebsmo* g) {
  const Launch L = launch_of(g);
  const int c0 = g->rank;
  const int c1 = std::min(c0 + g->dr, g->r);
  const int cnt = c1 - c0;
  const void* src = g->stages == 0 ? g->D : g->R;   // D = X before any S update
  launch_small_init(L, g->st, cnt);
  launch_copy_panel(L, g->f64, g->rp, g->Om + (size_t)g->n * c0, g->n, g->pl.ldd, cnt, g->st,
                    g->P0);
  for (int j = 0; j < g->power; ++j) gram_orth(g, src);
  gb_put_cols(L, g->f64, g->rp, g->P0, g->n, c0, cnt, g->Vt);
  g->rank = c1;
  launch_small_init(L, g->st, c1);
}

// One inner iteration of Eq. 13.  last: the stage's last one, which also
// writes R (when another stage may follow) and the statistics.  In FP32 with
// r <= 8 the soft pass of every other step also forms the next step's
// D V^T partials (mfma_soft_mm_a), so that step starts at their reduction.
void inner_step(godec_grebsmo* g, bool last) {
  const bool with_r = last && g->rank < g->r;
  // fused soft pass + next D V^T (FP32, r <= 8, not the stage's last step)
  const bool fuse = !last && !g->f64 && g->rp <= 8;
  const Launch L = launch_of(g);
  const int64_t ldd = g->pl.ldd, mpad = g->pl.mpad, m = g->m;
  // W = D V^T
  if (g->f64) {
    launch_apply(L, F64, g->rp, g->D, ldd, m, g->Vt, g->W);
  } else {
    if (!g->w_ready) {
      mfma_to_t(L, false, g->Vt, ldd, g->rp, g->Zt);
      mfma_mm_a(L, false, g->D, ldd, mpad, g->Zt, g->Wtpart, g->pl.kc_a);
    }
    mfma_reduce_w(L, false, g->Wtpart, (int)g->pl.nct_a, mpad, m, g->rp, nullptr, (float*)g->W);
  }
  g->w_ready = false;
  // U = orth(W): two Cholesky QR rounds; the second also writes U^T for the
  // matrix-core pass
  launch_gram_tree(L, g->f64, g->rp, g->W, m, g->Gpart, g->gram_ctl, 1, g->st, nullptr, 0, 0);
  launch_apply_rinv(L, g->f64, g->rp, g->W, m, g->st, g->U, F64, nullptr, 0);
  launch_gram_tree(L, g->f64, g->rp, g->U, m, g->Gpart, g->gram_ctl, 1, g->st, nullptr, 0, 0);
  launch_apply_rinv(L, g->f64, g->rp, g->U, m, g->st, g->W, g->f64 ? F64 : F32,
                    g->f64 ? nullptr : g->Wt, mpad);
  std::swap(g->U, g->W);
  // V^T = D^T U
  if (g->f64) {
    launch_apply_t(L, F64, g->rp, g->D, ldd, m, g->U, g->Zpart, g->pl.rpc, g->pl.nchunks);
    launch_reduce_chunks(L, true, g->rp, g->Zpart, g->pl.nchunks, ldd, g->Vt);
  } else {
    mfma_mm_b(L, false, g->D, ldd, mpad, g->Wt, g->Zpart32, g->pl.rc_b, g->pl.nch_b, g->rp);
    if (fuse)   // the fused soft pass below reads V^T transposed
      gb_reduce_zt(L, g->Zpart32, g->pl.nch_b, ldd, g->rp, (float*)g->Vt, (float*)g->Zt);
    else
      mfma_reduce_z(L, g->Zpart32, g->pl.nch_b, ldd, g->rp, (float*)g->Vt);
  }
  // S = S_lambda(X - U V), D = X - S (and R = X - U V - S)
  if (fuse)
    g->w_ready = mfma_soft_mm_a(L, g->rp, g->Xp, ldd, mpad, (const float*)g->U,
                                (const float*)g->Vt, (float)g->lambda, (float*)g->D,
                                (const float*)g->Zt, g->Wtpart, g->pl.kc_a);
  if (!g->w_ready)
    gb_soft(L, g->f64, g->rp, g->X, g->ldx, g->U, g->Vt, m, g->n, g->lambda, g->D, ldd,
            with_r ? g->R : nullptr, last ? g->part : nullptr, last ? g->stats : nullptr);
  g->inner += 1;
}

godec_status run_stage(godec_grebsmo* g, int32_t K) {
  if (K < 1) return fail(GODEC_E_INVAL, "K must be >= 1");
  if (g->rank >= g->r) return fail(GODEC_E_STATE, "rank bound reached");
  greedy_step(g);
  for (int k = 0; k < K; ++k) inner_step(g, k == K - 1);
  g->stages += 1;
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

}  // namespace

extern "C" {

godec_status godec_grebsmo_workspace_size(int64_t m, int64_t n, int32_t r, godec_dtype dtype,
                                          size_t* bytes) {
  if (!bytes) return fail(GODEC_E_INVAL, "bytes is NULL");
  godec_status s = validate(m, n, r, dtype);
  if (s != GODEC_OK) return s;
  godec_grebsmo tmp;
  fill_params(&tmp, m, n, r, dtype, 256);
  *bytes = carve(&tmp, nullptr);
  return GODEC_OK;
}

godec_status godec_grebsmo_init(godec_grebsmo** out, const void* X_dev, godec_dtype dtype,
                                int64_t m, int64_t n, int64_t ldx, int32_t r, int32_t dr,
                                int32_t power, double lambda, uint64_t seed,
                                const double* omega_host, void* ws, size_t ws_bytes,
                                void* stream) {
  if (!out) return fail(GODEC_E_INVAL, "out is NULL");
  *out = nullptr;
  godec_status s = validate(m, n, r, dtype);
  if (s != GODEC_OK) return s;
  if (dr < 1) return fail(GODEC_E_INVAL, "dr must be >= 1");
  if (power < 1) return fail(GODEC_E_INVAL, "power must be >= 1");
  if (!(lambda >= 0.0) || !std::isfinite(lambda))
    return fail(GODEC_E_INVAL, "lambda must be finite and >= 0");
  if (!X_dev || !ws) return fail(GODEC_E_INVAL, "X or workspace is NULL");
  if (ldx < n) return fail(GODEC_E_INVAL, "ldx < n");
  if (((uintptr_t)ws) % 256 != 0) return fail(GODEC_E_INVAL, "workspace not 256-byte aligned");
  if (((uintptr_t)X_dev) % (dtype == GODEC_F64 ? 8 : 4) != 0)
    return fail(GODEC_E_INVAL, "X not aligned to its element size");
  godec_grebsmo* g = new godec_grebsmo();
  fill_params(g, m, n, r, dtype, 256);
  const size_t need = carve(g, nullptr);
  if (ws_bytes < need) {
    delete g;
    return fail(GODEC_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  carve(g, ws);
  g->ldx = ldx;
  g->dr = dr;
  g->power = power;
  g->lambda = lambda;
  g->X = X_dev;
  g->stream = (hipStream_t)stream;
  g->num_cu = device_cu_count();
  auto cleanup = [&](godec_status st, const std::string& msg) {
    delete g;
    return fail(st, msg);
  };
  // Omega, re-laid out stage by stage: block s holds columns [c0, c1) as an
  // n x (c1 - c0) row-major matrix at offset n * c0
  std::vector<double> om((size_t)n * r), blk((size_t)n * r);
  if (omega_host)
    std::memcpy(om.data(), omega_host, sizeof(double) * n * r);
  else
    godec_draw_a1(seed, n, r, om.data());
  for (int c0 = 0; c0 < r; c0 += dr) {
    const int cnt = std::min(dr, r - c0);
    for (int64_t i = 0; i < n; ++i)
      for (int c = 0; c < cnt; ++c)
        blk[(size_t)n * c0 + (size_t)i * cnt + c] = om[(size_t)i * r + c0 + c];
  }
  const Launch L = launch_of(g);
  const int64_t ldd = g->pl.ldd, mpad = g->pl.mpad;
  hipError_t e = hipMemcpyAsync(g->Om, blk.data(), sizeof(double) * n * r,
                                hipMemcpyHostToDevice, g->stream);
  if (e == hipSuccess) e = hipMemsetAsync(g->R, 0, (size_t)mpad * ldd * g->ta, g->stream);
  if (e == hipSuccess) e = hipMemsetAsync(g->Vt, 0, (size_t)ldd * g->rp * g->ta, g->stream);
  if (e == hipSuccess) e = hipMemsetAsync(g->U, 0, (size_t)mpad * g->rp * g->ta, g->stream);
  if (e == hipSuccess) e = hipMemsetAsync(g->W, 0, (size_t)mpad * g->rp * g->ta, g->stream);
  if (e == hipSuccess && g->Wt) e = hipMemsetAsync(g->Wt, 0, (size_t)32 * mpad * 4, g->stream);
  if (e == hipSuccess) e = hipMemsetAsync(g->gram_ctl, 0, sizeof(GramCtl), g->stream);
  if (e == hipSuccess) e = hipMemsetAsync(g->stats, 0, 4 * 8, g->stream);
  if (e == hipSuccess) e = hipMemsetAsync(g->nonfinite, 0, 8, g->stream);
  if (e != hipSuccess) return cleanup(GODEC_E_DEVICE, hipGetErrorString(e));
  launch_init_d(L, g->f64 ? F64 : F32, g->f64, g->D, ldd, X_dev, ldx, m, n, mpad);
  if (g->Xp) launch_init_d(L, F32, false, g->Xp, ldd, X_dev, ldx, m, n, mpad);
  launch_small_init(L, g->st, 1);
  launch_norm_check(L, g->f64, X_dev, ldx, m, n, g->stats + 3, g->nonfinite, g->nrm_part);
  e = hipGetLastError();
  if (e != hipSuccess) return cleanup(GODEC_E_DEVICE, hipGetErrorString(e));
  int bad = 0;
  e = hipMemcpyAsync(&bad, g->nonfinite, sizeof(int), hipMemcpyDeviceToHost, g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) return cleanup(GODEC_E_DEVICE, hipGetErrorString(e));
  if (bad) return cleanup(GODEC_E_NUMERIC, "X contains NaN or Inf");
  *out = g;
  return GODEC_OK;
}

godec_status godec_grebsmo_stage(godec_grebsmo* g, int32_t K) {
  if (!g) return fail(GODEC_E_INVAL, "handle is NULL");
  return run_stage(g, K);
}

godec_status godec_grebsmo_get_info(godec_grebsmo* g, godec_grebsmo_info* info) {
  if (!g || !info) return fail(GODEC_E_INVAL, "NULL argument");
  double h[4];
  HIP_TRY(hipMemcpyAsync(h, g->stats, sizeof(h), hipMemcpyDeviceToHost, g->stream));
  HIP_TRY(hipStreamSynchronize(g->stream));
  info->rank = g->rank;
  info->stages = g->stages;
  info->inner_iters = g->inner;
  info->nnz = (int64_t)h[2];
  info->rel_err_sq = h[3] > 0.0 ? h[0] / h[3] : 0.0;
  info->l1 = h[1];
  return GODEC_OK;
}

godec_status godec_grebsmo_solve(godec_grebsmo* g, int32_t K, double tau,
                                 godec_grebsmo_info* info) {
  if (!g) return fail(GODEC_E_INVAL, "handle is NULL");
  if (K < 1) return fail(GODEC_E_INVAL, "K must be >= 1");
  if (!(tau >= 0.0)) return fail(GODEC_E_INVAL, "tau must be >= 0");
  while (g->rank < g->r) {
    godec_status s = run_stage(g, K);
    if (s != GODEC_OK) return s;
    if (tau > 0.0) {
      godec_grebsmo_info cur;
      s = godec_grebsmo_get_info(g, &cur);
      if (s != GODEC_OK) return s;
      if (cur.rel_err_sq <= tau) break;
    }
  }
  if (info) return godec_grebsmo_get_info(g, info);
  return GODEC_OK;
}

godec_status godec_grebsmo_get_factors(godec_grebsmo* g, void* U_dev, void* Vt_dev) {
  if (!g || !U_dev || !Vt_dev) return fail(GODEC_E_INVAL, "NULL argument");
  if (g->rank < 1) return fail(GODEC_E_STATE, "no stage has run");
  const Launch L = launch_of(g);
  launch_cast_panel(L, g->f64, g->rp, g->U, g->m, g->rank, U_dev);
  launch_cast_panel(L, g->f64, g->rp, g->Vt, g->n, g->rank, Vt_dev);
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

godec_status godec_grebsmo_get_S(godec_grebsmo* g, void* S_dev, int64_t lds) {
  if (!g || !S_dev) return fail(GODEC_E_INVAL, "NULL argument");
  if (lds < g->n) return fail(GODEC_E_INVAL, "lds < n");
  if (g->inner < 1) return fail(GODEC_E_STATE, "no S update has run");
  gb_soft_s(launch_of(g), g->f64, g->rp, g->X, g->ldx, g->U, g->Vt, g->m, g->n, g->lambda,
            S_dev, lds);
  HIP_TRY(hipGetLastError());
  return GODEC_OK;
}

godec_status godec_grebsmo_destroy(godec_grebsmo* g) {
  delete g;
  return GODEC_OK;
}

}  // extern "C"
