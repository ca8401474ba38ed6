/*
 * godec.h -- C ABI of libgodec, GoDec by bilateral random projection on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Zhou & Tao, "Unmixing Incoherent Structures of Big Data by
 * Randomized or Greedy Decomposition" (arXiv 1309.0302).  GoDec splits a
 * dense m x n matrix X into a low-rank part L (rank <= r) and a sparse part
 * S (at most k nonzeros) by minimising ||X - L - S||_F^2 (Sec. 2, Eq. 1-2)
 * with the alternating updates of Algorithm 1 (Sec. 3.1.3):
 *   L_t = BRP power-scheme approximation of X - S_{t-1}  (Eq. 5-9),
 *   S_t = P_Omega(X - L_t), Omega = the nonzero subset of the k largest
 *         entries of |X - L_t|                             (Eq. 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are row-major.  X has leading dimension ldx >= n (elements).
 * - Pointers named *_dev are device pointers (HIP device memory on the
 *   current device); *_host are host pointers.
 * - The caller owns all memory.  The library never allocates device memory:
 *   every device buffer it needs lives in the caller's workspace, whose size
 *   godec_workspace_size() reports.  X is borrowed: it must stay alive and
 *   unmodified until godec_destroy().
 * - All device work is enqueued on the stream given in godec_opts.stream
 *   (a hipStream_t; NULL means the default stream).  Calls that return host
 *   values synchronise that stream; the others are asynchronous.
 * - Errors are returned as godec_status codes; nothing is thrown across the
 *   ABI.  godec_last_error() gives a message for the calling thread's last
 *   failure.  On an error no device work has been enqueued by that call
 *   unless the code is GODEC_E_DEVICE.
 * - Tie-break of the sparse step (Eq. 4 and Algorithm 1 leave it open):
 *   entries are ordered by |R| descending then by row-major linear index
 *   i*n + j ascending; exact zeros are never selected, so
 *   nnz(S) = min(k, number of nonzero residuals).
 * - Rank check (Algorithm 1, "if rank(A2^T Y1) < r"): the numerical rank of
 *   C = A2^T Y1 = Y2^T Y2 is the number of squared singular values of Y2
 *   above rank_tol times the largest; default rank_tol = r * 2^-52 (the
 *   MATLAB rank() default for an r x r matrix).  On a drop the current
 *   iteration keeps the leading r' singular directions and later iterations
 *   use the first r' columns of A1.
 */
#ifndef GODEC_H
#define GODEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GODEC_OK = 0,
  GODEC_E_INVAL = 1,       /* invalid argument (sizes, pointers, options) */
  GODEC_E_NOMEM = 2,       /* workspace smaller than godec_workspace_size */
  GODEC_E_DEVICE = 3,      /* a HIP runtime call failed */
  GODEC_E_NUMERIC = 4,     /* NaN/Inf in X, or a non-finite r x r core */
  GODEC_E_STATE = 5,       /* call not valid in the context's state */
  GODEC_E_UNSUPPORTED = 6  /* valid request outside the library's limits */
} godec_status;

typedef enum { GODEC_F64 = 0, GODEC_F32 = 1 } godec_dtype;

/* Arithmetic of the panel passes.  NATIVE computes in the dtype of X.
 * BF16_REFINE (X must be GODEC_F32) keeps a bfloat16 copy of X - S and runs
 * the panel products on the matrix cores with FP32 accumulation; the last
 * refine_iters iterations redo the final subspace pass, the B chain and the
 * residual in FP32.  The r x r core is FP64 in every mode. */
typedef enum { GODEC_PREC_NATIVE = 0, GODEC_PREC_BF16_REFINE = 1 } godec_prec;

#define GODEC_MAX_RANK 32   /* largest r the library supports */

typedef struct {
  uint32_t size;          /* sizeof(godec_opts); set by godec_opts_default */
  int32_t prec;           /* godec_prec */
  int32_t refine_iters;   /* BF16_REFINE only: trailing FP32 iterations (>= 0) */
  int32_t lstep;          /* L update: 0 = the root form of Algorithm 1 (Eq. 9);
                             1 = the projection form L = (X - S) P_{Y2} that
                             App. II (Thm. 4) bounds: U_L = (X - S) Q2,
                             V_L = Q2, no B chain, core or rank check
                             (dependent directions come out as zero columns) */
  double rank_tol;        /* <= 0: default r * 2^-52 (see above) */
  const double* a1_host;  /* optional n x r row-major A1 replacing the seeded
                             draw (test hook); copied during godec_init */
  void* stream;           /* hipStream_t, NULL = default stream */
  /* Matrix completion (Sec. 2: the cardinality constraint replaced by a fixed
   * support set).  When support_nnz > 0 or support_dev != NULL, the S update
   * is S_t = P_support(X - L_t) on the support_nnz row-major linear indices
   * i*n + j at support_dev (device memory, strictly ascending, in [0, m*n),
   * borrowed and unmodified until destroy; checked during godec_init).  The
   * support is the set of unobserved entries: D = X - S_t then holds X on
   * the observed entries and L_t on the others.  Requires k == support_nnz;
   * either precision form (with BF16_REFINE the bf16 copy of D is rewritten
   * on the support every iteration and the refinement iterations rebuild
   * the FP32 copy from X and S).  info.rel_err_sq is the squared error on
   * the observed entries over ||X||_F^2; info.threshold is 0. */
  const int64_t* support_dev;
  int64_t support_nnz;
  /* 1: every power chain after the first starts from the previous
   * iteration's Q2 (whose span is that of Y2) instead of A1 -- a variant
   * outside the paper that lets a smaller q reach the same fixed point;
   * 0 (default): A1 every iteration, as Algorithm 1. */
  int32_t warm_start;
  /* 1: iteration t (counted from 0 over the context's life) draws its own
   * A1 from the seed seed + t with the generator of godec_draw_a1, as the
   * MSE training of Algorithm 4 redraws it every iteration; after a rank
   * drop to r' the first r' columns of each new draw are used.  Iteration 0
   * uses the seed's own draw, so the first step equals that of the default
   * mode.  0 (default): A1 is drawn once from the seed and kept (Algorithm 1
   * does not redraw it).  The draws are made on the host, four iterations at
   * a time, while the device runs the iterations queued before; each chunk
   * is uploaded on a stream of the library's own into two workspace slots
   * (counted by godec_workspace_size), and each draw is copied into place
   * on opts->stream ahead of its iteration.  godec_init sets this up and
   * draws iterations 1 .. 4.
   * Excludes warm_start and a1_host; single-problem contexts only (the
   * batched form, the layer and godec_solve_static reject it). */
  int32_t redraw_a1;
} godec_opts;

typedef struct {
  int64_t iters;          /* iterations completed */
  int64_t nnz;            /* nonzeros of the current S */
  int32_t rank_eff;       /* r after the rank checks so far */
  int32_t flags;          /* bit 0: NaN/Inf seen; bit 1: rank dropped;
                             bit 2: selection took the slow exact path */
  double rel_err_sq;      /* ||X - L - S||_F^2 / ||X||_F^2 (Sec. 5 measure) */
  double threshold;       /* |R| of the last selected entry (the k-th key) */
  double sum_r2;          /* ||X - L||_F^2 of the last iteration */
  double norm_x2;         /* ||X||_F^2 */
} godec_info;

typedef struct godec_ctx godec_ctx;

/* Fill *opts with defaults: NATIVE, refine_iters = 1, default rank_tol,
 * seeded A1, default stream. */
void godec_opts_default(godec_opts* opts);

/* Bytes of device workspace godec_init needs for this problem.
 * Errors: GODEC_E_INVAL for m, n < 1, r < 1, r > min(m, n), k < 0,
 * k > m*n, q < 0, bad dtype/prec; GODEC_E_UNSUPPORTED for r > GODEC_MAX_RANK. */
godec_status godec_workspace_size(int64_t m, int64_t n, int32_t r, int64_t k,
                                  int32_t q, godec_dtype dtype,
                                  const godec_opts* opts, size_t* bytes);

/* Set up a decomposition of X_dev (m x n, leading dimension ldx, dtype).
 * Draws A1 (n x r standard Gaussian) from `seed` with the counter-based
 * generator of godec_draw_a1 unless opts->a1_host is given, computes
 * ||X||_F^2, checks X for NaN/Inf (GODEC_E_NUMERIC), and sets S_0 = 0.
 * workspace_dev must be 256-byte aligned and at least the size reported by
 * godec_workspace_size for the same arguments (else GODEC_E_NOMEM).
 * Synchronises the stream once (for the NaN check).  *out receives a host
 * handle freed by godec_destroy. */
godec_status godec_init(godec_ctx** out, const void* X_dev, godec_dtype dtype,
                        int64_t m, int64_t n, int64_t ldx, int32_t r,
                        int64_t k, int32_t q, uint64_t seed,
                        void* workspace_dev, size_t workspace_bytes,
                        const godec_opts* opts);

/* Run `iters` iterations of Algorithm 1 (both updates each).  Asynchronous.
 * In BF16_REFINE mode, `total_iters` (>= the iterations run so far + iters)
 * tells which iterations are the trailing refine_iters ones; pass 0 to use
 * the iterations of this call as the total. */
godec_status godec_step(godec_ctx* ctx, int32_t iters, int32_t total_iters);

/* Convenience: init, `iters` steps, copy the results out, destroy.
 * UL_dev (m x r) and VL_dev (n x r) receive L = UL * VL^T (dtype of X);
 * S_idx_dev (int64, capacity k) and S_val_dev (dtype of X, capacity k)
 * receive S sorted by linear index; info (may be NULL) the final state. */
godec_status godec_solve(const void* X_dev, godec_dtype dtype, int64_t m,
                         int64_t n, int64_t ldx, int32_t r, int64_t k,
                         int32_t q, uint64_t seed, int32_t iters,
                         void* workspace_dev, size_t workspace_bytes,
                         const godec_opts* opts, void* UL_dev, void* VL_dev,
                         int64_t* S_idx_dev, void* S_val_dev,
                         godec_info* info);

/* As godec_solve, but iterating until the loop test of Algorithm 1 holds:
 * after each iteration ||X - L - S||_F^2 / ||X||_F^2 (godec_info.rel_err_sq,
 * Sec. 5 measure) is compared with eps, and the loop stops at the first
 * iteration where it is <= eps, or after max_iters iterations.  In
 * BF16_REFINE mode the tested iterations use the BF16 panels and
 * opts->refine_iters FP32 refinement iterations follow the last one (they
 * count toward max_iters).  Synchronises the stream once per iteration.
 * info->iters reports the iterations run.  Errors as godec_solve, plus
 * GODEC_E_INVAL for max_iters < 1 or eps < 0. */
godec_status godec_solve_tol(const void* X_dev, godec_dtype dtype, int64_t m,
                             int64_t n, int64_t ldx, int32_t r, int64_t k,
                             int32_t q, uint64_t seed, int32_t max_iters, double eps,
                             void* workspace_dev, size_t workspace_bytes,
                             const godec_opts* opts, void* UL_dev, void* VL_dev,
                             int64_t* S_idx_dev, void* S_val_dev,
                             godec_info* info);

/* godec_solve without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The workspace is a device array inside
 * the library of GODEC_STATIC_SCRATCH_BYTES bytes (128 MiB), one copy per
 * GPU the library runs on, held until the process ends.  The call allocates
 * no device memory and calls no allocating routine; the caller still passes
 * X and the outputs, exactly as for godec_solve.
 * Limit: problems whose godec_workspace_size exceeds the scratch are
 * rejected with GODEC_E_UNSUPPORTED (the 500 x 500 FP64 and 25 344 x 200
 * FP32 workloads fit; 10 000 x 10 000 does not), and so is
 * opts->redraw_a1 (its draws are staged in pinned host memory).
 * Sharing: every call on one GPU uses that GPU's single array, which keeps
 * the last call's contents; calls that overlap on one GPU (several streams
 * or host threads) race and must be serialised by the caller.  The call
 * synchronises opts->stream before returning (as godec_solve does).
 * Errors as godec_solve, plus GODEC_E_DEVICE if the array's device address
 * cannot be obtained. */
#define GODEC_STATIC_SCRATCH_BYTES (128ull << 20)
godec_status godec_solve_static(const void* X_dev, godec_dtype dtype, int64_t m,
                                int64_t n, int64_t ldx, int32_t r, int64_t k,
                                int32_t q, uint64_t seed, int32_t iters,
                                const godec_opts* opts, void* UL_dev, void* VL_dev,
                                int64_t* S_idx_dev, void* S_val_dev,
                                godec_info* info);

/* L = UL * VL^T: UL_dev m x r, VL_dev n x r, row-major, dtype of X.
 * Columns past rank_eff are zero.  Asynchronous. */
godec_status godec_get_factors(godec_ctx* ctx, void* UL_dev, void* VL_dev);

/* Dense L (m x n, leading dimension ldl >= n, dtype of X).  Asynchronous. */
godec_status godec_get_L_dense(godec_ctx* ctx, void* L_dev, int64_t ldl);

/* Current S as linear indices (int64, ascending) and values (dtype of X);
 * both buffers need capacity k.  Synchronises; *nnz_host gets the count. */
godec_status godec_get_S(godec_ctx* ctx, int64_t* idx_dev, void* val_dev,
                         int64_t* nnz_host);

/* Residual R = X - L of the last iteration, computed with exactly the
 * arithmetic the selection used (m x n, leading dimension ldr, dtype of X;
 * FP32 in BF16_REFINE mode).  Asynchronous. */
godec_status godec_get_residual(godec_ctx* ctx, void* R_dev, int64_t ldr);

/* Copy the n x r A1 in use (FP64, row-major) to the host: with redraw_a1,
 * the draw of the last iteration run (of iteration 0 before any).
 * Synchronous. */
godec_status godec_get_A1(godec_ctx* ctx, double* a1_host);

/* Synchronise the stream and report the state. */
godec_status godec_get_info(godec_ctx* ctx, godec_info* info);

/* Release the handle (no device memory is freed: the caller owns it). */
godec_status godec_destroy(godec_ctx* ctx);

/* Message for the calling thread's last error ("" if none). */
const char* godec_last_error(void);

/* Host-only: draw the n x r standard Gaussian A1 for `seed` (row-major):
 * element (i, c) is Gaussian number i*r + c of the SplitMix64 stream
 * (Steele, Lea, Flood 2014) mapped to 53-bit uniforms in (0,1) and paired
 * by the Box-Muller transform.  Needs no GPU. */
godec_status godec_draw_a1(uint64_t seed, int64_t n, int32_t r,
                           double* a1_host);

/* ---- Per-kernel timing (tracing) -------------------------------------
 * While enabled, the library records a pair of HIP events on its stream
 * around every launch of the streaming kernels, grouped by class.  Timing
 * adds no host synchronisation; godec_profile_read synchronises the stream
 * and reports, per class, the launch count, the summed event time and the
 * algorithmic bytes one launch must move (the m x n operand it streams). */
typedef struct {
  char name[32];            /* kernel class */
  int64_t launches;
  double total_ms;
  double bytes_per_launch;
} godec_kernel_stat;

/* enable != 0 starts (and clears) collection; 0 stops it. */
godec_status godec_profile(godec_ctx* ctx, int32_t enable);
/* Copy up to cap class records into out; *count receives the number of
 * classes with at least one launch.  Synchronous. */
godec_status godec_profile_read(godec_ctx* ctx, godec_kernel_stat* out,
                                int32_t cap, int32_t* count);

/* ---- Graph replay of the iteration -------------------------------------
 * enable != 0: godec_step records each steady iteration shape (the two
 * parities of the double-buffered S lists, with or without the FP32 copy of
 * D in step) once into a HIP graph, on a private stream of the context, and
 * from then on launches that graph on the context's stream: the same kernels
 * with the same arguments and results, one host call per iteration and a
 * shorter dispatch gap between kernels (measured on MI355X: about 1.5 us per
 * kernel against 2.4 us launched one by one).  The first iteration, the
 * refinement iterations of GODEC_PREC_BF16_REFINE and iterations run while
 * per-kernel timing is enabled are launched directly.  Recording and
 * instantiating allocate host and device memory: a caller that must not
 * allocate leaves replay off, the default.  An error while recording leaves
 * the context unusable (destroy it).  Not to be called concurrently with other
 * calls on the same context. */
godec_status godec_set_graphs(godec_ctx* ctx, int32_t enable);

/* ---- Batched form: many independent FP32 problems ----------------------
 * Runs Algorithm 1 (Sec. 3.1.3) on `count` independent problems at once: every
 * phase of an iteration (the Gram passes of the power scheme, Eq. 6-9; the
 * Cholesky QR steps; the r x r core; the top-k step of Eq. 4) is one launch
 * over all problems, and one iteration's launches are captured once into a
 * HIP graph that godec_batch_step replays.  The same readings as the
 * single-problem form apply (A1 drawn once per problem from its seed, the
 * rank check, ties by row-major index, zeros never selected).
 * Limits: FP32 only; r <= 8; n <= 512 columns (the batched Gram pass keeps a
 * whole row of the problem in on-chip memory).  Each problem's S list has
 * capacity k and its candidate buffer m * n entries (all in the workspace).
 * An autotuner times the Gram pass for several row counts per work item
 * during godec_batch_init and keeps the fastest (godec_batch_tuning); the
 * choice is remembered for the life of the process per device and batch
 * shape (q and every problem's m and n), and later batches of that shape
 * reuse it without timing. */
typedef struct {
  const void* X_dev;      /* m x n FP32, leading dimension ldx (borrowed) */
  int64_t m, n, ldx;
  int32_t r;              /* 1 <= r <= min(8, m, n) */
  int32_t reserved;
  int64_t k;              /* 0 <= k <= m * n */
  uint64_t seed;          /* seed of this problem's A1 (godec_draw_a1) */
} godec_problem;

typedef struct godec_batch godec_batch;

/* Workspace bytes for the batch.  Errors as godec_workspace_size, plus
 * GODEC_E_UNSUPPORTED for r > 8 or n > 512, GODEC_E_INVAL for count < 1. */
godec_status godec_batch_workspace_size(const godec_problem* probs, int32_t count, int32_t q,
                                        const godec_opts* opts, size_t* bytes);

/* Set up the batch (FP32 X only; opts->prec must be NATIVE; opts->a1_host is
 * ignored).  Draws every A1, copies X to the working copies, checks X for
 * NaN/Inf (GODEC_E_NUMERIC), runs the autotuner and captures the iteration
 * graph.  Synchronises the stream.  opts->stream must not be NULL (a graph
 * cannot be captured on the legacy default stream); NULL gives E_INVAL. */
godec_status godec_batch_init(godec_batch** out, const godec_problem* probs, int32_t count,
                              int32_t q, void* workspace_dev, size_t workspace_bytes,
                              const godec_opts* opts);

/* Run `iters` iterations on every problem (graph replays; asynchronous). */
godec_status godec_batch_step(godec_batch* b, int32_t iters);

/* The same iterations enqueued as ordinary launches instead of graph
 * replays (test hook: graph and eager runs must agree bit for bit). */
godec_status godec_batch_step_eager(godec_batch* b, int32_t iters);

/* Problem i: L = UL * VL^T (UL_dev m x r, VL_dev n x r, FP32, row-major;
 * columns past rank_eff are zero).  Asynchronous. */
godec_status godec_batch_get_factors(godec_batch* b, int32_t i, void* UL_dev, void* VL_dev);

/* Problem i: S as ascending linear indices and values (capacity k each).
 * Synchronous; *nnz_host receives the count. */
godec_status godec_batch_get_S(godec_batch* b, int32_t i, int64_t* idx_dev, void* val_dev,
                               int64_t* nnz_host);

/* Problem i: the residual X - L the last selection used (m x n, ldr).  Async. */
godec_status godec_batch_get_residual(godec_batch* b, int32_t i, void* R_dev, int64_t ldr);

/* Problem i: its A1 (n x r, FP64) on the host.  Synchronous. */
godec_status godec_batch_get_A1(godec_batch* b, int32_t i, double* a1_host);

/* Problem i: state after the last iteration.  Synchronous. */
godec_status godec_batch_get_info(godec_batch* b, int32_t i, godec_info* info);

/* Rows per work item the autotuner chose and the number of work items. */
godec_status godec_batch_tuning(godec_batch* b, int32_t* rows_per_item, int32_t* items);

/* Release the handle and its graphs (the workspace stays the caller's). */
godec_status godec_batch_destroy(godec_batch* b);

/* ------------------------------------------------------------------------
 * Differentiable layer: T unrolled iterations of Algorithm 1 (Sec. 3.1.3) on
 * a batch of equally shaped problems, with a backward pass.
 *
 * The forward pass runs T iterations on each problem b (X_b = X_dev + b*m*n,
 * row-major, leading dimension n; A1 drawn from seed + b) and keeps the
 * support and values of every S_t.  The backward pass differentiates the
 * unrolled map with the supports M_t held fixed:
 *   S_0 = 0,  L_t = f(X - S_{t-1}),  S_t = M_t * (X - L_t),
 * where f is the power-scheme low-rank update (Eq. 6-9), written exactly as
 * f(D) = D A^q Q (Q^T A^p Q)^a Q^T with A = D^T D, p = 2q + 1,
 * Q = orth(A^p A1), a = -(p - 1) / (2p) (the range of Q is that of Y2 and
 * the core's power gives the (2q+1)-th root of Eq. 9).  Selection is
 * piecewise constant in X, so its derivative is zero almost everywhere.
 * The adjoints are hand-written (eigen-function derivative of the r x r core,
 * orthonormal-range derivative, power-chain terms) and run in the dtype of X
 * with the r x r algebra in FP64.  Limits: r <= 8; the sketch must keep full
 * rank r in every iteration (else GODEC_E_UNSUPPORTED from the forward).
 * ------------------------------------------------------------------------ */
typedef struct godec_layer godec_layer;

/* Workspace bytes for a layer (batch problems of m x n, T iterations). */
godec_status godec_layer_workspace_size(int32_t batch, int64_t m, int64_t n, int32_t r,
                                        int64_t k, int32_t q, int32_t T, godec_dtype dtype,
                                        size_t* bytes);

/* Forward pass.  X_dev: batch x m x n (dtype), borrowed until destroy.
 * L_dev, S_dev (optional, batch x m x n dense, dtype of X) receive L_T and
 * S_T.  opts may be NULL; opts->prec must be NATIVE and opts->a1_host NULL;
 * opts->rank_tol and opts->stream are used.  Synchronous. */
godec_status godec_layer_forward(godec_layer** out, const void* X_dev, godec_dtype dtype,
                                 int32_t batch, int64_t m, int64_t n, int32_t r, int64_t k,
                                 int32_t q, int32_t T, uint64_t seed, void* workspace_dev,
                                 size_t workspace_bytes, const godec_opts* opts, void* L_dev,
                                 void* S_dev);

/* Backward pass: dX_dev = d/dX of <dL, L_T> + <dS, S_T> (all batch x m x n
 * dense, dtype of X; dX is overwritten).  May be called several times.
 * GODEC_E_NUMERIC when a Cholesky pivot or core eigenvalue is not positive.
 * Synchronous. */
godec_status godec_layer_backward(godec_layer* l, const void* dL_dev, const void* dS_dev,
                                  void* dX_dev);

/* Support of S_t (1 <= t <= T) of problem b: ascending linear indices into
 * idx_host (capacity k; may be NULL to query the count), count in *nnz_host. */
godec_status godec_layer_get_mask(godec_layer* l, int32_t b, int32_t t, int64_t* idx_host,
                                  int64_t* nnz_host);

/* A1 (n x r, FP64, row-major) of problem b. */
godec_status godec_layer_get_A1(godec_layer* l, int32_t b, double* a1_host);

/* Release the layer (the workspace stays the caller's). */
godec_status godec_layer_destroy(godec_layer* l);

/* ------------------------------------------------------------------------
 * GreBsmo: greedy bilateral smoothing (Sec. 3.2.1 within the greedy bilateral
 * paradigm of Algorithm 2).  X (m x n) = U V + S + noise is fitted by
 * minimising 1/2 ||X - U V - S||_F^2 + lambda ||S||_1 with rank(U V) <= r
 * (Eq. 10).  Each rank stage appends rows to V, then runs K inner iterations
 * of Eq. 13:
 *   U = Q with (X - S) V^T = Q R,   V = Q^T (X - S),   S = S_lambda(X - U V)
 * (S_lambda: element-wise soft thresholding, Eq. 12).  The appended rows are
 * an orthonormal basis of (R^T R)^power Omega_s, the random-projection
 * estimate of the top right singular vectors of R = X - U V - S (Eq. 14),
 * with Omega_s = columns [s*dr, min((s+1)*dr, r)) of an n x r standard
 * Gaussian matrix drawn from seed (the generator of godec_draw_a1).  V
 * starts empty, so stage 0 uses R = X.
 *
 * Storage: U (m x r) and V^T (n x r) are kept as zero-padded panels in the
 * dtype of X; D = X - S and R are dense m x n copies in the workspace.  The
 * orthonormal bases come from two Cholesky QR rounds with an FP64 Gram
 * matrix; a direction that is numerically dependent on the others comes out
 * as a zero column (the rank reported stays the number of rows appended).
 * ------------------------------------------------------------------------ */
typedef struct godec_grebsmo godec_grebsmo;

typedef struct {
  int32_t rank;          /* rows of V appended so far */
  int32_t stages;        /* rank stages completed */
  int64_t inner_iters;   /* Eq. 13 iterations completed (all stages) */
  int64_t nnz;           /* nonzeros of S after the last S update */
  double rel_err_sq;     /* ||X - U V - S||_F^2 / ||X||_F^2 after it */
  double l1;             /* ||S||_1 after it */
} godec_grebsmo_info;

/* Workspace bytes for an m x n problem of rank bound r (1 <= r <= 32). */
godec_status godec_grebsmo_workspace_size(int64_t m, int64_t n, int32_t r, godec_dtype dtype,
                                          size_t* bytes);

/* Set up a decomposition of X_dev (m x n, leading dimension ldx, borrowed
 * until destroy).  dr >= 1 rows per stage, power >= 1, lambda >= 0 finite.
 * omega_host (n x r FP64 row-major) replaces the seeded draw when not NULL.
 * The workspace must be 256-byte aligned.  stream: a hipStream_t or NULL.
 * Synchronous (checks X for NaN / Inf: GODEC_E_NUMERIC). */
godec_status godec_grebsmo_init(godec_grebsmo** out, const void* X_dev, godec_dtype dtype,
                                int64_t m, int64_t n, int64_t ldx, int32_t r, int32_t dr,
                                int32_t power, double lambda, uint64_t seed,
                                const double* omega_host, void* workspace_dev,
                                size_t workspace_bytes, void* stream);

/* One rank stage: the greedy step, then K >= 1 inner iterations.
 * GODEC_E_STATE once the rank has reached r.  Asynchronous. */
godec_status godec_grebsmo_stage(godec_grebsmo* g, int32_t K);

/* Stages of K inner iterations until the rank reaches r or, when tau > 0,
 * until the relative error is <= tau (read back after each stage, which
 * synchronises).  info may be NULL; when given it is filled (synchronises). */
godec_status godec_grebsmo_solve(godec_grebsmo* g, int32_t K, double tau,
                                 godec_grebsmo_info* info);

/* U (m x rank, row-major) and V^T (n x rank, row-major), so L = U (V^T)^T;
 * dtype of X.  Asynchronous. */
godec_status godec_grebsmo_get_factors(godec_grebsmo* g, void* U_dev, void* Vt_dev);

/* Dense S (m x n, leading dimension lds >= n, dtype of X), recomputed from
 * X, U and V exactly as the last S update computed it.  Asynchronous. */
godec_status godec_grebsmo_get_S(godec_grebsmo* g, void* S_dev, int64_t lds);

/* Counters and objective terms of the last S update.  Synchronises. */
godec_status godec_grebsmo_get_info(godec_grebsmo* g, godec_grebsmo_info* info);

/* Release the handle (the workspace stays the caller's). */
godec_status godec_grebsmo_destroy(godec_grebsmo* g);

/* ---------------------------------------------------------------------------
 * MSE training (Sec. 4.2.1, Algorithm 4): the randomized decomposition of a
 * multi-label training matrix X (n samples x p features) as
 *   X = sum_i L^i + S,  rank(L^i_{Omega_i}) <= r_i,  L^i zero outside the
 *   rows Omega_i of the samples carrying label i,  card(S) <= K.
 * One iteration updates every label in index order (each sees the others'
 * latest values): N = rows Omega_i of X - sum_{j != i} L^j - S, A1 a fresh
 * p x r_i standard Gaussian, Y2 = N^T (N A1), L^i_{Omega_i} = N Q Q^T with
 * Q = orth(Y2) (= Y1 (A2^T Y1)^{-1} Y2^T with A2 = Y1); then
 * S = P_Phi(X - sum_j L^j) on the K entries of largest magnitude (signed
 * residual values; nonzero entries only; ties by row-major index i*p + j).
 * Initialisation: L^i_{Omega_i} = rows Omega_i of D^{-1} X (D = number of
 * labels of each sample, rows without a label are left to S and the
 * residual), S = 0.  A1 of iteration t (from 0) and label i is
 * godec_draw_a1(seed + t*k + i, p, r_i).  A dependent direction of Y2
 * (|Omega_i| < r_i or a rank-deficient N) gives a zero column of Q.
 * Conventions as for godec_init (caller workspace, X borrowed, stream).
 * Limits: r_i <= 8; p <= 512 (FP32) or 256 (FP64); labels may be empty.
 * ------------------------------------------------------------------------- */
typedef struct godec_mse godec_mse;

typedef struct {
  int64_t iters;          /* iterations completed */
  int64_t nnz;            /* nonzeros of S */
  double rel_err_sq;      /* ||X - sum L - S||_F^2 / ||X||_F^2 (Sec. 5) */
  double threshold;       /* |value| of the K-th kept entry of S */
  double sum_r2;          /* ||X - sum L||_F^2 before the last sparse step */
  double norm_x2;         /* ||X||_F^2 */
} godec_mse_info;

/* Workspace bytes.  label_ptr_host: k + 1 offsets into the concatenated row
 * lists (label i's rows are label_rows[label_ptr[i] .. label_ptr[i+1]));
 * ranks_host: r_i.  Errors: GODEC_E_INVAL for bad sizes or ranks,
 * GODEC_E_UNSUPPORTED beyond the limits above. */
godec_status godec_mse_workspace_size(int64_t n, int64_t p, int32_t k,
                                      const int32_t* ranks_host,
                                      const int64_t* label_ptr_host, int64_t K,
                                      godec_dtype dtype, size_t* bytes);

/* Set up training on X_dev (n x p, leading dimension ldx >= p).
 * label_rows_host: the concatenated row lists, each strictly ascending
 * within [0, n) (checked: GODEC_E_INVAL).  Computes the initial residual
 * and ||X||_F^2 on `stream` (a hipStream_t, NULL = default); checks X for
 * NaN/Inf (GODEC_E_NUMERIC, synchronises once). */
godec_status godec_mse_init(godec_mse** out, const void* X_dev, godec_dtype dtype,
                            int64_t n, int64_t p, int64_t ldx, int32_t k,
                            const int32_t* ranks_host, const int64_t* label_ptr_host,
                            const int64_t* label_rows_host, int64_t K, uint64_t seed,
                            void* workspace_dev, size_t workspace_bytes, void* stream);

/* Run `iters` iterations (asynchronous; A1 draws are staged through a
 * pinned host buffer of the handle). */
godec_status godec_mse_step(godec_mse* m, int32_t iters);

/* Label i's factors: L^i_{Omega_i} = U V^T with U_dev (n_i x r_i, rows in the
 * order of the label's row list) and V_dev (p x r_i, orthonormal columns,
 * zero past the numerical rank; V^T is C^i of Algorithm 4's output).
 * GODEC_E_STATE before the first iteration.  Asynchronous. */
godec_status godec_mse_get_factors(godec_mse* m, int32_t i, void* U_dev, void* V_dev);

/* S as ascending linear indices i*p + j (int64, capacity K) and values
 * (dtype of X); *nnz receives the count.  Synchronises the stream. */
godec_status godec_mse_get_S(godec_mse* m, int64_t* idx_dev, void* val_dev, int64_t* nnz);

/* The residual E = X - sum_j L^j - S into E_dev (n x ldo, ldo >= p). */
godec_status godec_mse_get_residual(godec_mse* m, void* E_dev, int64_t ldo);

godec_status godec_mse_get_info(godec_mse* m, godec_mse_info* info);

/* Release the handle and its pinned staging buffer. */
godec_status godec_mse_destroy(godec_mse* m);

/* Build information string (static storage). */
const char* godec_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GODEC_H */
