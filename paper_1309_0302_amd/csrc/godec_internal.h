// Internal declarations of libgodec (not part of the public ABI).
//
// Device data layout (all inside the caller's workspace):
//   D      mpad x ldd working copy of X - S_{t-1} in the panel storage type
//          (f64 / f32; plus a bf16 copy in the mixed-precision mode), zero
//          padded to mpad = round_up(m, 64) rows and ldd = round_up(n, 128)
//          columns so panel kernels need no row or column tails.
//   panels n_pad x RP and m x RP row-major (RP = r rounded up to a
//          supported width), compute type TA (double, or float for the f32
//          and bf16 modes); padding rows/columns are zero.
//   small  r x r FP64 state of the power chain and the core.
//   select histogram, plan, candidate list, two sparse lists (S_{t-1},
//          S_t) as (int64 linear index, value) pairs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace godec {

constexpr int kMaxRP = 32;
constexpr int kHistBits0 = 12;        // first radix digit of the key
constexpr int kHistBits = 11;         // later digits
constexpr int kHistBins = 1 << kHistBits0;
constexpr int kHistReplicas = 8;      // global histogram copies (contention)
constexpr int kMaxSeg = 4096;         // most candidate segments (waves of a full pass)
// Fixed-order partial sums: one slot per block of a full selection pass
// (kSelParts, at most kMaxSeg / 4 + 1 blocks), the same again for the
// compaction, and one per block of the norm check (kNormParts).
constexpr int kSelParts = kMaxSeg / 4 + 8;
constexpr int kNormParts = 2048;
constexpr int kBlock = 256;

// Supported padded panel widths.
inline int round_rp(int r) {
  const int w[] = {1, 2, 4, 8, 12, 16, 20, 24, 32};
  for (int x : w)
    if (r <= x) return x;
  return -1;
}

enum DType { F64 = 0, F32 = 1, BF16 = 2 };

// Selection plan, kept in device memory and advanced by the plan kernel.
enum SelMode : int {
  SEL_HIST = 0,      // next full-data pass histograms the next digit
  SEL_COLLECT = 1,   // next full-data pass writes candidates >= bucket low
  SEL_REFINE = 2,    // candidates hold the bucket; refine digits over them
  SEL_FINAL = 3,     // threshold resolved, candidates hold everything needed
  SEL_TIES = 4,      // threshold resolved but ties overflow the candidates:
                     // the next full pass collects the entries above it
  SEL_DONE = 5,      // S written by the index-ordered tie scan
  SEL_TSCAN = 6,     // entries above collected; the tie scan comes next
};

struct SelPlan {
  unsigned long long prefix;   // resolved high bits of the threshold key
  long long k_rem;             // entries still to take inside the bucket
  long long count_above;       // entries above the bucket (all taken)
  long long bucket_count;      // entries inside the bucket
  long long ncand;             // candidates written to the spill region
  long long cap;               // capacity of the segments and of the spill
  long long nnz;               // entries of S written by compaction
  int pbits;                   // number of resolved key bits
  int kbits;                   // key width (31 for f32, 63 for f64)
  int mode;                    // SelMode
  int slow;                    // a slow exact path was used
  int overflow;                // candidate buffer overflowed
  int nseg;                    // segments (= blocks of the full passes)
  int carry_used;              // 1: pass 0 used the carried window
  int carry_dlo;               // lowest level-0 digit histogrammed/collected
  double sum_r2;               // ||X - L||_F^2 (all entries)
  double sum_sel2;             // sum of R^2 over the selected entries
  double threshold;            // |R| of the threshold key
  double sum_obs2;             // fixed support only: sum of R^2 off the support
  unsigned int arrivals;       // blocks of a pass that finished (its last one plans)
  int spare;
};

// Threshold carried between iterations: the level-0 digit window start.
struct SelCarry {
  int valid;
  int dlo;
};

// Small FP64 state of one iteration.
struct SmallState {
  double R2[kMaxRP * kMaxRP];      // R factor of Y2 = (D^T D)^p A1
  double T[kMaxRP * kMaxRP];       // B chain: (D^T D)^q Q2 = Y_q T
  double Rq[kMaxRP * kMaxRP];      // R factor of the last Cholesky QR step
  double dinv[kMaxRP];             // 1 / diag(Rq), 0 on inactive columns
  double V[kMaxRP * kMaxRP];       // eigenvectors of B^T B (warm start)
  double K[kMaxRP * kMaxRP];       // core K' = T K (FP64 copy)
  double sigma[kMaxRP];            // singular values of B (descending)
  double sv_c[kMaxRP];             // singular values of Y2 (rank check)
  int r_eff;                       // current rank (columns of A1 in use)
  int r_keep;                      // directions kept by this iteration
  int flags;                       // bit0 non-finite, bit1 rank drop
  int v_valid;                     // V holds a usable warm start
  int active[kMaxRP];              // column is active in the chain
};

struct Launch {
  hipStream_t stream;
  int num_cu;
};

// ---- panel kernels (k_panel.hip) ----
// W = D Z  (m x RP), D rows of length ldd (padded), Z ldd x RP.
void launch_apply(const Launch& L, DType td, int rp, const void* D,
                  int64_t ldd, int64_t m, const void* Z, void* W);
// Zpart[c] = D[chunk c]^T W[chunk c]  (nchunks x ldd x RP).
void launch_apply_t(const Launch& L, DType td, int rp, const void* D,
                    int64_t ldd, int64_t m, const void* W, void* Zpart,
                    int64_t rows_per_chunk, int64_t nchunks);
// Zo = sum_c Zpart[c]  (rows x RP).
void launch_reduce_chunks(const Launch& L, bool f64, int rp,
                          const void* Zpart, int64_t nchunks, int64_t rows,
                          void* Zo);
// Gram G = P^T P (FP64) of a rows x RP panel in one launch: row blocks
// write partials, a two-level arrival tree adds them in a fixed order, and
// the final G lands in Gpart slot kGramFinal.  With `chol` set, the last
// block then runs the Cholesky step of Cholesky QR (G = R^T R with
// dependent-column detection) and stores R and 1/diag(R) in st->Rq,
// st->dinv, and folds R into acc (acc <- R acc, or R when reset_acc),
// rescaled by a power of two when normalise is set.  ctl must be zero
// before the first launch; every launch leaves it zero.
constexpr int kGramRows = 64;        // rows per block
constexpr int kGramGroup = 16;       // blocks per first-level group
constexpr int kGramMaxBlocks = 256;
constexpr int kGramFinal = kGramMaxBlocks + kGramMaxBlocks / kGramGroup;
constexpr int kGramSlots = kGramFinal + 1;   // partial slots of RP x RP doubles
constexpr int kGramMaxChunks = 16;   // row-chunk partials k_gram_tree can add up
struct GramCtl {
  unsigned int grp[kGramMaxBlocks / kGramGroup];
  unsigned int top;
  unsigned int pad[15];
};
// Zpart (optional, FP32 only): form P first as the sum of nch (<= 16)
// row-chunk partials Zpart (nch x rows x 32, chunk-ascending order) and store
// it, instead of reading it.
void launch_gram_tree(const Launch& L, bool f64, int rp, const void* P, int64_t rows,
                      double* Gpart, GramCtl* ctl, int chol, SmallState* st, double* acc,
                      int reset_acc, int normalise, const float* Zpart = nullptr,
                      int nch = 0);
// Out = P R^{-1} with R = st->Rq (upper triangular; zero rows and dinv = 0 on
// inactive columns), by forward substitution in FP64, rows x RP in the
// panel type; when Zt is given, also its transpose (32 x ldz, bf16 or f32,
// rows >= RP zero) for the next matrix-core pass.
void launch_apply_rinv(const Launch& L, bool f64, int rp, const void* P, int64_t rows,
                       const SmallState* st, void* Out, DType zt_type, void* Zt, int64_t ldz);
// Out = P K  (rows x RP), K is RP x RP in the panel type.
void launch_apply_small(const Launch& L, bool f64, int rp, const void* P,
                        int64_t rows, const void* K, void* Out);
// dst (rows_pad x RP) <- src (rows x r, FP64) with columns >= st->r_eff zeroed.
void launch_copy_panel(const Launch& L, bool f64, int rp, const double* src,
                       int64_t rows, int64_t rows_pad, int r,
                       const SmallState* st, void* dst);
// ---- r x r FP64 kernels (k_small.hip) ----
void launch_core(const Launch& L, bool f64, int rp, const double* Gpart,
                 int nparts, SmallState* st, int p, double rank_tol,
                 int t_identity, void* k_panel);
void launch_small_init(const Launch& L, SmallState* st, int r);

// ---- selection and sparse state (k_select.hip) ----
struct SelectArgs {
  const void* X;        // m x ldx (f64 or f32)
  int64_t ldx;
  const void* UL;       // m x RP
  const void* VL;       // ldd x RP
  const void* VLt;      // RP x ldv (transpose of VL, for coalesced reads)
  int64_t ldv;
  int64_t m, n;
  int64_t k;
  SelPlan* plan;
  unsigned long long* hist;      // kHistRep x kHistBins counters
  unsigned long long* counters;  // [0] above threshold, [1] ties
  // candidates: 2*cap entries; [0, cap) is split into one segment per block
  // of the full-data passes, [cap, 2*cap) is the shared spill region
  int64_t* cand_idx;
  void* cand_val;
  void* cand_x;         // X at each candidate (so D updates need no X reads)
  unsigned int* seg_count;  // kMaxSeg entries: fill of each segment
  int64_t cap;
  int64_t* s_idx;       // output S list (unordered)
  void* s_val;
  void* s_x;
  int64_t* tie_idx;     // scratch for ties (cap entries)
  SelCarry* carry;      // persists across iterations
  double* s2part;       // 2 * kSelParts partial sums (pass 0, then compaction)
  hipEvent_t ev_a = nullptr, ev_b = nullptr;  // optional: bracket pass 0
  // optional (FP32 X only): pass 0 also writes bf16(x) at the entries of the
  // previous S (index list ridx, X values rx, count rplan->nnz) into this
  // mpad x ldd16 copy, restoring X there
  uint16_t* r16 = nullptr;
  int64_t ldd16 = 0;
  const int64_t* ridx = nullptr;
  const float* rx = nullptr;
  const SelPlan* rplan = nullptr;
  // optional: x - s is written into these working copies of D (ldd x n,
  // row-major; the bf16 copy for FP32 X only) at every entry of the new S:
  // by the compaction for the entries it takes below the plan's
  // count_above, by the tie-value pass for the rest (the ties, or every
  // entry when the threshold scan wrote the list)
  void* dwn = nullptr;      // in the type of X
  uint16_t* dw16 = nullptr;
  int64_t lddw = 0;
};
void launch_select(const Launch& L, bool f64, int rp, const SelectArgs& a);
void launch_transpose_panel(const Launch& L, bool f64, const void* VL, int64_t rows, int rp,
                            void* VLt);
// R = X - UL VL^T (dense_l = 0) or L = UL VL^T (dense_l = 1).
void launch_residual(const Launch& L, bool f64, int rp, const void* X,
                     int64_t ldx, const void* UL, const void* VL, int64_t m,
                     int64_t n, void* R, int64_t ldr, int dense_l);
// D (mpad x ldd) <- X with zero padding rows and columns.
void launch_init_d(const Launch& L, DType td, bool xf64, void* D,
                   int64_t ldd, const void* X, int64_t ldx, int64_t m,
                   int64_t n, int64_t mpad);
// D[idx] <- x - val (val != nullptr) or x, for the plan's nnz entries, with
// x the stored value of X at idx.
void launch_update_d(const Launch& L, DType td, void* D, int64_t ldd, int64_t n,
                     const int64_t* idx, const void* val, const void* xv, const SelPlan* plan,
                     int64_t kmax);
// *out2 = ||X||_F^2 summed in a fixed order through `part` (kNormParts
// doubles of scratch); *nonfinite |= 1 on a NaN/Inf entry.
void launch_norm_check(const Launch& L, bool f64, const void* X, int64_t ldx,
                       int64_t m, int64_t n, double* out2, int* nonfinite, double* part);
void launch_sort_s(const Launch& L, bool f64, const int64_t* idx,
                   const void* val, const SelPlan* plan, int64_t mn,
                   int64_t kmax, uint32_t* bitmap, uint32_t* wpre,
                   uint32_t* bsum, unsigned long long* boff, int64_t* out_idx,
                   void* out_val);
// ---- matrix-core panel products (k_mfma.hip), f32 and bf16 storage ----
void mfma_to_t(const Launch& L, bool bf16, const void* Z, int64_t ldd, int rp, void* Zt);
// ev_a/ev_b (optional) receive the kernel's own start and end timestamps.
void mfma_mm_a(const Launch& L, bool bf16, const void* D, int64_t ldd, int64_t mpad,
               const void* Zt, float* Wtpart, int64_t KC, hipEvent_t ev_a = nullptr,
               hipEvent_t ev_b = nullptr);
void mfma_reduce_w(const Launch& L, bool bf16, const float* Wtpart, int nct, int64_t mpad,
                   int64_t m, int rp, void* Wt, float* Wrow);
// Row-chunk partials Zpart[ch] are ldd x zpart_stride(rp) floats.
void mfma_mm_b(const Launch& L, bool bf16, const void* D, int64_t ldd, int64_t mpad,
               const void* Wt, float* Zpart, int64_t RC, int64_t nch, int rp,
               hipEvent_t ev_a = nullptr, hipEvent_t ev_b = nullptr);
void mfma_reduce_z(const Launch& L, const float* Zpart, int64_t nch, int64_t ldd, int rp,
                   float* Zo);
// GreBsmo: D <- Xp - S_lambda(Xp - U V) (Xp: X zero padded to mpad x ldd, U
// mpad x RP, Vt = V^T ldd x RP) and, in the same pass, the column-tile
// partials Wtpart of (D V^T)^T with Zt = (V^T)^T.  Returns false (nothing
// launched) when rp > 8.
bool mfma_soft_mm_a(const Launch& L, int rp, const float* Xp, int64_t ldd, int64_t mpad,
                    const float* U, const float* Vt, float lam, float* D, const float* Zt,
                    float* Wtpart, int64_t KC);

void launch_cast_panel(const Launch& L, bool f64, int rp, const void* src,
                       int64_t rows, int r, void* dst);


// ---- batched form: many independent FP32 problems (k_batch.hip, k_small.hip) ----
// Every phase of an iteration is one launch over all problems.  Streaming
// phases walk a flat list of work items (a problem and a row range); the r x r
// phases run one workgroup per problem.  Panels are kBatchRP = 8 columns
// wide for every problem (columns at or past the problem's rank are zero).
constexpr int kBatchRP = 8;
constexpr int kBatchSub = 16;          // rows of D staged per step of a work item
constexpr int kBatchMaxN = 512;        // widest problem (columns) a work item handles
constexpr int kBatchMaxRows = 1024;    // most rows of one work item

// BS_CARRY: one pass histograms and collects the carried window of level-0
// digits below the previous threshold; BS_HIST: full level-0 histogram
// (first iteration, or the window missed); BS_COLLECT: collect the bucket.
enum BSelMode : int {
  BS_COLLECT = 0, BS_REFINE = 1, BS_FINAL = 2, BS_NONE = 3, BS_HIST = 4, BS_CARRY = 5
};

struct BSel {                          // per-problem selection state
  unsigned long long prefix;           // resolved high bits of the threshold key
  long long k_rem;                     // entries still to take inside the bucket
  long long count_above;               // entries above the bucket
  unsigned long long ncand;            // candidates written (atomic)
  unsigned long long nabove;           // S entries above the threshold (atomic)
  unsigned long long nties;            // tied entries collected (atomic)
  long long nnz;                       // entries of S_t
  long long nnz_list[2];               // entries of each S list
  int pbits;                           // resolved key bits
  int mode;                            // BSelMode
  double sum_r2;                       // ||X - L||_F^2
  double sum_sel2;                     // sum of S_t^2
  double threshold;                    // |R| of the k-th entry
  double rel_err_sq;                   // (sum_r2 - sum_sel2) / ||X||_F^2
  double norm_x2;                      // ||X||_F^2
  int nonfinite;                       // NaN/Inf seen in X
  int s2_done;                         // sum_r2 already taken this iteration
  int carry_valid;                     // carry_dlo holds a window (persists)
  int carry_dlo;                       // lowest level-0 digit of the window
};

struct BProb {                         // device view of one problem
  int64_t m, n, ldx, ldd, k;
  double rank_tol;                     // rank check tolerance (r * 2^-52 by default)
  int32_t r, item0;                    // rank bound; first work item of the problem
  int32_t nitems, pad;                 // work items of the problem
  const float* X;                      // m x ldx (caller's)
  float* D;                            // m x ldd working copy of X - S
  float* P0;                           // n x 8 panels
  float* P1;
  float* VL;                           // V_L = Q2
  float* Bp;                           // m x 8: B' = D Y_q
  float* UL;                           // m x 8: U_L = B' K'
  float* Kp;                           // 8 x 8: K' = T K (FP32 copy)
  const double* A1;                    // n x r
  SmallState* st;
  BSel* sel;
  unsigned int* hist;                  // 4096 bins
  int64_t rowcap;                      // candidate slots per row of X
  int32_t* cand_idx;                   // (m + 3) rowcap candidates: linear index
  float* cand_val;                     //   residual
  float* cand_x;                       //   X
  int32_t* tie_idx;                    // candidate positions of the tied entries
  int64_t* s_idx[2];                   // S lists (k entries each)
  float* s_val[2];
  float* s_x[2];
};

struct BItem {                         // one work item: rows [i0, i1) of a problem
  int32_t prob, pad;
  int64_t i0, i1;
  int64_t zoff;                        // offset of its n x 8 partial in the slot array
};

struct BatchArgs {
  const BProb* probs;
  int nprob;
  const BItem* items;
  int nitems;
  int max_items;                       // most work items of one problem
  unsigned int* seg_count;             // candidates written per (work item, wave)
  float* zslots;                       // Gram-pass partials (n x 8 per item)
  double* gslots;                      // FP64 Gram partials of B' (8 x 8 per item)
  int* iter;                           // device iteration counter
  // fixed-order partial sums: [0, items_cap) sum R^2 per work item,
  // [items_cap, 2 items_cap) ||X||^2 per work item (init), then 64 per
  // problem for the compaction's sum S^2
  double* dslots;
  int64_t items_cap;
  int q, p;
  int rows_per_item;                   // most rows of a work item
};

// chain
void bl_copy_a1(const Launch& L, const BatchArgs& a, int64_t max_n);
// in: panel pointer selector (0 = P0, 1 = P1, 2 = VL); mode 0 = Gram pass
// (partials into zslots), 1 = W = D Y into Bp
void bl_pass(const Launch& L, const BatchArgs& a, int in, int mode);
// one workgroup per problem: out = orth(sum of the problem's partials) (or
// of panel `in` when from_slots == 0), R folded into R2 (acc 0) or T (acc 1)
void bl_chol(const Launch& L, const BatchArgs& a, int from_slots, int in, int out, int acc,
             int reset);
void bl_core(const Launch& L, const BatchArgs& a, int t_identity);
void bl_apply_k(const Launch& L, const BatchArgs& a, int64_t max_m);
// P1 = sum of each problem's Gram-pass partials
void bl_reduce_slots(const Launch& L, const BatchArgs& a, int64_t max_n);
// sparse step
void bl_select(const Launch& L, const BatchArgs& a, int cur, int64_t max_k);
// D = X on the old S list (after the last pass that reads D; the selection
// reads X); kb_compact then writes X - S on the new list's entries above the
// threshold and bl_update_d on its ties (and advances the device iteration
// counter)
void bl_restore_d(const Launch& L, const BatchArgs& a, int cur, int64_t max_k);
void bl_update_d(const Launch& L, const BatchArgs& a, int cur, int64_t max_k);
void bl_init(const Launch& L, const BatchArgs& a);   // D = X, norms, state
void bl_copy_lists(const Launch& L, const BProb* probs_dev, int nprob, int list, int64_t kmax,
                   int64_t* idx_out, float* val_out, int64_t kstride, int64_t* nnz_out);
// every problem's U_L (m x r) and V_L (n x r) into dense panels at U + b sU, V + b sV
void bl_copy_factors(const Launch& L, const BProb* probs_dev, int nprob, int64_t max_elems,
                     float* U, int64_t sU, float* V, int64_t sV);
// out[2i], out[2i + 1] = problem i's non-finite flag and current rank
void bl_gather_state(const Launch& L, const BProb* probs_dev, int nprob, int* out);
void bl_residual(const Launch& L, const BProb* prob_dev, int64_t m, int64_t n, float* R,
                 int64_t ldr);
void bl_small_init(const Launch& L, const BatchArgs& a);


// ---- differentiable layer (k_layer.hip) ----
constexpr int kLayerMaxRank = 8;   // r x r algebra held in registers
// Batched row-major GEMM C = alpha op(A) op(B) + beta C over nb problems
// (batch strides sA, sB, sC); ta / tb: A stored K x M / B stored N x K.
// Splits long K ranges over `part` (part_cap elements) when the output is small.
void lk_gemm(const Launch& L, bool f64, int nb, int M, int N, int K, const void* A, int64_t lda,
             int64_t sA, int ta, const void* B, int64_t ldb, int64_t sB, int tb, double alpha,
             double beta, void* C, int64_t ldc, int64_t sC, void* part, int64_t part_cap);
void lk_fill(const Launch& L, bool f64, int nb, void* P, int64_t count, int64_t stride, double v);
void lk_copy(const Launch& L, bool f64, int nb, const void* S, void* D, int64_t count,
             int64_t stride);
void lk_scatter(const Launch& L, bool f64, int nb, void* P, int64_t stride, const int64_t* idx,
                const void* v, int64_t kstride, int64_t kmax, const int64_t* nnz, int mode,
                double s);
void lk_gather(const Launch& L, bool f64, int nb, const void* G, int64_t stride,
               const int64_t* idx, int64_t kstride, int64_t kmax, const int64_t* nnz, void* out);
// D = X per problem (count entries); zeroes the bitmap words when bits != nullptr.
void lk_rebuild_d(const Launch& L, bool f64, int nb, const void* X, void* D, int64_t count,
                  uint32_t* bits, int64_t words);
// D[idx] -= v over each problem's list, and the list's bits set in the bitmap.
void lk_sub_mark(const Launch& L, bool f64, int nb, void* D, int64_t stride, const int64_t* idx,
                 const void* v, int64_t kstride, int64_t kmax, const int64_t* nnz,
                 uint32_t* bits, int64_t words);
// Row-pass products over a dense m x n matrix D (row stride n; n <= 512 in
// FP32, <= 128 in FP64; r <= 8), each problem in one read of D (k_dpass.hip):
//   Y = D P'  (m x ny, row stride ldy) when Y is given, and
//   Z = D^T Y[:, :r]  (n x r, row stride r) when Z is given (Y may then be
//   nullptr unless pair),
// with P n x r (pair false) or n x 2r (pair true: P' = P with its two r-column
// halves swapped, ny = 2r), row stride ldp.  False when the shape is outside
// the kernel's range (nothing launched).
bool lk_dpass(const Launch& L, bool f64, int nb, int m, int n, int r, const void* D, bool pair,
              const void* P, int64_t ldp, int64_t sP, void* Y, int64_t ldy, int64_t sY, void* Z,
              void* part, int64_t part_cap);
// C = A B' with B' column j = column (j + rot) mod N of B (B K x N, row stride
// ldb), for a long A (M >= 256 rows, K <= 512, N <= 8); false when the shape is
// outside that range (nothing launched).
bool lk_dmul_rot(const Launch& L, bool f64, int nb, int M, int N, int K, const void* A,
                 int64_t lda, int64_t sA, const void* B, int64_t ldb, int64_t sB, int rot,
                 void* C, int64_t ldc, int64_t sC);
// X += U V^T off the support and Lbar = U V^T on it (0 off it); bits ==
// nullptr: X += U V^T everywhere (X = U V^T when accumulate is 0).  U m x w,
// V n x w, row stride w.
void lk_uvt_update(const Launch& L, bool f64, int nb, int m, int n, int w, const void* U,
                   int64_t sU, const void* V, int64_t sV, void* X, int64_t ldx, int64_t sX,
                   int accumulate, const uint32_t* bits, int64_t wstride, void* Lbar,
                   int64_t sL);
void lk_put_cols(const Launch& L, bool f64, int nb, const void* P0, const void* P1, int64_t sP,
                 int r, void* O, int64_t sO, int w, int c0, int64_t rows);
// Fused steps of the backward, one block per problem (k_lfuse.hip; r <= 8,
// r-column panels row-major unless a row stride w is given):
// Z_0 = A1, Rc_0 = I
void lf_chain_init(const Launch& L, bool f64, int nb, int n, int r, const double* A1, void* Z0,
                   double* rc0);
// P^T P = U^T U, Z = P U^{-1}, rc_out = U rc_in; flag |= 1 on a bad pivot
void lf_cholqr(const Launch& L, bool f64, int nb, int rows, int r, const void* P,
               const double* rc_in, double* rc_out, void* Z, int* flag);
// B^T B = V diag(lam) V^T: C^a, V and divided differences F; flag |= 2 if lam <= 0
void lf_gram_eig(const Launch& L, bool f64, int nb, int rows, int r, const void* B, double a,
                 void* calpha, double* v, double* f, int* flag);
// Bbar = LQ C^a + B S2 (S2 from B^T LQ by Daleckii-Krein), also into Uf[:, 0:r]
void lf_bbar(const Launch& L, bool f64, int nb, int m, int r, const void* B, const void* LQ,
             const void* Ca, const double* v, const double* f, void* Bbar, void* Uf, int w);
// Qbar = (LtB C^a + cur) projected off the range of Q
void lf_qbar(const Launch& L, bool f64, int nb, int n, int r, const void* LtB, const void* Ca,
             const void* cur, const void* Q, void* Qbar);
// Vf[:, col:col+r] = Zj Rc Rtot^{-1}, Vf[:, col+r:col+2r] = cur
void lf_pterm(const Launch& L, bool f64, int nb, int n, int r, const void* Zj, const double* rc,
              const double* rtot, const void* cur, void* Vf, int w, int col);

// ---- matrix completion (k_complete.hip) ----
// S update on a fixed support (ascending; row_ptr: m x (ceil(n/256) + 1)
// starts of its runs per row and 256-column block): lists
// s_idx / s_val / s_x and plan (nnz, sum_r2, sum_sel2) as the selection
// would leave them, in one pass over X.  scratch: at least
// fixed_support_scratch_doubles() doubles.
void launch_fixed_support(const Launch& L, bool f64, int rp, const void* X, int64_t ldx,
                          const void* UL, const void* VL, int64_t m, int64_t n,
                          const int64_t* support, const int64_t* row_ptr, int64_t nnz,
                          int64_t* s_idx, void* s_val, void* s_x, SelPlan* plan,
                          double* scratch);
int64_t fixed_support_scratch_doubles();

// ---- GreBsmo (k_grebsmo.hip) ----
// Blocks of the soft pass (= partial triples it writes).
int64_t gb_soft_blocks(int64_t m, int64_t n);
// Soft-thresholding pass of Eq. 12 with L = U V (U m x RP, Vt = V^T ldd x RP
// panels): D <- X - S, optionally R <- X - U V - S (padded layout, ld ldd),
// stats[0..2] <- sum e^2, sum |s|, nnz(S) (deterministic order, through part;
// both null: no statistics).
void gb_soft(const Launch& L, bool f64, int rp, const void* X, int64_t ldx, const void* U,
             const void* Vt, int64_t m, int64_t n, double lam, void* D, int64_t ldd, void* R,
             double* part, double* stats);
// The same S written densely to S (ld lds).
void gb_soft_s(const Launch& L, bool f64, int rp, const void* X, int64_t ldx, const void* U,
               const void* Vt, int64_t m, int64_t n, double lam, void* S, int64_t lds);
// V^T = sum of the row-chunk partials Zpart (nch x ldd x 32) into Vt
// (ldd x rp) and into rows j < rp of Zt (32 x ldd).
void gb_reduce_zt(const Launch& L, const float* Zpart, int64_t nch, int64_t ldd, int rp,
                  float* Vt, float* Zt);
// Vt[:, c0 + c] <- P[:, c], c < cnt (rows x RP panels).
void gb_put_cols(const Launch& L, bool f64, int rp, const void* P, int64_t rows, int c0,
                 int cnt, void* Vt);


// ---------------------------------------------------------------------------
// MSE training (Sec. 4.2.1, Algorithm 4): one label update and helpers.
// ---------------------------------------------------------------------------
struct MseLabelArgs {
  void* E;                  // n x lde working residual X - sum L - S
  int64_t lde;
  const void* X;            // n x ldx
  int64_t ldx;
  const void* cnt;          // n: labels per sample (type of X)
  const int64_t* rows;      // the label's rows (ascending)
  int64_t nrows;
  int64_t p;
  int S;                    // columns per lane: p <= 64 S, S in {1, 2, 4, 8}
  int first;                // the label still holds its initial value
  int r;                    // the label's rank bound (<= 8)
  int nblk;                 // blocks of the Y2 row pass (one partial each)
  void* U;                  // nrows x 8 (read, then overwritten)
  const void* Vold;         // 64 S x 8 current basis
  void* Vnew;               // 64 S x 8 new basis (output)
  const void* A1;           // 64 S x 8 random matrix of this update
  void* part;               // nblk x 64 S x 8 partials
  double* y2;               // 64 S x 8: Y2 (FP64)
  unsigned int* ctl;        // arrival counter of km_reduce_orth (zero between launches)
};
void launch_mse_label(const Launch& L, bool f64, const MseLabelArgs& a);
void launch_mse_init_e(const Launch& L, bool f64, void* E, int64_t lde, const void* X,
                       int64_t ldx, const void* cnt, int64_t n, int64_t p);
void launch_mse_add_s(const Launch& L, bool f64, void* E, int64_t lde, int64_t p,
                      const int64_t* idx, const void* val, const SelPlan* plan, int64_t kmax);
void launch_mse_copy_factors(const Launch& L, bool f64, const void* U, const void* V,
                             int64_t ni, int64_t p, int r, void* Uo, void* Vo);
void launch_mse_copy_e(const Launch& L, bool f64, const void* E, int64_t lde, int64_t n,
                       int64_t p, void* out, int64_t ldo);

}  // namespace godec
