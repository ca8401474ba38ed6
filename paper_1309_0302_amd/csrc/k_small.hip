// r x r FP64 work of the low-rank step (one workgroup each).
//
// Paper background (Sec. 3.1.2, Eq. 6-9; Algorithm 1): the power-scheme BRP
// needs the QR factors of Y2 = L~^T Y1 and Y1 = L~ Y2, the inverse of the
// r x r matrix A2^T Y1, a rank check on it, and the (2q+1)-th root of the
// r x r core.  With A2 = Y1 these are, exactly:
//   Y2 = (D^T D)^p A1 = Q2 R2        (R2 tracked through the passes below),
//   A2^T Y1 = R2^T R2                (rank check on the singular values of R2),
//   core = R factor of B = L~ Q2     (so L = U_B S_B^{1/p} V_B^T Q2^T).
// The power chain orthonormalises every pass (Cholesky QR with an FP64
// Gram) and keeps the product of the R factors in FP64, rescaled by exact
// powers of two.  B is handled through K = V diag(s^{(1-p)/p}) V^T from
// the eigen-decomposition of B^T B, so that U_L = B K and V_L = Q2.
#include "godec_internal.h"
#include "k_common.h"
#include "k_mmb.h"

namespace godec {

constexpr int kSmallThreads = 384;   // the core: one thread per Jacobi item of a round (r = 20: 300)

// Sum of entry e over nparts partial matrices of `stride` doubles, with
// independent accumulators so the loads overlap.
__device__ __forceinline__ double sum_parts(const double* __restrict__ P, int nparts, int stride,
                                            int e) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int b = 0;
  for (; b + 3 < nparts; b += 4) {
    a0 += P[(int64_t)(b + 0) * stride + e];
    a1 += P[(int64_t)(b + 1) * stride + e];
    a2 += P[(int64_t)(b + 2) * stride + e];
    a3 += P[(int64_t)(b + 3) * stride + e];
  }
  for (; b < nparts; ++b) a0 += P[(int64_t)b * stride + e];
  return (a0 + a1) + (a2 + a3);
}

// ---------------------------------------------------------------------------
// Gram of a panel and the Cholesky step of Cholesky QR.
//
// Block b sums P[i]^T P[i] over its kGramRows-row slice into partial b (each
// thread owns a 2 x 2 tile of G; the rows are split over NG thread groups
// when the tiles do not fill the block).  The last block of each group of
// kGramGroup blocks adds the group's partials, and the last group leader
// adds the group sums: a fixed order, so G is the same bits on every run.
// Every load of a reduction level is issued at once, so a level costs one
// memory round trip.
//
// Cholesky (one wavefront of the final block, lane j holds column j of G in
// registers, broadcasts by readlane): G = R^T R, upper R.  A column is
// inactive when it lies at or past r_eff, is zero, or is numerically
// dependent on the columns before it: its pivot (the squared norm of its
// component orthogonal to them) is at most tau * G_jj with
// tau = RP * max(u^2, 2^-53), the resolution of a Gram of panel-type data
// accumulated in FP64.  An inactive column gets a zero row in R and
// dinv = 0, so the orthonormalised panel has a zero column, which stays zero
// in every later product.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lane_bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Global inputs of wave_chol (the active width and, lane j, column j of the
// accumulated factor), loaded ahead so that their latency overlaps other work.
template <int RP> struct CholIn {
  int reff;
  double b[RP];
};
template <int RP>
__device__ __forceinline__ void chol_prefetch(CholIn<RP>& in, const SmallState* st,
                                              const double* acc, int reset_acc) {
  const int lane = threadIdx.x & 63;
  in.reff = st->r_eff;
#pragma unroll
  for (int l = 0; l < RP; ++l)
    in.b[l] = (acc != nullptr && !reset_acc && lane < RP) ? acc[l * RP + lane] : 0.0;
}

// One wavefront (lanes 0..63); G is RP x RP row-major in LDS, and is
// overwritten with R (LDS scratch for the broadcast reads of R below).
template <typename TA, int RP>
__device__ void wave_chol(double* G, SmallState* st, double* acc, int reset_acc,
                          int normalise, const CholIn<RP>& in) {
  const int lane = threadIdx.x & 63;
  const bool col = lane < RP;
  const int reff = in.reff;
  double g[RP];
#pragma unroll
  for (int i = 0; i < RP; ++i) g[i] = col ? G[i * RP + lane] : 0.0;
  const double g0 = col ? G[lane * RP + lane] : 0.0;
  const double u = sizeof(TA) == 8 ? 0x1p-53 : 0x1p-24;
  const double tau = (double)RP * fmax(u * u, 0x1p-53);
  int act = (col && lane < reff && g0 > 0.0) ? 1 : 0;
  double rcol[RP];   // rcol[k] = R[k][lane]
  double rdiag = 0.0;
#pragma unroll
  for (int k = 0; k < RP; ++k) {
    const double piv = lane_bcast(g[k], k);
    const double g0k = lane_bcast(g0, k);
    const int actk = __builtin_amdgcn_readlane(act, k) && piv > tau * g0k;
    if (lane == k) act = actk;
    if (actk) {
      const double inv = rsqrt_nr(piv);
      const double rkk = piv * inv;
      const double rkj = lane > k ? g[k] * inv : (lane == k ? rkk : 0.0);
      if (lane == k) rdiag = rkk;
      rcol[k] = rkj;
#pragma unroll
      for (int i = k + 1; i < RP; ++i) g[i] -= lane_bcast(rkj, i) * rkj;
    } else {
      rcol[k] = 0.0;
    }
  }
  if (col) {
#pragma unroll
    for (int k = 0; k < RP; ++k) st->Rq[k * RP + lane] = rcol[k];
    st->dinv[lane] = act ? 1.0 / rdiag : 0.0;
  }
  if (acc == nullptr) return;
  // acc <- R acc (or R); lane j owns column j
  double a[RP];
  if (reset_acc) {
#pragma unroll
    for (int i = 0; i < RP; ++i) a[i] = rcol[i];
  } else {
    // R through LDS (G is no longer needed): every lane reads R[i][l] at the
    // same address, a broadcast, instead of a readlane pair per term
    __builtin_amdgcn_wave_barrier();
    if (col) {
#pragma unroll
      for (int i = 0; i < RP; ++i) G[i * RP + lane] = rcol[i];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < RP; ++i) {
      double s = 0.0;
#pragma unroll
      for (int l = i; l < RP; ++l) s += G[i * RP + l] * in.b[l];
      a[i] = s;
    }
  }
  // R2 only enters through ratios of its singular values, so it may be
  // rescaled by a power of two; T must keep its scale (B = B' T).
  if (normalise) {
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < RP; ++i) mx = fmax(mx, fabs(a[i]));
    mx = wave_max(mx);
    int e = 0;
    if (mx > 0.0 && isfinite(mx)) frexp(mx, &e);
    const double sc = ldexp(1.0, -e);
#pragma unroll
    for (int i = 0; i < RP; ++i) a[i] *= sc;
  }
  if (col) {
#pragma unroll
    for (int i = 0; i < RP; ++i) acc[i * RP + lane] = a[i];
  }
}

template <typename TA, int RP>
__device__ void wave_chol(double* G, SmallState* st, double* acc, int reset_acc,
                          int normalise) {
  CholIn<RP> in;
  chol_prefetch<RP>(in, st, acc, reset_acc);
  wave_chol<TA, RP>(G, st, acc, reset_acc, normalise, in);
}

// With Zpart (FP32 panels only), the panel is first formed here: row i,
// column c of P is the sum over h < nch of Zpart[(h rows + i) 32 + c] in
// ascending h (the row-chunk partials of a matrix-core Gram pass), and is
// also stored to P.

template <typename TA, int RP>
__global__ __launch_bounds__(256) void k_gram_tree(const TA* __restrict__ P, int64_t rows,
                                                   double* __restrict__ Gpart,
                                                   GramCtl* __restrict__ ctl, int chol,
                                                   SmallState* st, double* acc, int reset_acc,
                                                   int normalise,
                                                   const float* __restrict__ Zpart, int nch) {
  constexpr int RH = (RP + 1) / 2;    // tiles per side
  constexpr int RW = 2 * RH;          // padded width
  constexpr int NT = RH * RH;         // tiles
  constexpr int NG = 256 / NT;        // row groups
  constexpr int CH = kGramRows;
  constexpr int E = RP * RP;
  __shared__ double ps[CH * RW];
  __shared__ double red[NG * NT * 4];
  __shared__ int flag;
  const int tid = threadIdx.x;
  const int tile = tid % NT, grp = tid / NT;
  const bool active = grp < NG;
  const int ta = 2 * (tile / RH), tb = 2 * (tile % RH);
  // ---- partial of this block's rows ----
  double a00 = 0.0, a01 = 0.0, a10 = 0.0, a11 = 0.0;
  const int64_t per = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = (r0 + per) < rows ? (r0 + per) : rows;
  for (int64_t i0 = r0; i0 < r1; i0 += CH) {
    const int nr = (r1 - i0) < CH ? (int)(r1 - i0) : CH;
    __syncthreads();
    if (Zpart != nullptr) {
      // every entry of the thread and every chunk partial in flight at once;
      // the partials are added in ascending chunk order
      constexpr int PER = (CH * RW + 255) / 256;
      float z[PER];
      bool ok[PER];
      int64_t off[PER];
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int e = tid + 256 * j;
        const int row = e / RW, c = e % RW;
        ok[j] = e < CH * RW && row < nr && c < RP;
        off[j] = ok[j] ? (i0 + row) * zpart_stride(RP) + c : 0;
        z[j] = 0.f;
      }
      const int64_t hstride = rows * zpart_stride(RP);
      float v[kGramMaxChunks][PER];
#pragma unroll
      for (int h = 0; h < kGramMaxChunks; ++h)
#pragma unroll
        for (int j = 0; j < PER; ++j)
          v[h][j] = (h < nch && ok[j]) ? Zpart[h * hstride + off[j]] : 0.f;
#pragma unroll
      for (int h = 0; h < kGramMaxChunks; ++h)
#pragma unroll
        for (int j = 0; j < PER; ++j)
          if (h < nch) z[j] += v[h][j];
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int e = tid + 256 * j;
        if (e < CH * RW) {
          const int row = e / RW, c = e % RW;
          if (ok[j]) const_cast<TA*>(P)[(i0 + row) * RP + c] = (TA)z[j];
          ps[e] = ok[j] ? (double)z[j] : 0.0;
        }
      }
    } else {
      for (int e = tid; e < CH * RW; e += 256) {
        const int row = e / RW, c = e % RW;
        ps[e] = (row < nr && c < RP) ? (double)P[(i0 + row) * RP + c] : 0.0;
      }
    }
    __syncthreads();
    if (active) {
      for (int ii = grp; ii < nr; ii += NG) {
        const double x0 = ps[ii * RW + ta], x1 = ps[ii * RW + ta + 1];
        const double y0 = ps[ii * RW + tb], y1 = ps[ii * RW + tb + 1];
        a00 = fma(x0, y0, a00);
        a01 = fma(x0, y1, a01);
        a10 = fma(x1, y0, a10);
        a11 = fma(x1, y1, a11);
      }
    }
  }
  if (active) {
    double* q = red + (grp * NT + tile) * 4;
    q[0] = a00; q[1] = a01; q[2] = a10; q[3] = a11;
  }
  __syncthreads();
  for (int e = tid; e < E; e += 256) {
    const int a = e / RP, b = e % RP;
    const int t = (a / 2) * RH + b / 2, slot = (a & 1) * 2 + (b & 1);
    double s = 0.0;
    for (int q = 0; q < NG; ++q) s += red[(q * NT + t) * 4 + slot];
    publish(Gpart + (int64_t)blockIdx.x * E + e, s);
  }
  // ---- level 1: the last block of the group adds the group's partials ----
  const int nb = (int)gridDim.x;
  const int gi = (int)blockIdx.x / kGramGroup;
  const int g0 = gi * kGramGroup;
  const int gsz = (nb - g0) < kGramGroup ? (nb - g0) : kGramGroup;
  stores_done();
  __syncthreads();
  if (tid == 0) flag = arrive(&ctl->grp[gi]) == (unsigned int)(gsz - 1);
  __syncthreads();
  if (!flag) return;
  for (int e = tid; e < E; e += 256) {
    double v[kGramGroup];
#pragma unroll
    for (int q = 0; q < kGramGroup; ++q) v[q] = q < gsz ? fetch(Gpart + (int64_t)(g0 + q) * E + e) : 0.0;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kGramGroup; ++q) s += v[q];
    publish(Gpart + (int64_t)(kGramMaxBlocks + gi) * E + e, s);
  }
  // ---- level 2: the last group leader adds the group sums ----
  const int ngr = (nb + kGramGroup - 1) / kGramGroup;
  stores_done();
  __syncthreads();
  if (tid == 0) {
    publish_u32(&ctl->grp[gi], 0u);
    flag = arrive(&ctl->top) == (unsigned int)(ngr - 1);
  }
  __syncthreads();
  if (!flag) return;
  // the Cholesky step's global inputs, in flight during the fetch below
  CholIn<RP> cin;
  if (chol && tid < 64) chol_prefetch<RP>(cin, st, acc, reset_acc);
  double* Gs = ps;   // E <= 1024 doubles fit in ps
  for (int e = tid; e < E; e += 256) {
    double v[kGramMaxBlocks / kGramGroup];
#pragma unroll
    for (int q = 0; q < kGramMaxBlocks / kGramGroup; ++q)
      v[q] = q < ngr ? fetch(Gpart + (int64_t)(kGramMaxBlocks + q) * E + e) : 0.0;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kGramMaxBlocks / kGramGroup; ++q) s += v[q];
    Gs[e] = s;
    Gpart[(int64_t)kGramFinal * E + e] = s;
  }
  if (tid == 0) publish_u32(&ctl->top, 0u);
  if (!chol) return;
  __syncthreads();
  if (tid >= 64) return;
  wave_chol<TA, RP>(Gs, st, acc, reset_acc, normalise, cin);
}

// Rotation threshold of the Jacobi sweeps: an off-diagonal entry below
// 4 u sqrt(|a_pp a_qq|) (u = 2^-53) is already at rounding level.
constexpr double kJacobiTol = 4.0 * 0x1p-53;
// A sweep whose rotations all had |a_pq| <= 2^-34 sqrt(a_pp a_qq) leaves the
// off-diagonal at about the square of that (quadratic convergence of cyclic
// Jacobi), far below kJacobiTol, so the confirming sweep is skipped.
constexpr double kJacobiQuad = 0x1p-34;

// Round-robin pairing (circle method) over N (even) players.
__device__ __forceinline__ void rr_pair(int round, int k, int N, int& a, int& b) {
  auto pos = [&](int i) { return i == 0 ? 0 : 1 + ((i - 1 + round) % (N - 1)); };
  a = pos(k);
  b = pos(N - 1 - k);
}

// Two-sided cyclic Jacobi on the symmetric matrix A (LDS, stride LD),
// accumulating V <- V J.  A is zero outside its leading n x n block and V is
// the identity there, so the sweeps run over the full RP x RP at compile-time
// sizes: a pair that touches the padding has a_pq = 0 and is never rotated.
// Parallel over disjoint pairs in each round: the rotations of a round are
// computed first, then one pass applies them, a thread per 2 x 2 block of A
// (the column rotation of the block's column pair, then the row rotation of
// its row pair) and a thread per (row, pair) of V.  The rotation itself is
// one short FP64 chain (reciprocal square roots refined by Newton steps,
// thresholds compared on squares): the rounds are latency-bound.
template <int RP>
__device__ void jacobi_eig(double* A, double* V, int n, double* cs, int* rot) {
  constexpr int LD = RP + 1;
  constexpr int N = (RP + 1) & ~1;
  constexpr int NP = N / 2;
  constexpr int NBLK = NP * NP;
  __shared__ int pq[2 * NP];
  (void)n;
  auto pos = [](int i, int round) {
    if (i == 0) return 0;
    int x = i - 1 + round;
    if (x >= N - 1) x -= N - 1;
    return 1 + x;
  };
  for (int sweep = 0; sweep < 40; ++sweep) {
    int nrot = 0, nbig = 0;   // wave 0's counts (every pair lives in wave 0)
    for (int round = 0; round < N - 1; ++round) {
      if (threadIdx.x < 64) {
        const int k = threadIdx.x;
        bool did = false, big = false;
        if (k < NP) {
          // circle method: position i plays at 0 (fixed) or 1 + (i - 1 + round) mod (N - 1)
          int p = pos(k, round), q = pos(N - 1 - k, round);
          if (p > q) { const int t = p; p = q; q = t; }
          double c = 1.0, sn = 0.0;
          if (q < RP) {
            const double apq = A[p * LD + q];
            const double app = A[p * LD + p], aqq = A[q * LD + q];
            // |a_pq| > tol sqrt(|a_pp a_qq|), compared on squares
            const double prod = fabs(app * aqq), apq2 = apq * apq;
            if (apq2 > kJacobiTol * kJacobiTol * prod && apq != 0.0) {
              // tan of the rotation t = sgn(d) h / (|d| + r), d = a_qq - a_pp,
              // h = 2 a_pq, r = hypot(d, h); with w = sqrt(2 r (r + |d|)):
              // c = (r + |d|) / w, s = sgn(d) h / w.
              const double d = aqq - app, h = 2.0 * apq;
              const double mx = fmax(fabs(d), fabs(h));
              if (mx > 0x1p-450 && mx < 0x1p450) {
                const double r2 = d * d + h * h;
                const double r = r2 * rsqrt_nr(r2);
                const double iw = rsqrt_nr(2.0 * r * (r + fabs(d)));
                c = (r + fabs(d)) * iw;
                sn = (d >= 0.0 ? h : -h) * iw;
              } else {
                const double th = d / h;
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                c = 1.0 / sqrt(t * t + 1.0);
                sn = t * c;
              }
              did = true;
              big = apq2 > kJacobiQuad * kJacobiQuad * prod;
            }
          }
          cs[2 * k + 0] = c;
          cs[2 * k + 1] = sn;
          pq[2 * k + 0] = p;
          pq[2 * k + 1] = q;
        }
        nrot += __popcll(__ballot(did));
        nbig += __popcll(__ballot(big));
      }
      __syncthreads();
      for (int e = threadIdx.x; e < NBLK + RP * NP; e += blockDim.x) {
        if (e >= NBLK) {
          // V <- V J
          const int f = e - NBLK;
          const int i = f / NP, k = f % NP;
          const double c = cs[2 * k], sn = cs[2 * k + 1];
          const int p = pq[2 * k], q = pq[2 * k + 1];
          if (q >= RP || sn == 0.0) continue;
          const double vip = V[i * LD + p], viq = V[i * LD + q];
          V[i * LD + p] = c * vip - sn * viq;
          V[i * LD + q] = sn * vip + c * viq;
          continue;
        }
        // A <- J^T A J on the block (row pair k1) x (column pair k2)
        const int k1 = e / NP, k2 = e % NP;
        const double c1 = cs[2 * k1], s1 = cs[2 * k1 + 1];
        const double c2 = cs[2 * k2], s2 = cs[2 * k2 + 1];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const int p1 = pq[2 * k1], q1 = pq[2 * k1 + 1];
        const int p2 = pq[2 * k2], q2 = pq[2 * k2 + 1];
        const bool rq = q1 < RP, cq = q2 < RP;   // the partner may be the padding index
        double a = A[p1 * LD + p2];
        double b = cq ? A[p1 * LD + q2] : 0.0;
        double cc = rq ? A[q1 * LD + p2] : 0.0;
        double d = (rq && cq) ? A[q1 * LD + q2] : 0.0;
        if (s2 != 0.0) {
          const double a2 = c2 * a - s2 * b, b2 = s2 * a + c2 * b;
          const double c3 = c2 * cc - s2 * d, d2 = s2 * cc + c2 * d;
          a = a2; b = b2; cc = c3; d = d2;
        }
        if (s1 != 0.0) {
          const double a2 = c1 * a - s1 * cc, c3 = s1 * a + c1 * cc;
          const double b2 = c1 * b - s1 * d, d2 = s1 * b + c1 * d;
          a = a2; cc = c3; b = b2; d = d2;
        }
        A[p1 * LD + p2] = a;
        if (cq) A[p1 * LD + q2] = b;
        if (rq) A[q1 * LD + p2] = cc;
        if (rq && cq) A[q1 * LD + q2] = d;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) rot[0] = (nrot == 0 || nbig == 0) ? 1 : 0;
    __syncthreads();
    if (rot[0]) break;
    __syncthreads();
  }
}

// One-sided (Hestenes) Jacobi: orthogonalise the columns of M (n x n);
// afterwards the column norms are the singular values.
template <int RP>
__device__ void jacobi_svd_values(double* M, int n, double* out, double* cs, int* rot) {
  constexpr int LD = RP + 1;
  const int N = (n + 1) & ~1;
  const int npairs = N / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (threadIdx.x == 0) *rot = 0;
    __syncthreads();
    for (int round = 0; round < N - 1; ++round) {
      if (threadIdx.x < npairs) {
        int p, q;
        rr_pair(round, threadIdx.x, N, p, q);
        double c = 1.0, s = 0.0;
        if (p < n && q < n) {
          double al = 0, be = 0, ga = 0;
          for (int i = 0; i < n; ++i) {
            const double x = M[i * LD + p], y = M[i * LD + q];
            al += x * x; be += y * y; ga += x * y;
          }
          if (ga != 0.0 && fabs(ga) > kJacobiTol * sqrt(al * be)) {
            const double ze = (be - al) / (2.0 * ga);
            const double t = (ze >= 0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
            c = 1.0 / sqrt(1.0 + t * t);
            s = c * t;
            atomicAdd(rot, 1);
          }
        }
        cs[4 * threadIdx.x + 0] = c;
        cs[4 * threadIdx.x + 1] = s;
        cs[4 * threadIdx.x + 2] = (double)p;
        cs[4 * threadIdx.x + 3] = (double)q;
      }
      __syncthreads();
      for (int e = threadIdx.x; e < n * npairs; e += blockDim.x) {
        const int i = e / npairs, k = e % npairs;
        const double c = cs[4 * k], s = cs[4 * k + 1];
        const int p = (int)cs[4 * k + 2], q = (int)cs[4 * k + 3];
        if (p >= n || q >= n || s == 0.0) continue;
        const double x = M[i * LD + p], y = M[i * LD + q];
        M[i * LD + p] = c * x - s * y;
        M[i * LD + q] = s * x + c * y;
      }
      __syncthreads();
    }
    if (*rot == 0) break;
    __syncthreads();
  }
  if (threadIdx.x < n) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += M[i * LD + threadIdx.x] * M[i * LD + threadIdx.x];
    out[threadIdx.x] = sqrt(s);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Core of the low-rank step.  Inputs: Gpart of B' = D Y_q (so B = B' T),
// st->T, st->R2.  Output: K' = T K in the panel type, such that
// U_L = B' K' and L = U_L Q2^T.
// ---------------------------------------------------------------------------
template <typename TA, int RP>
__device__ void core_body(const double* __restrict__ Gpart, int nparts, SmallState* st, int p,
                          double rank_tol, int t_identity, TA* k_panel) {
  constexpr int LD = RP + 1;
  __shared__ double G[RP * LD];
  __shared__ double H[RP * LD];
  __shared__ double T[RP * LD];
  __shared__ double V[RP * LD];
  __shared__ double W[RP * LD];
  __shared__ double cs[4 * 16 + 4];
  __shared__ double ev[RP];
  __shared__ double fk[RP];
  __shared__ double sv[RP];
  __shared__ int order[RP];
  __shared__ int rot[2];
  __shared__ int sh_keep;
  __shared__ double red[4];
  __shared__ double redA[kSmallThreads / 64], redB[kSmallThreads / 64];
  const int tid = threadIdx.x;
  const int n = st->r_eff;             // active leading columns
  for (int e = tid; e < RP * RP; e += blockDim.x) {
    double s = 0.0;
    s = sum_parts(Gpart, nparts, RP * RP, e);
    const int i = e / RP, j = e % RP;
    G[i * LD + j] = s;
    T[i * LD + j] = t_identity ? (i == j ? 1.0 : 0.0) : st->T[e];
    W[i * LD + j] = st->R2[e];
  }
  __syncthreads();

  // ---- rank check on R2 (A2^T Y1 = R2^T R2) ----
  // Certificate first: s_min(R2) >= 1/||R2^{-1}||_F and s_max <= ||R2||_F.
  // R2^{-1} (upper triangular, active block) by back substitution, one lane
  // per column in registers, into H; a zero diagonal fails the certificate.
  if (tid == 0) {
    int ok = n > 0;
    for (int i = 0; i < n; ++i)
      if (!(W[i * LD + i] != 0.0)) ok = 0;
    red[1] = ok;
    sh_keep = n;
  }
  for (int e = tid; e < RP * RP; e += blockDim.x) {
    const int i = e / RP, c = e % RP;
    H[i * LD + c] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid < n) fk[tid] = 1.0 / W[tid * LD + tid];
  __syncthreads();
  if (red[1] != 0.0 && tid < n) {
    // column tid of R2^{-1}: each lane substitutes its own column in registers
    double h[RP];
#pragma unroll
    for (int i = 0; i < RP; ++i) h[i] = (i == tid) ? 1.0 : 0.0;
#pragma unroll
    for (int i = RP - 1; i >= 0; --i) {
      if (i < n) {
        h[i] *= fk[i];
#pragma unroll
        for (int l = 0; l < i; ++l) h[l] -= W[l * LD + i] * h[i];
      }
    }
#pragma unroll
    for (int i = 0; i < RP; ++i) H[i * LD + tid] = h[i];
  }
  __syncthreads();
  {
    double fr = 0.0, fi = 0.0;
    for (int e = tid; e < n * n; e += blockDim.x) {
      const int i = e / n, c = e % n;
      if (c >= i) {
        fr += W[i * LD + c] * W[i * LD + c];
        fi += H[i * LD + c] * H[i * LD + c];
      }
    }
    fr = wave_sum(fr);
    fi = wave_sum(fi);
    __syncthreads();
    if ((tid & 63) == 0) { redA[tid >> 6] = fr; redB[tid >> 6] = fi; }
    __syncthreads();
    if (tid == 0) {
      double a = 0, b = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { a += redA[w]; b += redB[w]; }
      const bool ok = red[1] != 0.0 && isfinite(a) && isfinite(b) && (1.0 / b) > rank_tol * a;
      red[0] = ok ? 1.0 : 0.0;
    }
    __syncthreads();
  }
  if (red[0] == 0.0 && n > 0) {
    jacobi_svd_values<RP>(W, n, sv, cs, rot);
    if (tid == 0) {
      double smax = 0.0;
      for (int i = 0; i < n; ++i) smax = fmax(smax, sv[i]);
      int keep = 0;
      for (int i = 0; i < n; ++i)
        if (smax > 0.0 && sv[i] * sv[i] > rank_tol * smax * smax) ++keep;
      sh_keep = keep;
    }
    __syncthreads();
  }

  // ---- G_B = T^T G' T on the active block ----
  for (int e = tid; e < RP * RP; e += blockDim.x) {
    const int i = e / RP, j = e % RP;
    double s = 0.0;
    for (int l = 0; l <= j; ++l) s += G[i * LD + l] * T[l * LD + j];
    H[i * LD + j] = s;
  }
  __syncthreads();
  for (int e = tid; e < RP * RP; e += blockDim.x) {
    const int i = e / RP, j = e % RP;
    double s = 0.0;
    for (int l = 0; l <= i; ++l) s += T[l * LD + i] * H[l * LD + j];
    W[i * LD + j] = (i < n && j < n) ? s : 0.0;
  }
  __syncthreads();
  // symmetrise and set V (warm start from the previous iteration if valid)
  const int warm = st->v_valid;
  for (int e = tid; e < RP * RP; e += blockDim.x) {
    const int i = e / RP, j = e % RP;
    G[i * LD + j] = 0.5 * (W[i * LD + j] + W[j * LD + i]);
    V[i * LD + j] = warm ? st->V[e] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (warm) {
    // A = V^T G V
    for (int e = tid; e < RP * RP; e += blockDim.x) {
      const int i = e / RP, j = e % RP;
      double s = 0.0;
      for (int l = 0; l < n; ++l) s += G[i * LD + l] * V[l * LD + j];
      H[i * LD + j] = s;
    }
    __syncthreads();
    for (int e = tid; e < RP * RP; e += blockDim.x) {
      const int i = e / RP, j = e % RP;
      double s = 0.0;
      for (int l = 0; l < n; ++l) s += V[l * LD + i] * H[l * LD + j];
      W[i * LD + j] = s;
    }
    __syncthreads();
    for (int e = tid; e < RP * RP; e += blockDim.x) {
      const int i = e / RP, j = e % RP;
      G[i * LD + j] = 0.5 * (W[i * LD + j] + W[j * LD + i]);
    }
    __syncthreads();
  }
  jacobi_eig<RP>(G, V, n, cs, rot);
  // sort eigenvalues descending (rank of each by counting; ties by index)
  if (tid < n) {
    const double mine = G[tid * LD + tid];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double o = G[j * LD + j];
      rank += (o > mine || (o == mine && j < tid)) ? 1 : 0;
    }
    order[rank] = tid;
    ev[rank] = mine;
  }
  __syncthreads();
  const int keep = sh_keep;
  // K = sum_{i < keep, ev_i > 0} v_i ev_i^{(1-p)/(2p)} v_i^T
  const double ex = (1.0 - (double)p) / (2.0 * (double)p);
  if (tid < n) {
    const double lam = ev[tid];
    fk[tid] = (tid < keep && lam > 0.0) ? ((p == 1) ? 1.0 : pow(lam, ex)) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < RP * RP; e += blockDim.x) {
    const int a = e / RP, b = e % RP;
    double s = 0.0;
    if (a < n && b < n) {
      for (int i = 0; i < keep; ++i) {
        if (!(ev[i] > 0.0)) continue;
        s += V[a * LD + order[i]] * fk[i] * V[b * LD + order[i]];
      }
    }
    H[a * LD + b] = s;
  }
  __syncthreads();
  // K' = T K ; store eigenvectors (sorted) for the next warm start
  int bad = 0;
  for (int e = tid; e < RP * RP; e += blockDim.x) {
    const int i = e / RP, j = e % RP;
    double s = 0.0;
    for (int l = i; l < RP; ++l) s += T[i * LD + l] * H[l * LD + j];
    if (!isfinite(s)) bad = 1;
    st->K[e] = s;
    k_panel[e] = (TA)s;
    st->V[e] = (j < n && i < n) ? V[i * LD + order[j]] : (i == j ? 1.0 : 0.0);
  }
  if (bad) atomicOr(&st->flags, 1);
  if (tid < RP) {
    st->sigma[tid] = (tid < n && ev[tid] > 0.0) ? sqrt(ev[tid]) : 0.0;
    st->sv_c[tid] = 0.0;
  }
  if (tid == 0) {
    st->r_keep = keep;
    st->v_valid = (keep == n) ? 1 : 0;
    if (keep < n) {
      st->r_eff = keep;
      atomicOr(&st->flags, 2);
    }
  }
}

template <typename TA, int RP>
__global__ __launch_bounds__(kSmallThreads) void k_core(const double* __restrict__ Gpart,
                                                        int nparts, SmallState* st, int p,
                                                        double rank_tol, int t_identity,
                                                        TA* k_panel) {
  core_body<TA, RP>(Gpart, nparts, st, p, rank_tol, t_identity, k_panel);
}

__global__ void k_small_init(SmallState* st, int r) {
  const int tid = threadIdx.x;
  for (int e = tid; e < kMaxRP * kMaxRP; e += blockDim.x) {
    st->R2[e] = 0.0; st->T[e] = 0.0; st->Rq[e] = 0.0; st->V[e] = 0.0; st->K[e] = 0.0;
  }
  if (tid < kMaxRP) {
    st->sigma[tid] = 0.0; st->sv_c[tid] = 0.0; st->dinv[tid] = 0.0; st->active[tid] = tid < r;
  }
  if (tid == 0) { st->r_eff = r; st->r_keep = r; st->flags = 0; st->v_valid = 0; }
}

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

void launch_gram_tree(const Launch& L, bool f64, int rp, const void* P, int64_t rows,
                      double* Gpart, GramCtl* ctl, int chol, SmallState* st, double* acc,
                      int reset_acc, int normalise, const float* Zpart, int nch) {
  int64_t nb = (rows + kGramRows - 1) / kGramRows;
  if (nb > kGramMaxBlocks) nb = kGramMaxBlocks;
  if (nb < 1) nb = 1;
  GODEC_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((k_gram_tree<double, RP>), dim3((unsigned)nb), dim3(256), 0, L.stream,
                         (const double*)P, rows, Gpart, ctl, chol, st, acc, reset_acc,
                         normalise, nullptr, 0);
    else
      hipLaunchKernelGGL((k_gram_tree<float, RP>), dim3((unsigned)nb), dim3(256), 0, L.stream,
                         (const float*)P, rows, Gpart, ctl, chol, st, acc, reset_acc,
                         normalise, Zpart, nch);
  });
}


void launch_core(const Launch& L, bool f64, int rp, const double* Gpart,
                 int nparts, SmallState* st, int p, double rank_tol,
                 int t_identity, void* k_panel) {
  GODEC_RP_SWITCH(rp, {
    if (f64)
      hipLaunchKernelGGL((k_core<double, RP>), dim3(1), dim3(kSmallThreads), 0, L.stream, Gpart,
                         nparts, st, p, rank_tol, t_identity, (double*)k_panel);
    else
      hipLaunchKernelGGL((k_core<float, RP>), dim3(1), dim3(kSmallThreads), 0, L.stream, Gpart,
                         nparts, st, p, rank_tol, t_identity, (float*)k_panel);
  });
}

void launch_small_init(const Launch& L, SmallState* st, int r) {
  hipLaunchKernelGGL(k_small_init, dim3(1), dim3(256), 0, L.stream, st, r);
}

}  // namespace godec

namespace godec {

// ---------------------------------------------------------------------------
// Batched r x r work: one workgroup per problem, 8-column panels.
// ---------------------------------------------------------------------------
constexpr int RB = kBatchRP;

__device__ __forceinline__ float* bpanel_rw(const BProb& b, int which) {
  return which == 0 ? b.P0 : (which == 1 ? b.P1 : b.VL);
}

// out = orth(Z) by one Cholesky QR step with an FP64 Gram, Z = the sum of the
// problem's Gram-pass partials (fixed order) or panel `in`; R folded into
// R2 (acc 0, rescaled by powers of two) or T (acc 1).
__global__ __launch_bounds__(256) void kb_chol(const BProb* __restrict__ probs,
                                               const BItem* __restrict__ items,
                                               const float* __restrict__ zslots, int from_slots,
                                               int in, int out, int acc_sel, int reset) {
  __shared__ float zs[kBatchMaxN * RB];
  __shared__ double gp[4][RB * RB];
  __shared__ double G[RB * RB];
  __shared__ double rq[RB * RB];
  __shared__ double di[RB];
  const BProb& b = probs[blockIdx.x];
  const int tid = threadIdx.x;
  const int n = (int)b.n;
  const int ne = n * RB;
  if (from_slots) {
    for (int e = tid; e < ne; e += 256) {
      float s = 0.f;
      for (int it = 0; it < b.nitems; ++it) s += zslots[items[b.item0 + it].zoff + e];
      zs[e] = s;
    }
  } else {
    const float* P = bpanel_rw(b, in);
    for (int e = tid; e < ne; e += 256) zs[e] = P[e];
  }
  __syncthreads();
  {
    const int e = tid % (RB * RB), h = tid / (RB * RB);
    const int a = e / RB, c = e % RB;
    double s = 0.0;
    for (int j = h; j < n; j += 4) s = fma((double)zs[j * RB + a], (double)zs[j * RB + c], s);
    gp[h][e] = s;
  }
  __syncthreads();
  if (tid < RB * RB) G[tid] = (gp[0][tid] + gp[1][tid]) + (gp[2][tid] + gp[3][tid]);
  __syncthreads();
  if (tid < 64) {
    double* acc = acc_sel == 0 ? b.st->R2 : b.st->T;
    wave_chol<float, RB>(G, b.st, acc, reset, acc_sel == 0 ? 1 : 0);
  }
  __syncthreads();
  if (tid < RB * RB) rq[tid] = b.st->Rq[tid];
  if (tid < RB) di[tid] = b.st->dinv[tid];
  __syncthreads();
  float* O = bpanel_rw(b, out);
  for (int j = tid; j < n; j += 256) {
    double x[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c) {
      double s = (double)zs[j * RB + c];
#pragma unroll
      for (int l = 0; l < c; ++l) s = fma(-x[l], rq[l * RB + c], s);
      x[c] = s * di[c];
    }
#pragma unroll
    for (int c = 0; c < RB; ++c) O[j * RB + c] = (float)x[c];
  }
}

// Core of the low-rank step per problem: the Gram of B' from the apply
// pass's partials, then the shared FP64 core (rank certificate, Jacobi
// eigen-solver, K' = T K into Kp).
__global__ __launch_bounds__(kSmallThreads) void kb_core(const BProb* __restrict__ probs,
                                                         const double* __restrict__ gslots,
                                                         int p, int t_identity) {
  const BProb& b = probs[blockIdx.x];
  core_body<float, RB>(gslots + (int64_t)b.item0 * RB * RB, b.nitems, b.st, p, b.rank_tol,
                       t_identity, b.Kp);
}

__global__ void kb_small_init(const BProb* __restrict__ probs) {
  const BProb& b = probs[blockIdx.x];
  SmallState* st = b.st;
  const int tid = threadIdx.x;
  for (int e = tid; e < kMaxRP * kMaxRP; e += blockDim.x) {
    st->R2[e] = 0.0; st->T[e] = 0.0; st->Rq[e] = 0.0; st->V[e] = 0.0; st->K[e] = 0.0;
  }
  if (tid < kMaxRP) {
    st->sigma[tid] = 0.0; st->sv_c[tid] = 0.0; st->dinv[tid] = 0.0; st->active[tid] = tid < b.r;
  }
  if (tid == 0) { st->r_eff = b.r; st->r_keep = b.r; st->flags = 0; st->v_valid = 0; }
}

void bl_chol(const Launch& L, const BatchArgs& a, int from_slots, int in, int out, int acc,
             int reset) {
  hipLaunchKernelGGL(kb_chol, dim3((unsigned)a.nprob), dim3(256), 0, L.stream, a.probs, a.items,
                     a.zslots, from_slots, in, out, acc, reset);
}

void bl_core(const Launch& L, const BatchArgs& a, int t_identity) {
  hipLaunchKernelGGL(kb_core, dim3((unsigned)a.nprob), dim3(kSmallThreads), 0, L.stream, a.probs,
                     a.gslots, a.p, t_identity);
}

void bl_small_init(const Launch& L, const BatchArgs& a) {
  hipLaunchKernelGGL(kb_small_init, dim3((unsigned)a.nprob), dim3(256), 0, L.stream, a.probs);
}

}  // namespace godec
