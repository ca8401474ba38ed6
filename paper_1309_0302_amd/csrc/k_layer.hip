// Kernels of the differentiable GoDec layer (backward pass).
//
// With the supports M_t of the forward frozen, each unrolled iteration is
//   D_t = X - S_{t-1},  L_t = f(D_t),  S_t = M_t * (X - L_t),
// and f, the power-scheme BRP update of Algorithm 1 (Sec. 3.1.3, Eq. 6-9),
// equals exactly
//   f(D) = D A^q Q C^a Q^T,   A = D^T D,  Q = orth(A^p A1),  C = Q^T A^p Q,
//   p = 2q + 1,  a = -(p - 1) / (2p)
// (the range of Q is that of Y2; B = D A^q Q is L~ Q2; C^a = (B^T B)^a gives
// the (2q+1)-th root of the core).  Its adjoint is assembled from thin panel
// products (the batched GEMM below) and r x r FP64 algebra (one thread per
// problem): the eigen-function derivative of C^a (Daleckii-Krein), the
// derivative of an orthonormalised range, and the power-chain terms, each of
// rank r.
#include "godec_internal.h"
#include "k_common.h"

#include <algorithm>

namespace godec {

// ---------------------------------------------------------------------------
// Batched GEMM with optional split over K:
//   C[b] = alpha * op(A[b]) op(B[b]) + beta * C[b],  op(A) M x K, op(B) K x N,
// row-major storage; ta: A is stored K x M (op(A) = A^T); tb: B is stored
// N x K.  With nsplit > 1 the K range is cut into nsplit chunks whose
// products go to part[b][s] and are added in order by kl_gemm_reduce.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void kl_gemm(int M, int N, int K, const T* __restrict__ A,
                                               int64_t lda, int64_t sA, int ta,
                                               const T* __restrict__ B, int64_t ldb,
                                               int64_t sB, int tb, T alpha, T beta,
                                               T* __restrict__ C, int64_t ldc, int64_t sC,
                                               int nsplit, T* __restrict__ part) {
  __shared__ T As[16][17];
  __shared__ T Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int b = blockIdx.z / nsplit, s = blockIdx.z % nsplit;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  const int kc = (K + nsplit - 1) / nsplit;
  const int kb = s * kc;
  const int ke = (kb + kc) < K ? (kb + kc) : K;
  const T* Ab = A + (int64_t)b * sA;
  const T* Bb = B + (int64_t)b * sB;
  T acc = T(0);
  for (int k0 = kb; k0 < ke; k0 += 16) {
    if (!ta) {
      const int i = i0 + ty, k = k0 + tx;
      As[ty][tx] = (i < M && k < ke) ? Ab[(int64_t)i * lda + k] : T(0);
    } else {
      const int i = i0 + tx, k = k0 + ty;
      As[tx][ty] = (i < M && k < ke) ? Ab[(int64_t)k * lda + i] : T(0);
    }
    if (!tb) {
      const int k = k0 + ty, j = j0 + tx;
      Bs[ty][tx] = (k < ke && j < N) ? Bb[(int64_t)k * ldb + j] : T(0);
    } else {
      const int k = k0 + tx, j = j0 + ty;
      Bs[tx][ty] = (k < ke && j < N) ? Bb[(int64_t)j * ldb + k] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) acc += As[ty][kk] * Bs[kk][tx];
    __syncthreads();
  }
  const int i = i0 + ty, j = j0 + tx;
  if (i >= M || j >= N) return;
  if (nsplit > 1) {
    part[(((int64_t)b * nsplit + s) * M + i) * N + j] = acc;
  } else {
    T* Cb = C + (int64_t)b * sC;
    const T old = beta != T(0) ? Cb[(int64_t)i * ldc + j] : T(0);
    Cb[(int64_t)i * ldc + j] = alpha * acc + beta * old;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void kl_gemm_reduce(int M, int N, int nsplit,
                                                      const T* __restrict__ part, T alpha,
                                                      T beta, T* __restrict__ C, int64_t ldc,
                                                      int64_t sC) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  T acc = T(0);
  for (int s = 0; s < nsplit; ++s) acc += part[((int64_t)b * nsplit + s) * M * N + e];
  T* Cb = C + (int64_t)b * sC;
  const T old = beta != T(0) ? Cb[(int64_t)i * ldc + j] : T(0);
  Cb[(int64_t)i * ldc + j] = alpha * acc + beta * old;
}

// ---------------------------------------------------------------------------
// Elementwise and sparse helpers (one problem per blockIdx.y).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void kl_fill(T* __restrict__ P, int64_t count, int64_t stride,
                                               T v) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) P[(int64_t)blockIdx.y * stride + e] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void kl_copy(const T* __restrict__ S, T* __restrict__ D,
                                               int64_t count, int64_t stride) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) D[(int64_t)blockIdx.y * stride + e] = S[(int64_t)blockIdx.y * stride + e];
}

// P[idx[e]] = v[e]  (mode 0),  P[idx[e]] += s * v[e]  (mode 1)  over the list
// of problem b (idx/v with batch stride kstride, counts nnz[b]).
template <typename T>
__global__ __launch_bounds__(256) void kl_scatter(T* __restrict__ P, int64_t stride,
                                                  const int64_t* __restrict__ idx,
                                                  const T* __restrict__ v, int64_t kstride,
                                                  const int64_t* __restrict__ nnz, int mode,
                                                  T s) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nnz[b]) return;
  const int64_t at = idx[(int64_t)b * kstride + e];
  const T x = v[(int64_t)b * kstride + e];
  if (mode == 0) P[(int64_t)b * stride + at] = x;
  else P[(int64_t)b * stride + at] += s * x;
}

// out[e] = G[idx[e]] (gather from a dense matrix)
template <typename T>
__global__ __launch_bounds__(256) void kl_gather(const T* __restrict__ G, int64_t stride,
                                                 const int64_t* __restrict__ idx,
                                                 int64_t kstride,
                                                 const int64_t* __restrict__ nnz,
                                                 T* __restrict__ out) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nnz[b]) return;
  out[(int64_t)b * kstride + e] = G[(int64_t)b * stride + idx[(int64_t)b * kstride + e]];
}

// out[e] = sum_c U[i][c] V[j][c] at the list entries (i, j) = divmod(idx, n)
template <typename T>
__global__ __launch_bounds__(256) void kl_lowrank_at(const T* __restrict__ U, int64_t sU,
                                                     const T* __restrict__ V, int64_t sV,
                                                     int w, int64_t n,
                                                     const int64_t* __restrict__ idx,
                                                     int64_t kstride,
                                                     const int64_t* __restrict__ nnz,
                                                     T* __restrict__ out) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nnz[b]) return;
  const int64_t at = idx[(int64_t)b * kstride + e];
  const int64_t i = at / n, j = at % n;
  const T* u = U + (int64_t)b * sU + i * w;
  const T* v = V + (int64_t)b * sV + j * w;
  T s = T(0);
  for (int c = 0; c < w; ++c) s += u[c] * v[c];
  out[(int64_t)b * kstride + e] = s;
}

// Copy a panel (rows x r, ld r) into columns [c0, c0 + r) of a rows x w panel.
template <typename T>
__global__ __launch_bounds__(256) void kl_put_cols(const T* __restrict__ P, int64_t sP, int r,
                                                   T* __restrict__ O, int64_t sO, int w, int c0,
                                                   int64_t rows) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= rows * r) return;
  const int64_t i = e / r;
  const int c = (int)(e % r);
  O[(int64_t)b * sO + i * w + c0 + c] = P[(int64_t)b * sP + e];
}

// Y += X (count entries per problem).
template <typename T>
__global__ __launch_bounds__(256) void kl_axpy(const T* __restrict__ X, T* __restrict__ Y,
                                               int64_t count, int64_t stride) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) Y[(int64_t)blockIdx.y * stride + e] += X[(int64_t)blockIdx.y * stride + e];
}

// A1 (FP64, n x r) -> panel of type T.
template <typename T>
__global__ __launch_bounds__(256) void kl_cast_a1(const double* __restrict__ A1, int64_t sA,
                                                  T* __restrict__ P, int64_t sP, int64_t count) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) P[(int64_t)b * sP + e] = (T)A1[(int64_t)b * sA + e];
}

// ---------------------------------------------------------------------------
// r x r FP64 algebra, one thread per problem (r <= 8).
// ---------------------------------------------------------------------------
constexpr int LR = 8;

// Cholesky QR factor: Gram = R^T R; Rinv (T), and Rcum_out = R Rcum_in (FP64;
// also as T when rout_t is given).  flag set when a pivot is not positive.
template <typename T>
__global__ void ks_chol(int nb, int r, const T* __restrict__ gram, const double* __restrict__ rin,
                        T* __restrict__ rinv, double* __restrict__ rout, T* __restrict__ rout_t,
                        int* __restrict__ flag) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int E = r * r;
  double G[LR][LR], R[LR][LR], Ri[LR][LR];
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      G[i][j] = 0.5 * ((double)gram[b * E + i * r + j] + (double)gram[b * E + j * r + i]);
      R[i][j] = 0.0;
      Ri[i][j] = 0.0;
    }
  for (int j = 0; j < r; ++j) {
    double d = G[j][j];
    for (int l = 0; l < j; ++l) d -= R[l][j] * R[l][j];
    if (!(d > 0.0)) { atomicOr(flag, 1); d = 1e-300; }
    R[j][j] = sqrt(d);
    for (int c = j + 1; c < r; ++c) {
      double s = G[j][c];
      for (int l = 0; l < j; ++l) s -= R[l][j] * R[l][c];
      R[j][c] = s / R[j][j];
    }
  }
  // upper-triangular inverse
  for (int j = r - 1; j >= 0; --j) {
    Ri[j][j] = 1.0 / R[j][j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= j; ++l) s += R[i][l] * Ri[l][j];
      Ri[i][j] = -s / R[i][i];
    }
  }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      rinv[b * E + i * r + j] = (T)Ri[i][j];
      double s = 0.0;
      for (int l = 0; l < r; ++l) s += R[i][l] * rin[b * E + l * r + j];
      rout[b * E + i * r + j] = s;
      if (rout_t) rout_t[b * E + i * r + j] = (T)s;
    }
}

__device__ void jacobi_sym(double (&A)[LR][LR], double (&V)[LR][LR], int r) {
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < r; ++i) {
      dia += A[i][i] * A[i][i];
      for (int j = i + 1; j < r; ++j) off += A[i][j] * A[i][j];
    }
    if (off <= 1e-32 * dia) break;
    for (int p = 0; p < r; ++p)
      for (int q = p + 1; q < r; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < r; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < r; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < r; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
}

// C = V diag(lam) V^T:  C^a (T), and the Daleckii-Krein weights
// F_ij = (lam_i^a - lam_j^a) / (lam_i - lam_j)  (a lam^(a-1) when equal).
template <typename T>
__global__ void ks_eig(int nb, int r, const T* __restrict__ cmat, double a,
                       T* __restrict__ calpha, double* __restrict__ vout,
                       double* __restrict__ fout, int* __restrict__ flag) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int E = r * r;
  double A[LR][LR], V[LR][LR];
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j)
      A[i][j] = 0.5 * ((double)cmat[b * E + i * r + j] + (double)cmat[b * E + j * r + i]);
  jacobi_sym(A, V, r);
  double lam[LR], la[LR];
  for (int i = 0; i < r; ++i) {
    lam[i] = A[i][i];
    if (!(lam[i] > 0.0)) { atomicOr(flag, 2); lam[i] = 1e-300; }
    la[i] = pow(lam[i], a);
  }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int l = 0; l < r; ++l) s += V[i][l] * la[l] * V[j][l];
      calpha[b * E + i * r + j] = (T)s;
      vout[b * E + i * r + j] = V[i][j];
      const double d = lam[i] - lam[j];
      fout[b * E + i * r + j] =
          fabs(d) > 1e-12 * fmax(lam[i], lam[j]) ? (la[i] - la[j]) / d
                                                  : a * pow(0.5 * (lam[i] + lam[j]), a - 1.0);
    }
}

// S2 = 2 Cbar with Cbar = V (F o (V^T sym(Cbar_a) V)) V^T  (Daleckii-Krein).
template <typename T>
__global__ void ks_dk(int nb, int r, const T* __restrict__ cbar_a, const double* __restrict__ vin,
                      const double* __restrict__ fin, T* __restrict__ s2) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int E = r * r;
  double S[LR][LR], V[LR][LR], M[LR][LR], N[LR][LR];
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      S[i][j] = 0.5 * ((double)cbar_a[b * E + i * r + j] + (double)cbar_a[b * E + j * r + i]);
      V[i][j] = vin[b * E + i * r + j];
    }
  for (int i = 0; i < r; ++i)           // M = V^T S V
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int k = 0; k < r; ++k)
        for (int l = 0; l < r; ++l) s += V[k][i] * S[k][l] * V[l][j];
      M[i][j] = s * fin[b * E + i * r + j];
    }
  for (int i = 0; i < r; ++i)           // N = V M V^T
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int k = 0; k < r; ++k)
        for (int l = 0; l < r; ++l) s += V[i][k] * M[k][l] * V[j][l];
      N[i][j] = s;
    }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) s2[b * E + i * r + j] = (T)(N[i][j] + N[j][i]);
}

// out = Rc Rtot^{-1} for upper-triangular FP64 Rc, Rtot (T output).  Both
// are accumulated products of Cholesky factors, so their ratio stays well
// scaled where each alone grows with powers of the spectrum.
template <typename T>
__global__ void ks_rrel(int nb, int r, const double* __restrict__ rc,
                        const double* __restrict__ rtot, T* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int E = r * r;
  double R[LR][LR], Ri[LR][LR];
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) { R[i][j] = rtot[b * E + i * r + j]; Ri[i][j] = 0.0; }
  for (int j = r - 1; j >= 0; --j) {
    Ri[j][j] = 1.0 / R[j][j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= j; ++l) s += R[i][l] * Ri[l][j];
      Ri[i][j] = -s / R[i][i];
    }
  }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int l = 0; l < r; ++l) s += rc[b * E + i * r + l] * Ri[l][j];
      out[b * E + i * r + j] = (T)s;
    }
}

__global__ void ks_identity(int nb, int r, double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) out[b * r * r + i * r + j] = i == j ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// Tall-skinny products (the panel passes of the backward).
//
// kl_ts_nn: C[b] = alpha A[b] B[b] + beta C[b] with A M x K (row-major, one
// thread per row) and B K x NC (NC <= 8, K <= kTsMaxK) staged in LDS.
// kl_ts_tn: the K-chunk partials of A[b]^T B[b] with A stored K x M (one
// thread per column of A, rows of the chunk read coalesced) and B K x NC;
// kl_ts_reduce adds the chunks in order.
// ---------------------------------------------------------------------------
constexpr int kTsMaxK = 512;
constexpr int kTsChunk = 256;

template <typename T, int NC>
__global__ __launch_bounds__(256) void kl_ts_nn(int M, int K, const T* __restrict__ A,
                                                int64_t lda, int64_t sA, const T* __restrict__ B,
                                                int64_t sB, T alpha, T beta, T* __restrict__ C,
                                                int64_t ldc, int64_t sC) {
  __shared__ T bs[kTsMaxK * NC];
  const int b = blockIdx.y, tid = threadIdx.x;
  const T* Bb = B + (int64_t)b * sB;
  for (int e = tid; e < K * NC; e += 256) bs[e] = Bb[e];
  __syncthreads();
  const int i = blockIdx.x * 256 + tid;
  if (i >= M) return;
  const T* a = A + (int64_t)b * sA + (int64_t)i * lda;
  T acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = T(0);
  for (int k = 0; k < K; ++k) {
    const T x = a[k];
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j] += x * bs[k * NC + j];
  }
  T* c = C + (int64_t)b * sC + (int64_t)i * ldc;
#pragma unroll
  for (int j = 0; j < NC; ++j) c[j] = alpha * acc[j] + (beta != T(0) ? beta * c[j] : T(0));
}

template <typename T, int NC>
__global__ __launch_bounds__(256) void kl_ts_tn(int M, int K, const T* __restrict__ A,
                                                int64_t lda, int64_t sA, const T* __restrict__ B,
                                                int64_t sB, T* __restrict__ part) {
  __shared__ T bs[kTsChunk * NC];
  const int b = blockIdx.z, ch = blockIdx.y, tid = threadIdx.x;
  const int k0 = ch * kTsChunk;
  const int kn = (K - k0) < kTsChunk ? (K - k0) : kTsChunk;
  const T* Bb = B + (int64_t)b * sB + (int64_t)k0 * NC;
  for (int e = tid; e < kn * NC; e += 256) bs[e] = Bb[e];
  __syncthreads();
  const int c = blockIdx.x * 256 + tid;
  if (c >= M) return;
  const T* a = A + (int64_t)b * sA + (int64_t)k0 * lda + c;
  T acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = T(0);
  for (int k = 0; k < kn; ++k) {
    const T x = a[(int64_t)k * lda];
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j] += x * bs[k * NC + j];
  }
  T* o = part + (((int64_t)b * gridDim.y + ch) * M + c) * NC;
#pragma unroll
  for (int j = 0; j < NC; ++j) o[j] = acc[j];
}

template <typename T>
__global__ __launch_bounds__(256) void kl_ts_reduce(int M, int NC, int nch,
                                                    const T* __restrict__ part, T alpha, T beta,
                                                    T* __restrict__ C, int64_t ldc, int64_t sC) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * NC) return;
  T s = T(0);
  for (int ch = 0; ch < nch; ++ch) s += part[((int64_t)b * nch + ch) * M * NC + e];
  const int64_t i = e / NC, j = e % NC;
  T* c = C + (int64_t)b * sC + i * ldc + j;
  *c = alpha * s + (beta != T(0) ? beta * *c : T(0));
}

#define GODEC_NC_SWITCH(nc, ...)                              \
  switch (nc) {                                               \
    case 1: { constexpr int NC = 1; __VA_ARGS__; } break;     \
    case 2: { constexpr int NC = 2; __VA_ARGS__; } break;     \
    case 3: { constexpr int NC = 3; __VA_ARGS__; } break;     \
    case 4: { constexpr int NC = 4; __VA_ARGS__; } break;     \
    case 5: { constexpr int NC = 5; __VA_ARGS__; } break;     \
    case 6: { constexpr int NC = 6; __VA_ARGS__; } break;     \
    case 7: { constexpr int NC = 7; __VA_ARGS__; } break;     \
    case 8: { constexpr int NC = 8; __VA_ARGS__; } break;     \
    default: break;                                           \
  }

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
template <typename T>
void lk_gemm_t(const Launch& L, int nb, int M, int N, int K, const T* A, int64_t lda,
               int64_t sA, int ta, const T* B, int64_t ldb, int64_t sB, int tb, T alpha, T beta,
               T* C, int64_t ldc, int64_t sC, T* part, int64_t part_cap) {
  // tall-skinny cases: a long panel times a small N-column one
  if (!ta && !tb && N <= 8 && K <= kTsMaxK && ldb == N && M >= 256) {
    const dim3 grid((unsigned)((M + 255) / 256), (unsigned)nb);
    GODEC_NC_SWITCH(N, hipLaunchKernelGGL((kl_ts_nn<T, NC>), grid, dim3(256), 0, L.stream, M, K,
                                          A, lda, sA, B, sB, alpha, beta, C, ldc, sC));
    return;
  }
  const int nch_ts = (K + kTsChunk - 1) / kTsChunk;
  if (ta && !tb && N <= 8 && ldb == N && M >= 64 && (int64_t)nb * nch_ts * M * N <= part_cap) {
    const dim3 grid((unsigned)((M + 255) / 256), (unsigned)nch_ts, (unsigned)nb);
    GODEC_NC_SWITCH(N, hipLaunchKernelGGL((kl_ts_tn<T, NC>), grid, dim3(256), 0, L.stream, M, K,
                                          A, lda, sA, B, sB, part));
    const dim3 g2((unsigned)(((int64_t)M * N + 255) / 256), (unsigned)nb);
    hipLaunchKernelGGL(kl_ts_reduce<T>, g2, dim3(256), 0, L.stream, M, N, nch_ts, (const T*)part,
                       alpha, beta, C, ldc, sC);
    return;
  }
  const int tiles = ((M + 15) / 16) * ((N + 15) / 16) * nb;
  int nsplit = 1;
  if (tiles < 1024 && K > 512) {
    nsplit = std::min(64, (K + 511) / 512);
    while (nsplit > 1 && (int64_t)nb * nsplit * M * N > part_cap) --nsplit;
  }
  dim3 grid((unsigned)((N + 15) / 16), (unsigned)((M + 15) / 16), (unsigned)(nb * nsplit));
  hipLaunchKernelGGL(kl_gemm<T>, grid, dim3(256), 0, L.stream, M, N, K, A, lda, sA, ta, B, ldb,
                     sB, tb, alpha, beta, C, ldc, sC, nsplit, part);
  if (nsplit > 1) {
    dim3 g2((unsigned)(((int64_t)M * N + 255) / 256), (unsigned)nb);
    hipLaunchKernelGGL(kl_gemm_reduce<T>, g2, dim3(256), 0, L.stream, M, N, nsplit,
                       (const T*)part, alpha, beta, C, ldc, sC);
  }
}

void lk_gemm(const Launch& L, bool f64, int nb, int M, int N, int K, const void* A, int64_t lda,
             int64_t sA, int ta, const void* B, int64_t ldb, int64_t sB, int tb, double alpha,
             double beta, void* C, int64_t ldc, int64_t sC, void* part, int64_t part_cap) {
  if (f64)
    lk_gemm_t<double>(L, nb, M, N, K, (const double*)A, lda, sA, ta, (const double*)B, ldb, sB,
                      tb, alpha, beta, (double*)C, ldc, sC, (double*)part, part_cap);
  else
    lk_gemm_t<float>(L, nb, M, N, K, (const float*)A, lda, sA, ta, (const float*)B, ldb, sB, tb,
                     (float)alpha, (float)beta, (float*)C, ldc, sC, (float*)part, part_cap);
}

static dim3 g1(int64_t count, int nb) { return dim3((unsigned)((count + 255) / 256), (unsigned)nb); }

void lk_fill(const Launch& L, bool f64, int nb, void* P, int64_t count, int64_t stride, double v) {
  if (f64) hipLaunchKernelGGL(kl_fill<double>, g1(count, nb), dim3(256), 0, L.stream, (double*)P, count, stride, v);
  else hipLaunchKernelGGL(kl_fill<float>, g1(count, nb), dim3(256), 0, L.stream, (float*)P, count, stride, (float)v);
}

void lk_copy(const Launch& L, bool f64, int nb, const void* S, void* D, int64_t count, int64_t stride) {
  if (f64) hipLaunchKernelGGL(kl_copy<double>, g1(count, nb), dim3(256), 0, L.stream, (const double*)S, (double*)D, count, stride);
  else hipLaunchKernelGGL(kl_copy<float>, g1(count, nb), dim3(256), 0, L.stream, (const float*)S, (float*)D, count, stride);
}

void lk_axpy(const Launch& L, bool f64, int nb, const void* X, void* Y, int64_t count, int64_t stride) {
  if (f64) hipLaunchKernelGGL(kl_axpy<double>, g1(count, nb), dim3(256), 0, L.stream, (const double*)X, (double*)Y, count, stride);
  else hipLaunchKernelGGL(kl_axpy<float>, g1(count, nb), dim3(256), 0, L.stream, (const float*)X, (float*)Y, count, stride);
}

void lk_scatter(const Launch& L, bool f64, int nb, void* P, int64_t stride, const int64_t* idx,
                const void* v, int64_t kstride, int64_t kmax, const int64_t* nnz, int mode,
                double s) {
  if (f64)
    hipLaunchKernelGGL(kl_scatter<double>, g1(kmax, nb), dim3(256), 0, L.stream, (double*)P, stride, idx,
                       (const double*)v, kstride, nnz, mode, s);
  else
    hipLaunchKernelGGL(kl_scatter<float>, g1(kmax, nb), dim3(256), 0, L.stream, (float*)P, stride, idx,
                       (const float*)v, kstride, nnz, mode, (float)s);
}

void lk_gather(const Launch& L, bool f64, int nb, const void* G, int64_t stride, const int64_t* idx,
               int64_t kstride, int64_t kmax, const int64_t* nnz, void* out) {
  if (f64)
    hipLaunchKernelGGL(kl_gather<double>, g1(kmax, nb), dim3(256), 0, L.stream, (const double*)G, stride,
                       idx, kstride, nnz, (double*)out);
  else
    hipLaunchKernelGGL(kl_gather<float>, g1(kmax, nb), dim3(256), 0, L.stream, (const float*)G, stride,
                       idx, kstride, nnz, (float*)out);
}

void lk_lowrank_at(const Launch& L, bool f64, int nb, const void* U, int64_t sU, const void* V,
                   int64_t sV, int w, int64_t n, const int64_t* idx, int64_t kstride, int64_t kmax,
                   const int64_t* nnz, void* out) {
  if (f64)
    hipLaunchKernelGGL(kl_lowrank_at<double>, g1(kmax, nb), dim3(256), 0, L.stream, (const double*)U, sU,
                       (const double*)V, sV, w, n, idx, kstride, nnz, (double*)out);
  else
    hipLaunchKernelGGL(kl_lowrank_at<float>, g1(kmax, nb), dim3(256), 0, L.stream, (const float*)U, sU,
                       (const float*)V, sV, w, n, idx, kstride, nnz, (float*)out);
}

void lk_put_cols(const Launch& L, bool f64, int nb, const void* P, int64_t sP, int r, void* O,
                 int64_t sO, int w, int c0, int64_t rows) {
  if (f64)
    hipLaunchKernelGGL(kl_put_cols<double>, g1(rows * r, nb), dim3(256), 0, L.stream, (const double*)P, sP,
                       r, (double*)O, sO, w, c0, rows);
  else
    hipLaunchKernelGGL(kl_put_cols<float>, g1(rows * r, nb), dim3(256), 0, L.stream, (const float*)P, sP,
                       r, (float*)O, sO, w, c0, rows);
}

void lk_cast_a1(const Launch& L, bool f64, int nb, const double* A1, int64_t sA, void* P,
                int64_t sP, int64_t count) {
  if (f64)
    hipLaunchKernelGGL(kl_cast_a1<double>, g1(count, nb), dim3(256), 0, L.stream, A1, sA, (double*)P, sP, count);
  else
    hipLaunchKernelGGL(kl_cast_a1<float>, g1(count, nb), dim3(256), 0, L.stream, A1, sA, (float*)P, sP, count);
}

void lk_chol(const Launch& L, bool f64, int nb, int r, const void* gram, const double* rin,
             void* rinv, double* rout, void* rout_t, int* flag) {
  const unsigned g = (unsigned)((nb + 63) / 64);
  if (f64)
    hipLaunchKernelGGL(ks_chol<double>, dim3(g), dim3(64), 0, L.stream, nb, r, (const double*)gram, rin,
                       (double*)rinv, rout, (double*)rout_t, flag);
  else
    hipLaunchKernelGGL(ks_chol<float>, dim3(g), dim3(64), 0, L.stream, nb, r, (const float*)gram, rin,
                       (float*)rinv, rout, (float*)rout_t, flag);
}

void lk_eig(const Launch& L, bool f64, int nb, int r, const void* c, double a, void* calpha,
            double* v, double* f, int* flag) {
  const unsigned g = (unsigned)((nb + 63) / 64);
  if (f64)
    hipLaunchKernelGGL(ks_eig<double>, dim3(g), dim3(64), 0, L.stream, nb, r, (const double*)c, a,
                       (double*)calpha, v, f, flag);
  else
    hipLaunchKernelGGL(ks_eig<float>, dim3(g), dim3(64), 0, L.stream, nb, r, (const float*)c, a,
                       (float*)calpha, v, f, flag);
}

void lk_dk(const Launch& L, bool f64, int nb, int r, const void* cbar_a, const double* v,
           const double* f, void* s2) {
  const unsigned g = (unsigned)((nb + 63) / 64);
  if (f64)
    hipLaunchKernelGGL(ks_dk<double>, dim3(g), dim3(64), 0, L.stream, nb, r, (const double*)cbar_a, v, f,
                       (double*)s2);
  else
    hipLaunchKernelGGL(ks_dk<float>, dim3(g), dim3(64), 0, L.stream, nb, r, (const float*)cbar_a, v, f,
                       (float*)s2);
}

void lk_rrel(const Launch& L, bool f64, int nb, int r, const double* rc, const double* rtot,
             void* out) {
  const unsigned g = (unsigned)((nb + 63) / 64);
  if (f64)
    hipLaunchKernelGGL(ks_rrel<double>, dim3(g), dim3(64), 0, L.stream, nb, r, rc, rtot, (double*)out);
  else
    hipLaunchKernelGGL(ks_rrel<float>, dim3(g), dim3(64), 0, L.stream, nb, r, rc, rtot, (float*)out);
}

void lk_identity(const Launch& L, int nb, int r, double* out) {
  hipLaunchKernelGGL(ks_identity, dim3((unsigned)((nb + 63) / 64)), dim3(64), 0, L.stream, nb, r, out);
}

}  // namespace godec
