// Fused steps of the differentiable layer's backward, one block of 256
// threads per problem: each kernel forms an r x r inner product of thin
// panels, applies the FP64 r x r algebra of that step on one thread, and
// applies the result to the panel rows, so that a step of the recomputed
// forward or of the adjoint costs one launch instead of three to five.
//
// Inner products: each thread sums its rows (rows tid, tid + 256, ...); the
// sums are added across each wave by exchanges at lane distances 32 .. 1 and
// the four waves' totals in order.  Panels are row-major with r columns
// unless a row stride is given.
#include "godec_internal.h"
#include "k_common.h"
#include "k_rr.h"

namespace godec {
namespace {

#define GODEC_R_SWITCH(rr, ...)                            \
  switch (rr) {                                            \
    case 1: { constexpr int R = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int R = 2; __VA_ARGS__; } break;   \
    case 3: { constexpr int R = 3; __VA_ARGS__; } break;   \
    case 4: { constexpr int R = 4; __VA_ARGS__; } break;   \
    case 5: { constexpr int R = 5; __VA_ARGS__; } break;   \
    case 6: { constexpr int R = 6; __VA_ARGS__; } break;   \
    case 7: { constexpr int R = 7; __VA_ARGS__; } break;   \
    case 8: { constexpr int R = 8; __VA_ARGS__; } break;   \
    default: break;                                        \
  }

// gs[i R + j] = sum over rows of P[row][i] * P2[row][j] (all threads return
// after the block barrier with gs filled).
template <typename T, int R>
__device__ __forceinline__ void block_inner(int rows, const T* __restrict__ P,
                                            const T* __restrict__ P2, T* gs, T (*red)[R * R]) {
  const int tid = threadIdx.x;
  T acc[R][R];
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) acc[i][j] = T(0);
  for (int row = tid; row < rows; row += 256) {
    T x[R], y[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      x[i] = P[(int64_t)row * R + i];
      y[i] = P2[(int64_t)row * R + i];
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int j = 0; j < R; ++j) acc[i][j] += x[i] * y[j];
  }
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      T v = acc[i][j];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      acc[i][j] = v;
    }
  const int wave = tid >> 6, lane = tid & 63;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int j = 0; j < R; ++j) red[wave][i * R + j] = acc[i][j];
  }
  __syncthreads();
  if (tid < R * R) gs[tid] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
  __syncthreads();
}

// symmetric part of an r x r product, FP64
template <typename T, int R>
__device__ __forceinline__ void sym_of(const T* gs, double (&G)[R][R]) {
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) G[i][j] = 0.5 * ((double)gs[i * R + j] + (double)gs[j * R + i]);
}

// rows of out = P M (M r x r in LDS), sums in ascending k
template <typename T, int R>
__device__ __forceinline__ void row_times(const T* __restrict__ p, const T* M, T (&o)[R]) {
  T x[R];
#pragma unroll
  for (int k = 0; k < R; ++k) x[k] = p[k];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    T s = T(0);
#pragma unroll
    for (int k = 0; k < R; ++k) s += x[k] * M[k * R + j];
    o[j] = s;
  }
}

// Z_0 = A1 (as T) and Rc_0 = I.
template <typename T, int R>
__global__ __launch_bounds__(256) void kf_chain_init(int n, const double* __restrict__ A1,
                                                     T* __restrict__ Z0,
                                                     double* __restrict__ rc0) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t cnt = (int64_t)n * R;
  if (e < cnt) Z0[(int64_t)b * cnt + e] = (T)A1[(int64_t)b * cnt + e];
  if (blockIdx.x == 0 && threadIdx.x < R * R)
    rc0[b * R * R + threadIdx.x] = (threadIdx.x / R == threadIdx.x % R) ? 1.0 : 0.0;
}

// Cholesky QR of a panel: P^T P = U^T U, Z = P U^{-1}, rc_out = U rc_in.
template <typename T, int R>
__global__ __launch_bounds__(256) void kf_cholqr(int rows, const T* __restrict__ P,
                                                 const double* __restrict__ rc_in,
                                                 double* __restrict__ rc_out,
                                                 T* __restrict__ Z, int* __restrict__ flag) {
  __shared__ T gs[R * R], ui[R * R];
  __shared__ T red[4][R * R];
  const int b = blockIdx.x, tid = threadIdx.x;
  const T* Pb = P + (int64_t)b * rows * R;
  block_inner<T, R>(rows, Pb, Pb, gs, red);
  if (tid == 0) {
    double G[R][R], U[R][R], Ui[R][R];
    sym_of<T, R>(gs, G);
    if (!rr_chol<R>(G, U, Ui)) atomicOr(flag, 1);
    const double* ri = rc_in + (int64_t)b * R * R;
    double* ro = rc_out + (int64_t)b * R * R;
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int j = 0; j < R; ++j) {
        ui[i * R + j] = (T)Ui[i][j];
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < R; ++l) s += U[i][l] * ri[l * R + j];
        ro[i * R + j] = s;
      }
  }
  __syncthreads();
  T* Zb = Z + (int64_t)b * rows * R;
  for (int row = tid; row < rows; row += 256) {
    T o[R];
    row_times<T, R>(Pb + (int64_t)row * R, ui, o);
#pragma unroll
    for (int j = 0; j < R; ++j) Zb[(int64_t)row * R + j] = o[j];
  }
}

// C = B^T B = V diag(lam) V^T: C^a (T), V and the Daleckii-Krein weights
// F_ij = (lam_i^a - lam_j^a) / (lam_i - lam_j)  (a lam^(a-1) when equal).
template <typename T, int R>
__global__ __launch_bounds__(256) void kf_gram_eig(int rows, const T* __restrict__ B, double a,
                                                   T* __restrict__ calpha,
                                                   double* __restrict__ vout,
                                                   double* __restrict__ fout,
                                                   int* __restrict__ flag) {
  __shared__ T gs[R * R];
  __shared__ T red[4][R * R];
  const int b = blockIdx.x;
  const T* Bb = B + (int64_t)b * rows * R;
  block_inner<T, R>(rows, Bb, Bb, gs, red);
  if (threadIdx.x != 0) return;
  constexpr int E = R * R;
  double A[R][R], V[R][R];
  sym_of<T, R>(gs, A);
  rr_jacobi<R>(A, V);
  double lam[R], la[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    lam[i] = A[i][i];
    if (!(lam[i] > 0.0)) {
      atomicOr(flag, 2);
      lam[i] = 1e-300;
    }
    la[i] = pow(lam[i], a);
  }
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < R; ++l) s += V[i][l] * la[l] * V[j][l];
      calpha[b * E + i * R + j] = (T)s;
      vout[b * E + i * R + j] = V[i][j];
      const double d = lam[i] - lam[j];
      fout[b * E + i * R + j] =
          fabs(d) > 1e-12 * fmax(lam[i], lam[j]) ? (la[i] - la[j]) / d
                                                  : a * pow(0.5 * (lam[i] + lam[j]), a - 1.0);
    }
}

// Adjoint of B in L = B C^a Q^T with C = B^T B:
//   Cbar_a = B^T LQ,  S2 = 2 sym(V (F o (V^T sym(Cbar_a) V)) V^T)  (Daleckii-Krein),
//   Bbar = LQ C^a + B S2, written to Bbar and to columns [0, r) of Uf (row
//   stride w).
template <typename T, int R>
__global__ __launch_bounds__(256) void kf_bbar(int m, const T* __restrict__ B,
                                               const T* __restrict__ LQ,
                                               const T* __restrict__ Ca,
                                               const double* __restrict__ vin,
                                               const double* __restrict__ fin,
                                               T* __restrict__ Bbar, T* __restrict__ Uf, int w) {
  __shared__ T gs[R * R], s2s[R * R], cas[R * R];
  __shared__ T red[4][R * R];
  constexpr int E = R * R;
  const int b = blockIdx.x, tid = threadIdx.x;
  const T* Bb = B + (int64_t)b * m * R;
  const T* Lb = LQ + (int64_t)b * m * R;
  block_inner<T, R>(m, Bb, Lb, gs, red);
  if (tid < E) cas[tid] = Ca[b * E + tid];
  if (tid == 0) {
    double S[R][R], V[R][R], M[R][R];
    sym_of<T, R>(gs, S);
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int j = 0; j < R; ++j) V[i][j] = vin[b * E + i * R + j];
#pragma unroll
    for (int i = 0; i < R; ++i)  // M = F o (V^T S V)
#pragma unroll
      for (int j = 0; j < R; ++j) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
          for (int l = 0; l < R; ++l) s += V[k][i] * S[k][l] * V[l][j];
        M[i][j] = s * fin[b * E + i * R + j];
      }
    double N[R][R];
#pragma unroll
    for (int i = 0; i < R; ++i)  // N = V M V^T
#pragma unroll
      for (int j = 0; j < R; ++j) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k)
#pragma unroll
          for (int l = 0; l < R; ++l) s += V[i][k] * M[k][l] * V[j][l];
        N[i][j] = s;
      }
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int j = 0; j < R; ++j) s2s[i * R + j] = (T)(N[i][j] + N[j][i]);
  }
  __syncthreads();
  T* Ob = Bbar + (int64_t)b * m * R;
  T* Ub = Uf + (int64_t)b * m * w;
  for (int row = tid; row < m; row += 256) {
    T o1[R], o2[R];
    row_times<T, R>(Lb + (int64_t)row * R, cas, o1);
    row_times<T, R>(Bb + (int64_t)row * R, s2s, o2);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const T v = o2[j] + o1[j];
      Ob[(int64_t)row * R + j] = v;
      Ub[(int64_t)row * w + j] = v;
    }
  }
}

// Adjoint of Q: Qbar = LtB C^a + cur, then its part off the range of Q,
// Qbar - Q (Q^T Qbar).
template <typename T, int R>
__global__ __launch_bounds__(256) void kf_qbar(int n, const T* __restrict__ LtB,
                                               const T* __restrict__ Ca, const T* __restrict__ cur,
                                               const T* __restrict__ Q, T* __restrict__ Qbar) {
  __shared__ T gs[R * R], cas[R * R];
  __shared__ T red[4][R * R];
  constexpr int E = R * R;
  const int b = blockIdx.x, tid = threadIdx.x;
  const T* Lb = LtB + (int64_t)b * n * R;
  const T* Cb = cur + (int64_t)b * n * R;
  const T* Qb = Q + (int64_t)b * n * R;
  T* Ob = Qbar + (int64_t)b * n * R;
  if (tid < E) cas[tid] = Ca[b * E + tid];
  __syncthreads();
  for (int row = tid; row < n; row += 256) {
    T o[R];
    row_times<T, R>(Lb + (int64_t)row * R, cas, o);
#pragma unroll
    for (int j = 0; j < R; ++j) Ob[(int64_t)row * R + j] = o[j] + Cb[(int64_t)row * R + j];
  }
  __syncthreads();
  block_inner<T, R>(n, Qb, Ob, gs, red);
  for (int row = tid; row < n; row += 256) {
    T o[R];
    row_times<T, R>(Qb + (int64_t)row * R, gs, o);
#pragma unroll
    for (int j = 0; j < R; ++j) Ob[(int64_t)row * R + j] = -o[j] + Ob[(int64_t)row * R + j];
  }
}

// A pair of power-chain terms: W = Z_j (Rc_j Rtot^{-1}) and U = cur go to
// columns [col, col + r) and [col + r, col + 2r) of Vf (row stride w).
template <typename T, int R>
__global__ __launch_bounds__(256) void kf_pterm(int n, const T* __restrict__ Zj,
                                                const double* __restrict__ rc,
                                                const double* __restrict__ rtot,
                                                const T* __restrict__ cur, T* __restrict__ Vf,
                                                int w, int col) {
  __shared__ T rel[R * R];
  constexpr int E = R * R;
  const int b = blockIdx.x, tid = threadIdx.x;
  if (tid == 0) {
    double U[R][R], Ui[R][R];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int j = 0; j < R; ++j) U[i][j] = rtot[b * E + i * R + j];
    rr_triu_inv<R>(U, Ui);
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int j = 0; j < R; ++j) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < R; ++l) s += rc[b * E + i * R + l] * Ui[l][j];
        rel[i * R + j] = (T)s;
      }
  }
  __syncthreads();
  const T* Zb = Zj + (int64_t)b * n * R;
  const T* Cb = cur + (int64_t)b * n * R;
  T* Vb = Vf + (int64_t)b * n * w;
  for (int row = tid; row < n; row += 256) {
    T o[R];
    row_times<T, R>(Zb + (int64_t)row * R, rel, o);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      Vb[(int64_t)row * w + col + j] = o[j];
      Vb[(int64_t)row * w + col + R + j] = Cb[(int64_t)row * R + j];
    }
  }
}

}  // namespace

void lf_chain_init(const Launch& L, bool f64, int nb, int n, int r, const double* A1, void* Z0,
                   double* rc0) {
  const dim3 g((unsigned)(((int64_t)n * r + 255) / 256), (unsigned)nb);
  if (f64) {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_chain_init<double, R>), g, dim3(256), 0, L.stream,
                                         n, A1, (double*)Z0, rc0));
  } else {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_chain_init<float, R>), g, dim3(256), 0, L.stream, n,
                                         A1, (float*)Z0, rc0));
  }
}

void lf_cholqr(const Launch& L, bool f64, int nb, int rows, int r, const void* P,
               const double* rc_in, double* rc_out, void* Z, int* flag) {
  if (f64) {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_cholqr<double, R>), dim3((unsigned)nb), dim3(256), 0,
                                         L.stream, rows, (const double*)P, rc_in, rc_out,
                                         (double*)Z, flag));
  } else {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_cholqr<float, R>), dim3((unsigned)nb), dim3(256), 0,
                                         L.stream, rows, (const float*)P, rc_in, rc_out,
                                         (float*)Z, flag));
  }
}

void lf_gram_eig(const Launch& L, bool f64, int nb, int rows, int r, const void* B, double a,
                 void* calpha, double* v, double* f, int* flag) {
  if (f64) {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_gram_eig<double, R>), dim3((unsigned)nb), dim3(256),
                                         0, L.stream, rows, (const double*)B, a,
                                         (double*)calpha, v, f, flag));
  } else {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_gram_eig<float, R>), dim3((unsigned)nb), dim3(256),
                                         0, L.stream, rows, (const float*)B, a, (float*)calpha,
                                         v, f, flag));
  }
}

void lf_bbar(const Launch& L, bool f64, int nb, int m, int r, const void* B, const void* LQ,
             const void* Ca, const double* v, const double* f, void* Bbar, void* Uf, int w) {
  if (f64) {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_bbar<double, R>), dim3((unsigned)nb), dim3(256), 0,
                                         L.stream, m, (const double*)B, (const double*)LQ,
                                         (const double*)Ca, v, f, (double*)Bbar, (double*)Uf,
                                         w));
  } else {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_bbar<float, R>), dim3((unsigned)nb), dim3(256), 0,
                                         L.stream, m, (const float*)B, (const float*)LQ,
                                         (const float*)Ca, v, f, (float*)Bbar, (float*)Uf, w));
  }
}

void lf_qbar(const Launch& L, bool f64, int nb, int n, int r, const void* LtB, const void* Ca,
             const void* cur, const void* Q, void* Qbar) {
  if (f64) {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_qbar<double, R>), dim3((unsigned)nb), dim3(256), 0,
                                         L.stream, n, (const double*)LtB, (const double*)Ca,
                                         (const double*)cur, (const double*)Q, (double*)Qbar));
  } else {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_qbar<float, R>), dim3((unsigned)nb), dim3(256), 0,
                                         L.stream, n, (const float*)LtB, (const float*)Ca,
                                         (const float*)cur, (const float*)Q, (float*)Qbar));
  }
}

void lf_pterm(const Launch& L, bool f64, int nb, int n, int r, const void* Zj, const double* rc,
              const double* rtot, const void* cur, void* Vf, int w, int col) {
  if (f64) {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_pterm<double, R>), dim3((unsigned)nb), dim3(256), 0,
                                         L.stream, n, (const double*)Zj, rc, rtot,
                                         (const double*)cur, (double*)Vf, w, col));
  } else {
    GODEC_R_SWITCH(r, hipLaunchKernelGGL((kf_pterm<float, R>), dim3((unsigned)nb), dim3(256), 0,
                                         L.stream, n, (const float*)Zj, rc, rtot,
                                         (const float*)cur, (float*)Vf, w, col));
  }
}

}  // namespace godec
