// r x r FP64 algebra of the differentiable layer's backward (r = R <= 8), one
// thread per problem.  R is a template argument so that every loop unrolls
// and the matrices stay in registers.
#pragma once

#include <hip/hip_runtime.h>

namespace godec {

// Upper-triangular Cholesky factor U of the symmetric G (G = U^T U) and its
// inverse Ui.  A pivot that is not positive is replaced by 1e-300 and the
// function returns false.
template <int R>
__device__ __forceinline__ bool rr_chol(const double (&G)[R][R], double (&U)[R][R],
                                        double (&Ui)[R][R]) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) {
      U[i][j] = 0.0;
      Ui[i][j] = 0.0;
    }
#pragma unroll
  for (int j = 0; j < R; ++j) {
    double d = G[j][j];
#pragma unroll
    for (int l = 0; l < j; ++l) d -= U[l][j] * U[l][j];
    if (!(d > 0.0)) {
      ok = false;
      d = 1e-300;
    }
    U[j][j] = sqrt(d);
#pragma unroll
    for (int c = j + 1; c < R; ++c) {
      double s = G[j][c];
#pragma unroll
      for (int l = 0; l < j; ++l) s -= U[l][j] * U[l][c];
      U[j][c] = s / U[j][j];
    }
  }
#pragma unroll
  for (int j = R - 1; j >= 0; --j) {
    Ui[j][j] = 1.0 / U[j][j];
#pragma unroll
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
#pragma unroll
      for (int l = i + 1; l <= j; ++l) s += U[i][l] * Ui[l][j];
      Ui[i][j] = -s / U[i][i];
    }
  }
  return ok;
}

// Inverse of an upper-triangular U.
template <int R>
__device__ __forceinline__ void rr_triu_inv(const double (&U)[R][R], double (&Ui)[R][R]) {
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) Ui[i][j] = 0.0;
#pragma unroll
  for (int j = R - 1; j >= 0; --j) {
    Ui[j][j] = 1.0 / U[j][j];
#pragma unroll
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
#pragma unroll
      for (int l = i + 1; l <= j; ++l) s += U[i][l] * Ui[l][j];
      Ui[i][j] = -s / U[i][i];
    }
  }
}

// Cyclic Jacobi on the symmetric A (overwritten with its diagonalisation);
// V collects the rotations (A_in = V diag(A_out) V^T).
template <int R>
__device__ __forceinline__ void rr_jacobi(double (&A)[R][R], double (&V)[R][R]) {
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = 0; j < R; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      dia += A[i][i] * A[i][i];
#pragma unroll
      for (int j = i + 1; j < R; ++j) off += A[i][j] * A[i][j];
    }
    if (off <= 1e-32 * dia) break;
#pragma unroll
    for (int p = 0; p < R; ++p)
#pragma unroll
      for (int q = p + 1; q < R; ++q) {
        const double apq = A[p][q];
        if (apq != 0.0) {
          const double th = (A[q][q] - A[p][p]) / (2.0 * apq);
          const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const double akp = A[k][p], akq = A[k][q];
            A[k][p] = c * akp - s * akq;
            A[k][q] = s * akp + c * akq;
          }
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const double apk = A[p][k], aqk = A[q][k];
            A[p][k] = c * apk - s * aqk;
            A[q][k] = s * apk + c * aqk;
          }
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const double vkp = V[k][p], vkq = V[k][q];
            V[k][p] = c * vkp - s * vkq;
            V[k][q] = s * vkp + c * vkq;
          }
        }
      }
  }
}

}  // namespace godec
