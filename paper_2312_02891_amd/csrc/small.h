// Small dense FP64 kernels on r x r (r <= 8) and 2r x r matrices, run by a
// single thread.  They are __host__ __device__ so the host self-test can
// exercise exactly the code the GPU runs.
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#define LRADI_HD __host__ __device__
#else
#define LRADI_HD
#endif

namespace lradi {

// Upper Cholesky factor S of a symmetric positive semidefinite G (row-major
// n x n): G = S^T S.  A pivot below rel_floor * max_i G_ii (or not positive)
// is replaced by that floor and the rest of its row is zeroed; the returned
// count says how many pivots were replaced.  Returns -1 if G holds a NaN/Inf.
LRADI_HD inline int chol_upper_reg(const double* G, double* S, int n, double rel_floor) {
  double dmax = 0.0;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) {
      double g = G[i * n + j];
      if (!(g == g) || g - g != 0.0) return -1;
    }
    dmax = fmax(dmax, G[i * n + i]);
  }
  double fl = rel_floor * dmax;
  if (!(fl > 0.0)) fl = 1e-300;
  int reg = 0;
  for (int i = 0; i < n * n; ++i) S[i] = 0.0;
  for (int c = 0; c < n; ++c) {
    double d = G[c * n + c];
    for (int k = 0; k < c; ++k) d -= S[k * n + c] * S[k * n + c];
    if (d > fl) {
      double s = sqrt(d);
      S[c * n + c] = s;
      for (int q = c + 1; q < n; ++q) {
        double v = G[c * n + q];
        for (int k = 0; k < c; ++k) v -= S[k * n + c] * S[k * n + q];
        S[c * n + q] = v / s;
      }
    } else {
      S[c * n + c] = sqrt(fl);
      ++reg;
    }
  }
  return reg;
}

// X = S^{-1} for upper triangular S (row-major n x n); X is upper triangular.
LRADI_HD inline void tri_inv_upper(const double* S, double* X, int n) {
  for (int i = 0; i < n * n; ++i) X[i] = 0.0;
  for (int c = n - 1; c >= 0; --c) {
    X[c * n + c] = 1.0 / S[c * n + c];
    for (int q = c + 1; q < n; ++q) {
      double v = 0.0;
      for (int k = c + 1; k <= q; ++k) v += S[c * n + k] * X[k * n + q];
      X[c * n + q] = -v / S[c * n + c];
    }
  }
}

// C = A B for n x n row-major matrices (C distinct from A and B).
LRADI_HD inline void matmul_sq(const double* A, const double* B, double* C, int n) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += A[i * n + k] * B[k * n + j];
      C[i * n + j] = v;
    }
}

// Cyclic Jacobi eigenvalue iteration on a symmetric n x n row-major A
// (overwritten; its diagonal ends up holding the eigenvalues).  If Q is not
// null it receives the eigenvectors as columns.  At most 50 sweeps.
LRADI_HD inline void jacobi_eig(double* A, double* Q, int n) {
  if (Q)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) Q[i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        double a = A[p * n + q];
        tot += a * a;
        if (p != q) off += a * a;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0);
        double s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        if (Q)
          for (int k = 0; k < n; ++k) {
            double qkp = Q[k * n + p], qkq = Q[k * n + q];
            Q[k * n + p] = c * qkp - s * qkq;
            Q[k * n + q] = s * qkp + c * qkq;
          }
      }
  }
}

// Largest eigenvalue of a symmetric positive semidefinite n x n matrix
// (row-major, copied; G itself is left alone).
LRADI_HD inline double lambda_max_sym(const double* G, int n) {
  double A[64];
  for (int i = 0; i < n * n; ++i) A[i] = G[i];
  jacobi_eig(A, nullptr, n);
  double m = 0.0;
  for (int i = 0; i < n; ++i) m = fmax(m, A[i * n + i]);
  return m;
}

// Largest eigenvalue of the product Gw Gt of two symmetric positive
// semidefinite n x n matrices: with Gw = Q diag(l) Q^T it equals
// lambda_max(diag(sqrt l) Q^T Gt Q diag(sqrt l)), a symmetric matrix.  So
// ||W T^T||_2^2 = lambda_max((W^T W)(T^T T)) for tall blocks W, T.
LRADI_HD inline double lambda_max_prod(const double* Gw, const double* Gt, int n) {
  double A[64], Q[64], M[64], tmp[64];
  for (int i = 0; i < n * n; ++i) A[i] = Gw[i];
  jacobi_eig(A, Q, n);
  double sl[8];
  for (int i = 0; i < n; ++i) sl[i] = sqrt(fmax(A[i * n + i], 0.0));
  // tmp = Gt Q
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += Gt[i * n + k] * Q[k * n + j];
      tmp[i * n + j] = v;
    }
  // M = diag(sl) Q^T tmp diag(sl)
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v += Q[k * n + i] * tmp[k * n + j];
      M[i * n + j] = sl[i] * v * sl[j];
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double a = 0.5 * (M[i * n + j] + M[j * n + i]);
      M[i * n + j] = a;
      M[j * n + i] = a;
    }
  return lambda_max_sym(M, n);
}

// Householder QR of the 2n x n matrix M (row-major, overwritten with R in
// its top n rows and zeros below).  Q (2n x 2n, row-major) is returned
// explicitly with Q^T M_in = [R; 0].
LRADI_HD inline void householder_2nxn(double* M, double* Q, int n) {
  const int m = 2 * n;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) Q[i * m + j] = (i == j) ? 1.0 : 0.0;
  double v[16];
  for (int c = 0; c < n; ++c) {
    double nx = 0.0;
    for (int i = c; i < m; ++i) nx += M[i * n + c] * M[i * n + c];
    nx = sqrt(nx);
    if (nx == 0.0) continue;
    double x0 = M[c * n + c];
    double alpha = (x0 >= 0.0) ? -nx : nx;
    for (int i = 0; i < m; ++i) v[i] = 0.0;
    for (int i = c; i < m; ++i) v[i] = M[i * n + c];
    v[c] -= alpha;
    double vv = 0.0;
    for (int i = c; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    double beta = 2.0 / vv;
    // M <- H M on columns c..n-1
    for (int j = c; j < n; ++j) {
      double d = 0.0;
      for (int i = c; i < m; ++i) d += v[i] * M[i * n + j];
      d *= beta;
      for (int i = c; i < m; ++i) M[i * n + j] -= d * v[i];
    }
    for (int i = c + 1; i < m; ++i) M[i * n + c] = 0.0;
    M[c * n + c] = alpha;
    // Q <- Q H
    for (int i = 0; i < m; ++i) {
      double d = 0.0;
      for (int k = c; k < m; ++k) d += Q[i * m + k] * v[k];
      d *= beta;
      for (int k = c; k < m; ++k) Q[i * m + k] -= d * v[k];
    }
  }
}

}  // namespace lradi
