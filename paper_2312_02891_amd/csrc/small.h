// Small dense FP64 kernels on r x r (r <= 8) and 2r x r matrices, run by a
// single thread.  Each routine is a template on the dimension so that on the
// GPU every array is indexed with compile-time constants and lives in
// registers; the runtime-n wrappers dispatch to the instantiations.  They are
// __host__ __device__ so the host self-test exercises the code the GPU runs.
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#define LRADI_HD __host__ __device__
#else
#define LRADI_HD
#endif

#define LRADI_UNROLL _Pragma("unroll")

namespace lradi {

// Upper Cholesky factor S of a symmetric positive semidefinite G (row-major
// N x N): G = S^T S.  A pivot below rel_floor * max_i G_ii (or not positive)
// is replaced by that floor and the rest of its row is zeroed; the returned
// count says how many pivots were replaced.  Returns -1 if G holds a NaN/Inf.
template <int N>
LRADI_HD inline int chol_upper_reg_t(const double* G, double* S, double rel_floor) {
  double g[N * N], s[N * N];
  double dmax = 0.0;
  bool bad = false;
  LRADI_UNROLL for (int e = 0; e < N * N; ++e) {
    g[e] = G[e];
    bad = bad || !(g[e] == g[e]) || (g[e] - g[e] != 0.0);
    s[e] = 0.0;
  }
  if (bad) return -1;
  LRADI_UNROLL for (int i = 0; i < N; ++i) dmax = fmax(dmax, g[i * N + i]);
  double fl = rel_floor * dmax;
  if (!(fl > 0.0)) fl = 1e-300;
  int reg = 0;
  LRADI_UNROLL for (int c = 0; c < N; ++c) {
    double d = g[c * N + c];
    LRADI_UNROLL for (int k = 0; k < c; ++k) d -= s[k * N + c] * s[k * N + c];
    if (d > fl) {
      const double sc = sqrt(d);
      const double inv = 1.0 / sc;
      s[c * N + c] = sc;
      LRADI_UNROLL for (int q = c + 1; q < N; ++q) {
        double v = g[c * N + q];
        LRADI_UNROLL for (int k = 0; k < c; ++k) v -= s[k * N + c] * s[k * N + q];
        s[c * N + q] = v * inv;
      }
    } else {
      s[c * N + c] = sqrt(fl);
      ++reg;
    }
  }
  LRADI_UNROLL for (int e = 0; e < N * N; ++e) S[e] = s[e];
  return reg;
}

// X = S^{-1} for upper triangular S (row-major N x N).
template <int N>
LRADI_HD inline void tri_inv_upper_t(const double* S, double* X) {
  double s[N * N], x[N * N];
  LRADI_UNROLL for (int e = 0; e < N * N; ++e) {
    s[e] = S[e];
    x[e] = 0.0;
  }
  LRADI_UNROLL for (int c = N - 1; c >= 0; --c) {
    const double inv = 1.0 / s[c * N + c];
    x[c * N + c] = inv;
    LRADI_UNROLL for (int q = c + 1; q < N; ++q) {
      double v = 0.0;
      LRADI_UNROLL for (int k = c + 1; k <= q; ++k) v += s[c * N + k] * x[k * N + q];
      x[c * N + q] = -v * inv;
    }
  }
  LRADI_UNROLL for (int e = 0; e < N * N; ++e) X[e] = x[e];
}

// Cyclic Jacobi eigenvalue iteration on a symmetric N x N row-major matrix
// held in a (overwritten; its diagonal ends up holding the eigenvalues).  If
// WANTQ, q receives the eigenvectors as columns.  At most 50 sweeps.
template <int N, bool WANTQ>
LRADI_HD inline void jacobi_eig_t(double* a, double* q) {
  if (WANTQ) {
    LRADI_UNROLL for (int i = 0; i < N; ++i)
      LRADI_UNROLL for (int j = 0; j < N; ++j) q[i * N + j] = (i == j) ? 1.0 : 0.0;
  }
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0, tot = 0.0;
    LRADI_UNROLL for (int i = 0; i < N; ++i)
      LRADI_UNROLL for (int j = 0; j < N; ++j) {
        const double v = a[i * N + j];
        tot += v * v;
        if (i != j) off += v * v;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    LRADI_UNROLL for (int p = 0; p < N - 1; ++p)
      LRADI_UNROLL for (int r = p + 1; r < N; ++r) {
        const double apq = a[p * N + r];
        if (apq != 0.0) {
          const double theta = (a[r * N + r] - a[p * N + p]) / (2.0 * apq);
          const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          const double c = 1.0 / sqrt(t * t + 1.0);
          const double s = t * c;
          LRADI_UNROLL for (int k = 0; k < N; ++k) {
            const double akp = a[k * N + p], akq = a[k * N + r];
            a[k * N + p] = c * akp - s * akq;
            a[k * N + r] = s * akp + c * akq;
          }
          LRADI_UNROLL for (int k = 0; k < N; ++k) {
            const double apk = a[p * N + k], aqk = a[r * N + k];
            a[p * N + k] = c * apk - s * aqk;
            a[r * N + k] = s * apk + c * aqk;
          }
          if (WANTQ) {
            LRADI_UNROLL for (int k = 0; k < N; ++k) {
              const double qkp = q[k * N + p], qkq = q[k * N + r];
              q[k * N + p] = c * qkp - s * qkq;
              q[k * N + r] = s * qkp + c * qkq;
            }
          }
        }
      }
  }
}

// Largest eigenvalue of a symmetric positive semidefinite N x N matrix:
// Householder reduction to a tridiagonal matrix (scaled by a power of two
// so that no square overflows), then bisection on the Sturm count (the
// number of negative pivots of T - x I equals the number of eigenvalues
// below x) between max_i t_ii and the Gershgorin bound, to the last bit.
// The steps are separate so that the bisection can also be spread over
// the lanes of a wavefront (multisection, below).
template <int N>
struct LmaxTri {
  double d[N], off[N];  // diagonal and off-diagonal of the scaled tridiagonal
  double lo, hi;        // lambda_max in [lo, hi]
  double pivmin;        // smallest admitted pivot magnitude
  int ex;               // the matrix was scaled by 2^-ex
  bool done;            // value is final (N = 1, zero matrix, NaN)
  double value;
};

template <int N>
LRADI_HD inline void lmax_prepare(const double* G, LmaxTri<N>& t) {
  t.done = false;
  t.ex = 0;
  if (N == 1) {
    t.done = true;
    t.value = G[0];
    return;
  }
  double a[N * N];
  double amax = 0.0;
  LRADI_UNROLL for (int e = 0; e < N * N; ++e) amax = fmax(amax, fabs(G[e]));
  if (!(amax > 0.0)) {  // zero matrix, or NaN
    t.done = true;
    t.value = amax == 0.0 ? 0.0 : amax;
    return;
  }
  int ex;
  frexp(amax, &ex);
  t.ex = ex;
  LRADI_UNROLL for (int e = 0; e < N * N; ++e) a[e] = ldexp(G[e], -ex);
  double* d = t.d;
  double* off = t.off;
  LRADI_UNROLL for (int k = 0; k < N - 2; ++k) {
    double s2 = 0.0;
    LRADI_UNROLL for (int i = k + 1; i < N; ++i) s2 += a[i * N + k] * a[i * N + k];
    const double x0 = a[(k + 1) * N + k];
    const double alpha = s2 > 0.0 ? -copysign(sqrt(s2), x0) : 0.0;
    double v[N];
    LRADI_UNROLL for (int i = 0; i < N; ++i) v[i] = (i > k + 1) ? a[i * N + k] : 0.0;
    v[k + 1] = x0 - alpha;
    double vtv = 0.0;
    LRADI_UNROLL for (int i = k + 1; i < N; ++i) vtv += v[i] * v[i];
    off[k] = alpha;
    if (!(vtv > 0.0)) continue;  // the column is already reduced
    const double beta = 2.0 / vtv;
    // trailing block A22 <- H A22 H, H = I - beta v v^T: p = beta A22 v,
    // q = p - (beta v^T p / 2) v, A22 -= v q^T + q v^T
    double pv[N];
    double vtp = 0.0;
    LRADI_UNROLL for (int i = k + 1; i < N; ++i) {
      double s = 0.0;
      LRADI_UNROLL for (int j = k + 1; j < N; ++j) s += a[i * N + j] * v[j];
      pv[i] = beta * s;
      vtp += v[i] * pv[i];
    }
    const double K = 0.5 * beta * vtp;
    LRADI_UNROLL for (int i = k + 1; i < N; ++i) pv[i] -= K * v[i];
    LRADI_UNROLL for (int i = k + 1; i < N; ++i)
      LRADI_UNROLL for (int j = k + 1; j < N; ++j) a[i * N + j] -= v[i] * pv[j] + pv[i] * v[j];
  }
  LRADI_UNROLL for (int i = 0; i < N; ++i) d[i] = a[i * N + i];
  off[N - 2] = a[(N - 1) * N + (N - 2)];
  off[N - 1] = 0.0;
  double lo = d[0], hi = -1e300, e2max = 0.0;
  LRADI_UNROLL for (int i = 0; i < N; ++i) {
    lo = fmax(lo, d[i]);
    const double r = (i > 0 ? fabs(off[i - 1]) : 0.0) + (i < N - 1 ? fabs(off[i]) : 0.0);
    hi = fmax(hi, d[i] + r);
    if (i < N - 1) e2max = fmax(e2max, off[i] * off[i]);
  }
  t.lo = lo;
  t.hi = hi;
  t.pivmin = 2.2250738585072014e-308 * fmax(1.0, e2max);
}

// true when every eigenvalue of the tridiagonal lies below x (all N Sturm
// pivots of T - x I negative)
template <int N>
LRADI_HD inline bool lmax_above(const LmaxTri<N>& t, double x) {
  int below = 0;
  double q = t.d[0] - x;
  if (fabs(q) < t.pivmin) q = -t.pivmin;
  below += q < 0.0;
  LRADI_UNROLL for (int i = 1; i < N; ++i) {
    q = t.d[i] - x - t.off[i - 1] * t.off[i - 1] / q;
    if (fabs(q) < t.pivmin) q = -t.pivmin;
    below += q < 0.0;
  }
  return below == N;
}

// bisection of [lo, hi] down to adjacent doubles; the unscaled midpoint
template <int N>
LRADI_HD inline double lmax_finish(LmaxTri<N>& t) {
  for (int it = 0; it < 128 && t.hi > t.lo; ++it) {
    const double mid = 0.5 * (t.lo + t.hi);
    if (!(mid > t.lo && mid < t.hi)) break;  // adjacent doubles
    if (lmax_above<N>(t, mid)) t.hi = mid;
    else t.lo = mid;
  }
  return ldexp(0.5 * (t.lo + t.hi), t.ex);
}

template <int N>
LRADI_HD inline double lambda_max_sym_t(const double* G) {
  LmaxTri<N> t;
  lmax_prepare<N>(G, t);
  if (t.done) return t.value;
  return lmax_finish<N>(t);
}

// Multisection: one round tests the L points lo + (l + 1)(hi - lo)/(L + 1),
// l = 0..L-1, at once (one per lane) and keeps the sub-interval between
// the last point below lambda_max and the first above it; `above` has bit
// l set when point l lies above every eigenvalue.  Rounds run while all
// the points are distinct from the ends; the bisection then finishes.
LRADI_HD inline double msect_point(double lo, double hi, int l, int L) {
  return lo + (hi - lo) * ((double)(l + 1) / (double)(L + 1));
}
LRADI_HD inline bool msect_fits(double lo, double hi, int L) {
  return msect_point(lo, hi, 0, L) > lo && msect_point(lo, hi, L - 1, L) < hi;
}
LRADI_HD inline void msect_update(double& lo, double& hi, unsigned long long above, int L) {
  if (above == 0) {
    lo = msect_point(lo, hi, L - 1, L);
    return;
  }
  int f = 0;
  while (!((above >> f) & 1ull)) ++f;  // first point above
  const double nhi = msect_point(lo, hi, f, L);
  const double nlo = f > 0 ? msect_point(lo, hi, f - 1, L) : lo;
  lo = nlo;
  hi = nhi;
}

// the multisection with its L points tested one after another (the host
// check of the rounds the GPU runs across lanes)
template <int N, int L>
LRADI_HD inline double lambda_max_sym_ms_t(const double* G) {
  LmaxTri<N> t;
  lmax_prepare<N>(G, t);
  if (t.done) return t.value;
  for (int r = 0; r < 64 && msect_fits(t.lo, t.hi, L); ++r) {
    unsigned long long above = 0;
    for (int l = 0; l < L; ++l)
      if (lmax_above<N>(t, msect_point(t.lo, t.hi, l, L))) above |= 1ull << l;
    msect_update(t.lo, t.hi, above, L);
  }
  return lmax_finish<N>(t);
}

// Largest eigenvalue of the product Gw Gt of two symmetric positive
// semidefinite N x N matrices: with Gw = Q diag(l) Q^T it equals
// lambda_max(diag(sqrt l) Q^T Gt Q diag(sqrt l)), a symmetric matrix.  So
// ||W T^T||_2^2 = lambda_max((W^T W)(T^T T)) for tall blocks W, T.
template <int N>
LRADI_HD inline void prod_sym_t(const double* Gw, const double* Gt, double* m) {
  double a[N * N], q[N * N], t[N * N];
  LRADI_UNROLL for (int e = 0; e < N * N; ++e) {
    a[e] = Gw[e];
    t[e] = Gt[e];
  }
  jacobi_eig_t<N, true>(a, q);
  double sl[N];
  LRADI_UNROLL for (int i = 0; i < N; ++i) sl[i] = sqrt(fmax(a[i * N + i], 0.0));
  // a <- Gt Q
  LRADI_UNROLL for (int i = 0; i < N; ++i)
    LRADI_UNROLL for (int j = 0; j < N; ++j) {
      double v = 0.0;
      LRADI_UNROLL for (int k = 0; k < N; ++k) v += t[i * N + k] * q[k * N + j];
      a[i * N + j] = v;
    }
  LRADI_UNROLL for (int i = 0; i < N; ++i)
    LRADI_UNROLL for (int j = 0; j < N; ++j) {
      double v = 0.0;
      LRADI_UNROLL for (int k = 0; k < N; ++k) v += q[k * N + i] * a[k * N + j];
      m[i * N + j] = sl[i] * v * sl[j];
    }
  LRADI_UNROLL for (int i = 0; i < N; ++i)
    LRADI_UNROLL for (int j = i + 1; j < N; ++j) {
      const double v = 0.5 * (m[i * N + j] + m[j * N + i]);
      m[i * N + j] = v;
      m[j * N + i] = v;
    }
}
template <int N>
LRADI_HD inline double lambda_max_prod_t(const double* Gw, const double* Gt) {
  double m[N * N];
  prod_sym_t<N>(Gw, Gt, m);
  return lambda_max_sym_t<N>(m);
}

// The same largest eigenvalue through a Cholesky factor instead of an
// eigendecomposition: with Gw = L L^T (L lower triangular), Gw Gt and
// L^T Gt L have the same eigenvalues, and the latter is symmetric.  The
// factorization works in place on the lower triangle of a (row-major
// N x N, the upper triangle is zeroed); a pivot at or below N u max_i a_ii
// (u the unit roundoff) is taken as zero with its column, so rank-deficient
// Grams (dependent or zero columns of W) factor without breakdown, the
// dropped part being of the order of the rounding in Gw.  A NaN pivot is
// dropped too: callers check their Grams for NaN and Inf themselves.
template <int N>
LRADI_HD inline void psd_chol_lower_t(double* a) {
  double dmax = 0.0;
  LRADI_UNROLL for (int i = 0; i < N; ++i) dmax = fmax(dmax, a[i * N + i]);
  const double tiny = (double)N * 1.1102230246251565e-16 * dmax;
  LRADI_UNROLL for (int j = 0; j < N; ++j) {
    LRADI_UNROLL for (int i = 0; i < j; ++i) a[i * N + j] = 0.0;
    double d = a[j * N + j];
    LRADI_UNROLL for (int k = 0; k < j; ++k) d -= a[j * N + k] * a[j * N + k];
    const bool keep = d > tiny;
    const double ljj = keep ? sqrt(d) : 0.0;
    a[j * N + j] = ljj;
    LRADI_UNROLL for (int i = j + 1; i < N; ++i) {
      double t = a[i * N + j];
      LRADI_UNROLL for (int k = 0; k < j; ++k) t -= a[i * N + k] * a[j * N + k];
      a[i * N + j] = keep ? t / ljj : 0.0;
    }
  }
}

// entry (i, j) of L^T Gt L for lower-triangular L (row-major N x N), in a
// fixed summation order; i <= j gives the upper triangle, which callers
// mirror so that the matrix is exactly symmetric
template <int N>
LRADI_HD inline double prod_chol_entry_t(const double* L, const double* Gt, int i, int j) {
  double s = 0.0;
  for (int k = i; k < N; ++k) {  // L[k][i] = 0 for k < i
    double t = 0.0;
    for (int l = j; l < N; ++l) t += Gt[k * N + l] * L[l * N + j];
    s += L[k * N + i] * t;
  }
  return s;
}

template <int N>
LRADI_HD inline double lambda_max_prod_chol_t(const double* Gw, const double* Gt) {
  double a[N * N], m[N * N];
  LRADI_UNROLL for (int e = 0; e < N * N; ++e) a[e] = Gw[e];
  psd_chol_lower_t<N>(a);
  for (int i = 0; i < N; ++i)
    for (int j = i; j < N; ++j) {
      const double v = prod_chol_entry_t<N>(a, Gt, i, j);
      m[i * N + j] = v;
      m[j * N + i] = v;
    }
  return lambda_max_sym_t<N>(m);
}

// Householder QR of the 2N x N matrix M (row-major, overwritten with R in
// its top N rows and zeros below).  Q (2N x 2N, row-major) is returned
// explicitly with Q^T M_in = [R; 0].
template <int N>
LRADI_HD inline void householder_2nxn_t(double* M, double* Q) {
  constexpr int m = 2 * N;
  double a[m * N], qq[m * m], v[m];
  LRADI_UNROLL for (int e = 0; e < m * N; ++e) a[e] = M[e];
  LRADI_UNROLL for (int i = 0; i < m; ++i)
    LRADI_UNROLL for (int j = 0; j < m; ++j) qq[i * m + j] = (i == j) ? 1.0 : 0.0;
  LRADI_UNROLL for (int c = 0; c < N; ++c) {
    double nx = 0.0;
    LRADI_UNROLL for (int i = c; i < m; ++i) nx += a[i * N + c] * a[i * N + c];
    nx = sqrt(nx);
    if (nx != 0.0) {
      const double x0 = a[c * N + c];
      const double alpha = (x0 >= 0.0) ? -nx : nx;
      LRADI_UNROLL for (int i = 0; i < m; ++i) v[i] = (i >= c) ? a[i * N + c] : 0.0;
      v[c] -= alpha;
      double vv = 0.0;
      LRADI_UNROLL for (int i = c; i < m; ++i) vv += v[i] * v[i];
      if (vv != 0.0) {
        const double beta = 2.0 / vv;
        LRADI_UNROLL for (int j = c; j < N; ++j) {
          double d = 0.0;
          LRADI_UNROLL for (int i = c; i < m; ++i) d += v[i] * a[i * N + j];
          d *= beta;
          LRADI_UNROLL for (int i = c; i < m; ++i) a[i * N + j] -= d * v[i];
        }
        LRADI_UNROLL for (int i = c + 1; i < m; ++i) a[i * N + c] = 0.0;
        a[c * N + c] = alpha;
        LRADI_UNROLL for (int i = 0; i < m; ++i) {
          double d = 0.0;
          LRADI_UNROLL for (int k = c; k < m; ++k) d += qq[i * m + k] * v[k];
          d *= beta;
          LRADI_UNROLL for (int k = c; k < m; ++k) qq[i * m + k] -= d * v[k];
        }
      }
    }
  }
  LRADI_UNROLL for (int e = 0; e < m * N; ++e) M[e] = a[e];
  LRADI_UNROLL for (int e = 0; e < m * m; ++e) Q[e] = qq[e];
}

// ---- runtime-dimension wrappers ------------------------------------------
#define LRADI_SMALL_SWITCH(n, ...) \
  switch (n) {                      \
    case 1: { constexpr int NN = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int NN = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int NN = 3; __VA_ARGS__; } break; \
    case 4: { constexpr int NN = 4; __VA_ARGS__; } break; \
    case 5: { constexpr int NN = 5; __VA_ARGS__; } break; \
    case 6: { constexpr int NN = 6; __VA_ARGS__; } break; \
    case 7: { constexpr int NN = 7; __VA_ARGS__; } break; \
    default: { constexpr int NN = 8; __VA_ARGS__; } break; \
  }

LRADI_HD inline int chol_upper_reg(const double* G, double* S, int n, double rel_floor) {
  int r = 0;
  LRADI_SMALL_SWITCH(n, r = chol_upper_reg_t<NN>(G, S, rel_floor));
  return r;
}
LRADI_HD inline void tri_inv_upper(const double* S, double* X, int n) {
  LRADI_SMALL_SWITCH(n, tri_inv_upper_t<NN>(S, X));
}
LRADI_HD inline void jacobi_eig(double* A, double* Q, int n) {
  if (Q) {
    LRADI_SMALL_SWITCH(n, jacobi_eig_t<NN, true>(A, Q));
  } else {
    LRADI_SMALL_SWITCH(n, jacobi_eig_t<NN, false>(A, nullptr));
  }
}
LRADI_HD inline double lambda_max_sym(const double* G, int n) {
  double r = 0.0;
  LRADI_SMALL_SWITCH(n, r = lambda_max_sym_t<NN>(G));
  return r;
}
template <int L>
LRADI_HD inline double lambda_max_sym_ms(const double* G, int n) {
  double r = 0.0;
  LRADI_SMALL_SWITCH(n, r = (lambda_max_sym_ms_t<NN, L>(G)));
  return r;
}
LRADI_HD inline double lambda_max_prod(const double* Gw, const double* Gt, int n) {
  double r = 0.0;
  LRADI_SMALL_SWITCH(n, r = lambda_max_prod_t<NN>(Gw, Gt));
  return r;
}
LRADI_HD inline double lambda_max_prod_chol(const double* Gw, const double* Gt, int n) {
  double r = 0.0;
  LRADI_SMALL_SWITCH(n, r = lambda_max_prod_chol_t<NN>(Gw, Gt));
  return r;
}
LRADI_HD inline void householder_2nxn(double* M, double* Q, int n) {
  LRADI_SMALL_SWITCH(n, householder_2nxn_t<NN>(M, Q));
}

}  // namespace lradi
