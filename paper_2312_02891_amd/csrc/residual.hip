// True Sylvester residual of a factored solution X = Z D Y^T:
//     R = A X + X B + f g^T   (eq. (adi_res_inexact), first line),
// reported as ||R||_2 / ||f g^T||_2.  Sec. 4 estimates ||R||_2 after the
// iteration with eigs on R^T R; here the largest singular value comes from
// Golub-Kahan-Lanczos bidiagonalisation with full (twice repeated)
// reorthogonalisation, applying R and R^T through the factors:
//     R v   = A (Z D (Y^T v)) + Z D (Y^T (B v)) + f (g^T v)
//     R^T u = Y D (Z^T (A^T u)) + B^T (Y D (Z^T u)) + g (f^T u)
// so no n x m matrix is formed.  All arithmetic is FP64; every reduction has
// a fixed order.
#include <cmath>
#include <vector>

#include "internal.h"

namespace lradi {

void csr_transpose(int n, const int32_t* rp, const int32_t* ci, const double* v,
                   std::vector<int32_t>& trp, std::vector<int32_t>& tci, std::vector<double>& tv);

namespace {

constexpr int kRows = 1024;   // rows per workgroup of the projection kernel
constexpr int kMaxCoef = 1024; // max coefficients per projection (nb * r)

// part[w][c] = sum_{i in chunk w} X_c[i] v[i]  for the nb*r columns of a
// block-stacked n x r factor (column (b, q) of block b), or of nb contiguous
// vectors when r == 1 and stride == n.
__global__ __launch_bounds__(256) void k_proj(const double* __restrict__ X, int nb, int n, int r,
                                              size_t stride, const double* __restrict__ v,
                                              double* __restrict__ part) {
  __shared__ double red[256];
  const int w = blockIdx.x;
  const int i0 = w * kRows, i1 = min(n, i0 + kRows);
  const int ncol = nb * r;
  for (int c = 0; c < ncol; ++c) {
    const int b = c / r, q = c - b * r;
    const double* xb = X + (size_t)b * stride;
    double acc = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += 256) acc += xb[(size_t)i * r + q] * v[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)w * ncol + c] = red[0];
    __syncthreads();
  }
}

// out[c] = scale * sum_w part[w][c]
__global__ void k_proj_reduce(const double* __restrict__ part, int nwg, int ncol, double scale,
                              double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  double s = 0.0;
  for (int w = 0; w < nwg; ++w) s += part[(size_t)w * ncol + c];
  out[c] = scale * s;
}

// y = beta*y + sign * sum_b gam_b sum_q X_b[i][q] coef[b r + q]  (gam may be null)
__global__ __launch_bounds__(256) void k_expand(const double* __restrict__ X, int nb, int n, int r,
                                                size_t stride, const double* __restrict__ gam,
                                                const double* __restrict__ coef, double sign,
                                                double beta, double* __restrict__ y) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double* xb = X + (size_t)b * stride + (size_t)i * r;
    double t = 0.0;
    for (int q = 0; q < r; ++q) t += xb[q] * coef[b * r + q];
    acc += (gam ? gam[b] : 1.0) * t;
  }
  y[i] = (beta == 0.0 ? 0.0 : beta * y[i]) + sign * acc;
}

// y = A x (+ y if accumulate)
__global__ __launch_bounds__(256) void k_spmv(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                              const double* __restrict__ val, const double* __restrict__ x,
                                              double* __restrict__ y, int accumulate) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) acc += val[k] * x[ci[k]];
  y[i] = accumulate ? y[i] + acc : acc;
}

// y += a * x with a read from device memory (sign applied)
__global__ void k_axpy_dev(int n, const double* __restrict__ a, double sign, const double* __restrict__ x,
                           double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += sign * a[0] * x[i];
}

// alpha = sqrt(nrm2[0]); dst = src / alpha  (alpha stored to *alpha_out)
__global__ void k_normalize(int n, const double* __restrict__ nrm2, double* __restrict__ src,
                            double* __restrict__ dst, double* __restrict__ alpha_out) {
  const double a = sqrt(fmax(nrm2[0], 0.0));
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *alpha_out = a;
  if (i < n) dst[i] = (a > 0.0) ? src[i] / a : 0.0;
}

// start vector v[j] in [-1, 1] from the splitmix64 mixing function of j
__global__ void k_start(int m, double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  unsigned long long z = (unsigned long long)i + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  v[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Largest singular value of the upper bidiagonal matrix with diagonal
// alpha[0..j) and superdiagonal beta[0..j-1): the square root of the largest
// eigenvalue of the tridiagonal B^T B, by bisection on Sturm counts.
__global__ void k_bidiag_smax(const double* __restrict__ alpha, const double* __restrict__ beta, int j,
                              double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  // T = B^T B: d_i = alpha_i^2 + beta_{i-1}^2, e_i = alpha_i beta_i
  double hi = 0.0;
  for (int i = 0; i < j; ++i) {
    const double d = alpha[i] * alpha[i] + (i > 0 ? beta[i - 1] * beta[i - 1] : 0.0);
    const double e1 = (i > 0) ? fabs(alpha[i - 1] * beta[i - 1]) : 0.0;
    const double e2 = (i + 1 < j) ? fabs(alpha[i] * beta[i]) : 0.0;
    hi = fmax(hi, d + e1 + e2);
  }
  double lo = 0.0;
  for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
    const double x = 0.5 * (lo + hi);
    // number of eigenvalues of T greater than x
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < j; ++i) {
      const double d = alpha[i] * alpha[i] + (i > 0 ? beta[i - 1] * beta[i - 1] : 0.0);
      const double e2 = (i > 0) ? (alpha[i - 1] * beta[i - 1]) * (alpha[i - 1] * beta[i - 1]) : 0.0;
      q = (i == 0) ? d - x : d - x - e2 / q;
      if (q == 0.0) q = -1e-300;
      if (q > 0.0) ++cnt;
    }
    if (cnt > 0) lo = x; else hi = x;
  }
  out[0] = sqrt(hi);
}

struct Dev {
  hipStream_t st;
  double* part;
  int proj(const double* X, int nb, int n, int r, size_t stride, const double* v, double* out,
           double scale = 1.0) {
    const int nwg = (n + kRows - 1) / kRows;
    const int ncol = nb * r;
    if (ncol <= 0) return LRADI_OK;
    hipLaunchKernelGGL(k_proj, dim3(nwg), dim3(256), 0, st, X, nb, n, r, stride, v, part);
    hipLaunchKernelGGL(k_proj_reduce, dim3((ncol + 255) / 256), dim3(256), 0, st, part, nwg, ncol, scale,
                       out);
    LRADI_HIP(hipGetLastError());
    return LRADI_OK;
  }
  int expand(const double* X, int nb, int n, int r, size_t stride, const double* gam,
             const double* coef, double sign, double beta, double* y) {
    hipLaunchKernelGGL(k_expand, dim3((n + 255) / 256), dim3(256), 0, st, X, nb, n, r, stride, gam, coef,
                       sign, beta, y);
    LRADI_HIP(hipGetLastError());
    return LRADI_OK;
  }
  int spmv(const CsrRef& A, const double* x, double* y, int acc) {
    hipLaunchKernelGGL(k_spmv, dim3((A.n + 255) / 256), dim3(256), 0, st, A.n, A.rowptr, A.colind, A.val, x,
                       y, acc);
    LRADI_HIP(hipGetLastError());
    return LRADI_OK;
  }
};

// Workspace layout of one residual evaluation with at most J Lanczos steps
// (offsets in doubles, every region starting on a 256-byte boundary).
struct WsLayout {
  size_t part, U, V, tn, tn2, tn3, tm, tm2, tm3, coef, scal, total;
};

size_t ws_round(size_t x) { return (x + 31) & ~(size_t)31; }

WsLayout ws_layout(int n, int m, int J, bool hasM, bool hasC) {
  const size_t nwg_max = (size_t)(std::max(n, m) + kRows - 1) / kRows;
  WsLayout L{};
  size_t o = 0;
  auto take = [&](size_t cnt) {
    const size_t at = o;
    o += ws_round(std::max<size_t>(cnt, 1));
    return at;
  };
  L.part = take(nwg_max * (size_t)std::max(kMaxCoef, J + 2));
  L.U = take((size_t)n * (J + 1));
  L.V = take((size_t)m * (J + 2));
  L.tn = take(n);
  L.tn2 = take(n);
  L.tn3 = hasM ? take(n) : 0;
  L.tm = take(m);
  L.tm2 = take(m);
  L.tm3 = hasC ? take(m) : 0;
  L.coef = take(3 * (size_t)kMaxCoef + 2 * (size_t)(J + 2));
  // scalars: [0] nrm2, [1..J+1] alpha, [J+2..2J+2] beta, [2J+4] sigma
  L.scal = take(2 * (size_t)J + 8);
  L.total = o;
  return L;
}

}  // namespace

size_t residual_ws_bytes(int n, int m, int maxit, bool hasM, bool hasC) {
  return sizeof(double) * ws_layout(n, m, maxit, hasM, hasC).total;
}

int residual_norm_ws(hipStream_t st, const CsrRef& A, const CsrRef& At, const CsrRef& B, const CsrRef& Bt,
                     const double* f, const double* g, int r, const double* Z, const double* gam_d,
                     const double* Y, int k, int maxit, double* sigma_out, const CsrRef* M,
                     const CsrRef* Mt, const CsrRef* C, const CsrRef* Ct, double* ws) {
  const int n = A.n, m = B.n;
  const int J = maxit;
  if (k * r > kMaxCoef) return set_error("lradi_residual: k*r above %d", kMaxCoef), LRADI_EINVAL;
  const WsLayout W = ws_layout(n, m, J, M != nullptr, C != nullptr);
  Dev dv;
  dv.st = st;
  dv.part = ws + W.part;
  double* U = ws + W.U;
  double* V = ws + W.V;
  double* tn = ws + W.tn;
  double* tn2 = ws + W.tn2;
  double* tn3 = ws + W.tn3;
  double* tm = ws + W.tm;
  double* tm2 = ws + W.tm2;
  double* tm3 = ws + W.tm3;
  double* c1 = ws + W.coef;
  double* c2 = c1 + kMaxCoef;
  double* c3 = c2 + kMaxCoef;
  double* ho = c3 + kMaxCoef;  // reorthogonalisation coefficients
  double* S = ws + W.scal;
  double* nrm2 = S;
  double* alpha = S + 1;
  double* beta = S + 2 + J;
  double* sig = S + 2 * J + 4;
  const size_t sZ = (size_t)n * r, sY = (size_t)m * r;
  auto nb256 = [](int x) { return dim3((x + 255) / 256); };

  // R = A Z D Y^T C + M Z D Y^T B + f g^T (M, C = I when null)
  // R v -> p (n-vector); p must not be tn, tn3, tm or tm3
  auto apply_R = [&](const double* v, double* p) -> int {
    if (C) {
      LRADI_TRY(dv.spmv(*C, v, tm3, 0));   // tm3 = C v
      LRADI_TRY(dv.proj(Y, k, m, r, sY, tm3, c1));  // c1 = Y^T C v
    } else {
      LRADI_TRY(dv.proj(Y, k, m, r, sY, v, c1));        // c1 = Y^T v
    }
    LRADI_TRY(dv.spmv(B, v, tm, 0));       // tm = B v
    LRADI_TRY(dv.proj(Y, k, m, r, sY, tm, c2));  // c2 = Y^T B v
    LRADI_TRY(dv.proj(g, 1, m, r, sY, v, c3));          // c3 = g^T v
    LRADI_TRY(dv.expand(Z, k, n, r, sZ, gam_d, c1, 1.0, 0.0, tn));  // Z D c1
    LRADI_TRY(dv.spmv(A, tn, p, 0));       // p = A Z D c1
    if (M) {
      LRADI_TRY(dv.expand(Z, k, n, r, sZ, gam_d, c2, 1.0, 0.0, tn3));
      LRADI_TRY(dv.spmv(*M, tn3, p, 1));   // p += M Z D c2
    } else {
      LRADI_TRY(dv.expand(Z, k, n, r, sZ, gam_d, c2, 1.0, 1.0, p));
    }
    LRADI_TRY(dv.expand(f, 1, n, r, sZ, nullptr, c3, 1.0, 1.0, p));
    return LRADI_OK;
  };
  // R^T u -> q (m-vector); q must not be tn2, tn3, tm2 or tm3
  auto apply_Rt = [&](const double* u, double* q) -> int {
    LRADI_TRY(dv.spmv(At, u, tn2, 0));     // A^T u
    LRADI_TRY(dv.proj(Z, k, n, r, sZ, tn2, c1));  // Z^T A^T u
    if (M) {
      LRADI_TRY(dv.spmv(*Mt, u, tn3, 0));  // M^T u
      LRADI_TRY(dv.proj(Z, k, n, r, sZ, tn3, c2));  // Z^T M^T u
    } else {
      LRADI_TRY(dv.proj(Z, k, n, r, sZ, u, c2));        // Z^T u
    }
    LRADI_TRY(dv.proj(f, 1, n, r, sZ, u, c3));          // f^T u
    if (C) {
      LRADI_TRY(dv.expand(Y, k, m, r, sY, gam_d, c1, 1.0, 0.0, tm3));
      LRADI_TRY(dv.spmv(*Ct, tm3, q, 0));  // q = C^T Y D c1
    } else {
      LRADI_TRY(dv.expand(Y, k, m, r, sY, gam_d, c1, 1.0, 0.0, q));
    }
    LRADI_TRY(dv.expand(Y, k, m, r, sY, gam_d, c2, 1.0, 0.0, tm2));
    LRADI_TRY(dv.spmv(Bt, tm2, q, 1));
    LRADI_TRY(dv.expand(g, 1, m, r, sY, nullptr, c3, 1.0, 1.0, q));
    return LRADI_OK;
  };
  // x -= Q (Q^T x) twice, Q = the first cnt columns (contiguous, length len)
  auto reorth = [&](double* Q, int cnt, int len, double* x) -> int {
    for (int pass = 0; pass < 2 && cnt > 0; ++pass) {
      LRADI_TRY(dv.proj(Q, cnt, len, 1, (size_t)len, x, ho));
      LRADI_TRY(dv.expand(Q, cnt, len, 1, (size_t)len, nullptr, ho, -1.0, 1.0, x));
    }
    return LRADI_OK;
  };
  auto normalize = [&](double* src, int len, double* dst, double* store) -> int {
    LRADI_TRY(dv.proj(src, 1, len, 1, (size_t)len, src, nrm2));
    hipLaunchKernelGGL(k_normalize, nb256(len), dim3(256), 0, st, len, nrm2, src, dst, store);
    LRADI_HIP(hipGetLastError());
    return LRADI_OK;
  };

  // v_1
  hipLaunchKernelGGL(k_start, nb256(m), dim3(256), 0, st, m, tm);
  LRADI_TRY(normalize(tm, m, V, S + 2 * J + 6));
  // u_1 = R v_1 / alpha_1 (apply_R uses tn internally, so write into U)
  LRADI_TRY(apply_R(V, U));
  LRADI_TRY(normalize(U, n, U, alpha));
  double prev = -1.0, cur = 0.0;
  double hb[2] = {0.0, 0.0};
  int it = 1;
  for (; it <= J; ++it) {
    // v_{it+1} = (R^T u_it - alpha_it v_it) / beta_it
    double* vn = V + (size_t)it * m;
    LRADI_TRY(apply_Rt(U + (size_t)(it - 1) * n, vn));
    hipLaunchKernelGGL(k_axpy_dev, nb256(m), dim3(256), 0, st, m, alpha + it - 1, -1.0,
                       V + (size_t)(it - 1) * m, vn);
    LRADI_TRY(reorth(V, it, m, vn));
    LRADI_TRY(normalize(vn, m, vn, beta + it - 1));
    // u_{it+1} = (R v_{it+1} - beta_it u_it) / alpha_{it+1}
    double* un = U + (size_t)it * n;
    if (it < J) {
      LRADI_TRY(apply_R(vn, un));
      hipLaunchKernelGGL(k_axpy_dev, nb256(n), dim3(256), 0, st, n, beta + it - 1, -1.0,
                         U + (size_t)(it - 1) * n, un);
      LRADI_TRY(reorth(U, it, n, un));
      LRADI_TRY(normalize(un, n, un, alpha + it));
    }
    // sigma_max of the it x it leading block (diagonal alpha_0..it-1, super beta_0..it-2)
    hipLaunchKernelGGL(k_bidiag_smax, dim3(1), dim3(64), 0, st, alpha, beta, it, sig);
    LRADI_HIP(hipGetLastError());
    LRADI_HIP(hipMemcpyAsync(hb, sig, sizeof(double), hipMemcpyDeviceToHost, st));
    LRADI_HIP(hipMemcpyAsync(hb + 1, beta + it - 1, sizeof(double), hipMemcpyDeviceToHost, st));
    LRADI_HIP(hipStreamSynchronize(st));
    cur = hb[0];
    if (it >= 3 && std::fabs(cur - prev) <= 1e-12 * cur) break;
    if (hb[1] <= 1e-15 * cur) break;  // invariant subspace: exact
    prev = cur;
  }
  *sigma_out = cur;
  return LRADI_OK;
}

int residual_norm(hipStream_t st, const DevCSR& A, const DevCSR& At, const DevCSR& B, const DevCSR& Bt,
                  const double* f, const double* g, int r, const double* Z, const double* gam_d,
                  const double* Y, int k, int maxit, double* sigma_out, const DevCSR* M,
                  const DevCSR* Mt, const DevCSR* C, const DevCSR* Ct) {
  DevBuf ws;
  LRADI_TRY(ws.alloc(residual_ws_bytes(A.n, B.n, maxit, M != nullptr, C != nullptr)));
  const CsrRef rM = M ? csr_ref(*M) : CsrRef{}, rMt = Mt ? csr_ref(*Mt) : CsrRef{};
  const CsrRef rC = C ? csr_ref(*C) : CsrRef{}, rCt = Ct ? csr_ref(*Ct) : CsrRef{};
  return residual_norm_ws(st, csr_ref(A), csr_ref(At), csr_ref(B), csr_ref(Bt), f, g, r, Z, gam_d, Y, k,
                          maxit, sigma_out, M ? &rM : nullptr, Mt ? &rMt : nullptr, C ? &rC : nullptr,
                          Ct ? &rCt : nullptr, ws.as<double>());
}

}  // namespace lradi
