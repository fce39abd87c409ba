// Outer LR-ADI kernels: setup (rescaling of f, g and ||f g^T||), the
// tolerance controller before each step, the residual-factor update and
// append after the inner solves, and the norm / stop test (Algorithm 1,
// eqs. (lradi_basic), (adi_resexact), Sec. 3.2).
//
// A batch of problems maps problem p to inner systems 2p (A side: W, Z) and
// 2p+1 (B side: T, Y).  Row kernels reuse the inner solver's row table.  In
// the Lyapunov case (B = A^T, C = M^T, g = f, equal shifts) system 2p+1 owns
// no workgroups and stays finished; the A side's factors stand for both.
#include "adi.h"
#include "controller.h"
#include "small.h"
#include "wavesmall.h"

namespace lradi {
namespace {

#define LRADI_DISPATCH_R2(rv, ...)         \
  switch (rv) {                            \
    case 1: { constexpr int RR = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int RR = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int RR = 3; __VA_ARGS__; } break; \
    case 4: { constexpr int RR = 4; __VA_ARGS__; } break; \
    case 5: { constexpr int RR = 5; __VA_ARGS__; } break; \
    case 6: { constexpr int RR = 6; __VA_ARGS__; } break; \
    case 7: { constexpr int RR = 7; __VA_ARGS__; } break; \
    case 8: { constexpr int RR = 8; __VA_ARGS__; } break; \
    default: break;                        \
  }

template <int NV>
__device__ inline void bsum(double (&v)[NV], double* lds, double* out) {
  constexpr int P2 = pow2c(NV);
  using RS = WaveRS<P2, 1>;
  static_assert(RS::NOUT == 1, "at most 64 values");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double w[P2];
#pragma unroll
  for (int k = 0; k < P2; ++k) w[k] = k < NV ? v[k] : 0.0;
  wave_reduce_scatter<P2, 1>(w, lane);
  const int idx = wave_rs_base<P2, 1>(lane);
  if ((lane & RS::DUP) == 0 && idx < NV) lds[wave * NV + idx] = w[0];
  __syncthreads();
  for (int k = threadIdx.x; k < NV; k += kTPB)
    out[k] = ((lds[k] + lds[NV + k]) + lds[2 * NV + k]) + lds[3 * NV + k];
  __syncthreads();
}

// fixed-order sum of partS rows at column offset off (P <= 64 values)
__device__ inline void reduce_rows(const double* partS, int nwg, int off, int P, double* red_lds,
                                   double* out) {
  const int t = threadIdx.x;
  const int groups = kTPB / P;
  const int p = t % P, g = t / P;
  double acc = 0.0;
  if (g < groups) {
    const double* X = partS + off + p;
    // sixteen independent sums keep sixteen loads in flight per thread (a
    // workgroup's partials sit kPS doubles apart, one line each)
    double a[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) a[u] = 0.0;
    int w = g;
    for (; w + 15 * groups < nwg; w += 16 * groups) {
#pragma unroll
      for (int u = 0; u < 16; ++u) a[u] += X[(size_t)(w + u * groups) * kPS];
    }
    for (; w < nwg; w += groups) a[0] += X[(size_t)w * kPS];
#pragma unroll
    for (int h = 8; h > 0; h >>= 1)
#pragma unroll
      for (int u = 0; u < h; ++u) a[u] += a[u + h];
    acc = a[0];
  }
  red_lds[t] = acc;
  __syncthreads();
  if (t < P) {
    double s = 0.0;
    for (int q = 0; q < groups; ++q) s += red_lds[q * P + t];
    out[t] = s;
  }
  __syncthreads();
}

struct RowC {
  int s, w, row0, row1;
};
__device__ inline RowC rowc(const SysDesc* d, const int2* rowmap) {
  const int2 sc = rowmap[blockIdx.x];
  const SysDesc& D = d[sc.x];
  RowC c;
  c.s = sc.x;
  c.w = sc.y;
  c.row0 = sc.y * D.rows_per_wg;
  c.row1 = min(D.n, c.row0 + D.rows_per_wg);
  return c;
}

// Gram X^T X of rows of X (n x R) into partS[w][off..]
template <int R>
__device__ inline void gram_self(const double* X, const RowC& c, double* lds, double* dst) {
  double g2[R * R];
#pragma unroll
  for (int e = 0; e < R * R; ++e) g2[e] = 0.0;
  for (int i = c.row0 + threadIdx.x; i < c.row1; i += kTPB) {
    double x[R];
#pragma unroll
    for (int q = 0; q < R; ++q) x[q] = X[(size_t)i * R + q];
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int q = 0; q < R; ++q) g2[a * R + q] += x[a] * x[q];
  }
  bsum<R * R>(g2, lds, dst);
}

// setup 1: partial f^T f (A side) / g^T g (B side)
__global__ __launch_bounds__(kTPB) void k_adi_setup_gram(const SysDesc* __restrict__ d,
                                                         const int2* __restrict__ rowmap,
                                                         const AdiDesc* __restrict__ ad) {
  __shared__ double lds[4 * 64];
  const RowC c = rowc(d, rowmap);
  const SysDesc& D = d[c.s];
  const AdiDesc& P = ad[c.s >> 1];
  if (!P.setup) return;
  const double* X = (c.s & 1) ? P.g : P.f;
  RowC cm = c;  // complex systems: f, g have the matrix's rows only
  if (D.cplx) cm.row1 = min(c.row1, D.nmat);
  LRADI_DISPATCH_R2(D.r, gram_self<RR>(X, cm, lds, D.partS + (size_t)c.w * kPS));
}

// Arm the inner systems of problem P for outer step C.k + 1: tolerances of
// Sec. 3.2 from (||w||, ||t||, u, v), the step's shifts, the solution slots
// z_{k+1}, y_{k+1}, and fresh inner control blocks (Algorithm 1 loop body).
__device__ inline void arm_step(const AdiDesc& P, AdiCtl& C, SysCtl& A, SysCtl& B) {
  CtlParams cp;
  cp.eps = C.eps;
  cp.delta_min = P.delta_min;
  cp.delta_max = P.delta_max;
  cp.xi = P.xi;
  cp.delta_fixed = P.delta_fixed;
  cp.rho = P.rho;
  cp.kmax = P.kmax;
  cp.selection = P.selection;
  cp.backlook = P.backlook;
  cp.paper_abs = P.paper_abs;
  cp.balance = P.rescale == 2;
  double dA, dB;
  ctl_tolerances(cp, C.k + 1, C.nw, C.nt, C.u, C.v, &dA, &dB);
  // one solve serves both sides of a Lyapunov problem: it must meet both
  if (P.sym) dA = dB = fmin(dA, dB);
  C.dA = dA;
  C.dB = dB;
  const int js = C.k % P.nshifts;
  SysCtl* sides[2] = {&A, &B};
  const size_t hz = P.cplx ? 2 : 1;  // stacked [re; im] blocks when complex
  for (int side = 0; side < (P.sym ? 1 : 2); ++side) {
    SysCtl& S = *sides[side];
    S.Z = side ? P.Yf + (size_t)C.k * hz * P.m * P.r : P.Zf + (size_t)C.k * hz * P.n * P.r;
    S.shift = side ? P.shiftsB[js] : P.shiftsA[js];
    S.shift_im = P.cplx ? (side ? P.shiftsB_im[js] : P.shiftsA_im[js]) : 0.0;
    S.delta = side ? dB : dA;
    S.phase = PH_CYCLE_END;
    S.first = 1;
    S.j = 0;
    S.ncols = 0;
    S.steps = 0;
    S.cycles = 0;
    S.status = IS_OK;
    S.breakdowns = 0;
    S.est = 0.0;
    S.rnorm = 0.0;
    S.r0 = 0.0;
  }
}

__device__ inline bool gram_finite(double x) { return x == x && x - x == 0.0; }

__device__ inline void mark_done(const AdiDesc& P, AdiCtl& C, SysCtl& A, SysCtl& B) {
  C.done = 1;
  A.phase = PH_FINISHED;
  B.phase = PH_FINISHED;
  if (P.host_done) __hip_atomic_store(P.host_done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// a problem's step is complete once both of its inner solves finished
__device__ inline bool step_ready(const AdiCtl& C, const SysCtl& A, const SysCtl& B) {
  return !C.done && A.phase == PH_FINISHED && B.phase == PH_FINISHED;
}

// setup 2: norms, rescaling factors, ||f g^T||, initial state, arm step 1
__global__ __launch_bounds__(kTPB) void k_adi_setup(const SysDesc* __restrict__ d,
                                                    const AdiDesc* __restrict__ ad,
                                                    AdiCtl* __restrict__ ac, SysCtl* __restrict__ ctl) {
  __shared__ double red_lds[kTPB];
  __shared__ double Gf[64], Gg[64];
  const int p = blockIdx.x;
  const AdiDesc& P = ad[p];
  if (!P.setup) return;
  const SysDesc& DA = d[2 * p];
  const SysDesc& DB = d[2 * p + 1];
  const int R = P.r;
  reduce_rows(DA.partS, DA.nwg, 0, R * R, red_lds, Gf);
  if (P.sym) {
    for (int e = threadIdx.x; e < R * R; e += kTPB) Gg[e] = Gf[e];
    __syncthreads();
  } else {
    reduce_rows(DB.partS, DB.nwg, 0, R * R, red_lds, Gg);
  }
  // ||f g^T||_2^2 = lambda_max(L^T (g^T g) L) with f^T f = L L^T (see the
  // step end)
  __shared__ double LF[64], MF[64];
  if (threadIdx.x == 0) {
    LRADI_SMALL_SWITCH(R, {
      double a[NN * NN];
      for (int e = 0; e < NN * NN; ++e) a[e] = Gf[e];
      psd_chol_lower_t<NN>(a);
      for (int e = 0; e < NN * NN; ++e) LF[e] = a[e];
    });
  }
  __syncthreads();
  {
    const int t = (int)threadIdx.x;
    if (t < R * R && t / R <= t % R) {
      const int i = t / R, j = t % R;
      double v = 0.0;
      LRADI_SMALL_SWITCH(R, v = prod_chol_entry_t<NN>(LF, Gg, i, j));
      MF[i * R + j] = v;
      MF[j * R + i] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    AdiCtl& C = ac[p];
    // a NaN or Inf in f or g shows in its Gram matrix; the eigenvalue
    // routines would turn it into a norm of 0 (fmax drops NaN), i.e. into
    // the exact solution X = 0, so it is caught here
    bool finite = true;
    for (int e = 0; e < R * R; ++e) finite = finite && gram_finite(Gf[e]) && gram_finite(Gg[e]);
    const double nf = sqrt(fmax(lambda_max_sym(Gf, R), 0.0));
    const double ng = sqrt(fmax(lambda_max_sym(Gg, R), 0.0));
    const double nfg = finite ? sqrt(fmax(lambda_max_sym(MF, R), 0.0)) : nan("");
    double sf = 1.0, sg = 1.0;
    if (P.rescale && nf > 0.0 && ng > 0.0) {
      sf = sqrt(ng / nf);
      sg = 1.0 / sf;
    }
    C.sf = sf;
    C.sg = sg;
    C.norm_fg = nfg;
    C.nw = nf * sf;
    C.nt = ng * sg;
    C.res = nfg;
    C.u = 0.0;
    C.v = 0.0;
    C.k = 0;
    C.winner = 0;
    C.status = LRADI_OK;
    C.eps = (P.eps_in > 0.0) ? P.eps_in : P.tol * nfg;
    C.done = 0;
    C.dA = 0.0;
    C.dB = 0.0;
    SysCtl& A = ctl[2 * p];
    SysCtl& B = ctl[2 * p + 1];
    if (!(nfg == nfg) || nfg - nfg != 0.0) {
      C.status = LRADI_ENAN;
      mark_done(P, C, A, B);
    } else if (nfg == 0.0) {
      mark_done(P, C, A, B);  // f g^T = 0: X = 0 is exact
    } else {
      arm_step(P, C, A, B);
    }
  }
}

// setup 3: W = sf f, T = sg g
__global__ __launch_bounds__(kTPB) void k_adi_init_wt(const SysDesc* __restrict__ d,
                                                      const int2* __restrict__ rowmap,
                                                      const AdiDesc* __restrict__ ad,
                                                      const AdiCtl* __restrict__ ac) {
  const RowC c = rowc(d, rowmap);
  const SysDesc& D = d[c.s];
  const int p = c.s >> 1;
  const AdiDesc& P = ad[p];
  if (!P.setup) return;
  const bool b = (c.s & 1) != 0;
  const double* X = b ? P.g : P.f;
  double* Y = b ? P.T : P.W;
  const double sc = b ? ac[p].sg : ac[p].sf;
  const size_t e1 = (size_t)c.row1 * D.r;
  // complex systems: the imaginary half of w_0 = f (t_0 = g) is zero
  const size_t ereal = (size_t)(D.cplx ? D.nmat : D.n) * D.r;
  for (size_t e = (size_t)c.row0 * D.r + threadIdx.x; e < e1; e += kTPB) Y[e] = e < ereal ? sc * X[e] : 0.0;
}

// complex form: W += gamma Z (A side) or T += conj(gamma) Y (B side) on the
// stacked blocks, local row i holding the real part at i and the imaginary
// part at nmat + i; partial Hermitian Grams of the new factor (S at 0, K at
// R^2) and of the new block (at 64 and 64 + R^2), S + i K = X^* X
template <int R>
__device__ inline void adi_update_rows_cplx(const SysDesc& D, double* Wt, const double* Zk, double gr,
                                            double gi, const RowC& c, double* lds, double* dst) {
  const int nm = D.nmat;
  double gw[2 * R * R], gz[2 * R * R];
#pragma unroll
  for (int e = 0; e < 2 * R * R; ++e) gw[e] = gz[e] = 0.0;
  const int i1 = min(c.row1, nm);
  for (int i = c.row0 + threadIdx.x; i < i1; i += kTPB) {
    double wr[R], wi[R], zr[R], zi[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      zr[q] = Zk[(size_t)i * R + q];
      zi[q] = Zk[(size_t)(nm + i) * R + q];
      wr[q] = Wt[(size_t)i * R + q] + (gr * zr[q] - gi * zi[q]);
      wi[q] = Wt[(size_t)(nm + i) * R + q] + (gr * zi[q] + gi * zr[q]);
      Wt[(size_t)i * R + q] = wr[q];
      Wt[(size_t)(nm + i) * R + q] = wi[q];
    }
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int q = 0; q < R; ++q) {
        gw[a * R + q] += wr[a] * wr[q] + wi[a] * wi[q];
        gw[R * R + a * R + q] += wr[a] * wi[q] - wi[a] * wr[q];
        gz[a * R + q] += zr[a] * zr[q] + zi[a] * zi[q];
        gz[R * R + a * R + q] += zr[a] * zi[q] - zi[a] * zr[q];
      }
  }
  bsum<2 * R * R>(gw, lds, dst);
  bsum<2 * R * R>(gz, lds, dst + 64);
}

// generalized equation (eq. (lradi_g)): W += gamma M Z with M's rows on the
// system's pattern, and the Gram of M Z in place of Z's for the gap
// recursion of eq. (upd_resgap)
template <int R>
__device__ inline void adi_update_rows_mass(const SysDesc& D, double* Wt, const double* Zk, double gamma,
                                            const RowC& c, double* lds, double* dst) {
  double g2[R * R], g3[R * R];
#pragma unroll
  for (int e = 0; e < R * R; ++e) g2[e] = g3[e] = 0.0;
  const int* __restrict__ rp = D.rowptr;
  const int* __restrict__ ci = D.colind;
  const double* __restrict__ mv = D.mval64;
  for (int i = c.row0 + threadIdx.x; i < c.row1; i += kTPB) {
    double mz[R];
#pragma unroll
    for (int q = 0; q < R; ++q) mz[q] = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const double a = mv[k];
      const double* z = Zk + (size_t)ci[k] * R;
#pragma unroll
      for (int q = 0; q < R; ++q) mz[q] += a * z[q];
    }
    double w[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      w[q] = Wt[(size_t)i * R + q] + gamma * mz[q];
      Wt[(size_t)i * R + q] = w[q];
    }
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int q = 0; q < R; ++q) {
        g2[a * R + q] += w[a] * w[q];
        g3[a * R + q] += mz[a] * mz[q];
      }
  }
  bsum<R * R>(g2, lds, dst);
  bsum<R * R>(g3, lds, dst + 64);
}

// after the inner solves: W += gamma Z (A side) or T += gamma Y (B side),
// partial Grams of the new factor (offset 0) and of the new block (offset 64)
template <int R>
__device__ inline void adi_update_rows(const SysDesc& D, double* Wt, const double* Zk, double gamma,
                                       const RowC& c, double* lds, double* dst) {
  if (D.mval64) {
    adi_update_rows_mass<R>(D, Wt, Zk, gamma, c, lds, dst);
    return;
  }
  double g2[R * R];
#pragma unroll
  for (int e = 0; e < R * R; ++e) g2[e] = 0.0;
  for (int i = c.row0 + threadIdx.x; i < c.row1; i += kTPB) {
    double w[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      w[q] = Wt[(size_t)i * R + q] + gamma * Zk[(size_t)i * R + q];
      Wt[(size_t)i * R + q] = w[q];
    }
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int q = 0; q < R; ++q) g2[a * R + q] += w[a] * w[q];
  }
  bsum<R * R>(g2, lds, dst);
  gram_self<R>(Zk, c, lds, dst + 64);
}

__global__ __launch_bounds__(kTPB) void k_adi_update(const SysDesc* __restrict__ d,
                                                     const int2* __restrict__ rowmap,
                                                     const AdiDesc* __restrict__ ad,
                                                     const AdiCtl* __restrict__ ac,
                                                     const SysCtl* __restrict__ ctl) {
  __shared__ double lds[4 * 64];
  const RowC c = rowc(d, rowmap);
  const SysDesc& D = d[c.s];
  const int p = c.s >> 1;
  if (!step_ready(ac[p], ctl[2 * p], ctl[2 * p + 1])) return;
  const AdiDesc& P = ad[p];
  const int js = ac[p].k % P.nshifts;
  const double gamma = -(P.shiftsA[js] + P.shiftsB[js]);
  double* Wt = (c.s & 1) ? P.T : P.W;
  const double* Zk = ctl[c.s].Z;
  if (P.cplx) {
    // gamma = -(pA + conj(pB)); the B side adds conj(gamma) (Algorithm 1)
    const double gi = -(P.shiftsA_im[js] - P.shiftsB_im[js]);
    const double gis = (c.s & 1) ? -gi : gi;
    LRADI_DISPATCH_R2(D.r, if constexpr (RR <= 4) adi_update_rows_cplx<RR>(D, Wt, Zk, gamma, gis, c, lds, D.partS + (size_t)c.w * kPS));
    return;
  }
  LRADI_DISPATCH_R2(D.r, adi_update_rows<RR>(D, Wt, Zk, gamma, c, lds, D.partS + (size_t)c.w * kPS));
}

// norms, gap estimates u, v (eq. (upd_resgap)), history row, stop test; then
// either finish the problem or arm its next step
__global__ __launch_bounds__(kTPB) void k_adi_step_end(const SysDesc* __restrict__ d,
                                                       const AdiDesc* __restrict__ ad,
                                                       AdiCtl* __restrict__ ac, SysCtl* __restrict__ ctl) {
  __shared__ double red_lds[kTPB];
  __shared__ double GW[64], GZ[64], GT[64], GY[64];
  __shared__ double nrm[5];
  const int p = blockIdx.x;
  const AdiDesc& P = ad[p];
  AdiCtl& C = ac[p];
  SysCtl& A = ctl[2 * p];
  SysCtl& B = ctl[2 * p + 1];
  if (!step_ready(C, A, B)) return;
  const SysDesc& DA = d[2 * p];
  const SysDesc& DB = d[2 * p + 1];
  const int R = P.r;
  // complex form: each partial holds a Hermitian Gram S + i K (S at 0, K at
  // R^2); its real form [S -K; K S] (2R x 2R, symmetric) has the same
  // eigenvalues twice, and the real forms multiply as the complex matrices
  // do, so every norm below runs unchanged on the 2R x 2R real forms
  const int PG = P.cplx ? 2 * R * R : R * R;
  const int NE = P.cplx ? 2 * R : R;
  reduce_rows(DA.partS, DA.nwg, 0, PG, red_lds, GW);
  reduce_rows(DA.partS, DA.nwg, 64, PG, red_lds, GZ);
  if (P.sym) {  // t_k = w_k, y_k = z_k
    for (int e = threadIdx.x; e < PG; e += kTPB) {
      GT[e] = GW[e];
      GY[e] = GZ[e];
    }
    __syncthreads();
  } else {
    reduce_rows(DB.partS, DB.nwg, 0, PG, red_lds, GT);
    reduce_rows(DB.partS, DB.nwg, 64, PG, red_lds, GY);
  }
  bool finite = true;
  for (int e = 0; e < PG; ++e)
    finite = finite && gram_finite(GW[e]) && gram_finite(GT[e]) && gram_finite(GZ[e]) && gram_finite(GY[e]);
  if (P.cplx) {
    __shared__ double EW[64], EZ[64], ET[64], EY[64];
    for (int e = threadIdx.x; e < NE * NE; e += kTPB) {
      const int a = e / NE, b = e % NE, ha = a / R, hb = b / R, o = (a % R) * R + b % R;
      const double sg = (ha == hb) ? 0.0 : (ha == 0 ? -1.0 : 1.0);
      EW[e] = sg == 0.0 ? GW[o] : sg * GW[R * R + o];
      EZ[e] = sg == 0.0 ? GZ[o] : sg * GZ[R * R + o];
      ET[e] = sg == 0.0 ? GT[o] : sg * GT[R * R + o];
      EY[e] = sg == 0.0 ? GY[o] : sg * GY[R * R + o];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NE * NE; e += kTPB) {
      GW[e] = EW[e];
      GZ[e] = EZ[e];
      GT[e] = ET[e];
      GY[e] = EY[e];
    }
    __syncthreads();
  }
  // ||w t^T||_2^2 = lambda_max(L^T (T^T T) L) with W^T W = L L^T: one thread
  // factors, the second wavefront forms the symmetric matrix entry by entry
  // (registers for one small matrix per lane, not three)
  __shared__ double LW[64], MP[64];
  if (threadIdx.x == 64) {
    LRADI_SMALL_SWITCH(NE, {
      double a[NN * NN];
      for (int e = 0; e < NN * NN; ++e) a[e] = GW[e];
      psd_chol_lower_t<NN>(a);
      for (int e = 0; e < NN * NN; ++e) LW[e] = a[e];
    });
  }
  __syncthreads();
  {
    const int t = (int)threadIdx.x - 64;
    if (t >= 0 && t < NE * NE && t / NE <= t % NE) {
      const int i = t / NE, j = t % NE;
      double v = 0.0;
      LRADI_SMALL_SWITCH(NE, v = prod_chol_entry_t<NN>(LW, GT, i, j));
      MP[i * NE + j] = v;
      MP[j * NE + i] = v;
    }
  }
  __syncthreads();
  // the five small eigenvalue problems run concurrently: the four Grams on
  // four 16-lane groups of the first wavefront, the product's symmetric form
  // on the whole second wavefront (each with its bisection spread over its
  // lanes)
  if (threadIdx.x < 64) {
    const int g = threadIdx.x / 16, l = threadIdx.x % 16;
    const double* G = g == 0 ? GW : g == 1 ? GT : g == 2 ? GZ : GY;
    const double v = sqrt(fmax(lambda_max_sym_lanes<16>(G, NE, l, g * 16), 0.0));
    if (l == 0) nrm[g] = v;
  } else if (threadIdx.x < 128) {
    const double v = sqrt(fmax(lambda_max_sym_lanes<64>(MP, NE, threadIdx.x - 64, 0), 0.0));
    if (threadIdx.x == 64) nrm[4] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int k = C.k;
    const int js = k % P.nshifts;
    const double gamma = -(P.shiftsA[js] + P.shiftsB[js]);
    const double gamma_im = P.cplx ? -(P.shiftsA_im[js] - P.shiftsB_im[js]) : 0.0;
    const double nw = nrm[0], nt = nrm[1], nz = nrm[2], ny = nrm[3], res = nrm[4];
    const double rA = A.rnorm, rB = P.sym ? A.rnorm : B.rnorm;
    double u = C.u, v = C.v;
    // eq. (upd_resgap) takes |gamma_k|, the modulus for complex shifts
    ctl_update_gap(&u, &v, P.cplx ? hypot(gamma, gamma_im) : gamma, nz, ny, rA, rB);
    double* h = P.hist + (size_t)k * kHistCols;
    const double nfg = C.norm_fg;
    h[0] = k + 1;
    h[1] = C.res / nfg;
    h[2] = C.dA;
    h[3] = C.dB;
    h[4] = rA;
    h[5] = rB;
    h[6] = A.steps;
    h[7] = P.sym ? 0 : B.steps;
    h[8] = u;
    h[9] = v;
    h[10] = C.nw;
    h[11] = C.nt;
    h[12] = nz;
    h[13] = ny;
    h[14] = gamma;
    h[15] = res / nfg;
    if (P.cplx) {
      P.gam[2 * k] = gamma;
      P.gam[2 * k + 1] = gamma_im;
    } else {
      P.gam[k] = gamma;
    }
    C.u = u;
    C.v = v;
    C.nw = nw;
    C.nt = nt;
    C.res = res;
    C.k = k + 1;
    if (A.status == IS_CAP || B.status == IS_CAP) C.winner = 1;
    const bool bad = !finite || !(res == res) || res - res != 0.0 || A.status == IS_NAN || B.status == IS_NAN;
    if (bad) {
      C.status = LRADI_ENAN;
      mark_done(P, C, A, B);
    } else if (res < P.tol * nfg) {
      mark_done(P, C, A, B);
    } else if (C.k >= P.kmax) {
      C.status = LRADI_WNOCONV;
      mark_done(P, C, A, B);
    } else {
      arm_step(P, C, A, B);
    }
  }
}

}  // namespace

int adi_launch_setup(hipStream_t st, const Batch& b, const AdiDesc* ad, AdiCtl* ac, int nprob) {
  hipLaunchKernelGGL(k_adi_setup_gram, dim3(b.rowgrid), dim3(kTPB), 0, st, b.d, b.rowmap, ad);
  hipLaunchKernelGGL(k_adi_setup, dim3(nprob), dim3(kTPB), 0, st, b.d, ad, ac, b.ctl);
  hipLaunchKernelGGL(k_adi_init_wt, dim3(b.rowgrid), dim3(kTPB), 0, st, b.d, b.rowmap, ad, ac);
  LRADI_HIP(hipGetLastError());
  return LRADI_OK;
}

int adi_launch_step_end(hipStream_t st, const Batch& b, const AdiDesc* ad, AdiCtl* ac, int nprob) {
  hipLaunchKernelGGL(k_adi_update, dim3(b.rowgrid), dim3(kTPB), 0, st, b.d, b.rowmap, ad, ac, b.ctl);
  hipLaunchKernelGGL(k_adi_step_end, dim3(nprob), dim3(kTPB), 0, st, b.d, ad, ac, b.ctl);
  LRADI_HIP(hipGetLastError());
  return LRADI_OK;
}

}  // namespace lradi
