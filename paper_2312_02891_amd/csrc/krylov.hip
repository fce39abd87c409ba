// Batched block GMRES(m) with FP64 iterative refinement for the shifted
// inner systems (A + s I) Z = W of the inexact LR-ADI iteration
// (Algorithm 1, eq. (gfadi_incsolves)).
//
// Every kernel serves all systems of a batch at once: row kernels map each
// workgroup to (system, row chunk) through a table, per-system kernels use one
// workgroup per system.  Each system carries a device-side phase, and a kernel
// returns at once for systems in a phase it does not serve, so the host can
// issue the same launch sequence ("tick") over and over without reading
// anything back per step.
//
// One Arnoldi step for the block V_j (n x r):
//   [P_j = M V_j                               optional right preconditioner]
//   U = (A + s I) V_j   (or (A + s I) P_j)     SpMM, basis precision
//   H1 = V^T U,  U -= V H1                     block classical Gram-Schmidt
//   H2 = V^T U,  U -= V H2                     ... repeated once (CGS2)
//   U = V_{j+1} S with S = S2 S1               CholQR2 (two Cholesky QR passes)
//   column block [H1 + H2; S] enters the incremental QR of the block
//   Hessenberg matrix (one 2r x 2r orthogonal factor per column block), the
//   rotated right-hand side gives the residual estimate.
// At the end of a cycle: Z += V y (P y when preconditioned),
// R = W - (A + s I) Z in FP64, ||R||_2 from
// the r x r Gram matrix, then stop or restart from R.
#include <cstdio>

#include "internal.h"
#include "small.h"
#include "wavesmall.h"

namespace lradi {
namespace {

#define LRADI_DISPATCH_R(rv, ...)          \
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

// RF > 0: the kernel is instantiated for that block width only (batches whose
// systems share r); RF == 0: dispatch on the system's r at run time.
#define LRADI_RSEL(RF, rv, ...)                               \
  if constexpr ((RF) > 0) {                                   \
    constexpr int RR = (RF);                                  \
    __VA_ARGS__;                                              \
  } else {                                                    \
    LRADI_DISPATCH_R(rv, __VA_ARGS__);                        \
  }

struct RowCtx {
  int s, w, row0, row1;
};

__device__ inline RowCtx row_ctx(const SysDesc* d, const int2* rowmap) {
  const int2 sc = rowmap[blockIdx.x];
  const SysDesc& D = d[sc.x];
  RowCtx c;
  c.s = sc.x;
  c.w = sc.y;
  c.row0 = sc.y * D.rows_per_wg;
  c.row1 = min(D.n, c.row0 + D.rows_per_wg);
  return c;
}

// one chunk (values C0 .. C0+N-1 of v) of block_sum_store_sym's
// reduce-scatter, into lds[wave * NV + C0 + ...]
template <int NV, int C0, int N>
__device__ inline void block_sum_chunk(const double (&v)[NV], double* lds) {
  constexpr int P2 = pow2c(N);
  using RS = WaveRS<P2, 1>;
  static_assert(RS::NOUT == 1, "at most 64 values");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double w[P2];
#pragma unroll
  for (int k = 0; k < P2; ++k) w[k] = k < N ? v[C0 + k] : 0.0;
  wave_reduce_scatter<P2, 1>(w, lane);
  const int idx = wave_rs_base<P2, 1>(lane);
  if ((lane & RS::DUP) == 0 && idx < N) lds[wave * NV + C0 + idx] = w[0];
}

// The Gram of a block's R columns from its packed upper triangle: v holds
// entry (a, q), a <= q, at a R - a (a - 1) / 2 + q - a.  Sums the packed
// values over the 256 threads in a fixed order (at most 32 values per
// reduce-scatter, so that the padded copies stay small) and stores the full
// symmetric R x R matrix to out.  lds needs 4 R (R + 1) / 2 doubles.
template <int R>
__device__ inline void block_sum_store_sym(double (&v)[R * (R + 1) / 2], double* lds, double* out) {
  constexpr int NV = R * (R + 1) / 2;
  constexpr int N0 = NV < 32 ? NV : 32;
  block_sum_chunk<NV, 0, N0>(v, lds);
  if constexpr (NV > N0) block_sum_chunk<NV, N0, NV - N0>(v, lds);
  __syncthreads();
  for (int k = threadIdx.x; k < NV; k += kTPB) {
    int a = 0, rem = k;
    while (rem >= R - a) {
      rem -= R - a;
      ++a;
    }
    const int q = a + rem;
    const double s = ((lds[k] + lds[NV + k]) + lds[2 * NV + k]) + lds[3 * NV + k];
    out[a * R + q] = s;
    out[q * R + a] = s;
  }
  __syncthreads();
}

// Sum NV per-thread values over the 256 threads of the workgroup in a fixed
// order and store the totals to out[0..NV).  lds needs 4*NV doubles.
template <int NV>
__device__ inline void block_sum_store(double (&v)[NV], double* lds, double* out) {
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

// Sum the per-workgroup r x r (P values) partial rows partS[w][0..P) over
// w in a fixed order with a 256-thread workgroup; result in out (shared).
// Each thread keeps sixteen independent partial sums so that its loads are in
// flight together.
__device__ inline void reduce_small(const double* src, int nwg, int P, double* red_lds, double* out) {
  const int t = threadIdx.x;
  const int groups = kTPB / P;  // P <= 64, so groups >= 4
  const int p = t % P, g = t / P;
  double acc = 0.0;
  if (g < groups) {
    const double* X = src + p;
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

__device__ inline void reduce_partS(const SysDesc& D, int P, double* red_lds, double* out) {
  reduce_small(D.partS, D.nwg, P, red_lds, out);
}

// ---------------------------------------------------------------------------
// 1. U = (A + s I) V_j  (PH_ARNOLDI)   or   U = R rounded  (PH_RESTART)
//
// One tile = kTPB / RL consecutive rows, a wavefront 64 / RL of them (two
// slices of the sliced ELL layout for RL = 1, one for RL = 2, half of one
// for RL = 4).  RL lanes work on each row, each for R / RL columns, and walk
// the slice's slots SU at a time with all gathers of a group in flight
// together; the column and value loads of a slot are contiguous across the
// slice's rows.  A row's terms are summed in its CSR order (padding slots
// add exact zeros), so the result does not depend on the tiling.
template <typename T>
struct SpmmUnroll {
  static constexpr int v = sizeof(T) == 8 ? 4 : 8;
};

template <bool NT, typename V>
__device__ inline V sell_ld(const V* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// Rows r0 .. r0 + kTPB / RL - 1 of Y = (A + shift M) X (M = I: diag).
// mass: the blocks carry M's values, the coefficient then is val + shift mv.
// Xc (nullable): complex systems' other half of the stacked block, added
// with coefficient cs (the imaginary shift's coupling, -s_im for the real
// rows and +s_im for the imaginary ones).  NT: matrix loads and output
// stores with the nontemporal hint.
template <typename T, int R, int RL, bool NT>
__device__ inline void sell_tile(int n, const int* __restrict__ sslot, const unsigned char* __restrict__ blk,
                                 bool mass, T shift, const T* __restrict__ X, T* __restrict__ Y, int r0,
                                 const T* __restrict__ Xc = nullptr, T cs = T(0)) {
  constexpr int RC = R / RL;
  constexpr int SU = SpmmUnroll<T>::v;
  const int lane = (int)threadIdx.x % 64;
  const int rw = r0 + ((int)threadIdx.x / 64) * (64 / RL);  // first row of this wavefront
  if (rw >= n) return;                                       // uniform per wavefront
  const int i = rw + lane / RL;
  const int nsl = (n + kSellH - 1) / kSellH;
  const int s = min(i / kSellH, nsl - 1);  // lanes past the last slice read its entries, store nothing
  const int b0 = sslot[s];
  const int w = sslot[s + 1] - b0;
  int wmax = w;
  if constexpr (RL == 1) wmax = max(w, __shfl_xor(w, 32));  // a wavefront spans two slices
  // this lane's row inside its slice: slot u's column at cp[u * cst], its
  // value at vp[u * vst] (M's at mp[u * vst])
  const int sb = sell_block_bytes((int)sizeof(T), mass);
  const unsigned char* base = blk + (size_t)b0 * sb;
  const int l = i % kSellH;
  const int* cp = reinterpret_cast<const int*>(base) + l;
  const T* vp = reinterpret_cast<const T*>(base + kSellH * 4) + l;
  const T* mp = reinterpret_cast<const T*>(base + kSellH * (4 + sizeof(T))) + l;
  const int cst = sb / 4, vst = sb / (int)sizeof(T);
  const int q0 = (lane % RL) * RC;
  T acc[RC];
#pragma unroll
  for (int q = 0; q < RC; ++q) acc[q] = T(0);
  for (int u = 0; u < wmax; u += SU) {
    int col[SU];
    T a[SU];
#pragma unroll
    for (int j = 0; j < SU; ++j) {
      const int uu = min(u + j, w - 1);
      col[j] = sell_ld<NT>(cp + uu * cst);
      T c = sell_ld<NT>(vp + uu * vst);
      if (mass) c = c + shift * sell_ld<NT>(mp + uu * vst);
      a[j] = c * (T)(u + j < w);
    }
    T xv[SU][RC];
#pragma unroll
    for (int j = 0; j < SU; ++j) {
      const T* x = X + (size_t)col[j] * R + q0;
#pragma unroll
      for (int q = 0; q < RC; ++q) xv[j][q] = x[q];
    }
#pragma unroll
    for (int j = 0; j < SU; ++j)
#pragma unroll
      for (int q = 0; q < RC; ++q) acc[q] += a[j] * xv[j][q];
  }
  if (i >= n) return;
  T out[RC];
  const T* xi = X + (size_t)i * R + q0;
  if (Xc) {
    const T* xc = Xc + (size_t)i * R + q0;
#pragma unroll
    for (int q = 0; q < RC; ++q) out[q] = (acc[q] + shift * xi[q]) + cs * xc[q];
  } else if (!mass) {
#pragma unroll
    for (int q = 0; q < RC; ++q) out[q] = acc[q] + shift * xi[q];
  } else {
#pragma unroll
    for (int q = 0; q < RC; ++q) out[q] = acc[q];
  }
  T* y = Y + (size_t)i * R + q0;
#pragma unroll
  for (int q = 0; q < RC; ++q) {
    if constexpr (NT) __builtin_nontemporal_store(out[q], y + q);
    else y[q] = out[q];
  }
}

// RL lanes per row; the kernel for group RL serves the systems whose tiling
// uses RL (RF > 0: all systems have r = RF; RF == 0: r read at run time).
// One workgroup per spmap entry (the host lists the entries in XCD bands).
template <typename T, int RF, int RL>
__global__ __launch_bounds__(kTPB) void k_spmm_arn(const SysDesc* __restrict__ d,
                                                   const SysCtl* __restrict__ ctl,
                                                   const int2* __restrict__ spmap,
                                                   unsigned long long* __restrict__ prof, int only) {
  const int2 e = spmap[blockIdx.x];
  const SysDesc& D = d[e.x];
  const int ph = ctl[e.x].phase;
  if (only >= 0 && ph != only) return;
  // complex systems: the tiles of each half of the stacked block apart
  // (tile e.y of th per half), local rows r0.. of A in that half
  const int tr = spmm_tile_rows(RL);
  const int th = D.cplx ? (D.nmat + tr - 1) / tr : 0;
  const int half = (D.cplx && e.y >= th) ? 1 : 0;
  const int r0 = (e.y - half * th) * tr;
  const size_t hoff = (size_t)half * D.nmat * D.r;
  T* U = static_cast<T*>(D.U);
  if (ph == PH_RESTART) {
    const size_t e1 = hoff + (size_t)min(D.cplx ? D.nmat : D.n, r0 + tr) * D.r;
    for (size_t q = hoff + (size_t)r0 * D.r + threadIdx.x; q < e1; q += kTPB) U[q] = (T)D.R[q];
    return;
  }
  if (ph != PH_ARNOLDI) return;
  // right preconditioning multiplies P_j = M V_j instead of V_j
  const T* Vj = static_cast<const T*>(D.rbrows ? D.P : D.V) + (size_t)ctl[e.x].j * D.n * D.r;
  const T sh = (T)ctl[e.x].shift;
  if (prof && e.y == 0 && threadIdx.x == 0) {
    // each nonzero's value (and M's value) and column index + input block +
    // output block (a complex system reads A once per half)
    const unsigned long long halves = D.cplx ? 2 : 1;
    const unsigned long long per_nz = sizeof(T) * (D.mvalT ? 2 : 1) + 4;
    const unsigned long long bytes = halves * (unsigned long long)D.nnz * per_nz + 2ull * sizeof(T) * D.n * D.r;
    atomicAdd(prof + LRADI_PROF_SPMM, bytes);
  }
  const bool mass = D.mvalT != nullptr;
  if (D.cplx) {
    const T si = (T)ctl[e.x].shift_im;
    const T* Xc = Vj + (size_t)(1 - half) * D.nmat * D.r;
    LRADI_RSEL(RF, D.r, if constexpr (RR % RL == 0) sell_tile<T, RR, RL, false>(D.nmat, D.sslot, D.sblk, false, sh, Vj + hoff, U + hoff, r0, Xc, half ? si : -si));
    return;
  }
  LRADI_RSEL(RF, D.r, if constexpr (RR % RL == 0) sell_tile<T, RR, RL, false>(D.n, D.sslot, D.sblk, mass, sh, Vj, U, r0));
}

// ---------------------------------------------------------------------------
// 0. Right preconditioner P_j = M V_j before the shifted product
//    (PH_ARNOLDI, systems with rbrows): red-black ILU(0) of S = A + s I,
//    S = [D_r E; F D_b] with the rows 2-coloured (every off-diagonal entry
//    joins a red and a black row), T = D_b - F D_r^{-1} E:
//      fwd    (black)  y = v_b - F D_r^{-1} v_r, 1/diag(T), z = y / diag(T)
//      sweep  (black)  z <- (y - T_off z) / diag(T)        (sweeps times)
//      back   (red)    z_r = D_r^{-1} (v_r - E z)
//    T_off (T without its diagonal, the two-hop black couplings) is built
//    explicitly once per inner solve, so a sweep is one one-hop launch.  A
//    workgroup's row chunk indexes the colour-ordered row list; the black
//    iterates alternate between P_j and a scratch block.  All gathers of a
//    row are issued together (clamped indices, selected contributions), and
//    each row sums its terms in a fixed order.
template <typename T>
struct RbCtx {
  const int* ci;  // slot-major colour-position table (rbw slots)
  const T* val;
  const T* tv;
  const T* dg;
  const T* ms;    // pencils: M's row sums, else null (weight 1)
  int w, n;
  T sh;
};

// diagonal of the matrix the preconditioner factors: a_jj + s, or
// a_jj + s (M 1)_j for a pencil
template <typename T>
__device__ inline T rb_dsh(const RbCtx<T>& x, int j) {
  return x.dg[j] + x.sh * (x.ms ? x.ms[j] : T(1));
}

template <typename T>
__device__ inline RbCtx<T> rb_ctx(const SysDesc& D, double shift) {
  RbCtx<T> x;
  x.ci = D.ellci;
  x.val = static_cast<const T*>(D.ellvalT);
  x.tv = static_cast<const T*>(D.elltvT);
  x.dg = static_cast<const T*>(D.diagT);
  x.ms = static_cast<const T*>(D.msT);
  x.w = D.rbw;
  x.n = D.n;
  x.sh = (T)shift;
  return x;
}

// gathers in flight per row: eight entries for narrow blocks, six (a 3-D
// Schur row's 18 couplings in three groups) for wide ones, three for r = 7,
// whose rows take one lane each (seven values per gather: six in flight
// needed 248 VGPRs, and kernels serving mixed widths inherit the widest
// variant's count)
template <int R>
struct RbUnroll {
  static constexpr int v = R == 7 ? 3 : R >= 5 ? 6 : 8;
};

// lanes that share one row in the stages of one sweep launch: each owns
// R / L consecutive columns, at least 16 bytes of every gathered row
template <typename T, int R>
struct RbLanes {
  static constexpr int v = (R % 4 == 0 && R * (int)sizeof(T) >= 64) ? 4
                           : (R % 2 == 0 && R * (int)sizeof(T) >= 32) ? 2 : 1;
};

// acc[q] += sum over the off-diagonal entries of row i (colour position p)
// of a_ik X[k][q0 + q], q < RQ; unused slots (col == i) are skipped by
// selection
template <typename T, int R, int RQ = R>
__device__ inline void rb_gather(const RbCtx<T>& x, int p, int i, const T* __restrict__ X, int q0,
                                 T (&acc)[RQ]) {
  constexpr int kRbUnroll = RbUnroll<R>::v;
  for (int u0 = 0; u0 < x.w; u0 += kRbUnroll) {
    int col[kRbUnroll];
    T a[kRbUnroll];
    bool ok[kRbUnroll];
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u) {
      const size_t e = (size_t)min(u0 + u, x.w - 1) * x.n + p;
      col[u] = x.ci[e];
      a[u] = x.val[e];
      ok[u] = (u0 + u < x.w) && col[u] != i;
    }
    T xv[kRbUnroll][RQ];
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u)
#pragma unroll
      for (int q = 0; q < RQ; ++q) xv[u][q] = X[(size_t)col[u] * R + q0 + q];
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u)
#pragma unroll
      for (int q = 0; q < RQ; ++q) acc[q] = ok[u] ? acc[q] + a[u] * xv[u][q] : acc[q];
  }
}

// black row i (position p): y = v_i - sum_j a_ij v_j / (d_j + s),
// diag(T)_i = d_i + s - sum_j a_ij a_ji / (d_j + s)
// (columns q0 .. q0 + RQ - 1 of y; td in full)
template <typename T, int R, int RQ = R>
__device__ inline void rb_black_fwd(const RbCtx<T>& x, int p, int i, const T* __restrict__ V, int q0,
                                    T (&y)[RQ], T& td) {
#pragma unroll
  for (int q = 0; q < RQ; ++q) y[q] = V[(size_t)i * R + q0 + q];
  td = rb_dsh(x, i);
  constexpr int kRbUnroll = RbUnroll<R>::v;
  for (int u0 = 0; u0 < x.w; u0 += kRbUnroll) {
    int col[kRbUnroll];
    T a[kRbUnroll], t[kRbUnroll], dj[kRbUnroll];
    bool ok[kRbUnroll];
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u) {
      const size_t e = (size_t)min(u0 + u, x.w - 1) * x.n + p;
      col[u] = x.ci[e];
      a[u] = x.val[e];
      t[u] = x.tv[e];
      ok[u] = (u0 + u < x.w) && col[u] != i;
    }
    T xv[kRbUnroll][RQ];
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u) {
      dj[u] = rb_dsh(x, col[u]);
#pragma unroll
      for (int q = 0; q < RQ; ++q) xv[u][q] = V[(size_t)col[u] * R + q0 + q];
    }
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u) {
      const T wgt = a[u] / dj[u];
      td = ok[u] ? td - wgt * t[u] : td;
#pragma unroll
      for (int q = 0; q < RQ; ++q) y[q] = ok[u] ? y[q] - wgt * xv[u][q] : y[q];
    }
  }
}

// diag(T)_i of black row i (colour position p), the forward stage's formula
template <typename T>
__device__ inline T rb_tdiag(const RbCtx<T>& x, int p, int i) {
  T td = rb_dsh(x, i);
  for (int u = 0; u < x.w; ++u) {
    const size_t e = (size_t)u * x.n + p;
    const int j = x.ci[e];
    if (j == i) continue;  // unused slot
    const T wgt = x.val[e] / rb_dsh(x, j);
    td = td - wgt * x.tv[e];
  }
  return td;
}

// Chebyshev steps on T z = y (the Golub-Varga semi-iterative method on the
// Jacobi splitting, J = I - diag(T)^{-1} T).  With J's spectrum real and in
// [lo, hi], hi < 1: the extrapolated step G x + gamma c, G = gamma J +
// (1 - gamma) I, c = diag(T)^{-1} y, gamma = 2 / (2 - lo - hi), has spectral
// radius sigma = (hi - lo) / (2 - lo - hi); from x_0 = 0, x_1 = gamma c and
// x_{k+1} = omega_{k+1} (G x_k + gamma c - x_{k-1}) + x_{k-1}, omega_2 =
// 2 / (2 - sigma^2), omega_{k+1} = 1 / (1 - sigma^2 omega_k / 4).  cb holds
// hi and -lo (SM_CHEB); gamma 0 means no dominance (hi >= 1): Jacobi steps.
__device__ inline double cheb_gamma(const double* cb) {
  const double hi = cb[0], lo = -cb[1];
  return hi < 1.0 ? 2.0 / (2.0 - lo - hi) : 0.0;
}

__device__ inline void cheb_table(double* cb, int k) {
  const double g = cheb_gamma(cb);
  cb[kChebGamma] = g;
  if (g == 0.0) return;
  const double hi = cb[0], lo = -cb[1];
  const double sg = (hi - lo) / (2.0 - lo - hi), s2 = sg * sg;
  double om = 0.0;
  for (int t = 1; t <= k; ++t) {
    om = t == 1 ? 2.0 / (2.0 - s2) : 1.0 / (1.0 - s2 * om / 4.0);
    cb[kChebOmega + t - 1] = om;
  }
}

// T's off-diagonal values of black position pb (row i, colour position p)
// for the current shift: slot q (column l) = -sum over the red neighbours j
// of i that neighbour l of a_ij a_jl / (d_j + s), walking i's and then j's
// slot tables in order (once per inner solve: the shift is fixed)
template <typename T>
__device__ inline void rb_build_t(const SysDesc& D, const RbCtx<T>& x, int p, int pb, int nb, int i) {
  T* tv = static_cast<T*>(D.t2val);
  for (int q = 0; q < D.t2w; ++q) tv[(size_t)q * nb + pb] = T(0);
  // rows of up to kT2Reg slots find a column's slot by comparing against
  // their columns held in registers, wider rows by reading the table
  constexpr int kT2Reg = 32;
  const bool reg = D.t2w <= kT2Reg;
  int cols[kT2Reg];
#pragma unroll
  for (int q = 0; q < kT2Reg; ++q) cols[q] = (reg && q < D.t2w) ? D.t2ci[(size_t)q * nb + pb] : -1;
  for (int u = 0; u < x.w; ++u) {
    const size_t e = (size_t)u * x.n + p;
    const int j = x.ci[e];
    if (j == i) continue;  // unused slot
    const T wj = x.val[e] / rb_dsh(x, j);
    const int pj = D.rbpos[j];
    for (int u2 = 0; u2 < x.w; ++u2) {
      const size_t e2 = (size_t)u2 * x.n + pj;
      const int l = x.ci[e2];
      if (l == j || l == i) continue;
      const int pl = D.rbpos[l] - D.nred;  // T's columns are black positions
      int slot = -1;
      if (reg) {
#pragma unroll
        for (int q = 0; q < kT2Reg; ++q) slot = (cols[q] == pl) ? q : slot;
      } else {
        for (int q = 0; q < D.t2w && slot < 0; ++q)
          if (D.t2ci[(size_t)q * nb + pb] == pl) slot = q;
      }
      if (slot >= 0) tv[(size_t)slot * nb + pb] -= wj * x.val[e2];
    }
  }
}

// acc = y_pb - sum_u T(pb, col_u) src(col_u) over T's off-diagonal slots of
// black position pb, with slot u's column at cols[u * cstride + crow] and
// unused slots (col == self) skipped; the one arithmetic of every Jacobi
// sweep, whichever table and source the columns refer to
// (columns q0 .. q0 + RQ - 1)
template <typename T, int R, typename Src, int RQ = R>
__device__ inline void rb_sweep_acc(const SysDesc& D, int pb, int nb, const int* __restrict__ cols, int cstride,
                                    int crow, int self, const Src& src, int q0, T (&acc)[RQ]) {
  const T* tv = static_cast<const T*>(D.t2val);
  const T* Y = static_cast<const T*>(D.Yb);
#pragma unroll
  for (int q = 0; q < RQ; ++q) acc[q] = Y[(size_t)pb * R + q0 + q];
  constexpr int kRbUnroll = RbUnroll<R>::v;
  for (int u0 = 0; u0 < D.t2w; u0 += kRbUnroll) {
    int col[kRbUnroll];
    T a[kRbUnroll];
    bool ok[kRbUnroll];
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u) {
      const int slot = min(u0 + u, D.t2w - 1);
      col[u] = cols[(size_t)slot * cstride + crow];
      a[u] = tv[(size_t)slot * nb + pb];
      ok[u] = (u0 + u < D.t2w) && col[u] != self;
    }
    T xv[kRbUnroll][RQ];
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u)
#pragma unroll
      for (int q = 0; q < RQ; ++q) xv[u][q] = src(col[u], q0 + q);
#pragma unroll
    for (int u = 0; u < kRbUnroll; ++u)
#pragma unroll
      for (int q = 0; q < RQ; ++q) acc[q] = ok[u] ? acc[q] - a[u] * xv[u][q] : acc[q];
  }
}

// a block of R values per black position, row-major
template <typename T, int R>
struct RbRows {
  const T* __restrict__ p;
  __device__ T operator()(int c, int q) const { return p[(size_t)c * R + q]; }
};

// one Jacobi sweep on T z = y for black position pb: dst row drow =
// (y_pb - sum_u T(pb, l_u) src_{l_u}) / diag(T)_pb, with y, 1/diag(T) and
// src in black-position order
template <typename T, int R, int RQ = R>
__device__ inline void rb_sweep_row(const SysDesc& D, int pb, int nb, const T* __restrict__ src,
                                    T* __restrict__ dst, size_t drow, int q0) {
  T acc[RQ];
  rb_sweep_acc<T, R, RbRows<T, R>, RQ>(D, pb, nb, D.t2ci, nb, pb, pb, RbRows<T, R>{src}, q0, acc);
  const T it = static_cast<const T*>(D.It)[pb];
#pragma unroll
  for (int q = 0; q < RQ; ++q) dst[drow * R + q0 + q] = acc[q] * it;
}

// one entry of a Chebyshev step: x_{s+1} = xp + om (G x_s + gamma c - xp)
// with G x_s + gamma c = xs + gamma (J x_s + c - xs), J x_s + c = acc * it
// the Jacobi update, xs = x_s and xp = x_{s-1}.  The fused multiply-adds
// are written out: left to contraction, a kernel that also forms acc * it
// for a Jacobi step may share that product and round differently, and
// single and paired steps must give the same bits.
template <typename T>
__device__ inline T cheb_entry(T acc, T it, T xs, T xp, T gam, T om) {
  const T g = fma(gam, fma(acc, it, -xs), xs);
  return fma(om, g - xp, xp);
}

// one Chebyshev step for black position pb: dst row drow from x_s = src
// and x_{s-1} = prev (null: x_0 = 0); prev and dst may be the same block
// (each row reads its own entries before writing them)
template <typename T, int R, int RQ = R>
__device__ inline void rb_cheb_row(const SysDesc& D, int pb, int nb, const T* __restrict__ src, const T* prev,
                                   T* dst, size_t drow, int q0, T gam, T om) {
  T acc[RQ];
  rb_sweep_acc<T, R, RbRows<T, R>, RQ>(D, pb, nb, D.t2ci, nb, pb, pb, RbRows<T, R>{src}, q0, acc);
  const T it = static_cast<const T*>(D.It)[pb];
#pragma unroll
  for (int q = 0; q < RQ; ++q) {
    const T xs = src[(size_t)pb * R + q0 + q];
    const T xp = prev ? prev[(size_t)pb * R + q0 + q] : T(0);
    dst[drow * R + q0 + q] = cheb_entry(acc[q], it, xs, xp, gam, om);
  }
}

// Spectral bounds of the Chebyshev steps for the current shift, once per
// inner solve after T's values and 1/diag(T) are built: per black position
// pb the row sum of the symmetrised J, sum_l sqrt(|T_pl T_lp| / |T_pp T_ll|),
// and P_pp / T_pp = S_pp / T_pp - 1 (P = F D_r^{-1} E); their maxima over the
// system (floored at 0) by integer atomic max of the non-negative doubles'
// bit patterns into SM_CHEB, which T's build cleared.  Both are Gershgorin
// bounds when T is diagonally similar to a symmetric matrix.
template <typename T>
__device__ inline void rb_bounds(const SysDesc& D, const RowCtx& c, const RbCtx<T>& x) {
  const int nb = D.n - D.nred;
  const int bc = (nb + D.nwg - 1) / D.nwg;
  const int sub = (bc + (int)gridDim.y - 1) / (int)gridDim.y;
  const int w0 = c.w * bc;
  const int p0 = w0 + (int)blockIdx.y * sub, p1 = min(nb, min(w0 + bc, p0 + sub));
  const T* tv = static_cast<const T*>(D.t2val);
  const T* It = static_cast<const T*>(D.It);
  double hi = 0.0, lr = 0.0;
  for (int pb = p0 + (int)threadIdx.x; pb < p1; pb += kTPB) {
    const double ip = (double)It[pb];
    double sum = 0.0;
    // kBGrp slots at a time, their loads issued together
    constexpr int kBGrp = 6;
    for (int u0 = 0; u0 < D.t2w; u0 += kBGrp) {
      int l[kBGrp], q[kBGrp];
      double a[kBGrp], b[kBGrp], il[kBGrp];
#pragma unroll
      for (int g = 0; g < kBGrp; ++g) {
        const size_t e = (size_t)min(u0 + g, D.t2w - 1) * nb + pb;
        l[g] = D.t2ci[e];
        q[g] = D.t2rev[e];  // T_lp: row l's slot with column pb
        a[g] = (double)tv[e];
      }
#pragma unroll
      for (int g = 0; g < kBGrp; ++g) {
        const bool ok = u0 + g < D.t2w && l[g] != pb && q[g] >= 0;  // (unused slots hold pb)
        b[g] = ok ? (double)tv[(size_t)max(q[g], 0) * nb + l[g]] : 0.0;
        il[g] = ok ? (double)It[l[g]] : 0.0;
      }
#pragma unroll
      for (int g = 0; g < kBGrp; ++g) sum += sqrt(fabs(a[g] * b[g] * ip * il[g]));
    }
    hi = fmax(hi, sum);
    lr = fmax(lr, (double)rb_dsh(x, D.rbrows[D.nred + pb]) * ip - 1.0);
  }
  for (int o = 32; o >= 1; o >>= 1) {
    hi = fmax(hi, __shfl_xor(hi, o));
    lr = fmax(lr, __shfl_xor(lr, o));
  }
  __shared__ double red[2][kTPB / 64];
  if (threadIdx.x % 64 == 0) {
    red[0][threadIdx.x / 64] = hi;
    red[1][threadIdx.x / 64] = lr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kTPB / 64; ++k) {
      hi = fmax(hi, red[0][k]);
      lr = fmax(lr, red[1][k]);
    }
    unsigned long long* cb = reinterpret_cast<unsigned long long*>(D.sm + SM_CHEB);
    atomicMax(cb, (unsigned long long)__double_as_longlong(hi));
    atomicMax(cb + 1, (unsigned long long)__double_as_longlong(lr));
  }
}

// black iterate t (< sweeps) in black-position order: two compact blocks in
// Eb, alternating; the last iterate goes to P_j's black rows instead
template <typename T>
__device__ inline T* rb_compact(const SysDesc& D, int nb, int t) {
  return static_cast<T*>(D.Eb) + (size_t)(t % 2) * nb * D.r;
}

// compact block holding the input of the sweep launch that starts with
// sweep `stage`: launches alternate between the two blocks, one sweep per
// launch, or two (pair) with a single last one for an odd count
__device__ inline int rb_launch_index(int stage, int pair) { return pair ? (stage - 1) / 2 : stage - 1; }

// Chebyshev steps of a system whose sweeps can run in pairs: Eb holds four
// compact blocks and iterate x_t (1 <= t <= sweeps) sits in block (t - 1)
// mod 4.  A paired launch reads x_s and x_{s-1} across its tile's region and
// writes x_{s+1} (the next launch's previous iterate) and x_{s+2}: four
// distinct blocks, so no workgroup overwrites what another still reads.
// Single steps keep the same places, so pairs and single steps mix.
__device__ inline bool rb_four(const SysDesc& D) { return D.poly && D.pair_lds > 0; }

template <typename T>
__device__ inline T* rb_iter4(const SysDesc& D, int nb, int t) {
  return static_cast<T*>(D.Eb) + (size_t)((t - 1) % 4) * nb * D.r;
}

// KIND 0: fwd (black rows); 1: Jacobi or Chebyshev sweep `stage` (black
// rows); 2: back (red rows); 5: T's values for the shift, and with Chebyshev
// steps 1/diag(T) (black rows, at the first Arnoldi step of an inner solve,
// in a launch of its own so that the forward stage keeps few registers)
template <typename T, int R, int KIND>
__device__ inline void rb_rows(const SysDesc& D, const RowCtx& c, const RbCtx<T>& x, const T* V, T* Pj,
                               int stage, int pair) {
  const int nb = D.n - D.nred;
  constexpr bool black = KIND != 2;
  const int off = black ? D.nred : 0;
  const int cnt = black ? nb : D.nred;
  // the colour's rows spread evenly over all of the system's workgroups
  // (about half a chunk each), not over the first half of them; each
  // workgroup's share is cut into gridDim.y slices, one per workgroup of
  // the launch's second grid dimension, and each row is served by L lanes
  // that own R / L columns each (every column sums its terms in the same
  // order whatever L, so the results do not depend on it)
  constexpr int L = KIND == 5 ? 1 : RbLanes<T, R>::v, RQ = R / L;
  const int bc = (cnt + D.nwg - 1) / D.nwg;
  const int sub = (bc + (int)gridDim.y - 1) / (int)gridDim.y;
  const int w0 = c.w * bc;
  const int p0 = w0 + (int)blockIdx.y * sub, p1 = min(cnt, min(w0 + bc, p0 + sub));
  const int lane = (int)threadIdx.x % L, q0 = lane * RQ;
  // Chebyshev steps (gamma 0: none, or the Jacobi fallback): the forward
  // stage's x_1 = gamma c, a sweep's gamma and omega_{stage+1}
  T cg = T(0), com = T(0);
  if constexpr (KIND == 0 || KIND == 1) {
    if (D.poly && D.sweeps > 0) {
      cg = (T)cheb_gamma(D.sm + SM_CHEB);
      if constexpr (KIND == 1) com = (T)D.sm[SM_CHEB + kChebOmega + stage - 1];
    }
  }
  // a step's blocks: x_stage (input), x_{stage+1} (output unless it is the
  // last step) and x_{stage-1} for a Chebyshev step (none at stage 1: x_0 =
  // 0); in the two-block layout x_{stage-1} is the output block, which each
  // row reads before writing
  const T* ssrc = nullptr;
  const T* sprev = nullptr;
  T* snxt = nullptr;
  if constexpr (KIND == 1) {
    if (rb_four(D)) {
      ssrc = rb_iter4<T>(D, nb, stage);
      snxt = rb_iter4<T>(D, nb, stage + 1);
      sprev = stage >= 2 ? rb_iter4<T>(D, nb, stage - 1) : nullptr;
    } else {
      const int ln = rb_launch_index(stage, pair);
      ssrc = rb_compact<T>(D, nb, ln);
      snxt = rb_compact<T>(D, nb, ln + 1);
      sprev = stage >= 2 ? snxt : nullptr;
    }
  }
  for (int pp = p0 + (int)threadIdx.x / L; pp < p1; pp += kTPB / L) {
    const int p = off + pp;  // colour position
    const int i = D.rbrows[p];
    if constexpr (KIND == 0) {
      T y[RQ], td;
      rb_black_fwd<T, R, RQ>(x, p, i, V, q0, y, td);
      const T it = T(1) / td;
      if (D.sweeps == 0) {
#pragma unroll
        for (int q = 0; q < RQ; ++q) Pj[(size_t)i * R + q0 + q] = y[q] * it;
      } else {
        T* z0 = rb_compact<T>(D, nb, 0);
        T* Y = static_cast<T*>(D.Yb);
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
          z0[(size_t)pp * R + q0 + q] = cg != T(0) ? cg * (y[q] * it) : y[q] * it;
          Y[(size_t)pp * R + q0 + q] = y[q];
        }
        if (lane == 0) static_cast<T*>(D.It)[pp] = it;
      }
    } else if constexpr (KIND == 5) {
      if (D.sweeps > 0) {
        rb_build_t<T>(D, x, p, pp, nb, i);
        if (D.poly) static_cast<T*>(D.It)[pp] = T(1) / rb_tdiag(x, p, i);
      }
    } else if constexpr (KIND == 1) {
      // (one call of each step kind, so that the kernel keeps one copy of
      // the gathers and its registers)
      T* dst = stage == D.sweeps ? Pj : snxt;
      const size_t drow = stage == D.sweeps ? (size_t)i : (size_t)pp;
      if (cg != T(0))
        rb_cheb_row<T, R, RQ>(D, pp, nb, ssrc, sprev, dst, drow, q0, cg, com);
      else
        rb_sweep_row<T, R, RQ>(D, pp, nb, ssrc, dst, drow, q0);
    } else {  // back: z_r = (v_r - E z) / (d_r + s)
      T g[RQ];
#pragma unroll
      for (int q = 0; q < RQ; ++q) g[q] = T(0);
      rb_gather<T, R, RQ>(x, p, i, Pj, q0, g);
      const T di = rb_dsh(x, i);
#pragma unroll
      for (int q = 0; q < RQ; ++q)
        Pj[(size_t)i * R + q0 + q] = (V[(size_t)i * R + q0 + q] - g[q]) / di;
    }
  }
}

// sweeps `stage` and `stage` + 1 for the black tile of workgroup c.w: the
// first over the tile's region (its rows and its halo, reading the launch's
// input block) into LDS, the second over its rows from LDS (the columns as
// region indices), to the other compact block or, when it is the last
// sweep, to P_j's black rows.  Each row's arithmetic is that of a single
// sweep (the slots summed in the same order), so the result equals two
// single-sweep launches bit for bit.  Chebyshev steps (four iterate blocks):
// the first step also reads the region's rows of x_{s-1} and writes the
// tile's rows of x_{s+1} for the next launch, the second reads its own rows
// of x_s.  FAST (every tile at most kTPB / LPR rows, T at most kPairRegSlots
// slots): each tile row has LPR lanes that hold its region columns in
// registers from the start, so the second sweep reads only LDS and cached
// operands.
template <typename T, int R, bool FAST>
__device__ inline void rb_pair(const SysDesc& D, const RowCtx& c, T* Pj, int stage, T* lds) {
  const int nb = D.n - D.nred;
  const int bc = (nb + D.nwg - 1) / D.nwg;
  const int p0 = c.w * bc, nin = min(nb, p0 + bc) - p0;
  if (nin <= 0) return;  // (uniform over the workgroup)
  const int h0 = D.halo_off[c.w], nreg = nin + (D.halo_off[c.w + 1] - h0);
  const int ln = rb_launch_index(stage, 1);
  const bool four = rb_four(D), last = stage + 1 == D.sweeps;
  const T* src = four ? rb_iter4<T>(D, nb, stage) : rb_compact<T>(D, nb, ln);
  T* dst = four ? (last ? nullptr : rb_iter4<T>(D, nb, stage + 2)) : rb_compact<T>(D, nb, ln + 1);
  T* out = last ? Pj : dst;
  // Chebyshev steps (gamma 0: the Jacobi fallback): omega_{stage+1} and
  // omega_{stage+2}, x_{stage-1} (none for stage 1: x_0 = 0) and the block
  // of x_{stage+1}, which only a later launch reads
  T gam = T(0), om1 = T(0), om2 = T(0);
  const T* prev = nullptr;
  T* mid = nullptr;
  if (four) {
    gam = (T)cheb_gamma(D.sm + SM_CHEB);
    om1 = (T)D.sm[SM_CHEB + kChebOmega + stage - 1];
    om2 = (T)D.sm[SM_CHEB + kChebOmega + stage];
    if (stage >= 2) prev = rb_iter4<T>(D, nb, stage - 1);
    if (!last) mid = rb_iter4<T>(D, nb, stage + 1);
  }
  const bool cheb = gam != T(0);
  const T* It = static_cast<const T*>(D.It);
  constexpr int kS = kPairRegSlots;
  // FAST: even blocks give each tile row two lanes (r/2 columns each), so
  // the second sweep keeps all four wavefronts busy
  constexpr int LPR = (R % 2 == 0) ? 2 : 1;
  int lc[kS];
  if constexpr (FAST) {
    const int k = min((int)threadIdx.x / LPR, nin - 1);
#pragma unroll
    for (int u = 0; u < kS; ++u) lc[u] = D.t2lc[(size_t)min(u, D.t2w - 1) * nb + p0 + k];
  }
  const int nhs = max(D.nhalo, 1);
  for (int k = threadIdx.x; k < nreg; k += kTPB) {
    // a halo row reads its columns from the halo's own table, so its
    // gathers do not wait for its position
    const bool in = k < nin;
    const int g = max(h0 + (k - nin), 0);  // (used by halo rows only)
    const int pb = in ? p0 + k : D.halo[g];
    T acc[R];
    rb_sweep_acc<T, R>(D, pb, nb, in ? D.t2ci : D.halo_ci, in ? nb : nhs, in ? pb : g, pb,
                       RbRows<T, R>{src}, 0, acc);
    const T it = It[pb];
    if (cheb) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const T xp = prev ? prev[(size_t)pb * R + q] : T(0);
        lds[k * R + q] = cheb_entry(acc[q], it, src[(size_t)pb * R + q], xp, gam, om1);
      }
      if (in && mid)
#pragma unroll
        for (int q = 0; q < R; ++q) mid[(size_t)pb * R + q] = lds[k * R + q];
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) lds[k * R + q] = acc[q] * it;
    }
  }
  __syncthreads();
  if constexpr (FAST) {
    constexpr int RQ = R / LPR;
    const int k = threadIdx.x / LPR, q0 = (threadIdx.x % LPR) * RQ;
    if (k >= nin) return;
    const int pb = p0 + k;
    const T* tv = static_cast<const T*>(D.t2val);
    const T* Y = static_cast<const T*>(D.Yb);
    T acc[RQ];
#pragma unroll
    for (int q = 0; q < RQ; ++q) acc[q] = Y[(size_t)pb * R + q0 + q];
    T a[kS], xv[kS][RQ];
#pragma unroll
    for (int u = 0; u < kS; ++u) {
      a[u] = tv[(size_t)min(u, D.t2w - 1) * nb + pb];
#pragma unroll
      for (int q = 0; q < RQ; ++q) xv[u][q] = lds[lc[u] * R + q0 + q];
    }
#pragma unroll
    for (int u = 0; u < kS; ++u) {
      const bool ok = u < D.t2w && lc[u] != k;
#pragma unroll
      for (int q = 0; q < RQ; ++q) acc[q] = ok ? acc[q] - a[u] * xv[u][q] : acc[q];
    }
    const T it = It[pb];
    const size_t row = last ? (size_t)D.rbrows[D.nred + pb] : (size_t)pb;
#pragma unroll
    for (int q = 0; q < RQ; ++q)
      out[row * R + q0 + q] =
          cheb ? cheb_entry(acc[q], it, lds[k * R + q0 + q], src[(size_t)pb * R + q0 + q], gam, om2) : acc[q] * it;
  } else {
    for (int k = threadIdx.x; k < nin; k += kTPB) {
      const int pb = p0 + k;
      T acc[R];
      rb_sweep_acc<T, R>(D, pb, nb, D.t2lc, nb, pb, k, RbRows<T, R>{lds}, 0, acc);
      const T it = It[pb];
      const size_t row = last ? (size_t)D.rbrows[D.nred + pb] : (size_t)pb;
#pragma unroll
      for (int q = 0; q < R; ++q)
        out[row * R + q] =
            cheb ? cheb_entry(acc[q], it, lds[k * R + q], src[(size_t)pb * R + q], gam, om2) : acc[q] * it;
    }
  }
}

// algorithmic bytes of one stage for one system (each array element read or
// written once; the once-per-solve build of T's values not counted); a
// pair of sweeps reads T once and the intermediate iterate never leaves
// LDS, so it counts one sweep plus its tables of region indices
template <typename T, int KIND>
__device__ inline unsigned long long rb_stage_bytes(const SysDesc& D) {
  if (KIND >= 5) return 0;  // once per inner solve, not per application
  const unsigned long long nr = D.nred, nb = D.n - D.nred, n = D.n, R = D.r, t = sizeof(T);
  const unsigned long long sweep = nb * 4 + D.t2w * nb * (4 + t) + 3 * nb * R * t + nb * t;
  if (KIND == 0)
    return nb * 4 + D.rbw * nb * (4 + 2 * t) + n * t + n * R * t + nb * R * t +
           (D.sweeps > 0 ? nb * R * t + nb * t : 0);
  // a Chebyshev step also reads its own rows of x_s and x_{s-1}
  if (KIND == 1) return sweep + (D.poly ? 2 * nb * R * t : 0);
  // (a pair of Chebyshev steps: x_{s-1} read and x_{s+1} written once)
  if (KIND >= 3)
    return sweep + D.t2w * nb * 4 + ((unsigned long long)D.nhalo + D.nwg + 1) * 4 + (D.poly ? 2 * nb * R * t : 0);
  return nr * 4 + D.rbw * nr * (4 + t) + nr * t + 2 * nr * R * t + nb * R * t;
}

// KIND 0: forward (stage 0), 1: sweep `stage`, 2: back, 3: sweeps `stage`
// and `stage` + 1, 4: the same with the region columns in registers (pair =
// 1: the launches of the sweeps are paired), 5: T's values for the shift,
// 6: the Chebyshev steps' spectral bounds (5 and 6 at the first Arnoldi step
// of an inner solve only); one instance per kind, so each allocates only the
// registers it needs.  The sweep kind at r = 8 is held to six waves per
// SIMD (80 VGPRs without spills, against 88 and five waves unbounded: its
// launches on the 3-D configuration ran about 1% faster); at other widths
// the same bound spills, so they keep the compiler's choice.
template <typename T, int RF, int KIND>
__global__ __launch_bounds__(kTPB) __attribute__((amdgpu_waves_per_eu(KIND == 1 && RF == 8 ? 6 : 1))) void k_precond(const SysDesc* __restrict__ d, const SysCtl* __restrict__ ctl,
                                                  const int2* __restrict__ rowmap, int stage, int pair,
                                                  unsigned long long* __restrict__ prof) {
  extern __shared__ double rb_lds[];  // KIND 3, 4: a tile region's iterate
  const RowCtx c = row_ctx(d, rowmap);
  const SysDesc& D = d[c.s];
  if (ctl[c.s].phase != PH_ARNOLDI || !D.rbrows) return;
  if (prof && c.w == 0 && blockIdx.y == 0 && threadIdx.x == 0)
    atomicAdd(prof + LRADI_PROF_PRECOND, rb_stage_bytes<T, KIND>(D));
  const int j = ctl[c.s].j;
  const RbCtx<T> x = rb_ctx<T>(D, ctl[c.s].shift);
  const size_t blk = (size_t)D.n * D.r;
  const T* V = static_cast<const T*>(D.V) + (size_t)j * blk;
  T* Pj = static_cast<T*>(D.P) + (size_t)j * blk;
  // the shift is fixed for an inner solve: T's values are built at its
  // first Arnoldi step (first cycle, j = 0) and kept over restarts
  const bool first = ctl[c.s].cycles == 1 && j == 0;
  if constexpr (KIND == 5 || KIND == 6) {
    if (!first) return;
  }
  if constexpr (KIND == 5) {
    // the bounds' maxima start from zero for each shift
    if (D.poly && c.w == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
      D.sm[SM_CHEB] = 0.0;
      D.sm[SM_CHEB + 1] = 0.0;
    }
  }
  if constexpr (KIND == 0) {
    // the coefficients, once the bounds' launch has finished
    if (D.poly && D.sweeps > 0 && first && c.w == 0 && blockIdx.y == 0 && threadIdx.x == 0)
      cheb_table(D.sm + SM_CHEB, D.sweeps);
  }
  if constexpr (KIND == 6) {
    if (D.poly && D.sweeps > 0) rb_bounds<T>(D, c, x);
  } else if constexpr (KIND == 3 || KIND == 4) {
    LRADI_RSEL(RF, D.r, (rb_pair<T, RR, KIND == 4>(D, c, Pj, stage, reinterpret_cast<T*>(rb_lds))));
  } else {
    LRADI_RSEL(RF, D.r, rb_rows<T, RR, KIND>(D, c, x, V, Pj, stage, pair));
  }
}

// ---------------------------------------------------------------------------
// 2. partial Gram  part[w][b][a][q] = sum_{i in chunk} V_b[i][a] U[i][q],
//    b = 0..j  (PH_ARNOLDI).  Lane layout: lane = (row offset, a) with the
//    column index padded to RP = next power of two >= R, so the sum over the
//    rows of a wavefront is an xor-shuffle butterfly over the high lane bits.
template <int R>
struct Pad {
  static constexpr int v = R <= 1 ? 1 : R <= 2 ? 2 : R <= 4 ? 4 : 8;
};

// Tile shape per block width: K rows per lane per super-row and G basis
// blocks per pass, so that K*G independent loads are in flight per lane.
// (Measured on the 3-D configuration at r = 8, FP64: K = 4, G = 4 25.4 us
// per launch; K = 2, G = 4 27.0; K = 1, G = 4 25.5; K = 2, G = 8 30.8.)
template <typename T, int R>
struct GramTile {
  static constexpr int K = 4;
  static constexpr int G = R >= 5 ? 4 : (sizeof(T) == 4 ? 8 : 4);
};

// Basis blocks per Gram workgroup: the launch grid's second dimension splits
// V_0..V_j into groups of this many blocks, so a short basis (small n)
// still spreads over many workgroups.
constexpr int kGramBlocks = 8;

template <typename T, int R>
__device__ inline void gram_vu_rows(const SysDesc& D, const RowCtx& c, int bfirst, int nb, double* lds) {
  constexpr int RP = Pad<R>::v;
  constexpr int RPW = 64 / RP;                  // rows per wavefront and row step
  constexpr int K = GramTile<T, R>::K, G = GramTile<T, R>::G;
  constexpr int SUPER = 4 * RPW * K;            // rows of one super-row
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ro = lane / RP, a = lane - ro * RP;
  const bool act = a < R;
  const auto V = gmem(static_cast<const T*>(D.V));
  const auto U = gmem(static_cast<const T*>(D.U));
  const size_t bs = (size_t)D.n * R;
  double* out = D.part + (size_t)c.w * D.pstride;
  for (int b0 = bfirst; b0 < nb; b0 += G) {
    const int gc = min(G, nb - b0);
    double acc[G][R];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int q = 0; q < R; ++q) acc[g][q] = 0.0;
    if (act) {
      for (int base = c.row0; base < c.row1; base += SUPER) {
        // every load is unconditional (row and block indices clamped into
        // range) and masked afterwards, so all K x G + K x R loads of a lane
        // are in flight together
        T ut[K][R];
        int rows[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          rows[k] = base + (k * 4 + wave) * RPW + ro;
          const size_t rc = (size_t)min(rows[k], c.row1 - 1);
#pragma unroll
          for (int q = 0; q < R; ++q) ut[k][q] = U[rc * R + q];
        }
        T x[K][G];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const size_t rc = (size_t)min(rows[k], c.row1 - 1);
#pragma unroll
          for (int g = 0; g < G; ++g) x[k][g] = V[(size_t)(b0 + min(g, gc - 1)) * bs + rc * R + a];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const bool okr = rows[k] < c.row1;
          double u[R];
#pragma unroll
          for (int q = 0; q < R; ++q) u[q] = okr ? (double)ut[k][q] : 0.0;
#pragma unroll
          for (int g = 0; g < G; ++g) {
            const double xv = (g < gc) ? (double)x[k][g] : 0.0;
#pragma unroll
            for (int q = 0; q < R; ++q) acc[g][q] += xv * u[q];
          }
        }
      }
    }
    // reduce-scatter over the row offset (lane bits >= log2 RP): afterwards
    // the lanes of column a hold the sums of (g, q) = index / R
    constexpr int NV = G * R, P2 = pow2c(NV);
    using RS = WaveRS<P2, RP>;
    double w[P2];
#pragma unroll
    for (int k = 0; k < P2; ++k) w[k] = k < NV ? acc[k / R][k % R] : 0.0;
    wave_reduce_scatter<P2, RP>(w, lane);
    if (act && (lane & RS::DUP) == 0) {
      const int base = wave_rs_base<P2, RP>(lane);
#pragma unroll
      for (int i = 0; i < RS::NOUT; ++i) {
        const int idx = base + i;
        if (idx < NV) lds[((wave * G + idx / R) * R + a) * R + idx % R] = w[i];
      }
    }
    __syncthreads();
    const int nout = gc * R * R;
    for (int o = threadIdx.x; o < nout; o += kTPB) {
      const int g = o / (R * R), rem = o - g * R * R;
      const double sum = ((lds[(0 * G + g) * R * R + rem] + lds[(1 * G + g) * R * R + rem]) +
                          lds[(2 * G + g) * R * R + rem]) + lds[(3 * G + g) * R * R + rem];
      out[(size_t)(b0 + g) * R * R + rem] = sum;
    }
    __syncthreads();
  }
}

template <typename T, int RF>
__global__ __launch_bounds__(kTPB) void k_gram_vu(const SysDesc* __restrict__ d,
                                                  const SysCtl* __restrict__ ctl,
                                                  const int2* __restrict__ rowmap,
                                                  unsigned long long* __restrict__ prof) {
  __shared__ double lds[4 * 8 * kMaxR * kMaxR];
  const RowCtx c = row_ctx(d, rowmap);
  const SysDesc& D = d[c.s];
  if (ctl[c.s].phase != PH_ARNOLDI) return;
  const int bfirst = (int)blockIdx.y * kGramBlocks;
  const int nb = min(ctl[c.s].j + 1, bfirst + kGramBlocks);
  if (bfirst >= nb) return;
  if (prof && c.w == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    // basis blocks V_0..V_j and the candidate block U
    const unsigned long long bytes = (unsigned long long)(ctl[c.s].j + 2) * sizeof(T) * D.n * D.r;
    atomicAdd(prof + LRADI_PROF_GRAM, bytes);
  }
  if constexpr (RF > 0) {
    gram_vu_rows<T, RF>(D, c, bfirst, nb, lds);
  } else {
    LRADI_DISPATCH_R(D.r, gram_vu_rows<T, RR>(D, c, bfirst, nb, lds));
  }
}

// 3. red = sum_w part[w]; hacc = red (first pass) or hacc += red (second).
//    One wavefront per coefficient: each lane sums every 64th workgroup's
//    partial with four independent accumulators, then a fixed-order xor
//    butterfly combines the lanes.
constexpr int kRedOut = 4;  // coefficients per workgroup (one per wavefront)
__global__ __launch_bounds__(kTPB) void k_reduce_vu(const SysDesc* __restrict__ d,
                                                    const SysCtl* __restrict__ ctl, int first) {
  const int s = blockIdx.x;
  const SysDesc& D = d[s];
  if (ctl[s].phase != PH_ARNOLDI) return;
  const int P = (ctl[s].j + 1) * D.r * D.r;
  const int p0 = blockIdx.y * kRedOut;
  if (p0 >= P) return;
  const int lane = threadIdx.x & 63;
  const int p = p0 + (threadIdx.x >> 6);
  double acc = 0.0;
  if (p < P) {
    const double* X = D.part + p;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int w = lane;
    for (; w + 192 < D.nwg; w += 256) {
      a0 += X[(size_t)w * D.pstride];
      a1 += X[(size_t)(w + 64) * D.pstride];
      a2 += X[(size_t)(w + 128) * D.pstride];
      a3 += X[(size_t)(w + 192) * D.pstride];
    }
    for (; w < D.nwg; w += 64) a0 += X[(size_t)w * D.pstride];
    acc = (a0 + a1) + (a2 + a3);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0 && p < P) {
    D.red[p] = acc;
    if (first)
      D.hacc[p] = acc;
    else
      D.hacc[p] += acc;
  }
}

// ---------------------------------------------------------------------------
// 4./7. U -= sum_b V_b red_b  (PH_ARNOLDI); the second pass also forms the
//       partial U^T U of the result into partS (PH_ARNOLDI and PH_RESTART).
template <typename T, int R, bool GRAM>
__device__ inline void update_rows(const SysDesc& D, const RowCtx& c, int nb, bool do_update,
                                   double* hl, double* lds) {
  // the coefficients, rounded once to the basis precision
  T* ht = reinterpret_cast<T*>(hl);
  if (do_update) {
    for (int e = threadIdx.x; e < nb * R * R; e += kTPB) ht[e] = (T)D.red[e];
    __syncthreads();
  }
  const auto V = gmem(static_cast<const T*>(D.V));
  const auto U = gmem_w(static_cast<T*>(D.U));
  const size_t bs = (size_t)D.n * R;
  constexpr int NG = R * (R + 1) / 2;  // the Gram's packed upper triangle
  double g2[GRAM ? NG : 1];
  if constexpr (GRAM) {
#pragma unroll
    for (int e = 0; e < NG; ++e) g2[e] = 0.0;
  }
  for (int i = c.row0 + threadIdx.x; i < c.row1; i += kTPB) {
    T u[R];
#pragma unroll
    for (int q = 0; q < R; ++q) u[q] = U[(size_t)i * R + q];
    if (do_update) {
      T acc[R];
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] = T(0);
      constexpr int UB = R >= 5 ? 2 : 4;  // blocks whose loads are in flight together
      int b = 0;
      for (; b + UB <= nb; b += UB) {
        T v[UB][R];
#pragma unroll
        for (int bb = 0; bb < UB; ++bb)
#pragma unroll
          for (int a = 0; a < R; ++a) v[bb][a] = V[(size_t)(b + bb) * bs + (size_t)i * R + a];
#pragma unroll
        for (int bb = 0; bb < UB; ++bb) {
          const T* h = ht + (b + bb) * R * R;
#pragma unroll
          for (int a = 0; a < R; ++a)
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] += v[bb][a] * h[a * R + q];
        }
      }
      for (; b < nb; ++b) {
        T v[R];
#pragma unroll
        for (int a = 0; a < R; ++a) v[a] = V[(size_t)b * bs + (size_t)i * R + a];
        const T* h = ht + b * R * R;
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
          for (int q = 0; q < R; ++q) acc[q] += v[a] * h[a * R + q];
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        u[q] -= acc[q];
        U[(size_t)i * R + q] = u[q];
      }
    }
    if constexpr (GRAM) {
      int e = 0;
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int q = a; q < R; ++q) g2[e++] += (double)u[a] * (double)u[q];
    }
  }
  if constexpr (GRAM) block_sum_store_sym<R>(g2, lds, D.partS + (size_t)c.w * kPS);
}

template <typename T, int RF, bool SECOND>
__global__ __launch_bounds__(kTPB) void k_update(const SysDesc* __restrict__ d,
                                                 const SysCtl* __restrict__ ctl,
                                                 const int2* __restrict__ rowmap, int only) {
  extern __shared__ double hl[];  // maxP doubles: the projection coefficients
  __shared__ double lds[4 * kMaxR * kMaxR];
  const RowCtx c = row_ctx(d, rowmap);
  const SysDesc& D = d[c.s];
  const int ph = ctl[c.s].phase;
  if (only >= 0 && ph != only) return;
  bool do_update;
  if (ph == PH_ARNOLDI) {
    do_update = true;
  } else if (ph == PH_RESTART && SECOND) {
    do_update = false;
  } else {
    return;
  }
  const int nb = ctl[c.s].j + 1;
  LRADI_RSEL(RF, D.r, update_rows<T, RR, SECOND>(D, c, nb, do_update, hl, lds));
}

// ---------------------------------------------------------------------------
// 8./10. Cholesky factor of the reduced U^T U (PH_ARNOLDI / PH_RESTART).
// S (upper Cholesky factor, regularised, of G) and its inverse into Sl, Sil;
// slot >= 0 also stores both to the system's small scratch for later
// kernels.  Returns chol_upper_reg_t's flag (< 0: not finite).
template <int R>
__device__ inline int chol_factor(const SysDesc& D, const double* G, double fl, double* Sl, double* Sil,
                                  int slot) {
  double S[R * R], Si[R * R];
  const int reg = chol_upper_reg_t<R>(G, S, fl);
  if (reg < 0) return reg;
  tri_inv_upper_t<R>(S, Si);
#pragma unroll
  for (int e = 0; e < R * R; ++e) {
    Sl[e] = S[e];
    Sil[e] = Si[e];
  }
  if (slot >= 0) {
    double* dst = D.sm + (slot == 0 ? SM_S1 : SM_S2);
    double* dsti = D.sm + (slot == 0 ? SM_S1I : SM_S2I);
#pragma unroll
    for (int e = 0; e < R * R; ++e) {
      dst[e] = S[e];
      dsti[e] = Si[e];
    }
  }
  return reg;
}

template <int R>
__device__ inline void chol_body(const SysDesc& D, SysCtl& C, int slot, double fl, const double* G) {
  double Sl[R * R], Sil[R * R];
  const int reg = chol_factor<R>(D, G, fl, Sl, Sil, slot);
  if (reg < 0) {
    C.status = IS_NAN;
    C.phase = PH_FINISHED;
    return;
  }
  if (reg > 0) C.breakdowns += 1;
}

__global__ __launch_bounds__(kTPB) void k_chol(const SysDesc* __restrict__ d, SysCtl* __restrict__ ctl,
                                               int slot, double rel_floor64, double rel_floor32, int only) {
  __shared__ double red_lds[kTPB];
  __shared__ double G[64];
  const int s = blockIdx.x;
  const SysDesc& D = d[s];
  const int ph = ctl[s].phase;
  if (ph != PH_ARNOLDI && ph != PH_RESTART) return;
  if (only >= 0 && ph != only) return;
  const int R = D.r;
  reduce_small(slot == 0 ? D.partS : D.partS2, D.nwg, R * R, red_lds, G);
  if (threadIdx.x == 0) {
    const double fl = (D.precision == LRADI_FP64) ? rel_floor64 : rel_floor32;
    LRADI_DISPATCH_R(R, chol_body<RR>(D, ctl[s], slot, fl, G));
  }
}

// 9./11. pass 0: the partial Gram of U S1^{-1} (rows formed in registers,
//        U itself is left as it is);
//        pass 1: V_{j+1} (PH_ARNOLDI) or V_0 (PH_RESTART) = (U S1^{-1}) S2^{-1},
//        U S1^{-1} formed again exactly as in pass 0 (rounded to the basis
//        precision in both), so the result equals writing U S1^{-1} back in
//        pass 0 and scaling it in pass 1, bit for bit, one write of U fewer.
template <int R>
struct PackedTri {
  // an upper-triangular R x R matrix's entries (a, q), a <= q, by rows
  double v[R * (R + 1) / 2];
  __device__ explicit PackedTri(const double* S) {
    int e = 0;
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int q = a; q < R; ++q) v[e++] = S[a * R + q];
  }
  // o = u S (row vector times the matrix)
  __device__ void apply(const double (&u)[R], double (&o)[R]) const {
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a <= q; ++a) s += u[a] * v[a * R - a * (a - 1) / 2 + (q - a)];
      o[q] = s;
    }
  }
};

template <typename T, int R, int PASS>
__device__ inline void scale_rows(const SysDesc& D, const RowCtx& c, const double* S1i, const double* S2i,
                                  T* dst, double* lds, double* gout) {
  const PackedTri<R> s1(S1i);
  const auto U = gmem(static_cast<const T*>(D.U));
  constexpr int NG = R * (R + 1) / 2;  // the Gram's packed upper triangle
  double g2[PASS == 0 ? NG : 1];
  if constexpr (PASS == 0) {
#pragma unroll
    for (int e = 0; e < NG; ++e) g2[e] = 0.0;
  }
  for (int i = c.row0 + threadIdx.x; i < c.row1; i += kTPB) {
    double u[R], o[R];
#pragma unroll
    for (int q = 0; q < R; ++q) u[q] = (double)U[(size_t)i * R + q];
    s1.apply(u, o);
    T ot[R];
#pragma unroll
    for (int q = 0; q < R; ++q) ot[q] = (T)o[q];
    if constexpr (PASS == 0) {
      int e = 0;
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int q = a; q < R; ++q) g2[e++] += (double)ot[a] * (double)ot[q];
    } else {
      const PackedTri<R> s2(S2i);
      double w[R];
#pragma unroll
      for (int q = 0; q < R; ++q) w[q] = (double)ot[q];
      s2.apply(w, o);
      const auto dg = gmem_w(dst);
#pragma unroll
      for (int q = 0; q < R; ++q) dg[(size_t)i * R + q] = (T)o[q];
    }
  }
  if constexpr (PASS == 0) block_sum_store_sym<R>(g2, lds, gout + (size_t)c.w * kPS);
}

template <typename T, int RF, int PASS>
__global__ __launch_bounds__(kTPB) void k_scale(const SysDesc* __restrict__ d,
                                                SysCtl* __restrict__ ctl,
                                                const int2* __restrict__ rowmap, int fuse,
                                                double fl64, double fl32, int only) {
  __shared__ double lds[4 * kMaxR * kMaxR];
  __shared__ double red_lds[kTPB];
  __shared__ double G[64];
  __shared__ double SS[2 * kMaxR * kMaxR];
  __shared__ int ok;
  const RowCtx c = row_ctx(d, rowmap);
  const SysDesc& D = d[c.s];
  const int ph = ctl[c.s].phase;
  if (ph != PH_ARNOLDI && ph != PH_RESTART) return;
  if (only >= 0 && ph != only) return;
  const double* Si = D.sm + (PASS == 0 ? SM_S1I : SM_S2I);
  const double* S1i = D.sm + SM_S1I;  // pass 1 applies S1^{-1} again
  if constexpr (RF >= 1 && RF <= 4) {
   if (fuse) {
    // this pass's Cholesky factor, formed by every workgroup from the small
    // Gram partials in the same order (identical in all of them); workgroup
    // 0 publishes it and the control-block updates
    reduce_small(PASS == 0 ? D.partS : D.partS2, D.nwg, D.r * D.r, red_lds, G);
    if (threadIdx.x == 0) {
      const double fl = (D.precision == LRADI_FP64) ? fl64 : fl32;
      int reg = 0;
      LRADI_RSEL(RF, D.r, reg = chol_factor<RR>(D, G, fl, SS, SS + RR * RR, c.w == 0 ? PASS : -1));
      ok = reg >= 0;
      if (c.w == 0) {
        SysCtl& C = ctl[c.s];
        if (reg < 0) {
          C.status = IS_NAN;
          C.phase = PH_FINISHED;
        } else if (reg > 0) {
          C.breakdowns += 1;
        }
      }
    }
    __syncthreads();
    if (!ok) return;
    Si = SS + D.r * D.r;
   }
  }
  T* dst = nullptr;
  if (PASS == 1) {
    const int tgt = (ph == PH_ARNOLDI) ? ctl[c.s].j + 1 : 0;
    dst = static_cast<T*>(D.V) + (size_t)tgt * D.n * D.r;
  }
  if constexpr (PASS == 0) {
    LRADI_RSEL(RF, D.r, scale_rows<T, RR, 0>(D, c, Si, nullptr, nullptr, lds, D.partS2));
  } else {
    LRADI_RSEL(RF, D.r, scale_rows<T, RR, 1>(D, c, S1i, Si, dst, lds, D.partS2));
  }
}

// ---------------------------------------------------------------------------
// 12. least-squares update (one workgroup per system).
//   PH_RESTART: G = [S; 0] with S = S2 S1, start a cycle.
//   PH_ARNOLDI: bring column block j of the block Hessenberg matrix,
//   [H_{0..j,j}; S], through the stored orthogonal factors Q_0..Q_{j-1},
//   factor its last 2r x r part (Householder, Q_j), rotate the right-hand
//   side, and take the residual estimate ||G_{j+1}||_F.  At the end of a
//   cycle solve the triangular system for y.

// threads of the least-squares workgroup: one lane per entry of a rotated
// 2r x r block; for r <= 5 that is a single wavefront, whose barriers are
// cheap, wider blocks (and batches of mixed r) take two
template <int RF>
struct LsqTPB {
  static constexpr int v = (RF > 0 && RF <= 5) ? 64 : 128;
};

// Householder QR of the 2R x R block hb (LDS, row-major, overwritten with
// [R_jj; 0]); Q (LDS, 2R x 2R row-major) receives the orthogonal factor.
// Run by wavefront 0; lane i < 2R owns row i of the block and of Q.  The
// column sums go through LDS (hw, 2R (R + 2) doubles): every lane writes its
// terms, then each lane adds all 2R of them in the same order, so all lanes
// hold the same sums.  One wavefront executes its LDS operations in order;
// wave_barrier keeps the compiler from moving them across each other.
template <int R>
__device__ inline void house_wave(double* hb, double* Q, double* hw) {
  constexpr int M2 = 2 * R;
  const int lane = threadIdx.x;
  const bool own = lane < M2;
  double* xs = hw;            // x (2R)
  double* vs = hw + M2;       // v (2R)
  double* pr = hw + 2 * M2;   // v * column jc (R x 2R)
  double mr[R], qr[M2];
#pragma unroll
  for (int c = 0; c < R; ++c) mr[c] = own ? hb[lane * R + c] : 0.0;
#pragma unroll
  for (int k = 0; k < M2; ++k) qr[k] = (own && k == lane) ? 1.0 : 0.0;
#pragma unroll
  for (int c = 0; c < R; ++c) {
    const double x = (own && lane >= c) ? mr[c] : 0.0;
    if (own) xs[lane] = x;
    __builtin_amdgcn_wave_barrier();
    double nx2 = 0.0;
#pragma unroll
    for (int k = c; k < M2; ++k) nx2 += xs[k] * xs[k];
    const double x0 = xs[c];
    __builtin_amdgcn_wave_barrier();
    if (nx2 == 0.0) continue;
    const double alpha = (x0 >= 0.0) ? -sqrt(nx2) : sqrt(nx2);
    const double v = x - ((lane == c) ? alpha : 0.0);
    // ||v||^2 = ||x||^2 - 2 alpha x0 + alpha^2, all terms >= 0
    const double vv = (nx2 - 2.0 * alpha * x0) + alpha * alpha;
    const double beta = 2.0 / vv;
    if (own) {
      vs[lane] = v;
#pragma unroll
      for (int jc = c + 1; jc < R; ++jc) pr[jc * M2 + lane] = v * mr[jc];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int jc = c + 1; jc < R; ++jc) {
      double dd = 0.0;
#pragma unroll
      for (int k = 0; k < M2; ++k) dd += pr[jc * M2 + k];
      mr[jc] -= beta * dd * v;
    }
    if (own && lane == c) mr[c] = alpha;
    else if (own && lane > c) mr[c] = 0.0;
    double vk[M2];
#pragma unroll
    for (int k = 0; k < M2; ++k) vk[k] = vs[k];
    __builtin_amdgcn_wave_barrier();
    double dq = 0.0;
#pragma unroll
    for (int k = 0; k < M2; ++k) dq += qr[k] * vk[k];
#pragma unroll
    for (int k = 0; k < M2; ++k) qr[k] -= beta * dq * vk[k];
  }
  if (own) {
#pragma unroll
    for (int c = 0; c < R; ++c) hb[lane * R + c] = mr[c];
#pragma unroll
    for (int k = 0; k < M2; ++k) Q[lane * M2 + k] = qr[k];
  }
}

template <int R, int kLsqTPB>
__device__ inline void lsq_body(const SysDesc& D, SysCtl& C, int ph, double* h, double* Sf,
                                double* Qj, double* hw, int* done_s) {
  constexpr int RR2 = R * R, twoR = 2 * R;
  // entries (a, q) of a 2r x r block per lane
  constexpr int NE = (twoR * R + kLsqTPB - 1) / kLsqTPB;
  static_assert(NE == 1, "one entry per lane");
  const int m = D.m, t = threadIdx.x;
  const int j = C.j;
  const int ldR = m * R;
  int ea[NE], eq[NE];
  bool ev[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = t + u * kLsqTPB;
    ev[u] = e < twoR * R;
    ea[u] = ev[u] ? e / R : 0;
    eq[u] = ev[u] ? e - (e / R) * R : 0;
  }
  // issue every independent load first: S = S2 S1, the Hessenberg column
  // block, the first orthogonal factor
  double s1c[R], s2r[R];
  if (t < RR2) {
    const int sa = t / R, sq = t - sa * R;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      s2r[k] = D.sm[SM_S2 + sa * R + k];
      s1c[k] = D.sm[SM_S1 + k * R + sq];
    }
  }
  double qa[NE][twoR], qn[NE][twoR];
  if (ph == PH_ARNOLDI) {
    for (int e = t; e < (j + 1) * RR2; e += kLsqTPB) h[e] = D.hacc[e];
    if (j > 0) {
#pragma unroll
      for (int u = 0; u < NE; ++u)
#pragma unroll
        for (int k = 0; k < twoR; ++k) qa[u][k] = ev[u] ? D.Qs[k * twoR + ea[u]] : 0.0;
    }
  }
  if (t < RR2) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) v += s2r[k] * s1c[k];
    Sf[t] = v;
    if (ph == PH_ARNOLDI) h[(j + 1) * RR2 + t] = v;
  }
  __syncthreads();
  if (ph == PH_RESTART) {
    for (int e = t; e < (m + 1) * RR2; e += kLsqTPB) D.Gv[e] = (e < RR2) ? Sf[e] : 0.0;
    if (t == 0) {
      C.j = 0;
      C.ncols = 0;
      C.est = C.r0;
      C.phase = PH_ARNOLDI;
    }
    return;
  }
  // apply Q_b^T to rows [b r, b r + 2r); the columns of Q_b a lane needs are
  // prefetched into registers one step ahead.  The workgroup is one
  // wavefront, so its barriers are cheap.
  for (int b = 0; b < j; ++b) {
    if (b + 1 < j) {
#pragma unroll
      for (int u = 0; u < NE; ++u)
#pragma unroll
        for (int k = 0; k < twoR; ++k)
          qn[u][k] = ev[u] ? D.Qs[(size_t)(b + 1) * 4 * RR2 + k * twoR + ea[u]] : 0.0;
    }
    double nv[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      nv[u] = 0.0;
#pragma unroll
      for (int k = 0; k < twoR; ++k) nv[u] += qa[u][k] * h[(b * R + k) * R + eq[u]];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NE; ++u)
      if (ev[u]) h[(b * R + ea[u]) * R + eq[u]] = nv[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NE; ++u)
#pragma unroll
      for (int k = 0; k < twoR; ++k) qa[u][k] = qn[u][k];
  }
  // the right-hand-side rows this step rotates (in flight during the QR)
  double gcol[NE][twoR];
#pragma unroll
  for (int u = 0; u < NE; ++u)
#pragma unroll
    for (int k = 0; k < twoR; ++k) gcol[u][k] = ev[u] ? D.Gv[(j * R + k) * R + eq[u]] : 0.0;
  // Householder QR of rows [j r, j r + 2r)
  if (t < 64) house_wave<R>(h + j * RR2, Qj, hw);
  __syncthreads();
  for (int e = t; e < 4 * RR2; e += kLsqTPB) D.Qs[(size_t)j * 4 * RR2 + e] = Qj[e];
  for (int e = t; e < (j + 1) * RR2; e += kLsqTPB) {
    const int row = e / R, qq = e - row * R;
    D.Rt[(size_t)(j * R + qq) * ldR + row] = h[e];
  }
  // rotate the right-hand side rows [j r, j r + 2r) (prefetched into gcol);
  // the new last block row also goes to LDS (Sf is free again) for the
  // residual estimate
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    if (!ev[u]) continue;
    double nv = 0.0;
#pragma unroll
    for (int k = 0; k < twoR; ++k) nv += Qj[k * twoR + ea[u]] * gcol[u][k];
    D.Gv[(j * R + ea[u]) * R + eq[u]] = nv;
    if (ea[u] >= R) Sf[(ea[u] - R) * R + eq[u]] = nv;
  }
  __syncthreads();
  if (t == 0) {
    double e2 = 0.0;
#pragma unroll
    for (int e = 0; e < RR2; ++e) {
      const double g = Sf[e];
      e2 += g * g;
    }
    const double est = sqrt(e2);
    C.steps += 1;
    C.ncols = j + 1;
    C.est = est;
    const double thr = fmax(C.delta, D.floor_rel * C.r0);
    const int done = (est <= thr) || (j + 1 >= m) || (C.steps >= D.max_inner) || !(est == est);
    *done_s = done;
    if (!done) C.j = j + 1;
  }
  __syncthreads();
  if (!*done_s) return;
  // back substitution R_t y = G(0 : (j+1) r), block by block
  const int nc = j + 1;
  double* g = h;
  for (int e = t; e < nc * RR2; e += kLsqTPB) g[e] = D.Gv[e];
  __syncthreads();
  for (int bj = nc - 1; bj >= 0; --bj) {
    if (t < R) {
      const int qq = t;
      for (int aa = R - 1; aa >= 0; --aa) {
        const int row = bj * R + aa;
        double v = g[row * R + qq];
        for (int k = aa + 1; k < R; ++k) v -= D.Rt[(size_t)(bj * R + k) * ldR + row] * g[(bj * R + k) * R + qq];
        v /= D.Rt[(size_t)row * ldR + row];
        g[row * R + qq] = v;
      }
    }
    __syncthreads();
    for (int e = t; e < bj * RR2; e += kLsqTPB) {
      const int row = e / R, qq = e - row * R;
      double v = g[e];
#pragma unroll
      for (int k = 0; k < R; ++k) v -= D.Rt[(size_t)(bj * R + k) * ldR + row] * g[(bj * R + k) * R + qq];
      g[e] = v;
    }
    __syncthreads();
  }
  for (int e = t; e < nc * RR2; e += kLsqTPB) D.yv[e] = g[e];
  if (t == 0) C.phase = PH_CYCLE_END;
}

template <int RF>
__global__ __launch_bounds__(LsqTPB<RF>::v) void k_lsq(const SysDesc* __restrict__ d, SysCtl* __restrict__ ctl, int only) {
  extern __shared__ double h[];  // maxP doubles: the Hessenberg column block
  __shared__ double Sf[64];
  __shared__ double Qj[16 * 16];
  __shared__ double hw[2 * kMaxR * (kMaxR + 2)];
  __shared__ int done_s;
  const int s = blockIdx.x;
  const SysDesc& D = d[s];
  SysCtl& C = ctl[s];
  const int ph = C.phase;
  if (ph != PH_ARNOLDI && ph != PH_RESTART) return;
  if (only >= 0 && ph != only) return;
  LRADI_RSEL(RF, D.r, lsq_body<RR, LsqTPB<RF>::v>(D, C, ph, h, Sf, Qj, hw, &done_s));
}

// ---------------------------------------------------------------------------
// 13. Z += sum_b V_b y_b  (PH_CYCLE_END, at least one column); with right
//     preconditioning Z += sum_b P_b y_b, P_b = M V_b
template <typename T, int R>
__device__ inline void zupdate_rows(const SysDesc& D, const RowCtx& c, double* Z, int nb,
                                    const double* yl) {
  const auto V = gmem(static_cast<const T*>(D.rbrows ? D.P : D.V));
  const size_t bs = (size_t)D.n * R;
  for (int i = c.row0 + threadIdx.x; i < c.row1; i += kTPB) {
    double acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0.0;
    for (int b = 0; b < nb; ++b) {
      double v[R];
#pragma unroll
      for (int a = 0; a < R; ++a) v[a] = (double)V[(size_t)b * bs + (size_t)i * R + a];
      const double* y = yl + b * R * R;
#pragma unroll
      for (int a = 0; a < R; ++a)
#pragma unroll
        for (int q = 0; q < R; ++q) acc[q] += v[a] * y[a * R + q];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) Z[(size_t)i * R + q] += acc[q];
  }
}

template <typename T, int RF>
__global__ __launch_bounds__(kTPB) void k_zupdate(const SysDesc* __restrict__ d,
                                                  const SysCtl* __restrict__ ctl,
                                                  const int2* __restrict__ rowmap) {
  extern __shared__ double yl[];  // maxP doubles: the least-squares solution
  const RowCtx c = row_ctx(d, rowmap);
  const SysDesc& D = d[c.s];
  if (ctl[c.s].phase != PH_CYCLE_END) return;
  const int nb = ctl[c.s].ncols;
  if (nb <= 0 || ctl[c.s].first) return;
  const int R = D.r;
  for (int e = threadIdx.x; e < nb * R * R; e += kTPB) yl[e] = D.yv[e];
  __syncthreads();
  LRADI_RSEL(RF, D.r, zupdate_rows<T, RR>(D, c, ctl[c.s].Z, nb, yl));
}

// 14. R = W - (A + s I) Z in FP64 and partial R^T R  (PH_CYCLE_END).
//     Before the first evaluation Z is set to zero and R = W.
template <int R>
__device__ inline void resid_rows(const SysDesc& D, const RowCtx& c, double shift, double* Z,
                                  bool first, double* lds) {
  const double* __restrict__ val = D.val64;
  const int* __restrict__ rp = D.rowptr;
  const int* __restrict__ ci = D.colind;
  constexpr int NG = R * (R + 1) / 2;  // R^T R's packed upper triangle
  double g2[NG];
#pragma unroll
  for (int e = 0; e < NG; ++e) g2[e] = 0.0;
  for (int i = c.row0 + threadIdx.x; i < c.row1; i += kTPB) {
    double rr[R];
#pragma unroll
    for (int q = 0; q < R; ++q) rr[q] = D.W[(size_t)i * R + q];
    if (first) {
#pragma unroll
      for (int q = 0; q < R; ++q) Z[(size_t)i * R + q] = 0.0;
    } else {
      double acc[R];
      const double* __restrict__ mv = D.mval64;
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] = mv ? 0.0 : shift * Z[(size_t)i * R + q];
      // the row's nonzeros four at a time, every gather of a group in
      // flight together (clamped indices, zero coefficients past the row);
      // the terms are added in the row's order
      constexpr int G = 4;
      const int k0 = rp[i], k1 = rp[i + 1];
      for (int k = k0; k < k1; k += G) {
        int col[G];
        double a[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int kk = min(k + u, k1 - 1);
          col[u] = ci[kk];
          a[u] = (mv ? val[kk] + shift * mv[kk] : val[kk]) * (double)(k + u < k1);
        }
        double z[G][R];
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
          for (int q = 0; q < R; ++q) z[u][q] = Z[(size_t)col[u] * R + q];
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
          for (int q = 0; q < R; ++q) acc[q] += a[u] * z[u][q];
      }
#pragma unroll
      for (int q = 0; q < R; ++q) rr[q] -= acc[q];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) D.R[(size_t)i * R + q] = rr[q];
    int e = 0;
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int q = a; q < R; ++q) g2[e++] += rr[a] * rr[q];
  }
  block_sum_store_sym<R>(g2, lds, D.partS + (size_t)c.w * kPS);
}

// complex systems: local row i < nmat gives both halves of the stacked
// residual, R_re = W_re - ((A + s) Z_re - s_im Z_im), R_im = W_im - ((A + s)
// Z_im + s_im Z_re), and the partials of the complex Gram R^* R: its real
// part S = R_re^T R_re + R_im^T R_im at [0, R^2), its imaginary part
// K = R_re^T R_im - R_im^T R_re at [R^2, 2 R^2)
template <int R>
__device__ inline void resid_rows_cplx(const SysDesc& D, const RowCtx& c, double shift, double shift_im,
                                       double* Z, bool first, double* lds) {
  const double* __restrict__ val = D.val64;
  const int* __restrict__ rp = D.rowptr;
  const int* __restrict__ ci = D.colind;
  const int nm = D.nmat;
  double g2[2 * R * R];
#pragma unroll
  for (int e = 0; e < 2 * R * R; ++e) g2[e] = 0.0;
  const int i1 = min(c.row1, nm);
  for (int i = c.row0 + threadIdx.x; i < i1; i += kTPB) {
    double re[R], im[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      re[q] = D.W[(size_t)i * R + q];
      im[q] = D.W[(size_t)(nm + i) * R + q];
    }
    if (first) {
#pragma unroll
      for (int q = 0; q < R; ++q) {
        Z[(size_t)i * R + q] = 0.0;
        Z[(size_t)(nm + i) * R + q] = 0.0;
      }
    } else {
      const double* Zr = Z;
      const double* Zi = Z + (size_t)nm * R;
      double ar[R], ai[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        ar[q] = shift * Zr[(size_t)i * R + q] - shift_im * Zi[(size_t)i * R + q];
        ai[q] = shift * Zi[(size_t)i * R + q] + shift_im * Zr[(size_t)i * R + q];
      }
      for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int col = ci[k];
        const double a = val[k];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          ar[q] += a * Zr[(size_t)col * R + q];
          ai[q] += a * Zi[(size_t)col * R + q];
        }
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        re[q] -= ar[q];
        im[q] -= ai[q];
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      D.R[(size_t)i * R + q] = re[q];
      D.R[(size_t)(nm + i) * R + q] = im[q];
    }
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int q = 0; q < R; ++q) {
        g2[a * R + q] += re[a] * re[q] + im[a] * im[q];
        g2[R * R + a * R + q] += re[a] * im[q] - im[a] * re[q];
      }
  }
  block_sum_store<2 * R * R>(g2, lds, D.partS + (size_t)c.w * kPS);
}

template <int RF>
__global__ __launch_bounds__(kTPB) void k_resid(const SysDesc* __restrict__ d,
                                                const SysCtl* __restrict__ ctl,
                                                const int2* __restrict__ rowmap) {
  __shared__ double lds[4 * kMaxR * kMaxR];
  const RowCtx c = row_ctx(d, rowmap);
  const SysDesc& D = d[c.s];
  if (ctl[c.s].phase != PH_CYCLE_END) return;
  if (D.cplx) {
    LRADI_RSEL(RF, D.r, if constexpr (RR <= 4) resid_rows_cplx<RR>(D, c, ctl[c.s].shift, ctl[c.s].shift_im, ctl[c.s].Z, ctl[c.s].first != 0, lds));
    return;
  }
  LRADI_RSEL(RF, D.r, resid_rows<RR>(D, c, ctl[c.s].shift, ctl[c.s].Z, ctl[c.s].first != 0, lds));
}

// 15. ||R||_2 from R^T R; finish or restart (PH_CYCLE_END).
__global__ __launch_bounds__(kTPB) void k_decide(const SysDesc* __restrict__ d, SysCtl* __restrict__ ctl) {
  __shared__ double red_lds[kTPB];
  __shared__ double G[64];
  const int s = blockIdx.x;
  const SysDesc& D = d[s];
  SysCtl& C = ctl[s];
  if (C.phase != PH_CYCLE_END) return;
  const int R = D.r;
  // complex systems: the Hermitian Gram S + i K of the complex residual;
  // its eigenvalues are those of the real symmetric [S -K; K S] (each
  // twice), so the same routine on 2R x 2R gives ||R||_2^2
  const int P = D.cplx ? 2 * R * R : R * R;
  __shared__ double E[64];
  reduce_partS(D, P, red_lds, G);
  bool bad = false;
  for (int e = 0; e < P; ++e)
    if (!(G[e] == G[e]) || G[e] - G[e] != 0.0) bad = true;
  const double* M = G;
  int NE = R;
  if (D.cplx) {
    NE = 2 * R;
    for (int e = threadIdx.x; e < NE * NE; e += kTPB) {
      const int a = e / NE, b = e % NE, ha = a / R, hb = b / R, aa = a % R, bb = b % R;
      const double sv = G[aa * R + bb], kv = G[R * R + aa * R + bb];
      E[e] = (ha == hb) ? sv : (ha == 0 ? -kv : kv);
    }
    __syncthreads();
    M = E;
  }
  // ||R||_2^2 on the first wavefront's 64 lanes (multisection)
  double lm = 0.0;
  if (!bad && threadIdx.x < 64) lm = lambda_max_sym_lanes<64>(M, NE, threadIdx.x, 0);
  if (threadIdx.x == 0) {
    if (bad) {
      C.status = IS_NAN;
      C.phase = PH_FINISHED;
      C.rnorm = G[0];
      return;
    }
    const double rn = sqrt(fmax(lm, 0.0));
    C.rnorm = rn;
    C.first = 0;
    if (rn <= C.delta) {
      C.phase = PH_FINISHED;
    } else if (C.steps >= D.max_inner) {
      C.status = IS_CAP;
      C.phase = PH_FINISHED;
    } else {
      C.cycles += 1;
      C.r0 = rn;
      C.phase = PH_RESTART;
    }
  }
}

// count of unfinished systems -> host-visible slot
__global__ __launch_bounds__(kTPB) void k_summary(const SysCtl* __restrict__ ctl, int nsys, int* slot) {
  __shared__ int cnt[kTPB];
  int c = 0;
  for (int s = threadIdx.x; s < nsys; s += kTPB) c += (ctl[s].phase != PH_FINISHED) ? 1 : 0;
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int off = kTPB / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) cnt[threadIdx.x] += cnt[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __hip_atomic_store(slot, cnt[0], __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// plain Y = (A + s I) X for one block (no phases); the same tile routine as
// the solver's shifted product, tiles in XCD bands
template <typename T, int R, int RL, bool NT>
__global__ __launch_bounds__(kTPB) void k_spmm_plain(int n, int ntiles, const int* __restrict__ sslot,
                                                     const unsigned char* __restrict__ blk, T shift,
                                                     const T* __restrict__ X, T* __restrict__ Y) {
  const int t = xcd_band_tile((int)blockIdx.x, (int)gridDim.x);
  if (t >= ntiles) return;
  sell_tile<T, R, RL, NT>(n, sslot, blk, false, shift, X, Y, t * spmm_tile_rows(RL));
}

template <typename T, int RF>
int tick_impl(hipStream_t st, const Batch& b, const TickProbe* pr) {
  const dim3 rg(b.rowgrid), tb(kTPB), sg(b.nsys);
  const dim3 redg(b.nsys, (b.maxP + kRedOut - 1) / kRedOut);
  const double fl64 = 1e-24, fl32 = 1e-10;
  if (pr) LRADI_HIP(hipEventRecord(pr->ev[6], st));
  if (b.precond) {
    // row stages: each workgroup's rows in pre_slices slices
    const dim3 rgs(b.rowgrid, b.pre_slices > 1 ? b.pre_slices : 1);
    if (b.sweeps > 0)
      hipLaunchKernelGGL((k_precond<T, RF, 5>), rgs, tb, 0, st, b.d, b.ctl, b.rowmap, 0, b.pairs, b.prof_bytes);
    if (b.sweeps > 0 && b.poly)
      hipLaunchKernelGGL((k_precond<T, RF, 6>), rgs, tb, 0, st, b.d, b.ctl, b.rowmap, 0, b.pairs, b.prof_bytes);
    hipLaunchKernelGGL((k_precond<T, RF, 0>), rgs, tb, 0, st, b.d, b.ctl, b.rowmap, 0, b.pairs, b.prof_bytes);
    int stage = 1;
    if (b.pairs)
      for (; stage + 1 <= b.sweeps; stage += 2) {
        if (b.pair_fast)
          hipLaunchKernelGGL((k_precond<T, RF, 4>), rg, tb, b.pair_lds, st, b.d, b.ctl, b.rowmap, stage, 1,
                             b.prof_bytes);
        else
          hipLaunchKernelGGL((k_precond<T, RF, 3>), rg, tb, b.pair_lds, st, b.d, b.ctl, b.rowmap, stage, 1,
                             b.prof_bytes);
      }
    for (; stage <= b.sweeps; ++stage)
      hipLaunchKernelGGL((k_precond<T, RF, 1>), rgs, tb, 0, st, b.d, b.ctl, b.rowmap, stage, b.pairs,
                         b.prof_bytes);
    hipLaunchKernelGGL((k_precond<T, RF, 2>), rgs, tb, 0, st, b.d, b.ctl, b.rowmap, b.sweeps + 1, b.pairs,
                       b.prof_bytes);
  }
  if (pr) LRADI_HIP(hipEventRecord(pr->ev[7], st));
  if (pr) LRADI_HIP(hipEventRecord(pr->ev[4], st));
  if (b.spcount[0] > 0)
    hipLaunchKernelGGL((k_spmm_arn<T, RF, 1>), dim3(b.spcount[0]), tb, 0, st, b.d, b.ctl,
                       b.spmap + b.spoff[0], b.prof_bytes, -1);
  if constexpr (RF == 0 || RF % 2 == 0)
    if (b.spcount[1] > 0)
      hipLaunchKernelGGL((k_spmm_arn<T, RF, 2>), dim3(b.spcount[1]), tb, 0, st, b.d, b.ctl,
                       b.spmap + b.spoff[1], b.prof_bytes, -1);
  if constexpr (RF == 0 || RF % 4 == 0)
    if (b.spcount[2] > 0)
      hipLaunchKernelGGL((k_spmm_arn<T, RF, 4>), dim3(b.spcount[2]), tb, 0, st, b.d, b.ctl,
                       b.spmap + b.spoff[2], b.prof_bytes, -1);
  if (pr) LRADI_HIP(hipEventRecord(pr->ev[5], st));
  const dim3 gg(b.rowgrid, (b.maxB + kGramBlocks - 1) / kGramBlocks);
  if (pr) LRADI_HIP(hipEventRecord(pr->ev[0], st));
  hipLaunchKernelGGL((k_gram_vu<T, RF>), gg, tb, 0, st, b.d, b.ctl, b.rowmap, b.prof_bytes);
  if (pr) LRADI_HIP(hipEventRecord(pr->ev[1], st));
  hipLaunchKernelGGL(k_reduce_vu, redg, tb, 0, st, b.d, b.ctl, 1);
  const size_t shP = sizeof(double) * (size_t)b.maxP;
  hipLaunchKernelGGL((k_update<T, RF, false>), rg, tb, shP, st, b.d, b.ctl, b.rowmap, -1);
  if (pr) LRADI_HIP(hipEventRecord(pr->ev[2], st));
  hipLaunchKernelGGL((k_gram_vu<T, RF>), gg, tb, 0, st, b.d, b.ctl, b.rowmap, b.prof_bytes);
  if (pr) LRADI_HIP(hipEventRecord(pr->ev[3], st));
  hipLaunchKernelGGL(k_reduce_vu, redg, tb, 0, st, b.d, b.ctl, 0);
  hipLaunchKernelGGL((k_update<T, RF, true>), rg, tb, shP, st, b.d, b.ctl, b.rowmap, -1);
  if (!b.fuse_chol) hipLaunchKernelGGL(k_chol, sg, tb, 0, st, b.d, b.ctl, 0, fl64, fl32, -1);
  hipLaunchKernelGGL((k_scale<T, RF, 0>), rg, tb, 0, st, b.d, b.ctl, b.rowmap, b.fuse_chol, fl64, fl32, -1);
  if (!b.fuse_chol) hipLaunchKernelGGL(k_chol, sg, tb, 0, st, b.d, b.ctl, 1, fl64, fl32, -1);
  hipLaunchKernelGGL((k_scale<T, RF, 1>), rg, tb, 0, st, b.d, b.ctl, b.rowmap, b.fuse_chol, fl64, fl32, -1);
  hipLaunchKernelGGL((k_lsq<RF>), sg, dim3(LsqTPB<RF>::v), shP, st, b.d, b.ctl, -1);
  hipLaunchKernelGGL((k_zupdate<T, RF>), rg, tb, shP, st, b.d, b.ctl, b.rowmap);
  hipLaunchKernelGGL((k_resid<RF>), rg, tb, 0, st, b.d, b.ctl, b.rowmap);
  hipLaunchKernelGGL(k_decide, sg, tb, 0, st, b.d, b.ctl);
  LRADI_HIP(hipGetLastError());
  return LRADI_OK;
}

// The tail of a tick, after the outer step ends: the first cycle end of the
// solves that were just armed (R = W, its norm, then restart or finish),
// then the rebuild of V_0 for every system that restarts (CholQR2 of R and
// the start of a cycle), so that every system enters the next tick in
// PH_ARNOLDI, PH_FINISHED or (when nothing was armed) unchanged, and an
// inner solve of s block steps takes s ticks.  The restart launches serve
// PH_RESTART only (systems in PH_ARNOLDI did their step in this tick).
template <typename T, int RF>
int tail_impl(hipStream_t st, const Batch& b) {
  const dim3 rg(b.rowgrid), tb(kTPB), sg(b.nsys);
  const double fl64 = 1e-24, fl32 = 1e-10;
  const size_t shP = sizeof(double) * (size_t)b.maxP;
  hipLaunchKernelGGL((k_resid<RF>), rg, tb, 0, st, b.d, b.ctl, b.rowmap);
  hipLaunchKernelGGL(k_decide, sg, tb, 0, st, b.d, b.ctl);
  if (b.spcount[0] > 0)
    hipLaunchKernelGGL((k_spmm_arn<T, RF, 1>), dim3(b.spcount[0]), tb, 0, st, b.d, b.ctl,
                       b.spmap + b.spoff[0], b.prof_bytes, (int)PH_RESTART);
  if constexpr (RF == 0 || RF % 2 == 0)
    if (b.spcount[1] > 0)
      hipLaunchKernelGGL((k_spmm_arn<T, RF, 2>), dim3(b.spcount[1]), tb, 0, st, b.d, b.ctl,
                         b.spmap + b.spoff[1], b.prof_bytes, (int)PH_RESTART);
  if constexpr (RF == 0 || RF % 4 == 0)
    if (b.spcount[2] > 0)
      hipLaunchKernelGGL((k_spmm_arn<T, RF, 4>), dim3(b.spcount[2]), tb, 0, st, b.d, b.ctl,
                         b.spmap + b.spoff[2], b.prof_bytes, (int)PH_RESTART);
  hipLaunchKernelGGL((k_update<T, RF, true>), rg, tb, shP, st, b.d, b.ctl, b.rowmap, (int)PH_RESTART);
  if (!b.fuse_chol) hipLaunchKernelGGL(k_chol, sg, tb, 0, st, b.d, b.ctl, 0, fl64, fl32, (int)PH_RESTART);
  hipLaunchKernelGGL((k_scale<T, RF, 0>), rg, tb, 0, st, b.d, b.ctl, b.rowmap, b.fuse_chol, fl64, fl32,
                     (int)PH_RESTART);
  if (!b.fuse_chol) hipLaunchKernelGGL(k_chol, sg, tb, 0, st, b.d, b.ctl, 1, fl64, fl32, (int)PH_RESTART);
  hipLaunchKernelGGL((k_scale<T, RF, 1>), rg, tb, 0, st, b.d, b.ctl, b.rowmap, b.fuse_chol, fl64, fl32,
                     (int)PH_RESTART);
  hipLaunchKernelGGL((k_lsq<RF>), sg, dim3(LsqTPB<RF>::v), shP, st, b.d, b.ctl, (int)PH_RESTART);
  LRADI_HIP(hipGetLastError());
  return LRADI_OK;
}

template <typename T>
int tail_dispatch(hipStream_t st, const Batch& b) {
  switch (b.rfix) {
    case 1: return tail_impl<T, 1>(st, b);
    case 2: return tail_impl<T, 2>(st, b);
    case 3: return tail_impl<T, 3>(st, b);
    case 4: return tail_impl<T, 4>(st, b);
    case 5: return tail_impl<T, 5>(st, b);
    case 6: return tail_impl<T, 6>(st, b);
    case 7: return tail_impl<T, 7>(st, b);
    case 8: return tail_impl<T, 8>(st, b);
    default: return tail_impl<T, 0>(st, b);
  }
}

template <typename T>
int tick_dispatch(hipStream_t st, const Batch& b, const TickProbe* pr) {
  switch (b.rfix) {
    case 1: return tick_impl<T, 1>(st, b, pr);
    case 2: return tick_impl<T, 2>(st, b, pr);
    case 3: return tick_impl<T, 3>(st, b, pr);
    case 4: return tick_impl<T, 4>(st, b, pr);
    case 5: return tick_impl<T, 5>(st, b, pr);
    case 6: return tick_impl<T, 6>(st, b, pr);
    case 7: return tick_impl<T, 7>(st, b, pr);
    case 8: return tick_impl<T, 8>(st, b, pr);
    default: return tick_impl<T, 0>(st, b, pr);
  }
}

}  // namespace

int launch_tick(hipStream_t st, const Batch& b, const TickProbe* probe) {
  if (b.precision == LRADI_FP64) return tick_dispatch<double>(st, b, probe);
  return tick_dispatch<float>(st, b, probe);
}

int launch_tick_tail(hipStream_t st, const Batch& b) {
  if (b.precision == LRADI_FP64) return tail_dispatch<double>(st, b);
  return tail_dispatch<float>(st, b);
}

int launch_summary(hipStream_t st, const Batch& b, int* host_slot) {
  hipLaunchKernelGGL(k_summary, dim3(1), dim3(kTPB), 0, st, b.ctl, b.nsys, host_slot);
  LRADI_HIP(hipGetLastError());
  return LRADI_OK;
}

namespace {
template <typename T, bool NT>
int spmm_plain_t(hipStream_t st, int n, int r, int lanes, const int* sslot, const unsigned char* blk, T shift,
                 const T* X, T* Y) {
  const int ntiles = (n + spmm_tile_rows(lanes) - 1) / spmm_tile_rows(lanes);
  const dim3 g(xcd_grid(ntiles)), tb(kTPB);
  LRADI_DISPATCH_R(r, {
    if (lanes == 1) {
      hipLaunchKernelGGL((k_spmm_plain<T, RR, 1, NT>), g, tb, 0, st, n, ntiles, sslot, blk, shift, X, Y);
    } else if (lanes == 2) {
      if constexpr (RR % 2 == 0)
        hipLaunchKernelGGL((k_spmm_plain<T, RR, 2, NT>), g, tb, 0, st, n, ntiles, sslot, blk, shift, X, Y);
    } else {
      if constexpr (RR % 4 == 0)
        hipLaunchKernelGGL((k_spmm_plain<T, RR, 4, NT>), g, tb, 0, st, n, ntiles, sslot, blk, shift, X, Y);
    }
  });
  LRADI_HIP(hipGetLastError());
  return LRADI_OK;
}
}  // namespace

int launch_spmm_plain(hipStream_t st, int n, int r, int precision, int lanes, const int* sslot,
                      const unsigned char* blk, double shift, const void* X, void* Y, bool nt) {
  if (n <= 0) return LRADI_OK;
  if (r < 1 || r > kMaxR || !(lanes == 1 || lanes == 2 || lanes == 4) || r % lanes != 0)
    return LRADI_EINVAL;
  if (precision == LRADI_FP64) {
    auto x = static_cast<const double*>(X);
    auto y = static_cast<double*>(Y);
    return nt ? spmm_plain_t<double, true>(st, n, r, lanes, sslot, blk, shift, x, y)
              : spmm_plain_t<double, false>(st, n, r, lanes, sslot, blk, shift, x, y);
  }
  auto x = static_cast<const float*>(X);
  auto y = static_cast<float*>(Y);
  return nt ? spmm_plain_t<float, true>(st, n, r, lanes, sslot, blk, (float)shift, x, y)
            : spmm_plain_t<float, false>(st, n, r, lanes, sslot, blk, (float)shift, x, y);
}

}  // namespace lradi
