// Internal declarations of the lradi library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/lradi.h"

namespace lradi {

constexpr int kMaxR = 8;        // widest right-hand-side block
constexpr int kMaxM = 64;       // longest block GMRES restart cycle (blocks)
constexpr int kTPB = 256;       // threads of a row workgroup (4 wavefronts)
constexpr int kSmallTPB = 64;   // threads of a per-system workgroup (1 wavefront)
constexpr int kHistCols = LRADI_HIST_COLS;
constexpr int kPS = 128;        // stride of the small Gram partial rows
// CholQR factors are formed inside the scale kernels when every system's
// small Gram partials (nwg x r^2 values) are at most this many
constexpr int kFuseCholMax = 8192;
// paired Schur sweeps: a tile's region (rows + halo) iterate must fit this
// many bytes of LDS, and the regions may hold at most kPairMaxRegion times
// the black rows.  Breadth-first tiles of 2-D five-point grids come to
// 1.2-1.4 times, of 3-D seven-point grids to 1.9-2.6 times; there the first
// sweep's halo rows cost more than the launch a pair saves (64^3 and 48^3,
// r = 8: 35 us per paired launch against 15 us per single one).
constexpr int kPairLdsMax = 64 * 1024;
// matrices of fewer rows keep their black rows in ascending order and do
// not pair: they are mostly solved in batches that fill the chip, where a
// sweep is throughput-bound and whole grid rows per wavefront gather with
// fuller cache lines than a tile's short row segments (256 problems of
// 32^2..128^2: 1.04 s in ascending order, 1.16 s in tile order)
constexpr int kPairMinRows = 32768;
// pairs pay while a launch is latency-bound: a batch whose preconditioned
// black rows exceed this many (about half the threads the chip holds)
// fills the chip, and there the halo rows' extra work costs more than the
// launch a pair saves (256 problems of 32^2..128^2: 1.16 s paired against
// 1.01 s with single sweeps)
constexpr long long kPairMaxRows = 262144;
constexpr int kPairRegSlots = 8;
constexpr double kPairMaxRegion = 1.6;

// Device pointers held in descriptor tables are generic (flat) to the
// compiler; casting them to the global address space lets it issue global
// loads (no LDS-aperture check, vector-memory counter only).
template <typename T>
__device__ inline const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ inline __attribute__((address_space(1))) T* gmem_w(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// ---------------------------------------------------------------------------
// Reduce-scatter of per-lane values across a wavefront.  Every lane holds
// NV (a power of two) values; the sum runs over the lanes that differ only
// in lane-index bits LO, 2 LO, ..., 32.  At each xor step a lane keeps one
// half of its values and adds the partner's copy of that half, so the step
// costs NV/2 shuffles instead of NV; once a lane holds one value the
// remaining steps are plain butterflies.  Afterwards v[0..NV >> H) (H =
// halving steps) hold complete sums of value indices wave_rs_base() + i.
// The order of every addition is fixed by the lane pattern alone.
constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }
constexpr int pow2c(int x) { return x <= 1 ? 1 : 2 * pow2c((x + 1) / 2); }

template <int CNT, int OFF, int LO, int NV>
__device__ inline void wave_rs_step(double (&v)[NV], int lane) {
  if constexpr (OFF >= LO) {
    if constexpr (CNT > 1) {
      constexpr int h = CNT / 2;
      const bool up = (lane & OFF) != 0;
#pragma unroll
      for (int i = 0; i < h; ++i) {
        const double send = up ? v[i] : v[i + h];
        const double keep = up ? v[i + h] : v[i];
        v[i] = keep + __shfl_xor(send, OFF, 64);
      }
      wave_rs_step<h, OFF / 2, LO, NV>(v, lane);
    } else {
      v[0] += __shfl_xor(v[0], OFF, 64);
      wave_rs_step<1, OFF / 2, LO, NV>(v, lane);
    }
  }
}

template <int NV, int LO>
__device__ inline void wave_reduce_scatter(double (&v)[NV], int lane) {
  wave_rs_step<NV, 32, LO, NV>(v, lane);
}

template <int NV, int LO>
struct WaveRS {
  static constexpr int S = ilog2c(64 / LO);               // xor steps
  static constexpr int H = S < ilog2c(NV) ? S : ilog2c(NV);  // halving steps
  static constexpr int NOUT = NV >> H;                    // sums left per lane
  static constexpr int DUP = (64 >> H) - LO;              // lane bits of equal copies
};

template <int NV, int LO>
__device__ inline int wave_rs_base(int lane) {
  int base = 0, cnt = NV;
#pragma unroll
  for (int off = 32; off >= LO; off >>= 1) {
    if (cnt > 1) {
      cnt >>= 1;
      if (lane & off) base += cnt;
    }
  }
  return base;
}

// Shifted-product tiling: `lanes` lanes share one matrix row, each owning
// r / lanes of its columns, so a tile covers kTPB / lanes rows (a wavefront
// 64 / lanes of them).  lanes is 1, 2 or 4 and divides r.
constexpr int spmm_tile_rows(int lanes) { return kTPB / lanes; }
// The shifted product reads the matrix in a blocked sliced ELL layout:
// slices of kSellH consecutive rows, each padded to its longest row (at
// least one slot), padding entries (own row, value 0).  A slice is a run of
// slot blocks, one per slot u: the kSellH column indices of slot u, then its
// kSellH values (then, for a pencil, M's kSellH values), so a wavefront's
// column and value loads of a slot are contiguous and adjacent, without
// staging through LDS.  Slice s owns slot blocks sslot[s] .. sslot[s+1]-1.
constexpr int kSellH = 32;
__host__ __device__ constexpr int sell_block_bytes(int tsz, bool mass) { return kSellH * (4 + tsz * (mass ? 2 : 1)); }
// Workgroup b of a launch runs on XCD b % 8.  Row chunks and product tiles
// are assigned to the XCDs in contiguous bands (the solver's tables by the
// host, the standalone product by xcd_band_tile), so that the rows a
// stencil couples across planes are gathered through the same L2.
constexpr int kXcds = 8;
__host__ __device__ constexpr int xcd_grid(int tiles) { return kXcds * ((tiles + kXcds - 1) / kXcds); }
__device__ inline int xcd_band_tile(int b, int grid) {
  const int band = grid / kXcds;
  return (b % kXcds) * band + b / kXcds;
}
// Default lanes per row: the widest split that still leaves each lane 32
// contiguous bytes of every gathered row of X (two 128-bit loads; narrower
// splits multiply the per-slot column and value loads without adding bytes
// in flight).
inline int spmm_rule_lanes(int r, int tsz) {
  int rl = 1;
  while (rl < 4 && r % (2 * rl) == 0 && r * tsz / (2 * rl) >= 32) rl *= 2;
  return rl;
}

// Phases of one inner solve; every kernel of the batched solver checks the
// phase of its system and returns at once when it is not the one it serves.
enum Phase : int {
  PH_ARNOLDI = 0,    // extend the basis by one block (block Arnoldi step)
  PH_RESTART = 1,    // (re)build V_0 from the refinement residual R
  PH_CYCLE_END = 2,  // update Z, recompute the FP64 residual, decide
  PH_FINISHED = 3,   // converged or out of budget; all kernels skip
};

enum InnerStatus : int { IS_OK = 0, IS_CAP = 1, IS_BREAKDOWN = 2, IS_NAN = 3 };

// Read-only description of one shifted block system (A + shift I) Z = W.
struct SysDesc {
  int n, r, m;          // rows, right-hand sides, restart length (blocks)
  int nwg;              // row workgroups of this system
  int rows_per_wg;      // rows handled by each of them
  int wg0;              // first of them in the batched row grid
  int precision;        // LRADI_FP64 / LRADI_FP32_INNER
  int max_inner;        // Arnoldi step cap
  const int* rowptr;
  const int* colind;
  const void* valT;     // values in the basis precision
  // the same matrix in the shifted product's blocked sliced ELL layout
  // (kSellH): slot-block starts per slice and the blocks (columns, values
  // and, for pencils, M's values in the basis precision)
  const int* sslot;
  const unsigned char* sblk;
  const double* val64;  // FP64 values (refinement residual)
  double floor_rel;     // a cycle stops once est <= floor_rel * (start norm)
  const double* W;      // right-hand side, n x r
  double* R;            // FP64 refinement residual, n x r
  void* V;              // basis, (m+1) blocks of n x r, basis precision
  void* U;              // candidate block, n x r, basis precision
  double* part;         // per-workgroup Gram partials, nwg x pstride
  double* partS;        // per-workgroup small Gram partials, nwg x kPS
  double* partS2;       // the same for the second CholQR pass, nwg x kPS
  double* red;          // reduced projection coefficients, (m+1) r^2
  double* hacc;         // Hessenberg column block being built, (m+1) r^2
  double* Rt;           // triangular factor, (m r) x (m r), column-major
  double* Qs;           // per column block orthogonal 2r x 2r factors, m x 4r^2
  double* Gv;           // rotated right-hand side, (m+1) r x r, row-major
  double* yv;           // least-squares solution, m r x r, row-major
  double* sm;           // small scratch (8 x 64 doubles)
  int pstride;          // stride of part rows (>= (m+1) r^2)
  int nnz;              // nonzeros of A
  int spmm_lanes;       // lanes per row of the shifted product (1, 2, 4)
  // generalized equation: the system is (A + shift M) Z = W with M's values
  // on A's (union) pattern; null for M = I (then the shift is added to the
  // diagonal)
  const void* mvalT;    // M's values in the basis precision
  const double* mval64; // M's values in FP64 (refinement residual, M z)
  // red-black ILU(0) right preconditioner (null rbrows: none): Arnoldi
  // multiplies S P_j with P_j = M V_j, and Z += sum_b P_b y_b
  const int* rbrows;    // red rows ascending, then black rows ascending
  int nred;             // number of red rows
  int sweeps;           // Jacobi sweeps on the Schur complement
  int poly;             // 1: the sweeps are Chebyshev steps (bounds and
                        // coefficients in sm + SM_CHEB), 0: Jacobi
  const void* diagT;    // diagonal of A per row, basis precision
  const void* msT;      // pencils: M's row sums (the preconditioner's shift
                        // weights), basis precision; null for M = I
  // off-diagonal entries by colour position p (row rbrows[p]), rbw slots
  // each, slot-major (slot u of position p at u * n + p); unused slots hold
  // the row itself with value 0
  int rbw;
  const int* ellci;
  const void* ellvalT;  // A's entry (i, col), basis precision
  const void* elltvT;   // A's entry (col, i), basis precision
  void* P;              // preconditioned basis blocks P_0..P_m, basis precision
  void* Yb;             // sweeps: y of the black rows by black position, basis precision
  void* Eb;             // sweeps: two black iterates by black position
                        // (four for Chebyshev steps with pair_lds > 0)
  void* It;             // sweeps: 1 / diag(T) by black position
  // sweeps: the off-diagonal entries of T = D_b - F D_r^{-1} E by black
  // position (pb = p - nred), slot-major with nb = n - nred: columns t2ci
  // as black positions (t2w slots, unused: its own) and values t2val, rebuilt for each
  // shift by walking two hops through the slot tables; rbpos[row] is the
  // row's colour position
  int t2w;
  const int* t2ci;
  const int* t2rev;     // the transposed entry's slot per slot (RbHost::t2rev)
  const int* rbpos;
  void* t2val;
  // paired sweeps: the black positions in tiles of ceil(nb / nwg), tile w
  // owned by row workgroup w; its halo (the black positions outside it
  // that its rows' T columns reach) at halo[halo_off[w] .. halo_off[w + 1]),
  // and t2lc, T's columns (slot-major like t2ci) as indices into the tile's
  // region, its own rows first, then its halo
  const int* halo_off;
  const int* halo;
  const int* t2lc;
  const int* halo_ci;   // the halo rows' T columns, slot-major over halo entries
  int nhalo;            // total halo entries
  int pair_lds;         // bytes of the largest region's iterate; 0: no pairs
  // complex shift (s + i s_im, Sec. 3.2.4's complex form): the system is the
  // real form of (A + (s + i s_im) I)(z_re + i z_im) = w_re + i w_im on the
  // stacked block [re; im] of n = 2 nmat rows,
  //   [A + s I, -s_im I; s_im I, A + s I] [z_re; z_im] = [w_re; w_im],
  // and ||.||_2 of a residual is the complex block's spectral norm
  int cplx;             // 1: complex system (r <= 4, no preconditioner)
  int nmat;             // rows of A (n / 2 when complex, else n)
};

// Mutable device-side control block of one inner solve.
struct SysCtl {
  double* Z;    // solution block, n x r (set per solve)
  double shift; // the system is (A + shift I) Z = W
  double shift_im;  // complex systems: imaginary part of the shift
  int phase;
  int j;        // Arnoldi step index inside the cycle (basis blocks V_0..V_j exist)
  int ncols;    // block columns of the current least-squares problem
  int steps;    // total block Arnoldi steps
  int cycles;   // restart cycles started
  int status;   // InnerStatus
  int breakdowns;
  int first;    // 1 before the first residual evaluation (Z = 0)
  double delta; // target ||W - S Z||_2
  double est;   // least-squares residual estimate of the current cycle
  double rnorm; // last FP64 ||W - S Z||_2
  double r0;    // ||R|| at the start of the current cycle
};

// small scratch slots (offsets into SysDesc::sm, 64 doubles each)
// SM_CHEB: the Chebyshev sweeps' spectral bounds of the current shift (hi,
// then max(0, max P_ii / T_ii), as non-negative doubles combined by integer
// atomic max), gamma (0: Jacobi fallback) and omega_2 .. omega_{sweeps+1}
enum SmSlot { SM_S1 = 0, SM_S1I = 64, SM_S2 = 128, SM_S2I = 192, SM_G = 256, SM_T = 320, SM_CHEB = 384 };
constexpr int kChebGamma = 2, kChebOmega = 3;  // offsets in SM_CHEB
constexpr int kSmDoubles = 512;  // per-system small scratch (doubles)
static_assert(SM_CHEB + kChebOmega + 64 <= kSmDoubles, "Chebyshev table exceeds the small scratch");

// ---------------------------------------------------------------------------
// error state
void set_error(const char* fmt, ...);
#define LRADI_HIP(call)                                                            \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::lradi::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),   \
                         __FILE__, __LINE__);                                     \
      return LRADI_EHIP;                                                          \
    }                                                                             \
  } while (0)

#define LRADI_TRY(expr)      \
  do {                       \
    int st_ = (expr);        \
    if (st_ < 0) return st_; \
  } while (0)

// ---------------------------------------------------------------------------
// device memory helper: a typed owning buffer
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  int alloc(size_t nbytes);
  void release();
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Device copy of a CSR matrix in FP64 and FP32.
// Red-black preconditioner data of one matrix: colour-ordered rows and each
// row's colour position, the diagonal, the off-diagonal entries by colour
// position in rbw slot-major slots (column, value, transposed value), and
// the Schur complement's column pattern on the black rows (t2w slots).
// A table inside another buffer (not owned).
struct DevView {
  void* p = nullptr;
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

struct RbData {
  DevBuf arena;  // every table below, in one allocation
  DevView rbrows, rbpos, diag64, diag32, ellci, ellval64, ellval32, elltv64, elltv32, t2ci, t2rev;
  // pencils A + s M: the preconditioner takes M's row sums (lumped mass)
  // as the per-row weight of the shift; null for M = I
  DevView ms64, ms32;
  // tiles of the black positions for paired sweeps (halo lists and T's
  // columns as region-local indices; see RbHost)
  DevView halo_off, halo, t2lc, halo_ci;
  int nred = 0, rbw = 0, t2w = 0;
  int tile = 0, ntile = 0, maxreg = 0, nhalo = 0;
};

struct DevCSR {
  int n = 0;
  int64_t nnz = 0;
  DevBuf rowptr, colind, val64, val32;
  DevBuf mval64, mval32;  // the mass matrix of a pencil, on the same pattern
  // blocked sliced ELL copy for the shifted product (kSellH rows per
  // slice): slot-block starts (nsl + 1) and the FP64 / FP32 blocks (with M's
  // values for a pencil); built by build_sell (upload() when asked for,
  // upload_pencil() once M's values are there)
  int nsl = 0;
  DevBuf sslot, sblk64, sblk32;
  bool has_sell() const { return sslot.p != nullptr; }
  int build_sell(const int32_t* host_rowptr, hipStream_t st, bool need32);
  // red-black preconditioner data (prepare_rb), shared with the context's
  // cache of prepared matrices
  std::shared_ptr<const RbData> rb;
  int upload(const lradi_csr* A, hipStream_t st, bool need32, bool sell = true);
  // the pencil (A, M): union pattern, A's values and M's values
  int upload_pencil(const lradi_csr* A, const lradi_csr* M, hipStream_t st, bool need32);
  bool has_mass() const { return mval64.p != nullptr; }
  // 2-colour the sparsity graph of A (the matrix uploaded here) and upload
  // the colour-ordered rows, A's diagonal and its transposed values;
  // LRADI_EINVAL if the graph is not bipartite
  // (M: the mass matrix of a pencil, or null)
  int prepare_rb(lradi_ctx* ctx, const lradi_csr* A, const lradi_csr* M, hipStream_t st, bool need32);
  bool has_rb() const { return rb != nullptr; }
};

// Borrowed view of a device CSR matrix (FP64 values).
struct CsrRef {
  int n = 0;
  const int* rowptr = nullptr;
  const int* colind = nullptr;
  const double* val = nullptr;
};
inline CsrRef csr_ref(const DevCSR& A) {
  return CsrRef{A.n, A.rowptr.as<int>(), A.colind.as<int>(), A.val64.as<double>()};
}

// True residual norm ||A X C + M X B + f g^T||_2 of X = Z diag(gam) Y^T by
// Golub-Kahan-Lanczos (residual.hip): residual_norm allocates its workspace,
// residual_norm_ws works in a caller-provided one of residual_ws_bytes.
size_t residual_ws_bytes(int n, int m, int maxit, bool hasM, bool hasC);
int residual_norm_ws(hipStream_t st, const CsrRef& A, const CsrRef& At, const CsrRef& B, const CsrRef& Bt,
                     const double* f, const double* g, int r, const double* Z, const double* gam_d,
                     const double* Y, int k, int maxit, double* sigma_out, const CsrRef* M,
                     const CsrRef* Mt, const CsrRef* C, const CsrRef* Ct, double* ws);
int residual_norm(hipStream_t st, const DevCSR& A, const DevCSR& At, const DevCSR& B, const DevCSR& Bt,
                  const double* f, const double* g, int r, const double* Z, const double* gam_d,
                  const double* Y, int k, int maxit, double* sigma_out, const DevCSR* M = nullptr,
                  const DevCSR* Mt = nullptr, const DevCSR* C = nullptr, const DevCSR* Ct = nullptr);

// ---------------------------------------------------------------------------
// kernel launchers (kernels.hip)
// Y = (A + shift I) X on the blocked sliced ELL copy of a DevCSR (no mass
// values); nt: matrix loads and output stores with the nontemporal hint
// (operands far beyond the last-level cache)
int launch_spmm_plain(hipStream_t st, int n, int r, int precision, int lanes, const int* sslot,
                      const unsigned char* sblk, double shift, const void* X, void* Y, bool nt);

// The batched inner solver: all systems of a batch share one precision.
struct Batch {
  const SysDesc* d;    // device array of nsys
  SysCtl* ctl;         // device array of nsys
  const int2* rowmap;  // device array of rowgrid entries (system, chunk)
  int nsys;
  int rowgrid;
  // shifted-product tiles (system, tile), grouped by lanes per row: group g
  // (lanes 1, 2, 4) holds spcount[g] entries starting at spmap + spoff[g]
  const int2* spmap;
  int spoff[3], spcount[3];
  int maxP;            // max over systems of (m+1) r^2
  int maxB;            // max over systems of m+1 (basis blocks)
  int precision;       // LRADI_FP64 / LRADI_FP32_INNER
  int rfix;            // common r of all systems, or 0 when they differ
  int precond;         // some system carries the red-black preconditioner
  int sweeps;          // its Jacobi sweeps (shared by the batch)
  int poly;            // some system takes Chebyshev steps (a launch of
                       // their spectral bounds per inner solve)
  int pairs;           // 1: two sweeps per launch (every preconditioned
                       // system has pair_lds > 0)
  int pair_lds;        // dynamic LDS bytes of a paired launch
  int pair_fast;       // 1: every tile fits one row per thread, T has at
                       // most kPairRegSlots slots and r is common and <= 4
                       // (the paired kernel keeps the second sweep's region
                       // columns in registers)
  int precond_launches;  // launches of one preconditioner application
  int pre_slices;      // slices per row workgroup of the preconditioner's
                       // row stages (second grid dimension, >= 1)
  int fuse_chol;       // 1: every scale workgroup reduces the small Gram
                       // partials and factors them itself (common r <= 4
                       // and small nwg r^2)
  unsigned long long* prof_bytes;  // device counters per kernel class, or null
};

// Optional timing events around the instrumented launches of one tick:
// [0,1] first projection, [2,3] second projection, [4,5] shifted product.
struct TickProbe {
  hipEvent_t ev[8];
};
// One scheduling tick: a block Arnoldi step (or the rebuild of V_0) for every
// system in PH_ARNOLDI / PH_RESTART, then the end-of-cycle work for every
// system in PH_CYCLE_END.
int launch_tick(hipStream_t st, const Batch& b, const TickProbe* probe = nullptr);
// After the outer step end of a tick: the first cycle end of the freshly
// armed solves and the V_0 rebuild of every restarting system.
int launch_tick_tail(hipStream_t st, const Batch& b);
// Count of systems not yet finished, written to a host-visible int.
int launch_summary(hipStream_t st, const Batch& b, int* host_slot);

}  // namespace lradi
