// Host side of the lradi library: context, device buffers, the batched
// inner-solve scheduler and the outer LR-ADI loop (Algorithm 1), and the
// C ABI entry points declared in include/lradi.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <list>
#include <functional>
#include <future>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "adi.h"
#include "internal.h"
#include "rbhost.h"

namespace lradi {

void csr_transpose(int n, const int32_t* rp, const int32_t* ci, const double* v,
                   std::vector<int32_t>& trp, std::vector<int32_t>& tci, std::vector<double>& tv);
void csr_union(int n, const int32_t* prp, const int32_t* pci, const double* pv, const int32_t* qrp,
               const int32_t* qci, const double* qv, std::vector<int32_t>& urp,
               std::vector<int32_t>& uci, std::vector<double>& upv, std::vector<double>& uqv);

// ---------------------------------------------------------------------------
// errors
static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}


// ---------------------------------------------------------------------------
// buffers
// device allocations made by the library since the process started
std::atomic<int64_t> g_alloc_count{0};

int DevBuf::alloc(size_t nbytes) {
  release();
  if (nbytes == 0) return LRADI_OK;
  g_alloc_count.fetch_add(1, std::memory_order_relaxed);
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    p = nullptr;
    set_error("hipMalloc(%zu bytes) failed: %s", nbytes, hipGetErrorString(e));
    return LRADI_ENOMEM;
  }
  bytes = nbytes;
  return LRADI_OK;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

// ---------------------------------------------------------------------------
// Scratch memory of lradi_residual_noalloc: a file-scope device array that
// each device holds from module load to process end.  Host code never uses
// its name as an address: the address on each device comes from
// hipGetSymbolAddress (looked up once per device when a context is created
// there) and is kept in g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;                  // guards g_scratch_ptr and serialises the calls per device
double* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` on each device
std::mutex g_scratch_call_mu[kMaxDevices];

// With `device` current: record the address of `scratch` on it (once).
int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return set_error("device ordinal %d above the scratch table", device), LRADI_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return LRADI_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    return LRADI_EHIP;
  }
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return LRADI_OK;
}

namespace {

__global__ void k_d2f(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// one thread per (padded) row: its slots of the slice's blocks, padding
// (own row, 0); mval null: no mass values
template <typename T>
__global__ void k_sell_fill(int n, int nsl, const int* __restrict__ rp, const int* __restrict__ sslot,
                            const int* __restrict__ ci, const double* __restrict__ val,
                            const double* __restrict__ mval, unsigned char* __restrict__ blk) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nsl * kSellH) return;
  const int i = (int)t, s = i / kSellH, l = i % kSellH;
  const int k0 = i < n ? rp[i] : 0;
  const int len = i < n ? rp[i + 1] - k0 : 0;
  const int sb = sell_block_bytes((int)sizeof(T), mval != nullptr);
  unsigned char* base = blk + (size_t)sslot[s] * sb;
  const int w = sslot[s + 1] - sslot[s];
  for (int u = 0; u < w; ++u) {
    unsigned char* b = base + (size_t)u * sb;
    const bool in = u < len;
    reinterpret_cast<int*>(b)[l] = in ? ci[k0 + u] : (i < n ? i : n - 1);
    reinterpret_cast<T*>(b + kSellH * 4)[l] = in ? (T)val[k0 + u] : T(0);
    if (mval) reinterpret_cast<T*>(b + kSellH * (4 + sizeof(T)))[l] = in ? (T)mval[k0 + u] : T(0);
  }
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

}  // namespace

int DevCSR::build_sell(const int32_t* rph, hipStream_t st, bool need32) {
  // slot-block starts per slice: each slice as wide as its longest row
  nsl = (n + kSellH - 1) / kSellH;
  std::vector<int> ss(nsl + 1);
  int64_t e = 0;
  for (int s = 0; s < nsl; ++s) {
    int w = 1;
    for (int i = s * kSellH; i < std::min(n, s * kSellH + kSellH); ++i) w = std::max(w, rph[i + 1] - rph[i]);
    ss[s] = (int)e;
    e += w;
    if (e > INT32_MAX) return set_error("sliced layout exceeds int32 slot indexing"), LRADI_EINVAL;
  }
  ss[nsl] = (int)e;
  const bool mass = has_mass();
  LRADI_TRY(sslot.alloc(sizeof(int) * ss.size()));
  LRADI_HIP(hipMemcpyAsync(sslot.p, ss.data(), sizeof(int) * ss.size(), hipMemcpyHostToDevice, st));
  const int tpb = 256;
  const dim3 g((unsigned)(((int64_t)nsl * kSellH + tpb - 1) / tpb)), tb(tpb);
  const double* mv = mass ? mval64.as<double>() : nullptr;
  LRADI_TRY(sblk64.alloc((size_t)e * sell_block_bytes(8, mass)));
  hipLaunchKernelGGL(k_sell_fill<double>, g, tb, 0, st, n, nsl, rowptr.as<int>(), sslot.as<int>(),
                     colind.as<int>(), val64.as<double>(), mv, sblk64.as<unsigned char>());
  LRADI_HIP(hipGetLastError());
  if (need32) {
    // FP32 values rounded from the FP64 ones, as val32
    LRADI_TRY(sblk32.alloc((size_t)e * sell_block_bytes(4, mass)));
    hipLaunchKernelGGL(k_sell_fill<float>, g, tb, 0, st, n, nsl, rowptr.as<int>(), sslot.as<int>(),
                       colind.as<int>(), val64.as<double>(), mv, sblk32.as<unsigned char>());
    LRADI_HIP(hipGetLastError());
  }
  // the host slot-block starts must outlive their copy
  LRADI_HIP(hipStreamSynchronize(st));
  return LRADI_OK;
}

int DevCSR::upload(const lradi_csr* A, hipStream_t st, bool need32, bool sell) {
  if (!A || A->nrows <= 0 || A->nrows != A->ncols || A->nnz < 0 || !A->rowptr ||
      (A->nnz > 0 && (!A->colind || !A->val))) {
    set_error("invalid csr argument (square, nrows > 0, non-null arrays required)");
    return LRADI_EINVAL;
  }
  if (A->nnz > INT32_MAX) {
    set_error("csr nnz exceeds int32 indexing");
    return LRADI_EINVAL;
  }
  n = A->nrows;
  nnz = A->nnz;
  const hipMemcpyKind kind = A->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (!A->on_device) {
    // host data: validate structure before it reaches a kernel
    const int32_t* rp = A->rowptr;
    if (rp[0] != 0 || rp[n] != nnz) {
      set_error("csr rowptr must start at 0 and end at nnz");
      return LRADI_EINVAL;
    }
    for (int i = 0; i < n; ++i)
      if (rp[i + 1] < rp[i]) {
        set_error("csr rowptr not monotone at row %d", i);
        return LRADI_EINVAL;
      }
    for (int64_t k = 0; k < nnz; ++k)
      if (A->colind[k] < 0 || A->colind[k] >= n) {
        set_error("csr column index out of range at %lld", (long long)k);
        return LRADI_EINVAL;
      }
  }
  LRADI_TRY(rowptr.alloc(sizeof(int32_t) * (n + 1)));
  LRADI_TRY(colind.alloc(sizeof(int32_t) * std::max<int64_t>(nnz, 1)));
  LRADI_TRY(val64.alloc(sizeof(double) * std::max<int64_t>(nnz, 1)));
  LRADI_HIP(hipMemcpyAsync(rowptr.p, A->rowptr, sizeof(int32_t) * (n + 1), kind, st));
  if (nnz > 0) {
    LRADI_HIP(hipMemcpyAsync(colind.p, A->colind, sizeof(int32_t) * nnz, kind, st));
    LRADI_HIP(hipMemcpyAsync(val64.p, A->val, sizeof(double) * nnz, kind, st));
  }
  if (A->on_device) {
    // device data: check the structure on a host copy of the index arrays
    std::vector<int32_t> rp(n + 1), ci(nnz);
    LRADI_HIP(hipMemcpyAsync(rp.data(), A->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, st));
    if (nnz > 0)
      LRADI_HIP(hipMemcpyAsync(ci.data(), A->colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st));
    LRADI_HIP(hipStreamSynchronize(st));
    if (rp[0] != 0 || rp[n] != nnz) {
      set_error("csr rowptr must start at 0 and end at nnz");
      return LRADI_EINVAL;
    }
    for (int i = 0; i < n; ++i)
      if (rp[i + 1] < rp[i]) {
        set_error("csr rowptr not monotone at row %d", i);
        return LRADI_EINVAL;
      }
    for (int64_t k = 0; k < nnz; ++k)
      if (ci[k] < 0 || ci[k] >= n) {
        set_error("csr column index out of range at %lld", (long long)k);
        return LRADI_EINVAL;
      }
  }
  if (need32) {
    LRADI_TRY(val32.alloc(sizeof(float) * std::max<int64_t>(nnz, 1)));
    if (nnz > 0) {
      const int tpb = 256;
      hipLaunchKernelGGL(k_d2f, dim3((unsigned)((nnz + tpb - 1) / tpb)), dim3(tpb), 0, st,
                         val64.as<double>(), val32.as<float>(), nnz);
      LRADI_HIP(hipGetLastError());
    }
  }
  if (sell) {
    std::vector<int32_t> hrp;
    const int32_t* rph = A->rowptr;
    if (A->on_device) {
      hrp.resize(n + 1);
      LRADI_HIP(hipMemcpy(hrp.data(), A->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
      rph = hrp.data();
    }
    LRADI_TRY(build_sell(rph, st, need32));
  }
  return LRADI_OK;
}

// ---------------------------------------------------------------------------
// pinned host ring for scheduler summaries
struct HostRing {
  int* h = nullptr;
  int* d = nullptr;
  int n = 0;
  ~HostRing() {
    if (h) (void)hipHostFree(h);
  }
  int init(int count) {
    if (h && n >= count) return LRADI_OK;
    if (h) (void)hipHostFree(h);
    h = nullptr;
    LRADI_HIP(hipHostMalloc((void**)&h, sizeof(int) * count, hipHostMallocMapped | hipHostMallocCoherent));
    LRADI_HIP(hipHostGetDevicePointer((void**)&d, h, 0));
    n = count;
    for (int i = 0; i < count; ++i) h[i] = -1;
    return LRADI_OK;
  }
};

}  // namespace lradi

using namespace lradi;

struct lradi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  HostRing ring;
  std::vector<hipEvent_t> events;
  // kernel measurements (opts.profile)
  std::vector<TickProbe> probes;
  DevBuf prof_dev;  // LRADI_PROF_CLASSES unsigned long long byte counters
  double prof_ms[LRADI_PROF_CLASSES] = {};
  int64_t prof_launches[LRADI_PROF_CLASSES] = {};
  // autotuned shifted-product tiling per (n, nnz, r, precision)
  std::map<std::array<int64_t, 4>, int> lanes_cache;
  // red-black preconditioner data of recently prepared matrices, most
  // recent first, keyed by content
  std::list<std::pair<uint64_t, std::shared_ptr<const lradi::RbData>>> rb_cache;
  // host halves of those tables built ahead of their upload by other threads
  // (a batch's matrices in parallel, the server's requests at submission),
  // same keys; an entry is taken by the upload that uses it
  std::mutex rb_pre_mu;
  std::list<std::pair<uint64_t, std::shared_ptr<const lradi::RbHost>>> rb_pre;
};

struct lradi_result {
  int n = 0, m = 0, r = 0, k = 0, kmax = 0;
  int status = LRADI_OK;
  double rel_res = 0.0, norm_fg = 0.0, seconds = 0.0;
  bool sym = false;  // Lyapunov case: Y is Z (Yf unallocated)
  bool cplx = false; // complex shifts: stacked [re; im] factor blocks, gam (re, im) pairs
  DevBuf Zf, Yf;
  std::vector<double> gam, hist;
  const DevBuf& Y() const { return sym ? Zf : Yf; }
};

namespace lradi {
namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int choose_rows_per_wg(int n) {
  int rpw = (n + 511) / 512;
  rpw = ((rpw + 255) / 256) * 256;
  return std::max(256, std::min(rpw, 8192));
}

// ---------------------------------------------------------------------------
// Standalone shifted product on a DevCSR's sliced layout.  Operands well
// beyond the 256 MB last-level cache stream with the nontemporal hint, so
// that the matrix and the output do not evict the rows of X the stencil
// gathers again.
constexpr double kLlcBytes = 256.0 * (1 << 20);
int spmm_plain_csr(hipStream_t st, const DevCSR& A, int r, int prec, int lanes, double shift, const void* X,
                   void* Y) {
  const double tsz = prec == LRADI_FP64 ? 8.0 : 4.0;
  const double bytes = (double)A.nnz * (tsz + 4.0) + 2.0 * tsz * A.n * r;
  if (A.has_mass()) return set_error("internal: plain shifted product of a pencil"), LRADI_EINVAL;
  const unsigned char* blk = prec == LRADI_FP64 ? A.sblk64.as<unsigned char>() : A.sblk32.as<unsigned char>();
  return launch_spmm_plain(st, A.n, r, prec, lanes, A.sslot.as<int>(), blk, shift, X, Y, bytes > 0.75 * kLlcBytes);
}

// Shifted-product autotuner: lanes per row (1, 2, 4 dividing r), timed with
// HIP events on the context's stream; results cached per matrix shape.
int spmm_time(lradi_ctx* c, const DevCSR& A, int r, int prec, int lanes, const void* X, void* Y,
              int reps, double* ms) {
  hipEvent_t e0, e1;
  LRADI_HIP(hipEventCreate(&e0));
  LRADI_HIP(hipEventCreate(&e1));
  int rc = spmm_plain_csr(c->stream, A, r, prec, lanes, 0.5, X, Y);  // warm-up
  if (rc == LRADI_OK) rc = hipEventRecord(e0, c->stream) == hipSuccess ? LRADI_OK : LRADI_EHIP;
  for (int i = 0; i < reps && rc == LRADI_OK; ++i) rc = spmm_plain_csr(c->stream, A, r, prec, lanes, 0.5, X, Y);
  if (rc == LRADI_OK) rc = hipEventRecord(e1, c->stream) == hipSuccess ? LRADI_OK : LRADI_EHIP;
  float t = 0.f;
  if (rc == LRADI_OK) rc = hipEventSynchronize(e1) == hipSuccess ? LRADI_OK : LRADI_EHIP;
  if (rc == LRADI_OK) rc = hipEventElapsedTime(&t, e0, e1) == hipSuccess ? LRADI_OK : LRADI_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != LRADI_OK) return set_error("shifted product: launch or event failure"), LRADI_EHIP;
  *ms = (double)t / reps;
  return LRADI_OK;
}

// policy: 0 autotune, -1 rule, 1/2/4 forced.  X is read, Y overwritten.
int spmm_lanes_for(lradi_ctx* c, const DevCSR& A, int r, int prec, int policy, const void* X, void* Y,
                   int* out) {
  const int tsz = prec == LRADI_FP64 ? 8 : 4;
  if (policy > 0) {
    if (!(policy == 1 || policy == 2 || policy == 4) || r % policy != 0)
      return set_error("spmm_lanes must be 1, 2 or 4 and divide r"), LRADI_EINVAL;
    *out = policy;
    return LRADI_OK;
  }
  const int rule = spmm_rule_lanes(r, tsz);
  const std::array<int64_t, 4> key{A.n, A.nnz, r, prec};
  auto it = c->lanes_cache.find(key);
  if (it != c->lanes_cache.end()) {
    *out = it->second;
    return LRADI_OK;
  }
  *out = rule;
  // small products are launch-bound: timing them is noise, and a batch whose
  // systems share one tiling needs one launch per tick instead of several
  if (policy < 0 || r == 1 || (int64_t)A.n * r * tsz < (8 << 20) || !X || !Y) return LRADI_OK;
  double best = 0.0;
  LRADI_TRY(spmm_time(c, A, r, prec, rule, X, Y, 3, &best));
  for (int lanes : {1, 2, 4}) {
    if (lanes == rule || r % lanes != 0) continue;
    double ms = 0.0;
    LRADI_TRY(spmm_time(c, A, r, prec, lanes, X, Y, 3, &ms));
    // the rule keeps anything within 8%: run-to-run noise of a few percent
    // must not flip a batch between one and two product launches per tick
    if (ms < 0.92 * best) {
      best = ms;
      *out = lanes;
    }
  }
  c->lanes_cache[key] = *out;
  return LRADI_OK;
}

// Workspace of one inner system: every device array the solver keeps for it
// across ticks.  Its address never changes while the system is alive, so the
// descriptor tables can be rebuilt (systems joining or leaving) at any point
// where the stream is drained.
struct SysWork {
  DevBuf buf;
  SysDesc d{};
  SysCtl c{};  // host copy of the control block, valid at drain points

  // sweeps < 0: no preconditioner; else A must carry the red-black data
  // cplx: the real form of a complex shifted system on 2 A->n rows (r <= 4,
  // no preconditioner)
  int init(const DevCSR* A, const double* W, int r, int m, int prec, int max_inner, double floor_rel,
           int sweeps = -1, bool pairs = false, bool cplx = false, int poly = 0) {
    if (r < 1 || r > kMaxR || m < 1 || m > kMaxM)
      return set_error("r must be in 1..%d and restart in 1..%d", kMaxR, kMaxM), LRADI_EINVAL;
    // a block of more columns than rows has no full-rank basis
    if (r > A->n) return set_error("r (%d) exceeds the system size (%d)", r, A->n), LRADI_EINVAL;
    if (cplx && (r > 4 || sweeps >= 0 || A->has_mass()))
      return set_error("complex shifts need r <= 4, M = C = I and no preconditioner"), LRADI_EINVAL;
    if (!A->has_sell()) return set_error("internal: matrix uploaded without its sliced layout"), LRADI_EINVAL;
    const size_t n = (cplx ? 2 : 1) * (size_t)A->n, rr = r, mm = m;
    const size_t tsz = (prec == LRADI_FP64) ? 8 : 4;
    const int rpw = choose_rows_per_wg((int)n);
    const int nwg = (int)((n + rpw - 1) / rpw);
    const size_t pstride = (mm + 1) * rr * rr;
    // pairs where the tiles are the row workgroups' black chunks and their
    // regions are small enough
    size_t nblack = n, plds = 0;
    bool fit = false;
    if (sweeps >= 0 && A->has_rb()) {
      const lradi::RbData& B = *A->rb;
      nblack = n - (size_t)B.nred;
      plds = (size_t)B.maxreg * rr * tsz;
      fit = pairs && sweeps >= 2 && B.ntile > 0 && B.tile == (int)((nblack + nwg - 1) / nwg) &&
            plds <= (size_t)kPairLdsMax && (double)(nblack + B.nhalo) <= kPairMaxRegion * (double)nblack;
    }
    // compact iterates: two, or four for Chebyshev steps that may run in
    // pairs (two read and two written per paired launch)
    const bool four = fit && sweeps > 0 && poly != 0;
    const size_t sizes[] = {(mm + 1) * n * rr * tsz,  // V
                            n * rr * tsz,              // U
                            n * rr * 8,                // R
                            (size_t)nwg * pstride * 8, // part
                            (size_t)nwg * kPS * 8,     // partS
                            (size_t)nwg * kPS * 8,     // partS2
                            pstride * 8,               // red
                            pstride * 8,               // hacc
                            mm * rr * mm * rr * 8,     // Rt
                            mm * 4 * rr * rr * 8,      // Qs
                            (mm + 1) * rr * rr * 8,    // Gv
                            mm * rr * rr * 8,          // yv
                            kSmDoubles * 8,            // sm
                            sweeps >= 0 ? (mm + 1) * n * rr * tsz : 0,  // P
                            sweeps > 0 ? n * rr * tsz : 0,              // Yb
                            sweeps > 0 ? (four ? 4 * nblack : 2 * n) * rr * tsz : 0,  // Eb
                            sweeps > 0 ? n * tsz : 0,                   // It
                            sweeps > 0 && A->has_rb()
                                ? (size_t)A->rb->t2w * std::max(n - (size_t)A->rb->nred, (size_t)1) * tsz
                                : 0};                                   // t2val
    size_t total = 0;
    for (size_t z : sizes) total += align256(z);
    LRADI_TRY(buf.alloc(total));
    char* p = buf.as<char>();
    auto take = [&](size_t bytes) {
      char* q = p;
      p += align256(bytes);
      return q;
    };
    d = SysDesc{};
    d.n = (int)n;
    d.cplx = cplx ? 1 : 0;
    d.nmat = A->n;
    d.r = r;
    d.m = m;
    d.nwg = nwg;
    d.rows_per_wg = rpw;
    d.precision = prec;
    d.max_inner = max_inner;
    d.rowptr = A->rowptr.as<int>();
    d.colind = A->colind.as<int>();
    d.valT = (prec == LRADI_FP64) ? (const void*)A->val64.p : (const void*)A->val32.p;
    d.val64 = A->val64.as<double>();
    d.mvalT = A->has_mass() ? ((prec == LRADI_FP64) ? (const void*)A->mval64.p : (const void*)A->mval32.p)
                            : nullptr;
    d.mval64 = A->has_mass() ? A->mval64.as<double>() : nullptr;
    d.sslot = A->sslot.as<int>();
    d.sblk = (prec == LRADI_FP64) ? A->sblk64.as<unsigned char>() : A->sblk32.as<unsigned char>();
    d.floor_rel = floor_rel;
    d.W = W;
    d.pstride = (int)pstride;
    d.nnz = (int)A->nnz;
    d.spmm_lanes = spmm_rule_lanes(r, (int)tsz);
    d.V = take(sizes[0]);
    d.U = take(sizes[1]);
    d.R = reinterpret_cast<double*>(take(sizes[2]));
    d.part = reinterpret_cast<double*>(take(sizes[3]));
    d.partS = reinterpret_cast<double*>(take(sizes[4]));
    d.partS2 = reinterpret_cast<double*>(take(sizes[5]));
    d.red = reinterpret_cast<double*>(take(sizes[6]));
    d.hacc = reinterpret_cast<double*>(take(sizes[7]));
    d.Rt = reinterpret_cast<double*>(take(sizes[8]));
    d.Qs = reinterpret_cast<double*>(take(sizes[9]));
    d.Gv = reinterpret_cast<double*>(take(sizes[10]));
    d.yv = reinterpret_cast<double*>(take(sizes[11]));
    d.sm = reinterpret_cast<double*>(take(sizes[12]));
    if (sweeps >= 0) {
      if (!A->has_rb()) return set_error("preconditioner data missing"), LRADI_EINVAL;
      d.P = take(sizes[13]);
      if (sweeps > 0) {
        d.Yb = take(sizes[14]);
        d.Eb = take(sizes[15]);
        d.It = take(sizes[16]);
        d.t2val = take(sizes[17]);
      }
      const lradi::RbData& B = *A->rb;
      d.t2w = B.t2w;
      d.t2ci = B.t2ci.as<int>();
      d.t2rev = B.t2rev.as<int>();
      d.rbpos = B.rbpos.as<int>();
      d.rbrows = B.rbrows.as<int>();
      d.nred = B.nred;
      d.sweeps = sweeps;
      d.poly = sweeps > 0 ? poly : 0;
      d.halo_off = B.halo_off.as<int>();
      d.halo = B.halo.as<int>();
      d.t2lc = B.t2lc.as<int>();
      d.halo_ci = B.halo_ci.as<int>();
      d.nhalo = B.nhalo;
      d.pair_lds = fit ? (int)plds : 0;
      d.diagT = (prec == LRADI_FP64) ? (const void*)B.diag64.p : (const void*)B.diag32.p;
      d.msT = B.ms64.p ? ((prec == LRADI_FP64) ? (const void*)B.ms64.p : (const void*)B.ms32.p) : nullptr;
      d.rbw = B.rbw;
      d.ellci = B.ellci.as<int>();
      d.ellvalT = (prec == LRADI_FP64) ? (const void*)B.ellval64.p : (const void*)B.ellval32.p;
      d.elltvT = (prec == LRADI_FP64) ? (const void*)B.elltv64.p : (const void*)B.elltv32.p;
    }
    c = SysCtl{};
    c.phase = PH_FINISHED;  // armed by the caller or by the outer kernels
    return LRADI_OK;
  }

  // the idle B side of a Lyapunov problem: no workgroups, no buffers, never
  // armed (its descriptor only keeps the table's per-problem pairing)
  void init_mirror(const SysWork& a) {
    d = SysDesc{};
    d.n = a.d.n;
    d.nmat = a.d.nmat;
    d.r = a.d.r;
    d.m = a.d.m;
    d.nwg = 0;
    d.rows_per_wg = a.d.rows_per_wg;
    d.precision = a.d.precision;
    d.max_inner = a.d.max_inner;
    d.pstride = a.d.pstride;
    d.spmm_lanes = a.d.spmm_lanes;
    c = SysCtl{};
    c.phase = PH_FINISHED;
  }

  // pick the shifted-product tiling (V's first two blocks serve as scratch;
  // the solver overwrites them before use)
  int tune(lradi_ctx* ctx, const DevCSR& A, int policy) {
    const size_t blk = (size_t)d.n * d.r * (d.precision == LRADI_FP64 ? 8 : 4);
    char* V = static_cast<char*>(d.V);
    if (policy == 0) LRADI_HIP(hipMemsetAsync(V, 0, blk, ctx->stream));
    return spmm_lanes_for(ctx, A, d.r, d.precision, policy, V, V + blk, &d.spmm_lanes);
  }

  // a standalone solve of (A + shift I) Z = W to ||R||_2 <= delta
  void arm(double* Z, double shift, double delta) {
    c = SysCtl{};
    c.Z = Z;
    c.shift = shift;
    c.delta = delta;
    c.phase = PH_CYCLE_END;
    c.first = 1;
  }
};

// Device tables of a set of systems: descriptors, control blocks, row map.
struct Table {
  std::vector<SysDesc> hd;
  std::vector<SysCtl> hc;
  std::vector<int2> hmap, hsp;
  DevBuf dd, dc, dmap, dsp;
  Batch b{};
};

// Workgroups are dispatched to the chip's 8 XCDs round-robin by workgroup
// index, and each XCD has its own L2.  Reorder a launch's (system, chunk)
// entries so that XCD x gets the x-th contiguous run of chunks: row chunks
// that gather each other's neighbours then meet in one L2.  Kernels index
// their partial results by chunk, never by workgroup, so results do not
// change.
void xcd_order(std::vector<int2>& v, size_t begin, size_t end) {
  const size_t G = end - begin;
  if (G <= (size_t)kXcds) return;
  std::vector<int2> nat(v.begin() + begin, v.begin() + end);
  const size_t q = G / kXcds, rem = G % kXcds;
  for (size_t b = 0; b < G; ++b) {
    const size_t x = b % kXcds, y = b / kXcds;
    v[begin + b] = nat[x * q + std::min(x, rem) + y];
  }
}

int upload_table(lradi_ctx* ctx, const std::vector<SysWork*>& ws, Table& t) {
  const int nsys = (int)ws.size();
  if (nsys == 0) return set_error("empty batch"), LRADI_EINVAL;
  const int prec = ws[0]->d.precision;
  t.hd.resize(nsys);
  t.hc.resize(nsys);
  t.hmap.clear();
  int maxP = 1, maxB = 1, rfix = ws[0]->d.r, fuse = 1, precond = 0, sweeps = 0, pairs = 1, pair_lds = 0,
      pair_fast = 1, poly = 0;
  long long black_rows = 0;
  int max_tile = 0, pre_slices = 1;
  for (int s = 0; s < nsys; ++s) {
    if (ws[s]->d.precision != prec) return set_error("all systems of a batch must use one precision"), LRADI_EINVAL;
    t.hd[s] = ws[s]->d;
    t.hd[s].wg0 = (int)t.hmap.size();
    t.hc[s] = ws[s]->c;
    for (int w = 0; w < ws[s]->d.nwg; ++w) t.hmap.push_back(make_int2(s, w));
    maxP = std::max(maxP, ws[s]->d.pstride);
    maxB = std::max(maxB, ws[s]->d.m + 1);
    if (ws[s]->d.nwg * ws[s]->d.r * ws[s]->d.r > kFuseCholMax) fuse = 0;
    if (ws[s]->d.r != rfix) rfix = 0;
    if (ws[s]->d.rbrows) {
      if (precond && ws[s]->d.sweeps != sweeps)
        return set_error("all preconditioned systems of a batch must use one sweep count"), LRADI_EINVAL;
      precond = 1;
      sweeps = ws[s]->d.sweeps;
      if (ws[s]->d.pair_lds == 0) pairs = 0;
      if (ws[s]->d.poly) poly = 1;
      pair_lds = std::max(pair_lds, ws[s]->d.pair_lds);
      const int nb = ws[s]->d.n - ws[s]->d.nred, tile = (nb + ws[s]->d.nwg - 1) / ws[s]->d.nwg;
      black_rows += nb;
      max_tile = std::max(max_tile, tile);
      if (ws[s]->d.t2w > kPairRegSlots) pair_fast = 0;
      // lanes per row of the row stages (the kernels' RbLanes): each lane
      // gathers at least 16 bytes of a row
      const int r = ws[s]->d.r, rb = r * (prec == LRADI_FP64 ? 8 : 4);
      const int lanes = (r % 4 == 0 && rb >= 64) ? 4 : (r % 2 == 0 && rb >= 32) ? 2 : 1;
      pre_slices = std::max(pre_slices, lanes);
    }
  }
  // shifted-product tiles, grouped by lanes per row
  t.hsp.clear();
  for (int g = 0; g < 3; ++g) {
    const int lanes = 1 << g;
    t.b.spoff[g] = (int)t.hsp.size();
    for (int s = 0; s < nsys; ++s) {
      if (ws[s]->d.spmm_lanes != lanes || ws[s]->d.nwg == 0) continue;
      if (ws[s]->d.r % lanes != 0) return set_error("lanes per row must divide r"), LRADI_EINVAL;
      const int tr = spmm_tile_rows(lanes);
      // (complex systems: the tiles of each half of the stacked block)
      const int tiles = ws[s]->d.cplx ? 2 * ((ws[s]->d.nmat + tr - 1) / tr) : (ws[s]->d.n + tr - 1) / tr;
      for (int w = 0; w < tiles; ++w) t.hsp.push_back(make_int2(s, w));
    }
    t.b.spcount[g] = (int)t.hsp.size() - t.b.spoff[g];
    xcd_order(t.hsp, t.b.spoff[g], t.hsp.size());
  }
  xcd_order(t.hmap, 0, t.hmap.size());
  if (t.dsp.bytes < sizeof(int2) * t.hsp.size()) LRADI_TRY(t.dsp.alloc(sizeof(int2) * t.hsp.size()));
  if (t.dd.bytes < sizeof(SysDesc) * nsys) LRADI_TRY(t.dd.alloc(sizeof(SysDesc) * nsys));
  if (t.dc.bytes < sizeof(SysCtl) * nsys) LRADI_TRY(t.dc.alloc(sizeof(SysCtl) * nsys));
  if (t.dmap.bytes < sizeof(int2) * t.hmap.size()) LRADI_TRY(t.dmap.alloc(sizeof(int2) * t.hmap.size()));
  hipStream_t st = ctx->stream;
  LRADI_HIP(hipMemcpyAsync(t.dd.p, t.hd.data(), sizeof(SysDesc) * nsys, hipMemcpyHostToDevice, st));
  LRADI_HIP(hipMemcpyAsync(t.dc.p, t.hc.data(), sizeof(SysCtl) * nsys, hipMemcpyHostToDevice, st));
  LRADI_HIP(hipMemcpyAsync(t.dmap.p, t.hmap.data(), sizeof(int2) * t.hmap.size(), hipMemcpyHostToDevice, st));
  LRADI_HIP(hipMemcpyAsync(t.dsp.p, t.hsp.data(), sizeof(int2) * t.hsp.size(), hipMemcpyHostToDevice, st));
  // the host vectors must outlive the copies
  LRADI_HIP(hipStreamSynchronize(st));
  t.b.d = t.dd.as<SysDesc>();
  t.b.ctl = t.dc.as<SysCtl>();
  t.b.rowmap = t.dmap.as<int2>();
  t.b.spmap = t.dsp.as<int2>();
  t.b.nsys = nsys;
  t.b.rowgrid = (int)t.hmap.size();
  t.b.maxP = maxP;
  t.b.maxB = maxB;
  // (the scale kernels carry the fused factor for narrow blocks only)
  t.b.fuse_chol = fuse && rfix >= 1 && rfix <= 4;
  t.b.precision = prec;
  t.b.rfix = rfix;
  t.b.precond = precond;
  t.b.sweeps = sweeps;
  t.b.poly = poly;
  t.b.pairs = precond && pairs && sweeps >= 2 && black_rows <= kPairMaxRows;
  t.b.pair_lds = t.b.pairs ? pair_lds : 0;
  // (the register-held columns with wider or mixed blocks would spill)
  // (even blocks take two lanes per tile row in that kernel)
  t.b.pair_fast =
      t.b.pairs && pair_fast && rfix >= 1 && rfix <= 4 && max_tile * (rfix % 2 == 0 ? 2 : 1) <= kTPB;
  // forward, back, the sweeps, and (with sweeps) the launches that build T
  // and the Chebyshev bounds
  t.b.precond_launches =
      precond ? 2 + (t.b.pairs ? (sweeps + 1) / 2 : sweeps) + (sweeps > 0 ? 1 + poly : 0) : 0;
  t.b.pre_slices = pre_slices;
  return LRADI_OK;
}

// Copy the device control blocks back into the workspaces (stream drained).
int download_table(lradi_ctx* ctx, const std::vector<SysWork*>& ws, Table& t) {
  const int nsys = (int)ws.size();
  LRADI_HIP(hipMemcpyAsync(t.hc.data(), t.dc.p, sizeof(SysCtl) * nsys, hipMemcpyDeviceToHost, ctx->stream));
  LRADI_HIP(hipStreamSynchronize(ctx->stream));
  for (int s = 0; s < nsys; ++s) ws[s]->c = t.hc[s];
  return LRADI_OK;
}

int probe_account(lradi_ctx* ctx, const TickProbe& p, const Batch& bt) {
  float a = 0.f, b = 0.f, c = 0.f, e = 0.f;
  LRADI_HIP(hipEventElapsedTime(&a, p.ev[0], p.ev[1]));
  LRADI_HIP(hipEventElapsedTime(&b, p.ev[2], p.ev[3]));
  LRADI_HIP(hipEventElapsedTime(&c, p.ev[4], p.ev[5]));
  ctx->prof_ms[LRADI_PROF_GRAM] += (double)a + (double)b;
  ctx->prof_launches[LRADI_PROF_GRAM] += 2;
  ctx->prof_ms[LRADI_PROF_SPMM] += (double)c;
  // one launch per tiling group that has tiles (lanes per row 1, 2, 4)
  ctx->prof_launches[LRADI_PROF_SPMM] += (bt.spcount[0] > 0) + (bt.spcount[1] > 0) + (bt.spcount[2] > 0);
  if (bt.precond) {
    LRADI_HIP(hipEventElapsedTime(&e, p.ev[6], p.ev[7]));
    ctx->prof_ms[LRADI_PROF_PRECOND] += (double)e;
    ctx->prof_launches[LRADI_PROF_PRECOND] += bt.precond_launches;
  }
  return LRADI_OK;
}

// Issue ticks (plus `after`, e.g. the outer step-end kernels) until every
// system of the table is finished, or until `stop` (checked at each read
// back) asks to return.  The host reads the unfinished count of tick t - L
// only after issuing tick t, so the device always has queued work; the
// extra ticks are no-ops.  Returns with the stream drained.
// Graphs of one tick each (tick, `after`, summary into ring slot s), captured
// on the context's stream; destroyed with the object.
struct TickGraphs {
  std::vector<hipGraphExec_t> exec;
  ~TickGraphs() {
    for (auto e : exec)
      if (e) (void)hipGraphExecDestroy(e);
  }
  // false: capture is not possible on this stream (launch directly instead)
  int build(lradi_ctx* ctx, const Batch& b, int slots, const std::function<int()>& after, bool summary,
            bool* ok) {
    *ok = false;
    hipStream_t st = ctx->stream;
    if (!st) return LRADI_OK;  // the null stream cannot be captured
    for (int s = 0; s < slots; ++s) {
      LRADI_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      int rc = launch_tick(st, b, nullptr);
      if (rc == LRADI_OK && after) rc = after();
      if (rc == LRADI_OK) rc = launch_tick_tail(st, b);
      if (rc == LRADI_OK && summary) rc = launch_summary(st, b, ctx->ring.d + s);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(st, &g);
      if (rc != LRADI_OK || ec != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return rc != LRADI_OK ? rc : LRADI_OK;  // capture unsupported: ok stays false
      }
      hipGraphExec_t e = nullptr;
      const hipError_t ei = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        (void)hipGetLastError();
        return LRADI_OK;
      }
      exec.push_back(e);
    }
    *ok = true;
    return LRADI_OK;
  }
};

// summary = false: no count of unfinished systems is produced; `stop` alone
// ends the loop (the outer engine reads its problems' completion flags).
int run_ticks(lradi_ctx* ctx, const Batch& b, int lookahead, long max_ticks, bool profile,
              const std::function<int()>& after, const std::function<bool()>& stop,
              bool use_graph = false, bool summary = true) {
  const int L = std::max(0, std::min(lookahead, 8));
  LRADI_TRY(ctx->ring.init(L + 1));
  while ((int)ctx->events.size() < L + 1) {
    hipEvent_t e;
    LRADI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->events.push_back(e);
  }
  if (profile) {
    while ((int)ctx->probes.size() < L + 1) {
      TickProbe p;
      for (auto& e : p.ev) LRADI_HIP(hipEventCreate(&e));
      ctx->probes.push_back(p);
    }
  }
  hipStream_t st = ctx->stream;
  // optional replay of captured ticks (not with per-launch timing events)
  TickGraphs graphs;
  bool graphed = false;
  if (use_graph && !profile) LRADI_TRY(graphs.build(ctx, b, L + 1, after, summary, &graphed));
  long t = 0;
  for (;; ++t) {
    const int slot = (int)(t % (L + 1));
    if (graphed) {
      LRADI_HIP(hipGraphLaunch(graphs.exec[slot], st));
    } else {
      LRADI_TRY(launch_tick(st, b, profile ? &ctx->probes[slot] : nullptr));
      if (after) LRADI_TRY(after());
      LRADI_TRY(launch_tick_tail(st, b));
      if (summary) LRADI_TRY(launch_summary(st, b, ctx->ring.d + slot));
    }
    LRADI_HIP(hipEventRecord(ctx->events[slot], st));
    if (t >= L) {
      const int rs = (int)((t - L) % (L + 1));
      LRADI_HIP(hipEventSynchronize(ctx->events[rs]));
      if (profile) LRADI_TRY(probe_account(ctx, ctx->probes[rs], b));
      if (summary && __atomic_load_n(ctx->ring.h + rs, __ATOMIC_ACQUIRE) == 0) break;
      if (stop && stop()) break;
    }
    if (t > max_ticks) {
      set_error("inner solver scheduler exceeded %ld ticks", max_ticks);
      return LRADI_EHIP;
    }
  }
  LRADI_HIP(hipStreamSynchronize(st));
  if (profile)  // ticks issued after the last one read back
    for (long u = std::max(0L, t - L + 1); u <= t; ++u)
      LRADI_TRY(probe_account(ctx, ctx->probes[u % (L + 1)], b));
  return LRADI_OK;
}

int prof_counters(lradi_ctx* ctx, bool profile, unsigned long long** out) {
  *out = nullptr;
  if (!profile) return LRADI_OK;
  if (!ctx->prof_dev.p) {
    LRADI_TRY(ctx->prof_dev.alloc(sizeof(unsigned long long) * LRADI_PROF_CLASSES));
    LRADI_HIP(hipMemset(ctx->prof_dev.p, 0, sizeof(unsigned long long) * LRADI_PROF_CLASSES));
  }
  *out = ctx->prof_dev.as<unsigned long long>();
  return LRADI_OK;
}

// Host copy of a (host or device) CSR matrix, validated.
int host_csr(const lradi_csr* M, std::vector<int32_t>& rp, std::vector<int32_t>& ci,
             std::vector<double>& v) {
  if (!M || !M->rowptr || M->nrows <= 0 || M->nrows != M->ncols || M->nnz < 0)
    return set_error("invalid csr"), LRADI_EINVAL;
  const int n = M->nrows;
  rp.resize(n + 1);
  ci.resize(M->nnz);
  v.resize(M->nnz);
  if (M->on_device) {
    LRADI_HIP(hipMemcpy(rp.data(), M->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
    if (M->nnz > 0) {
      LRADI_HIP(hipMemcpy(ci.data(), M->colind, sizeof(int32_t) * M->nnz, hipMemcpyDeviceToHost));
      LRADI_HIP(hipMemcpy(v.data(), M->val, sizeof(double) * M->nnz, hipMemcpyDeviceToHost));
    }
  } else {
    std::copy(M->rowptr, M->rowptr + n + 1, rp.begin());
    std::copy(M->colind, M->colind + M->nnz, ci.begin());
    std::copy(M->val, M->val + M->nnz, v.begin());
  }
  if (rp[0] != 0 || rp[n] != M->nnz) return set_error("csr rowptr must start at 0 and end at nnz"), LRADI_EINVAL;
  for (int i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) return set_error("csr rowptr not monotone"), LRADI_EINVAL;
  for (int64_t k = 0; k < M->nnz; ++k)
    if (ci[k] < 0 || ci[k] >= n) return set_error("csr column index out of range"), LRADI_EINVAL;
  return LRADI_OK;
}

// Upload a matrix and its transpose.
int upload_pair(const lradi_csr* M, hipStream_t st, DevCSR& dM, DevCSR& dMt) {
  std::vector<int32_t> rp, ci, trp, tci;
  std::vector<double> v, tv;
  LRADI_TRY(host_csr(M, rp, ci, v));
  const int n = M->nrows;
  csr_transpose(n, rp.data(), ci.data(), v.data(), trp, tci, tv);
  lradi_csr a{n, n, M->nnz, rp.data(), ci.data(), v.data(), 0};
  lradi_csr t{n, n, M->nnz, trp.data(), tci.data(), tv.data(), 0};
  LRADI_TRY(dM.upload(&a, st, false, false));
  LRADI_TRY(dMt.upload(&t, st, false, false));
  LRADI_HIP(hipStreamSynchronize(st));
  return LRADI_OK;
}

// transposed host copy of a (host or device) csr matrix
int host_csr_t(const lradi_csr* M, std::vector<int32_t>& trp, std::vector<int32_t>& tci,
               std::vector<double>& tv) {
  std::vector<int32_t> rp, ci;
  std::vector<double> v;
  LRADI_TRY(host_csr(M, rp, ci, v));
  csr_transpose(M->nrows, rp.data(), ci.data(), v.data(), trp, tci, tv);
  return LRADI_OK;
}

int check_opts(const lradi_opts& o) {
  if (!(o.tol > 0.0 && o.tol < 1.0)) return set_error("tol must be in (0,1)"), LRADI_EINVAL;
  if (o.kmax < 1 || o.kmax > 100000) return set_error("kmax must be in 1..100000"), LRADI_EINVAL;
  if (o.restart < 1 || o.restart > kMaxM) return set_error("restart must be in 1..%d", kMaxM), LRADI_EINVAL;
  if (o.max_inner < 1) return set_error("max_inner must be >= 1"), LRADI_EINVAL;
  if (o.precision != LRADI_FP64 && o.precision != LRADI_FP32_INNER)
    return set_error("unknown precision"), LRADI_EINVAL;
  if (o.selection < LRADI_SEL_RELATIVE || o.selection > LRADI_SEL_SYM)
    return set_error("unknown selection"), LRADI_EINVAL;
  if (!(o.delta_min > 0.0) || !(o.delta_max >= o.delta_min))
    return set_error("need 0 < delta_min <= delta_max"), LRADI_EINVAL;
  if (!(o.xi > 0.0 && o.xi <= 1.0)) return set_error("xi must be in (0,1]"), LRADI_EINVAL;
  if (o.lookahead < 0) return set_error("lookahead must be >= 0"), LRADI_EINVAL;
  if (o.rescale < 0 || o.rescale > 2) return set_error("rescale must be 0, 1 or 2"), LRADI_EINVAL;
  if (!(o.spmm_lanes >= -1 && o.spmm_lanes <= 4 && o.spmm_lanes != 3))
    return set_error("spmm_lanes must be -1, 0, 1, 2 or 4"), LRADI_EINVAL;
  if (o.precond != LRADI_PRECOND_NONE && o.precond != LRADI_PRECOND_RBILU0)
    return set_error("unknown preconditioner"), LRADI_EINVAL;
  if (o.precond_sweeps < 0 || o.precond_sweeps > 64)
    return set_error("precond_sweeps must be in 0..64"), LRADI_EINVAL;
  if (o.precond_pairs != 0 && o.precond_pairs != 1) return set_error("precond_pairs must be 0 or 1"), LRADI_EINVAL;
  if (o.precond_poly != 0 && o.precond_poly != 1) return set_error("precond_poly must be 0 or 1"), LRADI_EINVAL;
  return LRADI_OK;
}

int sweeps_for(const lradi_opts& o) { return o.precond == LRADI_PRECOND_RBILU0 ? o.precond_sweeps : -1; }

double floor_for(const lradi_opts& o) {
  return o.precision == LRADI_FP64 ? 1e-14 : (o.fp32_floor > 0.0 ? o.fp32_floor : 3e-6);
}

}  // namespace

int DevCSR::upload_pencil(const lradi_csr* A, const lradi_csr* M, hipStream_t st, bool need32) {
  std::vector<int32_t> arp, aci, mrp, mci, urp, uci;
  std::vector<double> av, mv, uav, umv;
  LRADI_TRY(host_csr(A, arp, aci, av));
  LRADI_TRY(host_csr(M, mrp, mci, mv));
  if (M->nrows != A->nrows) return set_error("mass matrix size differs from its operator"), LRADI_EINVAL;
  csr_union(A->nrows, arp.data(), aci.data(), av.data(), mrp.data(), mci.data(), mv.data(), urp, uci, uav,
            umv);
  lradi_csr U{A->nrows, A->nrows, (int64_t)uci.size(), urp.data(), uci.data(), uav.data(), 0};
  LRADI_TRY(upload(&U, st, need32, false));
  LRADI_TRY(mval64.alloc(sizeof(double) * std::max<int64_t>(nnz, 1)));
  if (nnz > 0)
    LRADI_HIP(hipMemcpyAsync(mval64.p, umv.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, st));
  if (need32) {
    LRADI_TRY(mval32.alloc(sizeof(float) * std::max<int64_t>(nnz, 1)));
    if (nnz > 0) {
      const int tpb = 256;
      hipLaunchKernelGGL(k_d2f, dim3((unsigned)((nnz + tpb - 1) / tpb)), dim3(tpb), 0, st,
                         mval64.as<double>(), mval32.as<float>(), nnz);
      LRADI_HIP(hipGetLastError());
    }
  }
  LRADI_TRY(build_sell(urp.data(), st, need32));
  LRADI_HIP(hipStreamSynchronize(st));  // the host vectors must outlive the copies
  return LRADI_OK;
}

// prepared preconditioner data kept per context (most recently used)
constexpr size_t kRbCacheEntries = 8;

// 64-bit content key of a CSR matrix (size, pattern, values, FP32 copies)
uint64_t csr_key(int n, int64_t nnz, const int32_t* rp, const int32_t* ci, const double* v, bool need32) {
  uint64_t h = 0x243F6A8885A308D3ull ^ ((uint64_t)n << 1) ^ ((uint64_t)nnz << 33) ^ (need32 ? 1u : 0u);
  auto mix = [&h](const void* p, size_t bytes) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    size_t i = 0;
    for (; i + 8 <= bytes; i += 8) {
      uint64_t x;
      std::memcpy(&x, c + i, 8);
      h = (h ^ (x * 0x9E3779B97F4A7C15ull)) * 0xBF58476D1CE4E5B9ull;
      h ^= h >> 31;
    }
    uint64_t x = 0;
    std::memcpy(&x, c + i, bytes - i);
    h = (h ^ (x * 0x9E3779B97F4A7C15ull)) * 0x94D049BB133111EBull;
    h ^= h >> 29;
  };
  if (rp) mix(rp, sizeof(int32_t) * (size_t)(n + 1));
  if (nnz > 0) {
    if (ci) mix(ci, sizeof(int32_t) * (size_t)nnz);
    if (v) mix(v, sizeof(double) * (size_t)nnz);
  }
  return h;
}

// The cache key of a matrix's preconditioner data (its contents, and a
// pencil's lumped mass), with M's row sums in lump and, for a device matrix,
// A's host copy in rp, ci, v.
int rb_key(const lradi_csr* A, const lradi_csr* M, bool need32, std::vector<int32_t>& rp,
           std::vector<int32_t>& ci, std::vector<double>& v, std::vector<double>& lump, uint64_t* key) {
  const int n = A->nrows;
  // pencil: M's row sums weight the shift inside the preconditioner
  if (M) {
    std::vector<int32_t> mrp, mci;
    std::vector<double> mv;
    LRADI_TRY(host_csr(M, mrp, mci, mv));
    if (M->nrows != n) return set_error("mass matrix size differs from its operator"), LRADI_EINVAL;
    lump.assign(n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int32_t k = mrp[i]; k < mrp[i + 1]; ++k) lump[i] += mv[k];
  }
  if (A->on_device) {
    LRADI_TRY(host_csr(A, rp, ci, v));
    *key = csr_key(n, (int64_t)ci.size(), rp.data(), ci.data(), v.data(), need32);
  } else {
    *key = csr_key(n, A->nnz, A->rowptr, A->colind, A->val, need32);
  }
  if (M) *key = (*key * 0x5851F42D4C957F2Dull) ^ csr_key(n, n, nullptr, nullptr, lump.data(), false);
  return LRADI_OK;
}

// the host tables of a (host) matrix: colouring, slot tables, Schur
// pattern, tiles (false: not bipartite)
bool rb_host_tables(int nn, const int32_t* rp, const int32_t* ci, const double* v, RbHost& h) {
  std::vector<int32_t> trp, tci;
  std::vector<double> tv;
  csr_transpose(nn, rp, ci, v, trp, tci, tv);
  // one tile of black rows per row workgroup of the inner solves (large
  // matrices only)
  const int rpw = choose_rows_per_wg(nn);
  const int tiles = nn >= kPairMinRows ? (nn + rpw - 1) / rpw : 0;
  return rb_host_build(nn, rp, ci, v, trp.data(), tci.data(), tv.data(), tiles, h);
}

constexpr size_t kRbPreEntries = 64;

// Build the host tables of a host-resident matrix ahead of its upload (any
// thread; device matrices and failures are left to prepare_rb).
void rb_prebuild(lradi_ctx* ctx, const lradi_csr* A, const lradi_csr* M, bool need32,
                 size_t cap = kRbPreEntries) {
  if (!A || A->on_device || (M && M->on_device) || A->nrows <= 0) return;
  std::vector<int32_t> rp, ci;
  std::vector<double> v, lump;
  uint64_t key = 0;
  if (rb_key(A, M, need32, rp, ci, v, lump, &key) != LRADI_OK) return;
  {
    std::lock_guard<std::mutex> lk(ctx->rb_pre_mu);
    for (auto& e : ctx->rb_pre)
      if (e.first == key) return;
  }
  if (host_csr(A, rp, ci, v) != LRADI_OK) return;
  auto h = std::make_shared<RbHost>();
  if (!rb_host_tables(A->nrows, rp.data(), ci.data(), v.data(), *h)) return;
  std::lock_guard<std::mutex> lk(ctx->rb_pre_mu);
  ctx->rb_pre.emplace_front(key, std::move(h));
  while (ctx->rb_pre.size() > std::max(cap, kRbPreEntries)) ctx->rb_pre.pop_back();
}

int DevCSR::prepare_rb(lradi_ctx* ctx, const lradi_csr* A, const lradi_csr* M, hipStream_t st, bool need32) {
  std::vector<int32_t> rp, ci;
  std::vector<double> v, lump;
  if (!A || A->nrows != n) return set_error("preconditioner: matrix size differs from the uploaded one"), LRADI_EINVAL;
  // a matrix already prepared on this context (same contents) is reused
  uint64_t key = 0;
  LRADI_TRY(rb_key(A, M, need32, rp, ci, v, lump, &key));
  // host tables built ahead by another thread (taken even when the device
  // data turns out to be cached, so that no entry is left behind)
  std::shared_ptr<const RbHost> hp;
  {
    std::lock_guard<std::mutex> lk(ctx->rb_pre_mu);
    for (auto it = ctx->rb_pre.begin(); it != ctx->rb_pre.end(); ++it)
      if (it->first == key) {
        hp = it->second;
        ctx->rb_pre.erase(it);
        break;
      }
  }
  for (auto it = ctx->rb_cache.begin(); it != ctx->rb_cache.end(); ++it)
    if (it->first == key) {
      rb = it->second;
      ctx->rb_cache.splice(ctx->rb_cache.begin(), ctx->rb_cache, it);
      return LRADI_OK;
    }
  auto R = std::make_shared<RbData>();
  const int nn = A->nrows;
  if (!hp) {
    if (!A->on_device) LRADI_TRY(host_csr(A, rp, ci, v));
    auto hb = std::make_shared<RbHost>();
    if (!rb_host_tables(nn, rp.data(), ci.data(), v.data(), *hb))
      return set_error("red-black preconditioner: the sparsity graph is not bipartite"), LRADI_EINVAL;
    hp = std::move(hb);
  }
  const RbHost& h = *hp;
  const size_t ne = (size_t)h.rbw * nn;
  const bool mass = !lump.empty();
  // every table in one allocation (256-byte aligned slices): a table slice
  // holds at least 4 bytes; the FP32 copies and the lumped mass are absent
  // (null) when not needed
  struct Slice {
    DevView* v;
    const void* src;
    size_t bytes;
    bool present;
  };
  const Slice sl[] = {
      {&R->t2ci, h.t2ci.data(), sizeof(int32_t) * h.t2ci.size(), true},
      {&R->t2rev, h.t2rev.data(), sizeof(int32_t) * h.t2rev.size(), true},
      {&R->t2lc, h.t2lc.data(), sizeof(int32_t) * h.t2lc.size(), true},
      {&R->halo_off, h.halo_off.data(), sizeof(int32_t) * h.halo_off.size(), true},
      {&R->halo, h.halo.data(), sizeof(int32_t) * h.halo.size(), true},
      {&R->halo_ci, h.halo_ci.data(), sizeof(int32_t) * h.halo_ci.size(), true},
      {&R->rbpos, h.pos.data(), sizeof(int32_t) * nn, true},
      {&R->rbrows, h.rows.data(), sizeof(int32_t) * nn, true},
      {&R->diag64, h.dg.data(), sizeof(double) * nn, true},
      {&R->ellci, h.eci.data(), sizeof(int32_t) * ne, true},
      {&R->ellval64, h.eval.data(), sizeof(double) * ne, true},
      {&R->elltv64, h.etv.data(), sizeof(double) * ne, true},
      {&R->ms64, mass ? lump.data() : nullptr, sizeof(double) * nn, mass},
      {&R->ms32, nullptr, sizeof(float) * nn, mass && need32},
      {&R->diag32, nullptr, sizeof(float) * nn, need32},
      {&R->ellval32, nullptr, sizeof(float) * ne, need32},
      {&R->elltv32, nullptr, sizeof(float) * ne, need32},
  };
  size_t total = 0;
  for (const Slice& x : sl)
    if (x.present) total += align256(std::max(x.bytes, (size_t)4));
  LRADI_TRY(R->arena.alloc(total));
  char* q = R->arena.as<char>();
  for (const Slice& x : sl) {
    x.v->p = nullptr;
    if (!x.present) continue;
    x.v->p = q;
    if (x.src && x.bytes) LRADI_HIP(hipMemcpyAsync(q, x.src, x.bytes, hipMemcpyHostToDevice, st));
    q += align256(std::max(x.bytes, (size_t)4));
  }
  const int tpb = 256;
  if (mass && need32)
    hipLaunchKernelGGL(k_d2f, dim3((unsigned)((nn + tpb - 1) / tpb)), dim3(tpb), 0, st, R->ms64.as<double>(),
                       R->ms32.as<float>(), (int64_t)nn);
  if (need32) {
    hipLaunchKernelGGL(k_d2f, dim3((unsigned)((nn + tpb - 1) / tpb)), dim3(tpb), 0, st, R->diag64.as<double>(),
                       R->diag32.as<float>(), (int64_t)nn);
    hipLaunchKernelGGL(k_d2f, dim3((unsigned)((ne + tpb - 1) / tpb)), dim3(tpb), 0, st, R->ellval64.as<double>(),
                       R->ellval32.as<float>(), (int64_t)ne);
    hipLaunchKernelGGL(k_d2f, dim3((unsigned)((ne + tpb - 1) / tpb)), dim3(tpb), 0, st, R->elltv64.as<double>(),
                       R->elltv32.as<float>(), (int64_t)ne);
  }
  LRADI_HIP(hipGetLastError());
  LRADI_HIP(hipStreamSynchronize(st));  // the host vectors must outlive the copies
  R->nred = h.nred;
  R->rbw = h.rbw;
  R->t2w = h.t2w;
  R->tile = h.tile;
  R->ntile = h.ntile;
  R->maxreg = h.maxreg;
  R->nhalo = (int)h.halo.size();
  rb = R;
  ctx->rb_cache.emplace_front(key, R);
  if (ctx->rb_cache.size() > kRbCacheEntries) ctx->rb_cache.pop_back();
  return LRADI_OK;
}


// Host tables of a problem's preconditioned matrices ahead of its set-up:
// side 0 is A (with M), side 1 the matrix the B-side solves use (B given
// as B^T, or B's host transpose, with C likewise).  Host matrices only.
void prebuild_side(lradi_ctx* c, const lradi_opts& o, const lradi_problem& P, int side, size_t cap) {
  if (sweeps_for(o) < 0 || P.shiftsA_im || P.shiftsB_im) return;  // (complex: no preconditioner)
  const bool f32 = o.precision == LRADI_FP32_INNER;
  if (side == 0) {
    rb_prebuild(c, P.A, P.M, f32, cap);
    return;
  }
  if (P.lyapunov || !P.B) return;
  if (o.b_is_transposed) {
    rb_prebuild(c, P.B, P.C, f32, cap);
    return;
  }
  if (P.B->on_device || (P.C && P.C->on_device)) return;
  std::vector<int32_t> trp, tci, crp, cci;
  std::vector<double> tv, cv;
  if (host_csr_t(P.B, trp, tci, tv) != LRADI_OK) return;
  lradi_csr Bt{P.B->nrows, P.B->nrows, (int64_t)tci.size(), trp.data(), tci.data(), tv.data(), 0};
  lradi_csr Ct{};
  if (P.C) {
    if (host_csr_t(P.C, crp, cci, cv) != LRADI_OK) return;
    Ct = lradi_csr{P.C->nrows, P.C->nrows, (int64_t)cci.size(), crp.data(), cci.data(), cv.data(), 0};
  }
  rb_prebuild(c, &Bt, P.C ? &Ct : nullptr, f32, cap);
}

// all of a batch's tables on up to 16 host threads
void prebuild_batch(lradi_ctx* c, const lradi_opts& o, const lradi_problem* probs, int nprob) {
  if (sweeps_for(o) < 0 || nprob < 2) return;
  const int hw = std::max(1, (int)std::thread::hardware_concurrency());
  const int nt = std::max(1, std::min({16, hw, 2 * nprob}));
  std::atomic<int> next{0};
  auto work = [&]() {
    for (int t; (t = next.fetch_add(1)) < 2 * nprob;) {
      try {
        prebuild_side(c, o, probs[t / 2], t % 2, 2 * (size_t)nprob);
      } catch (...) {
        // (the set-up builds this matrix's tables itself)
      }
    }
  };
  std::vector<std::thread> th;
  for (int i = 1; i < nt; ++i) th.emplace_back(work);
  work();
  for (auto& x : th) x.join();
}
}  // namespace lradi

// ---------------------------------------------------------------------------
// Outer engine: a set of Sylvester problems, each advancing through Algorithm 1
// on its own.  Problem p owns inner systems 2p (A side) and 2p+1 (B side) in
// the tables; after every tick the step-end kernels close the outer step of
// every problem whose two inner solves have finished and arm its next step,
// so no problem waits for another.  Problems join (setup kernels) and leave
// (finished, cancelled) at drain points, where the tables are rebuilt; their
// workspaces never move.
namespace lradi {
namespace {

struct PinnedInt {
  int* h = nullptr;
  int* d = nullptr;
  PinnedInt() = default;
  PinnedInt(const PinnedInt&) = delete;
  PinnedInt& operator=(const PinnedInt&) = delete;
  ~PinnedInt() {
    if (h) (void)hipHostFree(h);
  }
  int init() {
    LRADI_HIP(hipHostMalloc((void**)&h, sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
    LRADI_HIP(hipHostGetDevicePointer((void**)&d, h, 0));
    *h = 0;
    return LRADI_OK;
  }
  int get() const { return __atomic_load_n(h, __ATOMIC_ACQUIRE); }
};

struct Prob {
  DevCSR A, Bt;
  DevBuf fown, gown;   // owned copies of f, g (serving), else empty
  const double* f = nullptr;
  const double* g = nullptr;
  int n = 0, m = 0, r = 0, nshifts = 0;
  double tol = 0.0;
  DevBuf shA, shB, shAi, shBi, W, T, gam, hist;
  SysWork wa, wb;
  bool cplx = false;  // complex shifts (imaginary parts in shAi, shBi)
  PinnedInt done;
  std::unique_ptr<lradi_result> res;
  AdiCtl hc{};
  bool set_up = false;
  bool sym = false;  // Lyapunov case: wb is an idle mirror, T = W, Y = Z
  std::chrono::steady_clock::time_point t0;
};

// Validate and upload one problem (transposing B on the host when needed).
int prob_init(lradi_ctx* c, const lradi_opts& o, const lradi_problem& P0, bool copy_rhs, Prob& q) {
  hipStream_t st = c->stream;
  lradi_problem P = P0;
  q.sym = P.lyapunov != 0;
  if (q.sym) {  // B = A^T, C = M^T, g = f, alpha = beta: only the A side is stored
    P.B = P.A;
    P.g = P.f;
    P.shiftsB = P.shiftsA;
    P.C = nullptr;
  }
  if (!P.A || !P.B || !P.f || !P.g || !P.shiftsA || !P.shiftsB)
    return set_error("problem: null argument"), LRADI_EINVAL;
  if (P.r < 1 || P.r > kMaxR) return set_error("problem: r must be in 1..%d", kMaxR), LRADI_EINVAL;
  if (P.nshifts < 1) return set_error("problem: need at least one shift"), LRADI_EINVAL;
  for (int i = 0; i < P.nshifts; ++i)
    if (!std::isfinite(P.shiftsA[i]) || !std::isfinite(P.shiftsB[i]))
      return set_error("problem: non-finite shift"), LRADI_EINVAL;
  q.cplx = P.shiftsA_im != nullptr || P.shiftsB_im != nullptr;
  if (q.cplx) {
    if (!P.shiftsA_im || !P.shiftsB_im)
      return set_error("problem: complex shifts need both imaginary parts"), LRADI_EINVAL;
    for (int i = 0; i < P.nshifts; ++i)
      if (!std::isfinite(P.shiftsA_im[i]) || !std::isfinite(P.shiftsB_im[i]))
        return set_error("problem: non-finite shift"), LRADI_EINVAL;
    if (q.sym || P.M || P.C || P.r > 4 || sweeps_for(o) >= 0)
      return set_error("problem: complex shifts need r <= 4, M = C = I, no Lyapunov mirror and no "
                       "preconditioner"),
             LRADI_EINVAL;
  }
  const double tol = (P.tol > 0.0) ? P.tol : o.tol;
  if (!(tol > 0.0 && tol < 1.0)) return set_error("problem: tol must be in (0,1)"), LRADI_EINVAL;
  q.t0 = std::chrono::steady_clock::now();
  const bool f32 = o.precision == LRADI_FP32_INNER;
  if (P.M)
    LRADI_TRY(q.A.upload_pencil(P.A, P.M, st, f32));
  else
    LRADI_TRY(q.A.upload(P.A, st, f32));
  if (q.sym) {
    // no B side
  } else if (o.b_is_transposed) {
    if (P.C)
      LRADI_TRY(q.Bt.upload_pencil(P.B, P.C, st, f32));
    else
      LRADI_TRY(q.Bt.upload(P.B, st, f32));
  } else {
    std::vector<int32_t> trp, tci, crp, cci;
    std::vector<double> tv, cv;
    LRADI_TRY(host_csr_t(P.B, trp, tci, tv));
    const int mB = P.B->nrows;
    lradi_csr Bt{mB, mB, (int64_t)tci.size(), trp.data(), tci.data(), tv.data(), 0};
    if (P.C) {
      LRADI_TRY(host_csr_t(P.C, crp, cci, cv));
      const int mC = P.C->nrows;
      lradi_csr Ct{mC, mC, (int64_t)cci.size(), crp.data(), cci.data(), cv.data(), 0};
      LRADI_TRY(q.Bt.upload_pencil(&Bt, &Ct, st, f32));
    } else {
      LRADI_TRY(q.Bt.upload(&Bt, st, f32));
    }
    LRADI_HIP(hipStreamSynchronize(st));
  }
  const int sw = sweeps_for(o);
  if (sw >= 0) {
    // the preconditioner is built from the operators' own patterns (A, B^T);
    // a mass matrix enters through its row sums
    LRADI_TRY(q.A.prepare_rb(c, P.A, P.M, st, f32));
    if (!q.sym) {
      if (o.b_is_transposed) {
        LRADI_TRY(q.Bt.prepare_rb(c, P.B, P.C, st, f32));
      } else {
        std::vector<int32_t> trp, tci, crp, cci;
        std::vector<double> tv, cv;
        LRADI_TRY(host_csr_t(P.B, trp, tci, tv));
        const int mB = P.B->nrows;
        lradi_csr Bt{mB, mB, (int64_t)tci.size(), trp.data(), tci.data(), tv.data(), 0};
        lradi_csr Ct{};
        if (P.C) {
          LRADI_TRY(host_csr_t(P.C, crp, cci, cv));
          Ct = lradi_csr{P.C->nrows, P.C->nrows, (int64_t)cci.size(), crp.data(), cci.data(), cv.data(), 0};
        }
        LRADI_TRY(q.Bt.prepare_rb(c, &Bt, P.C ? &Ct : nullptr, st, f32));
      }
    }
  }
  q.n = q.A.n;
  q.m = q.sym ? q.A.n : q.Bt.n;
  q.r = P.r;
  q.nshifts = P.nshifts;
  q.tol = tol;
  const size_t n = q.n, m = q.m, r = q.r, K = o.kmax;
  if (copy_rhs) {
    LRADI_TRY(q.fown.alloc(sizeof(double) * n * r));
    LRADI_HIP(hipMemcpyAsync(q.fown.p, P.f, sizeof(double) * n * r, hipMemcpyDeviceToDevice, st));
    q.f = q.fown.as<double>();
    if (q.sym) {
      q.g = q.f;
    } else {
      LRADI_TRY(q.gown.alloc(sizeof(double) * m * r));
      LRADI_HIP(hipMemcpyAsync(q.gown.p, P.g, sizeof(double) * m * r, hipMemcpyDeviceToDevice, st));
      q.g = q.gown.as<double>();
    }
  } else {
    q.f = P.f;
    q.g = P.g;
  }
  q.res = std::make_unique<lradi_result>();
  q.res->n = q.n;
  q.res->m = q.m;
  q.res->r = q.r;
  q.res->kmax = o.kmax;
  q.res->sym = q.sym;
  q.res->cplx = q.cplx;
  const size_t hz = q.cplx ? 2 : 1;  // stacked [re; im] blocks when complex
  LRADI_TRY(q.res->Zf.alloc(sizeof(double) * K * hz * n * r));
  if (!q.sym) LRADI_TRY(q.res->Yf.alloc(sizeof(double) * K * hz * m * r));
  LRADI_TRY(q.W.alloc(sizeof(double) * hz * n * r));
  if (!q.sym) LRADI_TRY(q.T.alloc(sizeof(double) * hz * m * r));
  LRADI_TRY(q.shA.alloc(sizeof(double) * P.nshifts));
  LRADI_TRY(q.shB.alloc(sizeof(double) * P.nshifts));
  if (q.cplx) {
    LRADI_TRY(q.shAi.alloc(sizeof(double) * P.nshifts));
    LRADI_TRY(q.shBi.alloc(sizeof(double) * P.nshifts));
    LRADI_HIP(hipMemcpyAsync(q.shAi.p, P.shiftsA_im, sizeof(double) * P.nshifts, hipMemcpyHostToDevice, st));
    LRADI_HIP(hipMemcpyAsync(q.shBi.p, P.shiftsB_im, sizeof(double) * P.nshifts, hipMemcpyHostToDevice, st));
  }
  LRADI_TRY(q.gam.alloc(sizeof(double) * K * hz));
  LRADI_TRY(q.hist.alloc(sizeof(double) * K * kHistCols));
  LRADI_HIP(hipMemcpyAsync(q.shA.p, P.shiftsA, sizeof(double) * P.nshifts, hipMemcpyHostToDevice, st));
  LRADI_HIP(hipMemcpyAsync(q.shB.p, P.shiftsB, sizeof(double) * P.nshifts, hipMemcpyHostToDevice, st));
  const double fl = floor_for(o);
  LRADI_TRY(q.wa.init(&q.A, q.W.as<double>(), q.r, o.restart, o.precision, o.max_inner, fl, sw,
                      o.precond_pairs != 0, q.cplx, o.precond_poly));
  LRADI_TRY(q.wa.tune(c, q.A, o.spmm_lanes));
  if (q.sym) {
    q.wb.init_mirror(q.wa);
  } else {
    LRADI_TRY(q.wb.init(&q.Bt, q.T.as<double>(), q.r, o.restart, o.precision, o.max_inner, fl, sw,
                        o.precond_pairs != 0, q.cplx, o.precond_poly));
    LRADI_TRY(q.wb.tune(c, q.Bt, o.spmm_lanes));
  }
  LRADI_TRY(q.done.init());
  LRADI_HIP(hipStreamSynchronize(st));
  return LRADI_OK;
}

// Device bytes one problem holds while in flight: matrices, right-hand
// sides, residual and solution factors, and its two inner workspaces.
size_t prob_footprint(int n, int m, int r, int64_t nnzA, int64_t nnzB, const lradi_opts& o,
                      bool sym = false) {
  const size_t tsz = o.precision == LRADI_FP64 ? 8 : 4;
  const size_t K = o.kmax, mm = o.restart;
  auto mat = [&](int64_t nrow, int64_t nnz) {
    // (the preconditioner keeps transposed values beside the matrix)
    const size_t vals = (size_t)nnz * (8 + (tsz == 4 ? 4 : 0));
    return (size_t)(nrow + 1) * 4 + (size_t)nnz * 4 + vals +
           (sweeps_for(o) >= 0 ? (size_t)nnz * 4 + 2 * vals : 0);
  };
  const int sw = sweeps_for(o);
  auto inner = [&](size_t rows) {
    const size_t rpw = (size_t)choose_rows_per_wg((int)rows), nwg = (rows + rpw - 1) / rpw;
    // preconditioned: the basis P_0..P_m, a sweep block, colour order, diagonal
    const size_t pre = sw < 0 ? 0 : (mm + 1 + (sw > 0 ? 2 : 0)) * rows * r * tsz + rows * (4 + 8 + 2 * tsz);
    return (mm + 2) * rows * r * tsz + rows * r * 8 + nwg * ((mm + 1) * r * r + 2 * kPS) * 8 +
           (mm * r) * (mm * r) * 8 + 16 * (mm + 1) * r * r * 8 + 12 * 256 + 4096 + pre;
  };
  if (sym) return mat(n, nnzA) + (size_t)n * r * 8 * (2 + K) + K * (kHistCols + 1) * 8 + inner(n);
  return mat(n, nnzA) + mat(m, nnzB) + (size_t)(n + m) * r * 8 * (3 + K) + K * (kHistCols + 1) * 8 +
         inner(n) + inner(m);
}

struct Engine {
  lradi_ctx* c;
  lradi_opts o;
  std::vector<Prob*> act;
  std::vector<Prob*> finished;  // filled by drain(); the caller takes them
  std::vector<SysWork*> ws;
  Table tab;
  DevBuf dad, dac;
  std::vector<AdiCtl> hac;
  bool dirty = true;
  long ticks = 0;

  Engine(lradi_ctx* ctx, const lradi_opts& opts) : c(ctx), o(opts) {}

  int rebuild() {
    hipStream_t st = c->stream;
    const int np = (int)act.size();
    dirty = false;
    if (np == 0) return LRADI_OK;
    ws.clear();
    for (Prob* q : act) {
      ws.push_back(&q->wa);
      ws.push_back(&q->wb);
    }
    LRADI_TRY(upload_table(c, ws, tab));
    LRADI_TRY(prof_counters(c, o.profile != 0, &tab.b.prof_bytes));
    std::vector<AdiDesc> hd(np);
    hac.assign(np, AdiCtl{});
    bool any_setup = false;
    for (int p = 0; p < np; ++p) {
      Prob* q = act[p];
      AdiDesc& ad = hd[p];
      ad.n = q->n;
      ad.m = q->m;
      ad.r = q->r;
      ad.kmax = o.kmax;
      ad.nshifts = q->nshifts;
      ad.selection = o.selection;
      ad.backlook = o.backlook;
      ad.paper_abs = o.paper_abs;
      ad.rescale = o.rescale;
      ad.setup = q->set_up ? 0 : 1;
      ad.sym = q->sym ? 1 : 0;
      any_setup = any_setup || !q->set_up;
      ad.tol = q->tol;
      ad.eps_in = o.eps;
      // delta_min and delta_fixed are given for opts.tol (the paper's tau/20);
      // a problem with its own tolerance scales them with it
      const double ts = q->tol / o.tol;
      ad.delta_min = o.delta_min * ts;
      ad.delta_max = o.delta_max;
      ad.xi = o.xi;
      ad.delta_fixed = o.delta_fixed * ts;
      ad.rho = o.rho;
      ad.shiftsA = q->shA.as<double>();
      ad.shiftsB = q->shB.as<double>();
      ad.cplx = q->cplx ? 1 : 0;
      ad.shiftsA_im = q->cplx ? q->shAi.as<double>() : nullptr;
      ad.shiftsB_im = q->cplx ? q->shBi.as<double>() : nullptr;
      ad.f = q->f;
      ad.g = q->g;
      ad.W = q->W.as<double>();
      ad.T = q->sym ? ad.W : q->T.as<double>();
      ad.Zf = q->res->Zf.as<double>();
      ad.Yf = q->sym ? ad.Zf : q->res->Yf.as<double>();
      ad.gam = q->gam.as<double>();
      ad.hist = q->hist.as<double>();
      ad.host_done = q->done.d;
      hac[p] = q->hc;
    }
    if (dad.bytes < sizeof(AdiDesc) * np) LRADI_TRY(dad.alloc(sizeof(AdiDesc) * np));
    if (dac.bytes < sizeof(AdiCtl) * np) LRADI_TRY(dac.alloc(sizeof(AdiCtl) * np));
    LRADI_HIP(hipMemcpyAsync(dad.p, hd.data(), sizeof(AdiDesc) * np, hipMemcpyHostToDevice, st));
    LRADI_HIP(hipMemcpyAsync(dac.p, hac.data(), sizeof(AdiCtl) * np, hipMemcpyHostToDevice, st));
    if (any_setup) LRADI_TRY(adi_launch_setup(st, tab.b, dad.as<AdiDesc>(), dac.as<AdiCtl>(), np));
    LRADI_HIP(hipStreamSynchronize(st));
    for (Prob* q : act) q->set_up = true;
    return LRADI_OK;
  }

  int finalize(Prob* q) {
    lradi_result* R = q->res.get();
    const AdiCtl& h = q->hc;
    R->k = h.k;
    R->norm_fg = h.norm_fg;
    R->rel_res = h.norm_fg > 0.0 ? h.res / h.norm_fg : 0.0;
    const size_t ng = (size_t)std::max(h.k, 0) * (q->cplx ? 2 : 1);
    R->gam.assign(ng, 0.0);
    R->hist.assign((size_t)std::max(h.k, 0) * kHistCols, 0.0);
    if (h.k > 0) {
      LRADI_HIP(hipMemcpy(R->gam.data(), q->gam.p, sizeof(double) * ng, hipMemcpyDeviceToHost));
      LRADI_HIP(hipMemcpy(R->hist.data(), q->hist.p, sizeof(double) * h.k * kHistCols, hipMemcpyDeviceToHost));
    }
    int status = h.status;
    if (status == LRADI_OK && h.winner) status = LRADI_WINNER;
    // Thm 3: ||R_true|| <= ||w_k t_k^T|| + u_k + v_k; the stop test bounds
    // the first term by tol ||f g^T||, so the result is certified below
    // 2 tol only while the gap estimate stayed within epsilon
    if (status == LRADI_OK && h.u + h.v > h.eps) status = LRADI_WGAP;
    R->status = status;
    R->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - q->t0).count();
    return LRADI_OK;
  }

  // Stream drained: pull the control blocks back, move finished problems to
  // `finished`.
  int drain() {
    const int np = (int)act.size();
    if (np == 0) return LRADI_OK;
    LRADI_TRY(download_table(c, ws, tab));
    LRADI_HIP(hipMemcpy(hac.data(), dac.p, sizeof(AdiCtl) * np, hipMemcpyDeviceToHost));
    std::vector<Prob*> keep;
    for (int p = 0; p < np; ++p) {
      act[p]->hc = hac[p];
      if (hac[p].done) {
        LRADI_TRY(finalize(act[p]));
        finished.push_back(act[p]);
        dirty = true;
      } else {
        keep.push_back(act[p]);
      }
    }
    act.swap(keep);
    return LRADI_OK;
  }

  // Run ticks until every problem finished, or (retire > 0) until at least
  // `retire` problems finished, so the tables can shrink, or until `stop`
  // asks to return.  Ends drained.
  int run(int retire, const std::function<bool()>& stop) {
    if (dirty) LRADI_TRY(rebuild());
    if (act.empty()) return LRADI_OK;
    const int np = (int)act.size();
    auto after = [&]() { return adi_launch_step_end(c->stream, tab.b, dad.as<AdiDesc>(), dac.as<AdiCtl>(), np); };
    // the problems' completion flags (written by the device when a problem
    // finishes) end the run: all of them, or `retire` of them
    const int need = retire > 0 ? std::min(retire, np) : np;
    auto check = [&]() {
      if (stop && stop()) return true;
      int k = 0;
      for (Prob* q : act) k += q->done.get();
      return k >= need;
    };
    const long max_ticks = (3L * std::max(o.max_inner, 1) + 16) * (long)(o.kmax + 1);
    const int rc = run_ticks(c, tab.b, o.lookahead, max_ticks, o.profile != 0, after, check, o.use_graph != 0,
                             false);
    if (rc != LRADI_OK) {
      (void)hipStreamSynchronize(c->stream);
      return rc;
    }
    return drain();
  }
};

}  // namespace
}  // namespace lradi

// ===========================================================================
// C ABI
extern "C" {

void lradi_default_opts(lradi_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-8;
  o->eps = 0.0;
  o->delta_min = 1e-8 / 20.0;
  o->delta_max = 0.1;
  o->xi = 1.0;
  o->delta_fixed = 1e-8 / 20.0;
  o->rho = 1e-12;
  o->fp32_floor = 3e-6;
  o->kmax = 50;
  o->selection = LRADI_SEL_MID;
  o->backlook = 1;
  o->paper_abs = 0;
  o->precision = LRADI_FP64;
  o->restart = 30;
  o->max_inner = 20000;
  o->rescale = 2;
  o->b_is_transposed = 0;
  o->lookahead = 2;
  o->use_graph = 0;
  o->precond_pairs = 1;
  o->precond_poly = 0;
}

const char* lradi_strerror(int st) {
  switch (st) {
    case LRADI_OK: return "ok";
    case LRADI_EINVAL: return "invalid argument";
    case LRADI_ENOMEM: return "out of device memory";
    case LRADI_EHIP: return "HIP runtime error";
    case LRADI_ENAN: return "NaN or Inf in the iteration";
    case LRADI_EBREAKDOWN: return "Krylov breakdown";
    case LRADI_WNOCONV: return "outer iteration reached kmax";
    case LRADI_WINNER: return "an inner solve reached its step cap";
    case LRADI_WGAP: return "residual-gap estimate u + v above the budget epsilon";
    case LRADI_ECANCELED: return "request cancelled";
    default: return "unknown status";
  }
}

const char* lradi_last_error(void) { return g_err; }

int lradi_create(lradi_ctx** out, int device, void* stream) {
  if (!out) return set_error("lradi_create: null output"), LRADI_EINVAL;
  *out = nullptr;
  int ndev = 0;
  LRADI_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return set_error("lradi_create: no device %d", device), LRADI_EINVAL;
  LRADI_HIP(hipSetDevice(device));
  // the no-alloc entry point's scratch address on this device; a failure
  // here only disables that entry point (it looks the address up again and
  // reports the error), so the context is created regardless
  if (lradi::scratch_setup(device) != LRADI_OK) (void)hipGetLastError();
  auto* c = new lradi_ctx();
  c->device = device;
  if (stream) {
    c->stream = static_cast<hipStream_t>(stream);
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      set_error("hipStreamCreate failed: %s", hipGetErrorString(e));
      return LRADI_EHIP;
    }
    c->own_stream = true;
  }
  *out = c;
  return LRADI_OK;
}

int lradi_destroy(lradi_ctx* c) {
  if (!c) return LRADI_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto e : c->events) (void)hipEventDestroy(e);
  for (auto& p : c->probes)
    for (auto e : p.ev) (void)hipEventDestroy(e);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return LRADI_OK;
}

int lradi_spmm(lradi_ctx* c, const lradi_csr* A, double shift, const void* X, void* Y, int r,
               int precision) {
  if (!c || !X || !Y) return set_error("lradi_spmm: null argument"), LRADI_EINVAL;
  if (r < 1 || r > kMaxR) return set_error("lradi_spmm: r must be in 1..%d", kMaxR), LRADI_EINVAL;
  if (precision != LRADI_FP64 && precision != LRADI_FP32_INNER)
    return set_error("lradi_spmm: unknown precision"), LRADI_EINVAL;
  LRADI_HIP(hipSetDevice(c->device));
  DevCSR dA;
  LRADI_TRY(dA.upload(A, c->stream, precision == LRADI_FP32_INNER));
  int lanes = 1;
  LRADI_TRY(spmm_lanes_for(c, dA, r, precision, -1, nullptr, nullptr, &lanes));
  LRADI_TRY(spmm_plain_csr(c->stream, dA, r, precision, lanes, shift, X, Y));
  LRADI_HIP(hipStreamSynchronize(c->stream));
  return LRADI_OK;
}

int lradi_spmm_bench(lradi_ctx* c, const lradi_csr* A, double shift, const void* X, void* Y, int r,
                     int precision, int lanes, int reps, double* avg_ms, int64_t* bytes) {
  if (!c || !X || !Y || !avg_ms || reps < 1) return set_error("lradi_spmm_bench: bad argument"), LRADI_EINVAL;
  if (r < 1 || r > kMaxR) return set_error("lradi_spmm_bench: r must be in 1..%d", kMaxR), LRADI_EINVAL;
  if (precision != LRADI_FP64 && precision != LRADI_FP32_INNER)
    return set_error("lradi_spmm_bench: unknown precision"), LRADI_EINVAL;
  LRADI_HIP(hipSetDevice(c->device));
  DevCSR dA;
  LRADI_TRY(dA.upload(A, c->stream, precision == LRADI_FP32_INNER));
  int use = 1;
  LRADI_TRY(spmm_lanes_for(c, dA, r, precision, lanes, X, Y, &use));
  double ms = 0.0;
  LRADI_TRY(spmm_time(c, dA, r, precision, use, X, Y, reps, &ms));
  // leave Y = (A + shift I) X
  LRADI_TRY(spmm_plain_csr(c->stream, dA, r, precision, use, shift, X, Y));
  LRADI_HIP(hipStreamSynchronize(c->stream));
  *avg_ms = ms;
  const int64_t tsz = precision == LRADI_FP64 ? 8 : 4;
  if (bytes) *bytes = dA.nnz * (tsz + 4) + 2 * tsz * (int64_t)dA.n * r;
  return LRADI_OK;
}

int lradi_spmm_tune(lradi_ctx* c, const lradi_csr* A, int r, int precision, int* lanes) {
  if (!c || !lanes) return set_error("lradi_spmm_tune: null argument"), LRADI_EINVAL;
  if (r < 1 || r > kMaxR) return set_error("lradi_spmm_tune: r must be in 1..%d", kMaxR), LRADI_EINVAL;
  if (precision != LRADI_FP64 && precision != LRADI_FP32_INNER)
    return set_error("lradi_spmm_tune: unknown precision"), LRADI_EINVAL;
  LRADI_HIP(hipSetDevice(c->device));
  DevCSR dA;
  LRADI_TRY(dA.upload(A, c->stream, precision == LRADI_FP32_INNER));
  const size_t blk = (size_t)dA.n * r * (precision == LRADI_FP64 ? 8 : 4);
  DevBuf X, Y;
  LRADI_TRY(X.alloc(blk));
  LRADI_TRY(Y.alloc(blk));
  LRADI_HIP(hipMemsetAsync(X.p, 0, blk, c->stream));
  LRADI_TRY(spmm_lanes_for(c, dA, r, precision, 0, X.p, Y.p, lanes));
  LRADI_HIP(hipStreamSynchronize(c->stream));
  return LRADI_OK;
}

int lradi_shifted_solve(lradi_ctx* c, int nsys, const lradi_csr* const* A, const double* shift,
                        const double* const* W, double* const* Z, const int* r, const double* delta,
                        const lradi_opts* opts, lradi_inner_stats* stats) {
  if (!c || nsys < 1 || !A || !shift || !W || !Z || !r || !delta)
    return set_error("lradi_shifted_solve: null or empty argument"), LRADI_EINVAL;
  lradi_opts o;
  lradi_default_opts(&o);
  if (opts) o = *opts;
  if (o.restart < 1 || o.restart > kMaxM || o.max_inner < 1 ||
      (o.precision != LRADI_FP64 && o.precision != LRADI_FP32_INNER) ||
      (o.precond != LRADI_PRECOND_NONE && o.precond != LRADI_PRECOND_RBILU0) || o.precond_sweeps < 0 ||
      o.precond_sweeps > 64 || (o.precond_pairs != 0 && o.precond_pairs != 1) ||
      (o.precond_poly != 0 && o.precond_poly != 1))
    return set_error("lradi_shifted_solve: bad options"), LRADI_EINVAL;
  const int sw = sweeps_for(o);
  LRADI_HIP(hipSetDevice(c->device));
  std::vector<DevCSR> mats(nsys);
  std::vector<std::unique_ptr<SysWork>> work(nsys);
  std::vector<SysWork*> ws(nsys);
  for (int s = 0; s < nsys; ++s) {
    if (!W[s] || !Z[s] || !(delta[s] >= 0.0) || !std::isfinite(shift[s]))
      return set_error("lradi_shifted_solve: bad system %d", s), LRADI_EINVAL;
    LRADI_TRY(mats[s].upload(A[s], c->stream, o.precision == LRADI_FP32_INNER));
    if (sw >= 0) LRADI_TRY(mats[s].prepare_rb(c, A[s], nullptr, c->stream, o.precision == LRADI_FP32_INNER));
    work[s] = std::make_unique<SysWork>();
    LRADI_TRY(work[s]->init(&mats[s], W[s], r[s], o.restart, o.precision, o.max_inner, floor_for(o), sw,
                            o.precond_pairs != 0, false, o.precond_poly));
    LRADI_TRY(work[s]->tune(c, mats[s], o.spmm_lanes));
    work[s]->arm(Z[s], shift[s], delta[s]);
    ws[s] = work[s].get();
  }
  Table tab;
  LRADI_TRY(upload_table(c, ws, tab));
  LRADI_TRY(prof_counters(c, o.profile != 0, &tab.b.prof_bytes));
  const long max_ticks = 3L * o.max_inner + 16;
  const int rc = run_ticks(c, tab.b, o.lookahead, max_ticks, o.profile != 0, nullptr, nullptr, o.use_graph != 0);
  if (rc != LRADI_OK) {
    (void)hipStreamSynchronize(c->stream);
    return rc;
  }
  LRADI_TRY(download_table(c, ws, tab));
  int status = LRADI_OK;
  for (int s = 0; s < nsys; ++s) {
    const SysCtl& h = ws[s]->c;
    if (stats) {
      stats[s].steps = h.steps;
      stats[s].cycles = h.cycles;
      stats[s].status = h.status;
      stats[s].pad = h.breakdowns;
      stats[s].rnorm = h.rnorm;
    }
    if (h.status == IS_NAN) status = LRADI_ENAN;
    else if (h.status == IS_CAP && status == LRADI_OK) status = LRADI_WINNER;
  }
  return status;
}

int lradi_solve(lradi_ctx* c, const lradi_csr* A, const lradi_csr* B, const double* f,
                const double* g, int r, const double* shiftsA, const double* shiftsB, int nshifts,
                const lradi_opts* opts, lradi_result** out) {
  if (!out) return set_error("lradi_solve: null output"), LRADI_EINVAL;
  lradi_problem P{A, B, f, g, r, nshifts, shiftsA, shiftsB, 0.0, nullptr, nullptr};
  return lradi_batch_solve(c, 1, &P, opts, out);
}

int lradi_solve_gen(lradi_ctx* c, const lradi_csr* A, const lradi_csr* B, const lradi_csr* M,
                    const lradi_csr* C, const double* f, const double* g, int r,
                    const double* shiftsA, const double* shiftsB, int nshifts, const lradi_opts* opts,
                    lradi_result** out) {
  if (!out) return set_error("lradi_solve_gen: null output"), LRADI_EINVAL;
  lradi_problem P{A, B, f, g, r, nshifts, shiftsA, shiftsB, 0.0, M, C};
  return lradi_batch_solve(c, 1, &P, opts, out);
}

int lradi_solve_lyap(lradi_ctx* c, const lradi_csr* A, const lradi_csr* M, const double* f, int r,
                     const double* shifts, int nshifts, const lradi_opts* opts, lradi_result** out) {
  if (!out) return set_error("lradi_solve_lyap: null output"), LRADI_EINVAL;
  lradi_problem P{A, nullptr, f, nullptr, r, nshifts, shifts, nullptr, 0.0, M, nullptr, 1};
  return lradi_batch_solve(c, 1, &P, opts, out);
}

int lradi_solve_complex(lradi_ctx* c, const lradi_csr* A, const lradi_csr* B, const double* f,
                        const double* g, int r, const double* shiftsA_re, const double* shiftsA_im,
                        const double* shiftsB_re, const double* shiftsB_im, int nshifts,
                        const lradi_opts* opts, lradi_result** out) {
  if (!out) return set_error("lradi_solve_complex: null output"), LRADI_EINVAL;
  if (!shiftsA_im || !shiftsB_im) return set_error("lradi_solve_complex: null imaginary parts"), LRADI_EINVAL;
  lradi_problem P{};
  P.A = A;
  P.B = B;
  P.f = f;
  P.g = g;
  P.r = r;
  P.nshifts = nshifts;
  P.shiftsA = shiftsA_re;
  P.shiftsB = shiftsB_re;
  P.shiftsA_im = shiftsA_im;
  P.shiftsB_im = shiftsB_im;
  return lradi_batch_solve(c, 1, &P, opts, out);
}

int lradi_batch_solve(lradi_ctx* c, int nprob, const lradi_problem* probs, const lradi_opts* opts,
                      lradi_result** outs) {
  if (!c || nprob < 1 || !probs || !outs) return set_error("lradi_batch_solve: bad argument"), LRADI_EINVAL;
  for (int i = 0; i < nprob; ++i) outs[i] = nullptr;
  lradi_opts o;
  lradi_default_opts(&o);
  if (opts) o = *opts;
  LRADI_TRY(check_opts(o));
  LRADI_HIP(hipSetDevice(c->device));
  // the preconditioner's host tables of all problems in parallel first
  prebuild_batch(c, o, probs, nprob);
  std::vector<std::unique_ptr<Prob>> ps(nprob);
  for (int i = 0; i < nprob; ++i) {
    ps[i] = std::make_unique<Prob>();
    LRADI_TRY(prob_init(c, o, probs[i], false, *ps[i]));
  }
  Engine E(c, o);
  for (auto& q : ps) E.act.push_back(q.get());
  // each run retires at least one problem (or fails)
  for (int k = 0; k <= nprob && !E.act.empty(); ++k)
    LRADI_TRY(E.run(std::max(1, (int)E.act.size() / 8), nullptr));
  if (!E.act.empty()) return set_error("lradi_batch_solve: problems left unfinished"), LRADI_EHIP;
  int status = LRADI_OK;
  for (int i = 0; i < nprob; ++i) {
    const int st = ps[i]->res->status;
    if (st < 0 && (status >= 0 || st < status)) status = st;
    else if (status >= 0 && st > status) status = st;
    outs[i] = ps[i]->res.release();
  }
  return status;
}

int lradi_profile_read(lradi_ctx* c, int kc, lradi_kernel_profile* out) {
  if (!c || !out || kc < 0 || kc >= LRADI_PROF_CLASSES)
    return set_error("lradi_profile_read: bad argument"), LRADI_EINVAL;
  unsigned long long bytes[LRADI_PROF_CLASSES] = {};
  if (c->prof_dev.p) {
    LRADI_HIP(hipSetDevice(c->device));
    LRADI_HIP(hipMemcpy(bytes, c->prof_dev.p, sizeof(bytes), hipMemcpyDeviceToHost));
  }
  out->ms = c->prof_ms[kc];
  out->launches = c->prof_launches[kc];
  out->bytes = (int64_t)bytes[kc];
  return LRADI_OK;
}

int lradi_profile_reset(lradi_ctx* c) {
  if (!c) return set_error("lradi_profile_reset: null context"), LRADI_EINVAL;
  for (int k = 0; k < LRADI_PROF_CLASSES; ++k) {
    c->prof_ms[k] = 0.0;
    c->prof_launches[k] = 0;
  }
  if (c->prof_dev.p) {
    LRADI_HIP(hipSetDevice(c->device));
    LRADI_HIP(hipMemset(c->prof_dev.p, 0, sizeof(unsigned long long) * LRADI_PROF_CLASSES));
  }
  return LRADI_OK;
}

int lradi_result_info(const lradi_result* r, int* k, int* status, double* rel, double* nfg) {
  if (!r) return set_error("null result"), LRADI_EINVAL;
  if (k) *k = r->k;
  if (status) *status = r->status;
  if (rel) *rel = r->rel_res;
  if (nfg) *nfg = r->norm_fg;
  return LRADI_OK;
}

int lradi_result_factors(const lradi_result* r, const double** Z, const double** D, const double** Y,
                         int* n, int* m, int* rr) {
  if (!r) return set_error("null result"), LRADI_EINVAL;
  if (Z) *Z = r->Zf.as<double>();
  if (D) *D = r->gam.data();
  if (Y) *Y = r->Y().as<double>();
  if (n) *n = r->n;
  if (m) *m = r->m;
  if (rr) *rr = r->r;
  return LRADI_OK;
}

int lradi_result_copy(const lradi_result* r, double* Z, double* D, double* Y) {
  if (!r) return set_error("null result"), LRADI_EINVAL;
  const size_t hz = r->cplx ? 2 : 1;
  if (Z && r->k > 0)
    LRADI_HIP(hipMemcpy(Z, r->Zf.p, sizeof(double) * (size_t)r->k * hz * r->n * r->r, hipMemcpyDeviceToHost));
  if (Y && r->k > 0)
    LRADI_HIP(hipMemcpy(Y, r->Y().p, sizeof(double) * (size_t)r->k * hz * r->m * r->r, hipMemcpyDeviceToHost));
  if (D) std::copy(r->gam.begin(), r->gam.begin() + (size_t)r->k * hz, D);
  return LRADI_OK;
}

int lradi_result_is_complex(const lradi_result* r, int* is_complex) {
  if (!r || !is_complex) return set_error("null argument"), LRADI_EINVAL;
  *is_complex = r->cplx ? 1 : 0;
  return LRADI_OK;
}

int lradi_result_history(const lradi_result* r, double* rows, int max_rows, int* nrows) {
  if (!r || !rows) return set_error("null argument"), LRADI_EINVAL;
  const int k = std::min(r->k, std::max(max_rows, 0));
  std::copy(r->hist.begin(), r->hist.begin() + (size_t)k * kHistCols, rows);
  if (nrows) *nrows = k;
  return LRADI_OK;
}

int lradi_result_time(const lradi_result* r, double* seconds) {
  if (!r || !seconds) return set_error("null argument"), LRADI_EINVAL;
  *seconds = r->seconds;
  return LRADI_OK;
}

void lradi_result_free(lradi_result* r) { delete r; }

int lradi_residual_gen(lradi_ctx* c, const lradi_csr* A, const lradi_csr* B, const lradi_csr* M,
                       const lradi_csr* C, int b_is_transposed, const double* f, const double* g, int r,
                       const double* Z, const double* D, const double* Y, int k, double* rel) {
  if (!c || !A || !B || !f || !g || !rel || (k > 0 && (!Z || !D || !Y)))
    return set_error("lradi_residual: null argument"), LRADI_EINVAL;
  if (r < 1 || r > kMaxR || k < 0) return set_error("lradi_residual: bad r or k"), LRADI_EINVAL;
  LRADI_HIP(hipSetDevice(c->device));
  hipStream_t st = c->stream;
  DevCSR dA, dAt, dB, dBt, dM, dMt, dC, dCt;
  LRADI_TRY(upload_pair(A, st, dA, dAt));
  if (b_is_transposed) {
    LRADI_TRY(upload_pair(B, st, dBt, dB));
  } else {
    LRADI_TRY(upload_pair(B, st, dB, dBt));
  }
  if (M) {
    if (M->nrows != A->nrows) return set_error("lradi_residual: M size differs from A"), LRADI_EINVAL;
    LRADI_TRY(upload_pair(M, st, dM, dMt));
  }
  if (C) {
    if (C->nrows != B->nrows) return set_error("lradi_residual: C size differs from B"), LRADI_EINVAL;
    if (b_is_transposed)
      LRADI_TRY(upload_pair(C, st, dCt, dC));
    else
      LRADI_TRY(upload_pair(C, st, dC, dCt));
  }
  DevBuf gam;
  LRADI_TRY(gam.alloc(sizeof(double) * std::max(k, 1)));
  if (k > 0) LRADI_HIP(hipMemcpyAsync(gam.p, D, sizeof(double) * k, hipMemcpyHostToDevice, st));
  const int maxit = std::min(2 * k * r + r + 2, 400);
  double sres = 0.0, sfg = 0.0;
  const DevCSR* pM = M ? &dM : nullptr;
  const DevCSR* pMt = M ? &dMt : nullptr;
  const DevCSR* pC = C ? &dC : nullptr;
  const DevCSR* pCt = C ? &dCt : nullptr;
  LRADI_TRY(residual_norm(st, dA, dAt, dB, dBt, f, g, r, Z, gam.as<double>(), Y, k, maxit, &sres, pM, pMt,
                          pC, pCt));
  LRADI_TRY(residual_norm(st, dA, dAt, dB, dBt, f, g, r, Z, gam.as<double>(), Y, 0, r + 2, &sfg));
  LRADI_HIP(hipStreamSynchronize(st));
  *rel = (sfg > 0.0) ? sres / sfg : 0.0;
  return LRADI_OK;
}

int lradi_residual(lradi_ctx* c, const lradi_csr* A, const lradi_csr* B, int b_is_transposed,
                   const double* f, const double* g, int r, const double* Z, const double* D,
                   const double* Y, int k, double* rel) {
  return lradi_residual_gen(c, A, B, nullptr, nullptr, b_is_transposed, f, g, r, Z, D, Y, k, rel);
}

int64_t lradi_alloc_count(void) { return lradi::g_alloc_count.load(std::memory_order_relaxed); }

int64_t lradi_residual_noalloc_limit(void) { return (int64_t)lradi::kScratchBytes; }

int lradi_residual_noalloc(lradi_ctx* c, const lradi_csr* A, const lradi_csr* At, const lradi_csr* B,
                           const lradi_csr* Bt, const double* f, const double* g, int r, const double* Z,
                           const double* D, const double* Y, int k, double* rel) {
  using namespace lradi;
  if (!c || !A || !At || !B || !Bt || !f || !g || !rel || (k > 0 && (!Z || !D || !Y)))
    return set_error("lradi_residual_noalloc: null argument"), LRADI_EINVAL;
  if (r < 1 || r > kMaxR || k < 0) return set_error("lradi_residual_noalloc: bad r or k"), LRADI_EINVAL;
  for (const lradi_csr* X : {A, At, B, Bt})
    if (!X->on_device || X->nrows <= 0 || X->nrows != X->ncols || X->nnz < 0 || X->nnz > INT32_MAX ||
        !X->rowptr || (X->nnz > 0 && (!X->colind || !X->val)))
      return set_error("lradi_residual_noalloc: every matrix must be a square device csr (on_device = 1)"),
             LRADI_EINVAL;
  const int n = A->nrows, m = B->nrows;
  if (At->nrows != n || Bt->nrows != m || At->nnz != A->nnz || Bt->nnz != B->nnz)
    return set_error("lradi_residual_noalloc: At / Bt do not match A / B"), LRADI_EINVAL;
  const int maxit = std::min(2 * k * r + r + 2, 400);
  if (k * r > 1024) return set_error("lradi_residual_noalloc: k*r above 1024"), LRADI_EINVAL;
  // scratch: the k gammas, then one residual workspace (the two evaluations
  // run one after the other and share it)
  const size_t gam_bytes = ((sizeof(double) * (size_t)std::max(k, 1) + 255) / 256) * 256;
  const size_t need =
      gam_bytes + std::max(residual_ws_bytes(n, m, maxit, false, false), residual_ws_bytes(n, m, r + 2, false, false));
  if (need > kScratchBytes)
    return set_error("lradi_residual_noalloc: n = %d, m = %d, k*r = %d need %zu bytes of scratch, above the "
                     "%zu bytes this entry point holds (use lradi_residual)",
                     n, m, k * r, need, kScratchBytes),
           LRADI_EINVAL;
  LRADI_HIP(hipSetDevice(c->device));
  LRADI_TRY(scratch_setup(c->device));
  std::lock_guard<std::mutex> lk(g_scratch_call_mu[c->device]);
  double* base = g_scratch_ptr[c->device];
  double* gam = base;
  double* ws = base + gam_bytes / sizeof(double);
  hipStream_t st = c->stream;
  if (k > 0) LRADI_HIP(hipMemcpyAsync(gam, D, sizeof(double) * k, hipMemcpyHostToDevice, st));
  auto ref = [](const lradi_csr* X) {
    return CsrRef{X->nrows, X->rowptr, X->colind, X->val};
  };
  const CsrRef rA = ref(A), rAt = ref(At), rB = ref(B), rBt = ref(Bt);
  double sres = 0.0, sfg = 0.0;
  LRADI_TRY(residual_norm_ws(st, rA, rAt, rB, rBt, f, g, r, Z, gam, Y, k, maxit, &sres, nullptr, nullptr,
                             nullptr, nullptr, ws));
  LRADI_TRY(residual_norm_ws(st, rA, rAt, rB, rBt, f, g, r, Z, gam, Y, 0, r + 2, &sfg, nullptr, nullptr,
                             nullptr, nullptr, ws));
  LRADI_HIP(hipStreamSynchronize(st));
  *rel = (sfg > 0.0) ? sres / sfg : 0.0;
  return LRADI_OK;
}

// ---------------------------------------------------------------------------
// serving
}  // extern "C"

struct lradi_server {
  lradi_ctx* ctx = nullptr;
  lradi_opts opts{};
  int64_t budget = 0;
  int max_active = 0;
  int admit_ms = 2;
  // host copies of a submitted problem until the worker uploads it
  struct Pending {
    uint64_t ticket;
    std::vector<int32_t> arp, aci, brp, bci, mrp, mci, crp, cci;
    std::vector<double> aval, bval, mval, cval, f, g, sA, sB, sAi, sBi;
    bool hasM = false, hasC = false, lyap = false;
    int r = 0, n = 0, m = 0;
    double tol = 0.0;
    size_t footprint = 0;
    std::chrono::steady_clock::time_point t_submit;
    // the preconditioner's host tables, built by the preparation threads
    // from the arrays above (which keep their storage when the request
    // moves): waited for before admission and before the request is dropped
    std::shared_future<void> prep;
  };
  // a few host threads that build submitted requests' preconditioner tables
  // while the worker runs the device
  struct PrepPool {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::function<void()>> jobs;
    bool stop = false;
    std::vector<std::thread> th;
    void start(int n) {
      for (int i = 0; i < n; ++i) th.emplace_back([this] { loop(); });
    }
    void loop() {
      for (;;) {
        std::function<void()> f;
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return stop || !jobs.empty(); });
          if (jobs.empty()) return;  // (stop, and every job done)
          f = std::move(jobs.front());
          jobs.pop_front();
        }
        f();
      }
    }
    void push(std::function<void()> f) {
      {
        std::lock_guard<std::mutex> lk(mu);
        jobs.push_back(std::move(f));
      }
      cv.notify_one();
    }
    void finish() {
      {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
      }
      cv.notify_all();
      for (auto& t : th) t.join();
      th.clear();
    }
  };
  PrepPool pool;
  struct Done {
    lradi_result* res = nullptr;
    double latency = 0.0;
  };
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Pending> queue;
  std::map<uint64_t, Done> done;
  std::map<uint64_t, std::chrono::steady_clock::time_point> submitted;
  std::vector<uint64_t> cancel_req;
  uint64_t next_ticket = 1;
  bool stop = false;
  int worker_error = LRADI_OK;
  lradi_server_counters st{};
  std::thread worker;
  void run();
};

namespace lradi {
namespace {
struct Live {
  std::unique_ptr<Prob> prob;
  uint64_t ticket;
  size_t footprint;
};
}  // namespace
}  // namespace lradi

void lradi_server::run() {
  (void)hipSetDevice(ctx->device);
  Engine E(ctx, opts);
  std::map<Prob*, Live> live;
  int64_t used = 0;
  auto complete = [&](Prob* q, int status_override) {
    auto it = live.find(q);
    Live L = std::move(it->second);
    live.erase(it);
    used -= (int64_t)L.footprint;
    lradi_result* R = L.prob->res.release();
    if (status_override != 0) R->status = status_override;
    std::lock_guard<std::mutex> lk(mu);
    const auto now = std::chrono::steady_clock::now();
    Done d;
    d.res = R;
    d.latency = std::chrono::duration<double>(now - submitted[L.ticket]).count();
    submitted.erase(L.ticket);
    done[L.ticket] = d;
    st.completed += 1;
  };
  for (;;) {
    std::vector<Pending> admit;
    std::vector<uint64_t> cancels;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (E.act.empty() && queue.empty() && !stop)
        cv.wait_for(lk, std::chrono::milliseconds(50));
      if (stop) break;
      while (!queue.empty() && (max_active <= 0 || (int)E.act.size() + (int)admit.size() < max_active) &&
             used + (int64_t)queue.front().footprint <= budget) {
        used += (int64_t)queue.front().footprint;
        admit.push_back(std::move(queue.front()));
        queue.pop_front();
      }
      cancels.swap(cancel_req);
      st.queued = (int)queue.size();
    }
    for (Pending& P : admit) {
      if (P.prep.valid()) P.prep.wait();
      auto q = std::make_unique<Prob>();
      lradi_csr A{P.n, P.n, (int64_t)P.aci.size(), P.arp.data(), P.aci.data(), P.aval.data(), 0};
      lradi_csr B{P.m, P.m, (int64_t)P.bci.size(), P.brp.data(), P.bci.data(), P.bval.data(), 0};
      DevBuf fd, gd;
      int rc = fd.alloc(sizeof(double) * P.f.size());
      if (rc == LRADI_OK && !P.lyap) rc = gd.alloc(sizeof(double) * P.g.size());
      if (rc == LRADI_OK && hipMemcpy(fd.p, P.f.data(), sizeof(double) * P.f.size(), hipMemcpyHostToDevice) != hipSuccess)
        rc = LRADI_EHIP;
      if (rc == LRADI_OK && !P.lyap &&
          hipMemcpy(gd.p, P.g.data(), sizeof(double) * P.g.size(), hipMemcpyHostToDevice) != hipSuccess)
        rc = LRADI_EHIP;
      lradi_csr Mc{P.n, P.n, (int64_t)P.mci.size(), P.mrp.data(), P.mci.data(), P.mval.data(), 0};
      lradi_csr Cc{P.m, P.m, (int64_t)P.cci.size(), P.crp.data(), P.cci.data(), P.cval.data(), 0};
      lradi_problem pr{&A, &B, fd.as<double>(), gd.as<double>(), P.r, (int32_t)P.sA.size(), P.sA.data(),
                       P.sB.data(), P.tol, P.hasM ? &Mc : nullptr, P.hasC ? &Cc : nullptr,
                       P.lyap ? 1 : 0, P.sAi.empty() ? nullptr : P.sAi.data(),
                       P.sBi.empty() ? nullptr : P.sBi.data()};
      if (rc == LRADI_OK) rc = prob_init(ctx, opts, pr, true, *q);
      Prob* raw = q.get();
      live[raw] = Live{std::move(q), P.ticket, P.footprint};
      if (rc != LRADI_OK) {
        if (!raw->res) raw->res = std::make_unique<lradi_result>();
        complete(raw, rc);
        continue;
      }
      E.act.push_back(raw);
      E.dirty = true;
    }
    // cancellations of running problems
    if (!cancels.empty()) {
      std::vector<Prob*> keep;
      for (Prob* q : E.act) {
        const uint64_t t = live[q].ticket;
        if (std::find(cancels.begin(), cancels.end(), t) != cancels.end()) {
          E.dirty = true;
          if (E.finalize(q) == LRADI_OK) complete(q, LRADI_ECANCELED);
        } else {
          keep.push_back(q);
        }
      }
      E.act.swap(keep);
    }
    if (E.act.empty()) {
      std::lock_guard<std::mutex> lk(mu);
      st.active = 0;
      st.bytes_in_use = used;
      continue;
    }
    // Return to this loop as soon as a problem finished (its result goes
    // out at once), a cancellation or shutdown came in, or a queued request
    // fits; admissions are batched over at least admit_ms.
    const auto t_run = std::chrono::steady_clock::now();
    auto interrupt = [&]() {
      std::lock_guard<std::mutex> lk(mu);
      if (stop || !cancel_req.empty()) return true;
      if (queue.empty()) return false;
      if (max_active > 0 && (int)E.act.size() >= max_active) return false;
      if (used + (int64_t)queue.front().footprint > budget) return false;
      return std::chrono::steady_clock::now() - t_run > std::chrono::milliseconds(admit_ms);
    };
    const int rc = E.run(1, interrupt);
    {
      std::lock_guard<std::mutex> lk(mu);
      st.steps += 1;
    }
    if (rc < 0) {
      // a device error ends every problem in flight with that status
      std::vector<Prob*> all = E.act;
      E.act.clear();
      E.dirty = true;
      for (Prob* q : all) {
        (void)E.finalize(q);
        complete(q, rc);
      }
      std::lock_guard<std::mutex> lk(mu);
      worker_error = rc;
    }
    std::vector<Prob*> fin;
    fin.swap(E.finished);
    for (Prob* q : fin) complete(q, 0);
    std::lock_guard<std::mutex> lk(mu);
    st.active = (int)E.act.size();
    st.bytes_in_use = used;
  }
  // shutdown: cancel whatever is still running
  std::vector<Prob*> all = E.act;
  E.act.clear();
  for (Prob* q : all) {
    (void)E.finalize(q);
    complete(q, LRADI_ECANCELED);
  }
  (void)hipStreamSynchronize(ctx->stream);
}

extern "C" {

int lradi_server_create(lradi_ctx* c, const lradi_opts* opts, int64_t hbm_budget, int max_active,
                        lradi_server** out) {
  if (!c || !out) return set_error("lradi_server_create: null argument"), LRADI_EINVAL;
  *out = nullptr;
  lradi_opts o;
  lradi_default_opts(&o);
  if (opts) o = *opts;
  LRADI_TRY(check_opts(o));
  LRADI_HIP(hipSetDevice(c->device));
  if (hbm_budget <= 0) {
    size_t fr = 0, tot = 0;
    LRADI_HIP(hipMemGetInfo(&fr, &tot));
    hbm_budget = (int64_t)(0.8 * (double)fr);
  }
  auto* s = new lradi_server();
  s->ctx = c;
  s->opts = o;
  s->budget = hbm_budget;
  s->max_active = max_active;
  s->st.bytes_budget = hbm_budget;
  if (sweeps_for(o) >= 0)
    s->pool.start(std::max(2, std::min(8, (int)std::thread::hardware_concurrency() / 2)));
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return LRADI_OK;
}

int lradi_server_submit(lradi_server* s, const lradi_problem* P, uint64_t* ticket) {
  const bool lyap = P && P->lyapunov != 0;
  if (!s || !P || !ticket || !P->A || !P->f || !P->shiftsA || (!lyap && (!P->B || !P->g || !P->shiftsB)))
    return set_error("lradi_server_submit: null argument"), LRADI_EINVAL;
  if (P->r < 1 || P->r > kMaxR || P->nshifts < 1)
    return set_error("lradi_server_submit: bad r or nshifts"), LRADI_EINVAL;
  lradi_server::Pending q;
  q.r = P->r;
  q.tol = P->tol;
  q.lyap = lyap;
  LRADI_TRY(host_csr(P->A, q.arp, q.aci, q.aval));
  if (!lyap) LRADI_TRY(host_csr(P->B, q.brp, q.bci, q.bval));
  if (P->M) {
    LRADI_TRY(host_csr(P->M, q.mrp, q.mci, q.mval));
    q.hasM = true;
  }
  if (P->C && !lyap) {
    LRADI_TRY(host_csr(P->C, q.crp, q.cci, q.cval));
    q.hasC = true;
  }
  q.n = P->A->nrows;
  q.m = lyap ? q.n : P->B->nrows;
  q.f.resize((size_t)q.n * q.r);
  LRADI_HIP(hipMemcpy(q.f.data(), P->f, sizeof(double) * q.f.size(), hipMemcpyDeviceToHost));
  if (!lyap) {
    q.g.resize((size_t)q.m * q.r);
    LRADI_HIP(hipMemcpy(q.g.data(), P->g, sizeof(double) * q.g.size(), hipMemcpyDeviceToHost));
  }
  q.sA.assign(P->shiftsA, P->shiftsA + P->nshifts);
  q.sB.assign(lyap ? P->shiftsA : P->shiftsB, (lyap ? P->shiftsA : P->shiftsB) + P->nshifts);
  if (P->shiftsA_im) q.sAi.assign(P->shiftsA_im, P->shiftsA_im + P->nshifts);
  if (P->shiftsB_im) q.sBi.assign(P->shiftsB_im, P->shiftsB_im + P->nshifts);
  const bool cplx = P->shiftsA_im || P->shiftsB_im;
  // (a mass matrix adds its values on the union pattern: counted as extra
  // nonzeros of the operator)
  // (complex problems hold stacked blocks of twice the rows)
  q.footprint = prob_footprint((cplx ? 2 : 1) * q.n, (cplx ? 2 : 1) * q.m, q.r,
                               (int64_t)(q.aci.size() + 2 * q.mci.size()),
                               (int64_t)(q.bci.size() + 2 * q.cci.size()), s->opts, lyap);
  if ((int64_t)q.footprint > s->budget)
    return set_error("lradi_server_submit: footprint %zu bytes exceeds the budget", q.footprint), LRADI_ENOMEM;
  q.t_submit = std::chrono::steady_clock::now();
  if (!s->pool.th.empty() && !cplx) {
    // the preconditioner's host tables on a preparation thread, from views of
    // this request's arrays
    auto done = std::make_shared<std::promise<void>>();
    q.prep = done->get_future().share();
    const lradi_csr A{q.n, q.n, (int64_t)q.aci.size(), q.arp.data(), q.aci.data(), q.aval.data(), 0};
    const lradi_csr B{q.m, q.m, (int64_t)q.bci.size(), q.brp.data(), q.bci.data(), q.bval.data(), 0};
    const lradi_csr M{q.n, q.n, (int64_t)q.mci.size(), q.mrp.data(), q.mci.data(), q.mval.data(), 0};
    const lradi_csr C{q.m, q.m, (int64_t)q.cci.size(), q.crp.data(), q.cci.data(), q.cval.data(), 0};
    const bool hasM = q.hasM, hasC = q.hasC;
    lradi_ctx* ctx = s->ctx;
    const lradi_opts o = s->opts;
    s->pool.push([=] {
      try {
        lradi_problem pr{};
        pr.A = &A;
        pr.B = lyap ? nullptr : &B;
        pr.M = hasM ? &M : nullptr;
        pr.C = hasC ? &C : nullptr;
        pr.lyapunov = lyap ? 1 : 0;
        for (int side = 0; side < 2; ++side) prebuild_side(ctx, o, pr, side, kRbPreEntries);
      } catch (...) {
        // (the worker builds the tables itself)
      }
      done->set_value();
    });
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    q.ticket = s->next_ticket++;
    *ticket = q.ticket;
    s->submitted[q.ticket] = q.t_submit;
    s->queue.push_back(std::move(q));
    s->st.queued = (int)s->queue.size();
  }
  s->cv.notify_one();
  return LRADI_OK;
}

int lradi_server_poll(lradi_server* s, uint64_t ticket, lradi_result** out, double* latency) {
  if (!s || !out) return set_error("lradi_server_poll: null argument"), LRADI_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->done.find(ticket);
  if (it != s->done.end()) {
    *out = it->second.res;
    if (latency) *latency = it->second.latency;
    s->done.erase(it);
    return 0;
  }
  if (s->submitted.count(ticket)) return 1;
  return set_error("lradi_server_poll: unknown ticket"), LRADI_EINVAL;
}

int lradi_server_cancel(lradi_server* s, uint64_t ticket) {
  if (!s) return set_error("lradi_server_cancel: null server"), LRADI_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
    if (it->ticket == ticket) {
      if (it->prep.valid()) it->prep.wait();  // (its tables are read from the request's arrays)
      auto* R = new lradi_result();
      R->status = LRADI_ECANCELED;
      lradi_server::Done d;
      d.res = R;
      d.latency = std::chrono::duration<double>(std::chrono::steady_clock::now() - it->t_submit).count();
      s->done[ticket] = d;
      s->submitted.erase(ticket);
      s->queue.erase(it);
      s->st.completed += 1;
      s->st.queued = (int)s->queue.size();
      return LRADI_OK;
    }
  }
  if (!s->submitted.count(ticket)) return set_error("lradi_server_cancel: unknown ticket"), LRADI_EINVAL;
  s->cancel_req.push_back(ticket);
  return LRADI_OK;
}

int lradi_server_stats(lradi_server* s, lradi_server_counters* out) {
  if (!s || !out) return set_error("lradi_server_stats: null argument"), LRADI_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  return s->worker_error < 0 ? s->worker_error : LRADI_OK;
}

int lradi_server_destroy(lradi_server* s) {
  if (!s) return LRADI_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  s->pool.finish();  // (pending jobs read queued requests' arrays)
  for (auto& kv : s->done) delete kv.second.res;
  delete s;
  return LRADI_OK;
}

}  // extern "C"
