"""Thin ctypes binding of liblradi.so (include/lradi.h).

Only argument marshalling lives here: every step of the method runs in the
HIP library.  Dense arguments are torch tensors on the GPU (FP64, row-major
n x r); sparse matrices are host CSR triples (numpy) that the library copies
to the device.  Importing this module loads the library and raises if it has
not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblradi.so")

OK, EINVAL, ENOMEM, EHIP, ENAN, EBREAKDOWN, ECANCELED = 0, -1, -2, -3, -4, -5, -6
WNOCONV, WINNER, WGAP = 1, 2, 3
SEL_RELATIVE, SEL_FIXED, SEL_MID, SEL_TIGHT_A, SEL_TIGHT_B, SEL_SYM = 0, 1, 2, 3, 4, 5
FP64, FP32_INNER = 0, 1
PRECOND_NONE, PRECOND_RBILU0 = 0, 1
HIST_COLS = 16
HIST_NAMES = ["k", "res_before", "deltaA", "deltaB", "rA", "rB", "stepsA", "stepsB", "u", "v",
              "norm_w", "norm_t", "norm_z", "norm_y", "gamma", "res_after"]

SELECTIONS = {"relative": SEL_RELATIVE, "fixed": SEL_FIXED, "mid": SEL_MID,
              "tightA": SEL_TIGHT_A, "tightB": SEL_TIGHT_B, "sym": SEL_SYM}


class LradiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lradi status {status}: {msg}")
        self.status = status


class Csr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int32), ("ncols", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("on_device", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("eps", ctypes.c_double),
                ("delta_min", ctypes.c_double), ("delta_max", ctypes.c_double),
                ("xi", ctypes.c_double), ("delta_fixed", ctypes.c_double),
                ("rho", ctypes.c_double), ("fp32_floor", ctypes.c_double),
                ("kmax", ctypes.c_int32), ("selection", ctypes.c_int32),
                ("backlook", ctypes.c_int32), ("paper_abs", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("max_inner", ctypes.c_int32), ("rescale", ctypes.c_int32),
                ("b_is_transposed", ctypes.c_int32), ("lookahead", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("spmm_lanes", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("precond_sweeps", ctypes.c_int32), ("precond_pairs", ctypes.c_int32),
                ("precond_poly", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("A", ctypes.POINTER(Csr)), ("B", ctypes.POINTER(Csr)), ("f", ctypes.c_void_p),
                ("g", ctypes.c_void_p), ("r", ctypes.c_int32), ("nshifts", ctypes.c_int32),
                ("shiftsA", ctypes.POINTER(ctypes.c_double)),
                ("shiftsB", ctypes.POINTER(ctypes.c_double)), ("tol", ctypes.c_double),
                ("M", ctypes.POINTER(Csr)), ("C", ctypes.POINTER(Csr)),
                ("lyapunov", ctypes.c_int32),
                ("shiftsA_im", ctypes.POINTER(ctypes.c_double)),
                ("shiftsB_im", ctypes.POINTER(ctypes.c_double))]


class ServerCounters(ctypes.Structure):
    _fields_ = [("active", ctypes.c_int32), ("queued", ctypes.c_int32), ("completed", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("bytes_in_use", ctypes.c_int64),
                ("bytes_budget", ctypes.c_int64)]


class KernelProfile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("launches", ctypes.c_int64), ("bytes", ctypes.c_int64)]


PROF_GRAM, PROF_SPMM, PROF_PRECOND = 0, 1, 2


class InnerStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("cycles", ctypes.c_int32), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("rnorm", ctypes.c_double)]


def _load():
    # torch must be loaded first: its bundled HIP runtime (soname
    # libamdhip64.so.7) then satisfies the library's dependency, so the
    # process holds a single HIP/HSA runtime.  Loading the library first
    # would bring in a second runtime that cannot open the device.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2312_02891_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "lradi_default_opts": (None, [P(Opts)]),
        "lradi_strerror": (ctypes.c_char_p, [i32]),
        "lradi_last_error": (ctypes.c_char_p, []),
        "lradi_create": (i32, [P(vp), i32, vp]),
        "lradi_destroy": (i32, [vp]),
        "lradi_convdiff_size": (i32, [i32, i32, P(ctypes.c_int64), P(ctypes.c_int64)]),
        "lradi_gen_convdiff": (i32, [i32, i32, P(dbl), vp, vp, vp]),
        "lradi_gen_convdiff_scheme": (i32, [i32, i32, P(dbl), i32, vp, vp, vp]),
        "lradi_spmm": (i32, [vp, P(Csr), dbl, vp, vp, i32, i32]),
        "lradi_spmm_bench": (i32, [vp, P(Csr), dbl, vp, vp, i32, i32, i32, i32, P(dbl),
                                   P(ctypes.c_int64)]),
        "lradi_spmm_tune": (i32, [vp, P(Csr), i32, i32, P(i32)]),
        "lradi_shifted_solve": (i32, [vp, i32, P(P(Csr)), P(dbl), P(vp), P(vp), P(i32), P(dbl),
                                      P(Opts), P(InnerStats)]),
        "lradi_solve": (i32, [vp, P(Csr), P(Csr), vp, vp, i32, P(dbl), P(dbl), i32, P(Opts),
                              P(vp)]),
        "lradi_batch_solve": (i32, [vp, i32, P(Problem), P(Opts), P(vp)]),
        "lradi_solve_gen": (i32, [vp, P(Csr), P(Csr), P(Csr), P(Csr), vp, vp, i32, P(dbl), P(dbl), i32,
                                  P(Opts), P(vp)]),
        "lradi_solve_lyap": (i32, [vp, P(Csr), P(Csr), vp, i32, P(dbl), i32, P(Opts), P(vp)]),
        "lradi_solve_complex": (i32, [vp, P(Csr), P(Csr), vp, vp, i32, P(dbl), P(dbl), P(dbl), P(dbl), i32,
                                      P(Opts), P(vp)]),
        "lradi_result_is_complex": (i32, [vp, P(i32)]),
        "lradi_server_create": (i32, [vp, P(Opts), ctypes.c_int64, i32, P(vp)]),
        "lradi_server_submit": (i32, [vp, P(Problem), P(ctypes.c_uint64)]),
        "lradi_server_poll": (i32, [vp, ctypes.c_uint64, P(vp), P(dbl)]),
        "lradi_server_cancel": (i32, [vp, ctypes.c_uint64]),
        "lradi_server_stats": (i32, [vp, P(ServerCounters)]),
        "lradi_server_destroy": (i32, [vp]),
        "lradi_result_info": (i32, [vp, P(i32), P(i32), P(dbl), P(dbl)]),
        "lradi_result_factors": (i32, [vp, P(vp), P(vp), P(vp), P(i32), P(i32), P(i32)]),
        "lradi_result_copy": (i32, [vp, vp, vp, vp]),
        "lradi_result_history": (i32, [vp, vp, i32, P(i32)]),
        "lradi_result_time": (i32, [vp, P(dbl)]),
        "lradi_result_free": (None, [vp]),
        "lradi_profile_read": (i32, [vp, i32, P(KernelProfile)]),
        "lradi_profile_reset": (i32, [vp]),
        "lradi_residual": (i32, [vp, P(Csr), P(Csr), i32, vp, vp, i32, vp, P(dbl), vp, i32,
                                 P(dbl)]),
        "lradi_residual_gen": (i32, [vp, P(Csr), P(Csr), P(Csr), P(Csr), i32, vp, vp, i32, vp, P(dbl),
                                     vp, i32, P(dbl)]),
        "lradi_residual_noalloc": (i32, [vp, P(Csr), P(Csr), P(Csr), P(Csr), vp, vp, i32, vp, P(dbl), vp,
                                         i32, P(dbl)]),
        "lradi_residual_noalloc_limit": (ctypes.c_int64, []),
        "lradi_alloc_count": (ctypes.c_int64, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def _check(status, allow_warn=True):
    if status < 0 or (status > 0 and not allow_warn):
        raise LradiError(status, "%s: %s" % (_lib.lradi_strerror(status).decode(),
                                             _lib.lradi_last_error().decode()))
    return status


def default_opts(**kw) -> Opts:
    o = Opts()
    _lib.lradi_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "selection" and isinstance(v, str):
            v = SELECTIONS[v]
        if k == "precision" and isinstance(v, str):
            v = {"fp64": FP64, "fp32": FP32_INNER, "fp32-inner": FP32_INNER}[v]
        if k == "precond" and isinstance(v, str):
            v = {"none": PRECOND_NONE, "rbilu0": PRECOND_RBILU0}[v]
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def alloc_count() -> int:
    """Device allocations the library has made in this process."""
    return int(_lib.lradi_alloc_count())


def residual_noalloc_limit() -> int:
    """Bytes of the scratch array behind Context.residual_noalloc."""
    return int(_lib.lradi_residual_noalloc_limit())


class DeviceCsr:
    """CSR matrix whose arrays are torch tensors on the GPU (int32 row
    pointers and column indices, FP64 values), passed with on_device = 1."""

    def __init__(self, rowptr, colind, val):
        torch = _torch()
        self.rowptr = torch.as_tensor(np.ascontiguousarray(rowptr, dtype=np.int32)).cuda()
        self.colind = torch.as_tensor(np.ascontiguousarray(colind, dtype=np.int32)).cuda()
        self.val = torch.as_tensor(np.ascontiguousarray(val, dtype=np.float64)).cuda()
        self.n = self.rowptr.numel() - 1
        self.c = Csr(self.n, self.n, self.colind.numel(), self.rowptr.data_ptr(), self.colind.data_ptr(),
                     self.val.data_ptr(), 1)


class HostCsr:
    """Host CSR triple kept alive while the library reads it."""

    def __init__(self, rowptr, colind, val):
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        self.colind = np.ascontiguousarray(colind, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.n = len(self.rowptr) - 1
        self.c = Csr(self.n, self.n, len(self.colind), self.rowptr.ctypes.data,
                     self.colind.ctypes.data, self.val.ctypes.data, 0)

    @property
    def nnz(self):
        return len(self.colind)


SCHEME_UPWIND, SCHEME_CENTRAL = 0, 1


def convdiff(dim: int, N: int, omega: Sequence[float], scheme: int = SCHEME_UPWIND) -> HostCsr:
    """A = -L_h of the convection-diffusion operator (library generator),
    upwind or central first differences."""
    n = ctypes.c_int64()
    nnz = ctypes.c_int64()
    _check(_lib.lradi_convdiff_size(dim, N, ctypes.byref(n), ctypes.byref(nnz)))
    rp = np.empty(n.value + 1, dtype=np.int32)
    ci = np.empty(nnz.value, dtype=np.int32)
    v = np.empty(nnz.value, dtype=np.float64)
    om = (ctypes.c_double * dim)(*[float(w) for w in omega])
    _check(_lib.lradi_gen_convdiff_scheme(dim, N, om, int(scheme), rp.ctypes.data, ci.ctypes.data,
                                          v.ctypes.data), allow_warn=False)
    return HostCsr(rp, ci, v)


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Result:
    def __init__(self, handle, status):
        self.h = ctypes.c_void_p(handle)
        self.status = status
        k, st = ctypes.c_int(), ctypes.c_int()
        rel, nfg = ctypes.c_double(), ctypes.c_double()
        _check(_lib.lradi_result_info(self.h, ctypes.byref(k), ctypes.byref(st), ctypes.byref(rel),
                                      ctypes.byref(nfg)))
        self.k, self.rel_res, self.norm_fg = k.value, rel.value, nfg.value
        self.status = st.value
        n, m, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        zp, dp, yp = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(_lib.lradi_result_factors(self.h, ctypes.byref(zp), ctypes.byref(dp),
                                         ctypes.byref(yp), ctypes.byref(n), ctypes.byref(m),
                                         ctypes.byref(r)))
        self.n, self.m, self.r = n.value, m.value, r.value
        self.Zptr, self.Yptr = zp.value, yp.value
        sec = ctypes.c_double()
        _check(_lib.lradi_result_time(self.h, ctypes.byref(sec)))
        self.seconds = sec.value
        cx = ctypes.c_int()
        _check(_lib.lradi_result_is_complex(self.h, ctypes.byref(cx)))
        self.is_complex = bool(cx.value)

    def factors(self):
        """(Z n x kr, d kr, Y m x kr) as host numpy arrays (blocks side by
        side); complex arrays for complex results."""
        k, n, m, r = self.k, self.n, self.m, self.r
        if self.is_complex:
            Z = np.empty((k, 2 * n, r))
            Y = np.empty((k, 2 * m, r))
            D = np.empty(2 * max(k, 1))
            _check(_lib.lradi_result_copy(self.h, Z.ctypes.data, D.ctypes.data, Y.ctypes.data))
            Zc = Z[:, :n, :] + 1j * Z[:, n:, :]
            Yc = Y[:, :m, :] + 1j * Y[:, m:, :]
            Zc = np.concatenate([Zc[i] for i in range(k)], axis=1) if k else np.zeros((n, 0), complex)
            Yc = np.concatenate([Yc[i] for i in range(k)], axis=1) if k else np.zeros((m, 0), complex)
            d = np.repeat(D[0:2 * k:2] + 1j * D[1:2 * k:2], r)
            return Zc, d, Yc
        Z = np.empty((k, n, r))
        Y = np.empty((k, m, r))
        D = np.empty(max(k, 1))
        _check(_lib.lradi_result_copy(self.h, Z.ctypes.data, D.ctypes.data, Y.ctypes.data))
        Zc = np.concatenate([Z[i] for i in range(k)], axis=1) if k else np.zeros((n, 0))
        Yc = np.concatenate([Y[i] for i in range(k)], axis=1) if k else np.zeros((m, 0))
        d = np.repeat(D[:k], r)
        return Zc, d, Yc

    def gammas(self):
        if self.is_complex:
            D = np.empty(2 * max(self.k, 1))
            _check(_lib.lradi_result_copy(self.h, None, D.ctypes.data, None))
            return D[0:2 * self.k:2] + 1j * D[1:2 * self.k:2]
        D = np.empty(max(self.k, 1))
        _check(_lib.lradi_result_copy(self.h, None, D.ctypes.data, None))
        return D[: self.k]

    def history(self):
        rows = np.zeros((max(self.k, 1), HIST_COLS))
        nr = ctypes.c_int()
        _check(_lib.lradi_result_history(self.h, rows.ctypes.data, self.k, ctypes.byref(nr)))
        return rows[: nr.value]

    def device_factors(self):
        """Torch views (k, n, r) / (k, m, r) of the library-owned device factors
        (no copy); valid while this Result lives."""
        torch = _torch()

        class _View:
            def __init__(self, ptr, shape):
                self.__cuda_array_interface__ = {"shape": shape, "typestr": "<f8",
                                                 "data": (ptr, False), "version": 3,
                                                 "strides": None}

        k = max(self.k, 0)
        Z = torch.as_tensor(_View(self.Zptr, (k, self.n, self.r)), device="cuda")
        Y = torch.as_tensor(_View(self.Yptr, (k, self.m, self.r)), device="cuda")
        return Z, Y

    def __del__(self):
        try:
            if self.h:
                _lib.lradi_result_free(self.h)
                self.h = None
        except Exception:
            pass


class Context:
    """lradi_ctx bound to one device.  Calls synchronise torch's stream first
    and return after the library's own stream finished."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(_lib.lradi_create(ctypes.byref(h), device, None))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            _lib.lradi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync(self):
        _torch().cuda.synchronize(self.device)

    def profile_read(self, kernel_class: int):
        """(ms, launches, algorithmic bytes) accumulated for a kernel class."""
        p = KernelProfile()
        _check(_lib.lradi_profile_read(self.h, kernel_class, ctypes.byref(p)))
        return p.ms, p.launches, p.bytes

    def profile_reset(self):
        _check(_lib.lradi_profile_reset(self.h))

    def spmm(self, A: HostCsr, shift: float, X, precision: int = FP64):
        """Y = (A + shift I) X; X (n x r) FP64 or FP32 torch tensor on the GPU."""
        torch = _torch()
        assert X.is_cuda and X.is_contiguous() and X.dim() == 2
        prec = FP64 if X.dtype == torch.float64 else FP32_INNER
        Y = torch.empty_like(X)
        self._sync()
        _check(_lib.lradi_spmm(self.h, ctypes.byref(A.c), float(shift), _ptr(X), _ptr(Y),
                               X.shape[1], prec), allow_warn=False)
        return Y

    def spmm_bench(self, A: HostCsr, shift: float, X, reps: int = 20, lanes: int = 0, out=None):
        """(average ms per launch, algorithmic bytes per launch) of the
        shifted product on X (FP64 or FP32 CUDA tensor); lanes = 0 uses the
        tiling the solver would pick.  `out` (like X) receives the product."""
        torch = _torch()
        prec = FP64 if X.dtype == torch.float64 else FP32_INNER
        Y = torch.empty_like(X) if out is None else out
        assert Y.shape == X.shape and Y.dtype == X.dtype and Y.is_cuda and Y.is_contiguous()
        ms, nb = ctypes.c_double(), ctypes.c_int64()
        self._sync()
        _check(_lib.lradi_spmm_bench(self.h, ctypes.byref(A.c), float(shift), _ptr(X), _ptr(Y), X.shape[1],
                                     prec, lanes, reps, ctypes.byref(ms), ctypes.byref(nb)), allow_warn=False)
        return ms.value, nb.value

    def spmm_tune(self, A: HostCsr, r: int, precision: int = FP64) -> int:
        """Lanes per row the autotuner picks for A with r columns."""
        lanes = ctypes.c_int()
        self._sync()
        _check(_lib.lradi_spmm_tune(self.h, ctypes.byref(A.c), r, precision, ctypes.byref(lanes)),
               allow_warn=False)
        return lanes.value

    def shifted_solve(self, mats: List[HostCsr], shifts, Ws, deltas, opts: Optional[Opts] = None):
        """Batched (A_s + shift_s I) Z_s = W_s to ||R_s||_2 <= delta_s; returns (Zs, stats)."""
        torch = _torch()
        ns = len(mats)
        Zs = [torch.zeros_like(W) for W in Ws]
        Aarr = (ctypes.POINTER(Csr) * ns)(*[ctypes.pointer(M.c) for M in mats])
        sh = (ctypes.c_double * ns)(*[float(s) for s in shifts])
        Wp = (ctypes.c_void_p * ns)(*[W.data_ptr() for W in Ws])
        Zp = (ctypes.c_void_p * ns)(*[Z.data_ptr() for Z in Zs])
        rr = (ctypes.c_int * ns)(*[W.shape[1] for W in Ws])
        dl = (ctypes.c_double * ns)(*[float(d) for d in deltas])
        stats = (InnerStats * ns)()
        self._sync()
        st = _check(_lib.lradi_shifted_solve(self.h, ns, Aarr, sh, Wp, Zp, rr, dl,
                                             ctypes.byref(opts) if opts is not None else None,
                                             stats))
        return Zs, [dict(steps=s.steps, cycles=s.cycles, status=s.status, breakdowns=s.pad,
                         rnorm=s.rnorm) for s in stats], st

    @staticmethod
    def make_problem(A: HostCsr, B: Optional[HostCsr], f, g, shiftsA, shiftsB, tol=0.0, M=None, C=None,
                     lyapunov=False):
        """(Problem struct, keep-alive list) for batch and serving calls; M, C
        (HostCsr or None) give the generalized equation.  lyapunov=True: the
        case A X M^T + M X A^T = -f f^T, where B, g, shiftsB, C are not used
        (may be None)."""
        cx = np.iscomplexobj(shiftsA) or (shiftsB is not None and np.iscomplexobj(shiftsB))
        sA = np.ascontiguousarray(np.real(shiftsA), dtype=np.float64)
        sB = sA if lyapunov else np.ascontiguousarray(np.real(shiftsB), dtype=np.float64)
        sAi = np.ascontiguousarray(np.imag(shiftsA), dtype=np.float64) if cx else None
        sBi = np.ascontiguousarray(np.imag(shiftsB), dtype=np.float64) if cx else None
        dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None  # noqa: E731
        assert f.is_cuda and f.is_contiguous()
        if not lyapunov:
            assert g.is_cuda and g.is_contiguous()
        pr = Problem(ctypes.pointer(A.c), ctypes.pointer(B.c) if B is not None else None, f.data_ptr(),
                     g.data_ptr() if g is not None else None, f.shape[1],
                     len(sA), sA.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     sB.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(tol),
                     ctypes.pointer(M.c) if M is not None else None,
                     ctypes.pointer(C.c) if C is not None else None, 1 if lyapunov else 0,
                     dp(sAi), dp(sBi))
        return pr, [A, B, f, g, sA, sB, M, C, sAi, sBi]

    @staticmethod
    def lyap_problem(A: HostCsr, f, shifts, tol=0.0, M=None):
        """A Lyapunov problem A X M^T + M X A^T = -f f^T for batch_solve."""
        return dict(A=A, B=None, f=f, g=None, shiftsA=shifts, shiftsB=None, tol=tol, M=M,
                    lyapunov=True)

    def batch_solve(self, problems, opts: Optional[Opts] = None):
        """problems: list of (A, B, f, g, shiftsA, shiftsB[, tol, M, C]) or of
        make_problem keyword dicts (lyap_problem); returns (list of Result,
        overall status)."""
        structs, keep = [], []
        for pr in problems:
            s_, k_ = self.make_problem(**pr) if isinstance(pr, dict) else self.make_problem(*pr)
            structs.append(s_)
            keep.append(k_)
        n = len(structs)
        arr = (Problem * n)(*structs)
        outs = (ctypes.c_void_p * n)()
        self._sync()
        st = _lib.lradi_batch_solve(self.h, n, arr, ctypes.byref(opts) if opts is not None else None, outs)
        results = [Result(outs[i], 0) if outs[i] else None for i in range(n)]
        # per-problem failures (status in each result) still return every
        # result; an error before any problem ran raises
        if st < 0 and not any(outs[i] for i in range(n)):
            _check(st)
        return results, st

    def residual(self, A: HostCsr, B: HostCsr, f, g, result: "Result", b_is_transposed=False,
                 M: Optional[HostCsr] = None, C: Optional[HostCsr] = None):
        """True ||A X C + M X B + f g^T||_2 / ||f g^T||_2 of a solve result
        (M = C = I unless given; lradi_residual_gen on the result's device
        factors)."""
        D = np.ascontiguousarray(result.gammas(), dtype=np.float64)
        out = ctypes.c_double()
        self._sync()
        _check(_lib.lradi_residual_gen(self.h, ctypes.byref(A.c), ctypes.byref(B.c),
                                       ctypes.byref(M.c) if M is not None else None,
                                       ctypes.byref(C.c) if C is not None else None,
                                       int(bool(b_is_transposed)), _ptr(f), _ptr(g), f.shape[1],
                                       ctypes.c_void_p(result.Zptr),
                                       D.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       ctypes.c_void_p(result.Yptr), result.k, ctypes.byref(out)),
               allow_warn=False)
        return out.value

    def residual_noalloc(self, A: "DeviceCsr", At: "DeviceCsr", B: "DeviceCsr", Bt: "DeviceCsr", f, g,
                         result: "Result"):
        """lradi_residual_noalloc: the true residual of a result (M = C = I)
        with every matrix and its transpose already on the device; the call
        allocates no device memory."""
        D = np.ascontiguousarray(result.gammas(), dtype=np.float64)
        out = ctypes.c_double()
        self._sync()
        _check(_lib.lradi_residual_noalloc(self.h, ctypes.byref(A.c), ctypes.byref(At.c), ctypes.byref(B.c),
                                           ctypes.byref(Bt.c), _ptr(f), _ptr(g), f.shape[1],
                                           ctypes.c_void_p(result.Zptr),
                                           D.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           ctypes.c_void_p(result.Yptr), result.k, ctypes.byref(out)),
               allow_warn=False)
        return out.value

    def residual_lyap(self, A: HostCsr, f, result: "Result", M: Optional[HostCsr] = None):
        """True ||A X M^T + M X A^T + f f^T||_2 / ||f f^T||_2 of X = Z D Z^T:
        lradi_residual_gen with B^T = A, C^T = M, g = f and Y = Z."""
        D = np.ascontiguousarray(result.gammas(), dtype=np.float64)
        out = ctypes.c_double()
        self._sync()
        pM = ctypes.byref(M.c) if M is not None else None
        _check(_lib.lradi_residual_gen(self.h, ctypes.byref(A.c), ctypes.byref(A.c), pM, pM, 1,
                                       _ptr(f), _ptr(f), f.shape[1], ctypes.c_void_p(result.Zptr),
                                       D.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       ctypes.c_void_p(result.Zptr), result.k, ctypes.byref(out)),
               allow_warn=False)
        return out.value

    def residual_factors(self, A: HostCsr, B: HostCsr, f, g, Zs, gammas, Ys, b_is_transposed=False):
        """lradi_residual on device factor stacks Zs (k, n, r) and Ys (k, m, r)."""
        D = np.ascontiguousarray(gammas, dtype=np.float64)
        out = ctypes.c_double()
        self._sync()
        _check(_lib.lradi_residual(self.h, ctypes.byref(A.c), ctypes.byref(B.c), int(bool(b_is_transposed)),
                                   _ptr(f), _ptr(g), f.shape[1], _ptr(Zs),
                                   D.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(Ys),
                                   len(D), ctypes.byref(out)), allow_warn=False)
        return out.value

    def solve(self, A: HostCsr, B: HostCsr, f, g, shiftsA, shiftsB, opts: Optional[Opts] = None,
              M: Optional[HostCsr] = None, C: Optional[HostCsr] = None):
        """Algorithm 1 on A X + X B = -f g^T (f, g: FP64 CUDA tensors), or on
        A X C + M X B = -f g^T when M or C is given; B (and C) are the
        matrices themselves unless opts.b_is_transposed."""
        assert f.is_cuda and g.is_cuda and f.is_contiguous() and g.is_contiguous()
        r = f.shape[1]
        sA = np.ascontiguousarray(shiftsA, dtype=np.float64)
        sB = np.ascontiguousarray(shiftsB, dtype=np.float64)
        h = ctypes.c_void_p()
        self._sync()
        po = ctypes.byref(opts) if opts is not None else None
        psA = sA.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        psB = sB.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if M is None and C is None:
            st = _check(_lib.lradi_solve(self.h, ctypes.byref(A.c), ctypes.byref(B.c), _ptr(f), _ptr(g),
                                         r, psA, psB, len(sA), po, ctypes.byref(h)))
        else:
            pM = ctypes.byref(M.c) if M is not None else None
            pC = ctypes.byref(C.c) if C is not None else None
            st = _check(_lib.lradi_solve_gen(self.h, ctypes.byref(A.c), ctypes.byref(B.c), pM, pC,
                                             _ptr(f), _ptr(g), r, psA, psB, len(sA), po,
                                             ctypes.byref(h)))
        res = Result(h.value, st)
        return res

    def solve_complex(self, A: HostCsr, B: HostCsr, f, g, shiftsA, shiftsB, opts: Optional[Opts] = None):
        """Algorithm 1 with complex shifts (complex arrays pA added to A, pB
        added to B^T) in its complex form; the result's factors are complex."""
        assert f.is_cuda and g.is_cuda and f.is_contiguous() and g.is_contiguous()
        a = np.asarray(shiftsA, dtype=np.complex128)
        b = np.asarray(shiftsB, dtype=np.complex128)
        arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (a.real, a.imag, b.real, b.imag)]
        ptr = [x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for x in arr]
        h = ctypes.c_void_p()
        self._sync()
        st = _check(_lib.lradi_solve_complex(self.h, ctypes.byref(A.c), ctypes.byref(B.c), _ptr(f), _ptr(g),
                                             f.shape[1], ptr[0], ptr[1], ptr[2], ptr[3], len(a),
                                             ctypes.byref(opts) if opts is not None else None,
                                             ctypes.byref(h)))
        return Result(h.value, st)

    def solve_lyap(self, A: HostCsr, f, shifts, opts: Optional[Opts] = None, M: Optional[HostCsr] = None):
        """Lyapunov case A X M^T + M X A^T = -f f^T (M = I unless given): one
        inner solve per step, shifts added to A; the result's Y is its Z."""
        assert f.is_cuda and f.is_contiguous()
        sh = np.ascontiguousarray(shifts, dtype=np.float64)
        h = ctypes.c_void_p()
        self._sync()
        st = _check(_lib.lradi_solve_lyap(self.h, ctypes.byref(A.c), ctypes.byref(M.c) if M is not None else None,
                                          _ptr(f), f.shape[1], sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          len(sh), ctypes.byref(opts) if opts is not None else None,
                                          ctypes.byref(h)))
        return Result(h.value, st)


class Server:
    """Continuous-batching request loop (lradi_server_*) on a context that the
    caller must not use while the server lives."""

    def __init__(self, ctx: Context, opts: Optional[Opts] = None, hbm_budget: int = 0,
                 max_active: int = 0):
        h = ctypes.c_void_p()
        ctx._sync()
        _check(_lib.lradi_server_create(ctx.h, ctypes.byref(opts) if opts is not None else None,
                                        int(hbm_budget), int(max_active), ctypes.byref(h)))
        self.h = h
        self.ctx = ctx

    def submit(self, A: HostCsr, B: HostCsr, f, g, shiftsA, shiftsB, tol=0.0, M=None, C=None) -> int:
        pr, keep = Context.make_problem(A, B, f, g, shiftsA, shiftsB, tol, M, C)
        t = ctypes.c_uint64()
        # f and g are ready once the producing stream is (not a device-wide
        # sync, which would wait for the server's own work too)
        _torch().cuda.current_stream().synchronize()
        _check(_lib.lradi_server_submit(self.h, ctypes.byref(pr), ctypes.byref(t)))
        return t.value

    def submit_lyap(self, A: HostCsr, f, shifts, tol=0.0, M=None) -> int:
        pr, keep = Context.make_problem(A, None, f, None, shifts, None, tol, M, None, lyapunov=True)
        t = ctypes.c_uint64()
        _torch().cuda.current_stream().synchronize()
        _check(_lib.lradi_server_submit(self.h, ctypes.byref(pr), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """(Result, latency seconds) when done, else None."""
        out = ctypes.c_void_p()
        lat = ctypes.c_double()
        st = _lib.lradi_server_poll(self.h, ticket, ctypes.byref(out), ctypes.byref(lat))
        if st == 1:
            return None
        _check(st)
        return Result(out.value, 0), lat.value

    def cancel(self, ticket: int):
        _check(_lib.lradi_server_cancel(self.h, ticket))

    def stats(self):
        c = ServerCounters()
        _check(_lib.lradi_server_stats(self.h, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in ServerCounters._fields_}

    def close(self):
        if self.h:
            _lib.lradi_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
