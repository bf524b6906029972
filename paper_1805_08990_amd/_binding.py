"""ctypes binding of libdme.so (the C ABI declared in include/dme.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device arrays are torch CUDA float64 tensors; the library is column-major, so
a logical (rows x cols) matrix lives in a row-major (cols, rows) storage
tensor and is handed back as its transposed view.  Host arrays for the solve
calls are numpy float64 arrays (copied to Fortran order here).

If the library has not been built, importing this module raises ImportError:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdme.so")

DME_OK = 0
DME_EINVAL = -1
DME_ENOMEM = -2
DME_ERANK = -3
DME_ENUMERIC = -4
DME_EAGAIN = -5
DME_EHIP = -6
DME_EINTERNAL = -7

DME_LIE, DME_STRANG = 0, 1
DME_SPLIT_F12, DME_SPLIT_F1F2, DME_SPLIT_F1F3F2 = 0, 1, 2
DME_FP64, DME_MIXED = 0, 1

SCHEMES = {"lie": DME_LIE, "strang": DME_STRANG}
SPLITS = {"F12": DME_SPLIT_F12, "F1F2": DME_SPLIT_F1F2, "F1F3F2": DME_SPLIT_F1F3F2}
PRECISIONS = {"fp64": DME_FP64, "mixed": DME_MIXED}
DME_ACTION_DENSE, DME_ACTION_LEJA = 0, 1
ACTIONS = {"dense": DME_ACTION_DENSE, "leja": DME_ACTION_LEJA}

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -m paper_1805_08990_amd.build); there is no CPU fallback")

# PyTorch supplies device memory and streams, so the library must run on the
# HIP runtime torch has loaded: importing torch first makes the library's
# libamdhip64.so.7 dependency resolve (by soname) to that same runtime instead
# of loading a second one, which would not see the device.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

_p = ctypes.c_void_p
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_int = ctypes.c_int
_pd = ctypes.POINTER(ctypes.c_double)


class Problem(ctypes.Structure):
    _fields_ = [("n", _i64), ("m", _i64), ("p", _i64), ("r0", _i64),
                ("A", _p), ("B", _p), ("C", _p), ("R", _p), ("S", _p), ("L0", _p), ("D0", _p),
                ("M", _p), ("A_rowptr", _p), ("A_colind", _p), ("A_val", _p)]


class Opts(ctypes.Structure):
    _fields_ = [("T", _dbl), ("h", _dbl), ("tol", _dbl), ("scheme", _int), ("split", _int),
                ("precision", _int), ("quad_nodes", _int), ("max_rank", _i64), ("action", _int)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_lib_dme_create = _sig("dme_create", _int, [ctypes.POINTER(_p), _int, _p])
_lib_dme_destroy = _sig("dme_destroy", None, [_p])
_lib_dme_strerror = _sig("dme_strerror", ctypes.c_char_p, [_int])
_lib_dme_last_error = _sig("dme_last_error", ctypes.c_char_p, [])
_lib_dle_solve = _sig("dle_solve", _int, [_p, ctypes.POINTER(Problem), ctypes.POINTER(Opts), ctypes.POINTER(_p)])
_lib_dre_solve = _sig("dre_solve", _int, [_p, ctypes.POINTER(Problem), ctypes.POINTER(Opts), ctypes.POINTER(_p)])
_lib_solver_create = _sig("dme_solver_create", _int,
                          [_p, ctypes.POINTER(Problem), ctypes.POINTER(Opts), _int, ctypes.POINTER(_p)])
_lib_solver_step = _sig("dme_solver_step", _int, [_p, _i64])
_lib_solver_state = _sig("dme_solver_state", _int,
                         [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)])
_lib_solver_setup_info = _sig("dme_solver_setup_info", _int,
                              [_p, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), ctypes.POINTER(_i64)])
_lib_solver_result = _sig("dme_solver_result", _int, [_p, ctypes.POINTER(_p)])
_lib_solver_free = _sig("dme_solver_free", None, [_p])
_lib_solver_profile = _sig("dme_solver_profile", _int, [_p, _int])
_lib_solver_gain = _sig("dme_solver_gain", _int, [_p, _p, _i64])
_lib_solver_profile_get = _sig("dme_solver_profile_get", _int,
                               [_p, _int, ctypes.POINTER(_i64), ctypes.POINTER(_dbl),
                                ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)])
PHASES = {"step_gemm": 0, "compress": 1, "riccati": 2, "S": 3, "step_kernel": 4}
_lib_result_info = _sig("dme_result_info", _int,
                        [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                         ctypes.POINTER(_dbl)])
_lib_result_copy = _sig("dme_result_copy", _int, [_p, _p, _p])
_lib_result_free = _sig("dme_result_free", None, [_p])
_lib_expm = _sig("dme_expm", _int, [_p, _i64, _p, _dbl, _p, ctypes.POINTER(_int), ctypes.POINTER(_int)])
_lib_gemm = _sig("dme_gemm_f64", _int, [_p, ctypes.c_char, ctypes.c_char, _i64, _i64, _i64, _dbl,
                                        _p, _i64, _p, _i64, _dbl, _p, _i64])
_lib_gemm_mixed = _sig("dme_gemm_mixed", _int, [_p, _i64, _i64, _p, _p, _i64, _p, _i64])
_lib_compress = _sig("dme_compress", _int, [_p, _i64, _i64, _p, _p, _dbl, _i64, _p, _p, ctypes.POINTER(_i64)])
_lib_riccati = _sig("dme_riccati", _int, [_p, _i64, _i64, _i64, _p, _p, _p, _dbl, _p])
_lib_riccati_noalloc = _sig("dme_riccati_noalloc", _int, [_p, _i64, _i64, _i64, _p, _p, _p, _dbl, _p])
_lib_expmv_leja = _sig("dme_expmv_leja", _int, [_p, _i64, _p, _p, _p, _p, _dbl, _i64, _p, _p,
                                                 ctypes.POINTER(_int), ctypes.POINTER(_int)])
_lib_syev = _sig("dme_syev", _int, [_p, _i64, _p, _dbl, _i64, _p, _p, ctypes.POINTER(_i64)])

_lib_register = _sig("dme_register_operator", _int, [_p, _p, _i64, ctypes.POINTER(ctypes.c_uint64)])
_lib_server_start = _sig("dme_server_start", _int, [_p, ctypes.c_size_t, _int, ctypes.POINTER(_p)])
_lib_server_warm = _sig("dme_server_warm", _int, [_p, ctypes.c_uint64, _dbl, _int, _int])
_lib_submit = _sig("dme_submit", _int, [_p, ctypes.c_uint64, ctypes.POINTER(Problem), ctypes.POINTER(Opts),
                                        _int, ctypes.POINTER(ctypes.c_uint64)])
_lib_poll = _sig("dme_poll", _int, [_p, ctypes.c_uint64, ctypes.POINTER(_p)])
_lib_server_stop = _sig("dme_server_stop", _int, [_p])
_lib_result_serving = _sig("dme_result_serving", _int, [_p, ctypes.POINTER(_int), ctypes.POINTER(_int),
                                                        ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)])


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", _i64), ("failed", _i64), ("fallbacks", _i64), ("steps", _i64),
                ("cold_builds", _i64), ("in_flight", _i64), ("peak_bytes", _i64),
                ("p50_s", _dbl), ("p99_s", _dbl), ("queue_p50_s", _dbl), ("queue_p99_s", _dbl),
                ("req_per_s", _dbl), ("steps_per_s", _dbl), ("cold_build_s", _dbl)]


_lib_server_stats = _sig("dme_server_stats_get", _int, [_p, ctypes.POINTER(ServerStats)])


class DmeError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib_dme_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_lib_dme_strerror(code).decode()} ({code}): {msg}")


def _check(code: int, where: str):
    if code != DME_OK:
        raise DmeError(code, where)


# ---------------------------------------------------------------- helpers
def _torch():
    import torch
    return torch


def to_device_cm(x, device="cuda"):
    """Logical 2-D matrix -> column-major device storage (row-major (cols, rows))."""
    torch = _torch()
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
    x = x.to(device=device, dtype=torch.float64)
    if x.dim() == 1:
        x = x[:, None]
    return x.t().contiguous()


def empty_cm(rows: int, cols: int, device="cuda"):
    torch = _torch()
    return torch.empty((cols, rows), dtype=torch.float64, device=device)


def zeros_cm(rows: int, cols: int, device="cuda"):
    torch = _torch()
    return torch.zeros((cols, rows), dtype=torch.float64, device=device)


def from_cm(storage):
    """Column-major storage tensor -> logical view (rows x cols)."""
    return storage.t()


def _ptr(t) -> int:
    return int(t.data_ptr()) if t is not None and t.numel() > 0 else 0


def _host_f(x) -> Optional[np.ndarray]:
    if x is None:
        return None
    return np.asfortranarray(np.asarray(x, dtype=np.float64))


@dataclass
class SolveOptions:
    T: float
    h: float
    tol: float = 1e-10
    scheme: str = "strang"
    split: str = "F12"
    precision: str = "fp64"
    quad_nodes: int = 7
    max_rank: int = 0
    action: str = "dense"

    def to_c(self) -> Opts:
        return Opts(self.T, self.h, self.tol, SCHEMES[self.scheme], SPLITS[self.split],
                    PRECISIONS[self.precision], self.quad_nodes, self.max_rank, ACTIONS[self.action])


class _HostProblem:
    """Keeps Fortran-ordered host copies alive for the duration of a call.
    A may be a dense matrix or a CSR triple (rowptr, colind, values), e.g.
    from scipy.sparse's (indptr, indices, data); M is the optional dense mass
    matrix."""

    def __init__(self, A, C, B=None, R=None, S=None, L0=None, D0=None, n=None, M=None):
        self.csr = None
        if n is None and isinstance(A, tuple):
            rp, ci, va = A
            self.csr = (np.ascontiguousarray(rp, dtype=np.int64), np.ascontiguousarray(ci, dtype=np.int64),
                        np.ascontiguousarray(va, dtype=np.float64))
            n = len(self.csr[0]) - 1
            self.A = None
        else:
            self.A = _host_f(A) if n is None else None
        self.M = _host_f(M)
        self.C = _host_f(C)
        self.B = _host_f(B)
        self.R = _host_f(R)
        self.S = _host_f(S)
        self.L0 = _host_f(L0)
        self.D0 = _host_f(D0)
        n = self.A.shape[0] if n is None else int(n)
        p = self.C.shape[0]
        m = 0 if self.B is None else self.B.shape[1]
        r0 = 0 if self.L0 is None else self.L0.shape[1]
        if r0 == 0:
            self.L0 = None
            self.D0 = None

        def ptr(a):
            return a.ctypes.data if a is not None and a.size else None

        csr = [ptr(a) for a in self.csr] if self.csr is not None else [None, None, None]
        if self.csr is not None and self.csr[2].size == 0:
            raise ValueError("CSR A without entries")
        self.c = Problem(n, m, p, r0, ptr(self.A), ptr(self.B), ptr(self.C), ptr(self.R),
                         ptr(self.S), ptr(self.L0), ptr(self.D0), ptr(self.M), *csr)


class Result:
    def __init__(self, handle):
        self._h = handle

    def info(self):
        """(n, r, steps, err_est) of the result (dme_result_info)."""
        n, r, steps, err = _i64(), _i64(), _i64(), _dbl()
        _check(_lib_result_info(self._h, ctypes.byref(n), ctypes.byref(r), ctypes.byref(steps),
                                ctypes.byref(err)), "dme_result_info")
        return int(n.value), int(r.value), int(steps.value), float(err.value)

    def fetch(self):
        n, r, steps = _i64(), _i64(), _i64()
        _check(_lib_result_info(self._h, ctypes.byref(n), ctypes.byref(r), ctypes.byref(steps),
                                None), "dme_result_info")
        L = np.zeros((n.value, r.value), order="F")
        D = np.zeros((r.value, r.value), order="F")
        _check(_lib_result_copy(self._h, L.ctypes.data if L.size else None,
                                D.ctypes.data if D.size else None), "dme_result_copy")
        return L, D, int(steps.value)

    def __del__(self):
        if getattr(self, "_h", None):
            _lib_result_free(self._h)
            self._h = None


class Context:
    """A library context on one HIP device, enqueueing on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = _p()
        _check(_lib_dme_create(ctypes.byref(h), device, ctypes.c_void_p(int(stream.cuda_stream))),
               "dme_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib_dme_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # ------------------------------------------------ step-level calls
    def expm(self, X, t: float):
        """e^{tX} of a device matrix; returns (E, m, s)."""
        Xs = to_device_cm(X)
        n = Xs.shape[0]
        Es = empty_cm(n, n)
        m, s = _int(), _int()
        _check(_lib_expm(self._h, n, _ptr(Xs), float(t), _ptr(Es), ctypes.byref(m), ctypes.byref(s)),
               "dme_expm")
        return from_cm(Es), int(m.value), int(s.value)

    def gemm(self, A, B, alpha=1.0, beta=0.0, C=None, transa="N", transb="N"):
        # the same array twice is passed as one buffer (A^T A takes the library's Gram path)
        As = to_device_cm(A)
        Bs = As if B is A else to_device_cm(B)
        ra, ca = As.shape[1], As.shape[0]
        rb, cb = Bs.shape[1], Bs.shape[0]
        M, K = (ca, ra) if transa == "T" else (ra, ca)
        K2, N = (cb, rb) if transb == "T" else (rb, cb)
        if K != K2:
            raise ValueError("inner dimensions differ")
        Cs = to_device_cm(C) if C is not None else zeros_cm(M, N)
        _check(_lib_gemm(self._h, transa.encode(), transb.encode(), M, N, K, float(alpha),
                         _ptr(As), max(1, ra), _ptr(Bs), max(1, rb), float(beta), _ptr(Cs), max(1, M)),
               "dme_gemm_f64")
        return from_cm(Cs)

    def gemm_mixed(self, E, X):
        """Y = E X with the split-BF16 product of the mixed-precision mode."""
        Es, Xs = to_device_cm(E), to_device_cm(X)
        n, r = Xs.shape[1], Xs.shape[0]
        if Es.shape != (n, n):
            raise ValueError("E must be n x n with n = rows of X")
        Ys = zeros_cm(n, r)
        _check(_lib_gemm_mixed(self._h, n, r, _ptr(Es), _ptr(Xs), max(1, n), _ptr(Ys), max(1, n)),
               "dme_gemm_mixed")
        return from_cm(Ys)

    def compress(self, W, Dhat, tol: float, max_rank: Optional[int] = None):
        Ws = to_device_cm(W)
        Ds = to_device_cm(Dhat)
        n, k = Ws.shape[1], Ws.shape[0]
        mr = k if max_rank is None else int(max_rank)
        Ls = zeros_cm(n, max(mr, 1))
        Dout = zeros_cm(max(mr, 1), max(mr, 1))
        r = _i64()
        _check(_lib_compress(self._h, n, k, _ptr(Ws), _ptr(Ds), float(tol), mr, _ptr(Ls), _ptr(Dout),
                             ctypes.byref(r)), "dme_compress")
        rr = int(r.value)
        L = from_cm(Ls)[:, :rr]
        D = from_cm(Dout)[:rr, :rr]
        return L, D

    def riccati(self, L, B, R, t: float, D):
        Ls, Bs, Rs, Ds = to_device_cm(L), to_device_cm(B), to_device_cm(R), to_device_cm(D)
        n, r = Ls.shape[1], Ls.shape[0]
        m = Bs.shape[0]
        _check(_lib_riccati(self._h, n, r, m, _ptr(Ls), _ptr(Bs), _ptr(Rs), float(t), _ptr(Ds)),
               "dme_riccati")
        return from_cm(Ds)

    def expmv_leja(self, A, t: float, X):
        """Y = e^{t A^T} X by the Leja-interpolation action; A is a dense
        matrix (copied to the device) or a host CSR triple (rowptr, colind,
        values).  Returns (Y, S, m)."""
        Xs = to_device_cm(X)
        n, c = Xs.shape[1], Xs.shape[0]
        Ys = empty_cm(n, c)
        S, m = _int(), _int()
        if isinstance(A, tuple):
            rp = np.ascontiguousarray(A[0], dtype=np.int64)
            ci = np.ascontiguousarray(A[1], dtype=np.int64)
            va = np.ascontiguousarray(A[2], dtype=np.float64)
            _check(_lib_expmv_leja(self._h, n, None, rp.ctypes.data, ci.ctypes.data, va.ctypes.data,
                                   float(t), c, _ptr(Xs), _ptr(Ys), ctypes.byref(S), ctypes.byref(m)),
                   "dme_expmv_leja")
        else:
            As = to_device_cm(A)
            _check(_lib_expmv_leja(self._h, n, _ptr(As), None, None, None, float(t), c, _ptr(Xs),
                                   _ptr(Ys), ctypes.byref(S), ctypes.byref(m)), "dme_expmv_leja")
        return from_cm(Ys), int(S.value), int(m.value)

    def riccati_noalloc(self, L, B, R, t: float, D):
        """dme_riccati_noalloc: the Riccati update with the library's static
        device scratch (no device allocation inside the call)."""
        Ls, Bs, Rs, Ds = to_device_cm(L), to_device_cm(B), to_device_cm(R), to_device_cm(D)
        n, r = Ls.shape[1], Ls.shape[0]
        m = Bs.shape[0]
        _check(_lib_riccati_noalloc(self._h, n, r, m, _ptr(Ls), _ptr(Bs), _ptr(Rs), float(t),
                                    _ptr(Ds)), "dme_riccati_noalloc")
        return from_cm(Ds)

    def syev(self, M, tol: float = 0.0, max_keep: Optional[int] = None):
        Ms = to_device_cm(M)
        k = Ms.shape[0]
        mk = k if max_keep is None else int(max_keep)
        torch = _torch()
        lam = torch.zeros(max(k, 1), dtype=torch.float64, device="cuda")
        Vs = zeros_cm(max(k, 1), max(mk, 1))
        keep = _i64()
        _check(_lib_syev(self._h, k, _ptr(Ms), float(tol), mk, _ptr(lam), _ptr(Vs), ctypes.byref(keep)),
               "dme_syev")
        kk = int(keep.value)
        return lam[:k], from_cm(Vs)[:k, :kk], kk

    def register_operator(self, A) -> int:
        """Copy the operator A (n x n) to the device once; returns its id."""
        Ah = _host_f(A)
        op = ctypes.c_uint64()
        _check(_lib_register(self._h, Ah.ctypes.data, Ah.shape[0], ctypes.byref(op)),
               "dme_register_operator")
        return int(op.value)

    def server(self, hbm_budget_bytes: int, max_slots: int = 16) -> "Server":
        return Server(self, hbm_budget_bytes, max_slots)

    # ------------------------------------------------ whole solves
    def solve(self, kind: str, opts: SolveOptions, A, C, B=None, R=None, S=None, L0=None, D0=None,
              err_est: bool = False, M=None):
        """(L, D, steps) of a whole solve; with err_est=True also the result's
        estimated distance to the FP64 computation.  A is dense or a CSR
        triple (rowptr, colind, values); M the optional mass matrix."""
        hp = _HostProblem(A, C, B, R, S, L0, D0, M=M)
        o = opts.to_c()
        out = _p()
        fn = _lib_dre_solve if kind == "dre" else _lib_dle_solve
        _check(fn(self._h, ctypes.byref(hp.c), ctypes.byref(o), ctypes.byref(out)),
               "dre_solve" if kind == "dre" else "dle_solve")
        res = Result(out)
        L, D, steps = res.fetch()
        return (L, D, steps, res.info()[3]) if err_est else (L, D, steps)

    def solver(self, kind: str, opts: SolveOptions, A, C, B=None, R=None, S=None, L0=None, D0=None,
               M=None):
        return Solver(self, kind, opts, A, C, B, R, S, L0, D0, M=M)


class Solver:
    """Stepwise solve: setup once, then advance with all data in HBM."""

    def __init__(self, ctx: Context, kind, opts, A, C, B=None, R=None, S=None, L0=None, D0=None,
                 M=None):
        self.ctx = ctx
        hp = _HostProblem(A, C, B, R, S, L0, D0, M=M)
        o = opts.to_c()
        h = _p()
        _check(_lib_solver_create(ctx._h, ctypes.byref(hp.c), ctypes.byref(o), 1 if kind == "dre" else 0,
                                  ctypes.byref(h)), "dme_solver_create")
        self._h = h
        self.n = int(hp.c.n)
        self.m = int(np.asarray(B).shape[1]) if B is not None else 0

    def step(self, nsteps: int = 1):
        _check(_lib_solver_step(self._h, int(nsteps)), "dme_solver_step")

    def state(self):
        st, tot, r = _i64(), _i64(), _i64()
        _check(_lib_solver_state(self._h, ctypes.byref(st), ctypes.byref(tot), ctypes.byref(r)),
               "dme_solver_state")
        return int(st.value), int(tot.value), int(r.value)

    def setup_info(self):
        e, q, rq = _dbl(), _dbl(), _i64()
        _check(_lib_solver_setup_info(self._h, ctypes.byref(e), ctypes.byref(q), ctypes.byref(rq)),
               "dme_solver_setup_info")
        return {"expm_ms": e.value, "quad_ms": q.value, "rank_quad": int(rq.value)}

    def gain(self):
        """Feedback gain K = R^-1 B^T L D L^T (m x n) at the current step."""
        m, n = self.m, self.n
        K = np.zeros((max(m, 1), n), order="F")
        _check(_lib_solver_gain(self._h, K.ctypes.data_as(_p), max(m, 1)), "dme_solver_gain")
        return K

    def profile(self, enable: bool = True, kernel_only: bool = False):
        """Phase timing on (every phase, or only the step product kernel) or off."""
        level = (2 if kernel_only else 1) if enable else 0
        _check(_lib_solver_profile(self._h, level), "dme_solver_profile")

    def profile_get(self, phase: str):
        c, ms, fl, by = _i64(), _dbl(), _dbl(), _dbl()
        _check(_lib_solver_profile_get(self._h, PHASES[phase], ctypes.byref(c), ctypes.byref(ms),
                                       ctypes.byref(fl), ctypes.byref(by)), "dme_solver_profile_get")
        return {"count": int(c.value), "ms": ms.value, "flops": fl.value, "bytes": by.value}

    def result(self, err_est: bool = False):
        out = _p()
        _check(_lib_solver_result(self._h, ctypes.byref(out)), "dme_solver_result")
        res = Result(out)
        L, D, steps = res.fetch()
        return (L, D, steps, res.info()[3]) if err_est else (L, D, steps)

    def close(self):
        if getattr(self, "_h", None):
            _lib_solver_free(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Server:
    """Continuous-batching request server on a context (dme_server_*)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int = 16):
        self.ctx = ctx
        h = _p()
        _check(_lib_server_start(ctx._h, int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)),
               "dme_server_start")
        self._h = h
        self._keep = {}

    def register_operator(self, A) -> int:
        return self.ctx.register_operator(A)

    def warm(self, op_id: int, t: float, precision: str = "mixed", quad_nodes: int = 7):
        _check(_lib_server_warm(self._h, int(op_id), float(t), PRECISIONS[precision], int(quad_nodes)),
               "dme_server_warm")

    def submit(self, op_id: int, kind: str, opts: SolveOptions, C, n: int, B=None, R=None, S=None,
               L0=None, D0=None) -> int:
        hp = _HostProblem(np.zeros((n, 0)), C, B, R, S, L0, D0, n=n)
        o = opts.to_c()
        t = ctypes.c_uint64()
        _check(_lib_submit(self._h, int(op_id), ctypes.byref(hp.c), ctypes.byref(o),
                           1 if kind == "dre" else 0, ctypes.byref(t)), "dme_submit")
        return int(t.value)

    def poll(self, ticket: int):
        """None while in flight, else (L, D, steps, info dict); raises on failure."""
        out = _p()
        code = _lib_poll(self._h, int(ticket), ctypes.byref(out))
        if code == DME_EAGAIN:
            return None
        _check(code, "dme_poll")
        res = Result(out)
        prec, fb, lat, qs = _int(), _int(), _dbl(), _dbl()
        _check(_lib_result_serving(out, ctypes.byref(prec), ctypes.byref(fb), ctypes.byref(lat),
                                   ctypes.byref(qs)), "dme_result_serving")
        L, D, steps = res.fetch()
        info = {"precision": "mixed" if prec.value == DME_MIXED else "fp64", "fell_back": bool(fb.value),
                "latency_s": lat.value, "queue_s": qs.value, "err_est": res.info()[3]}
        return L, D, steps, info

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib_server_stats(self._h, ctypes.byref(st)), "dme_server_stats_get")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def stop(self):
        if getattr(self, "_h", None):
            _check(_lib_server_stop(self._h), "dme_server_stop")
            self._h = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass
