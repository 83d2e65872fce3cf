"""ctypes binding of libsgpc.so (the C interface declared in include/sg.h).

Argument marshalling only: every computation runs in the HIP library. Device
blocks are torch tensors of shape (P, n), float64, contiguous, on the CUDA
(HIP) device -- i.e. n x P column-major blocks with leading dimension n. The
library allocates no device memory; the workspace is a torch uint8 tensor.
If the library is not built this module raises on import.
"""

from __future__ import annotations

import ctypes
import os
import sys
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SGPC_LIBRARY") or os.path.join(_HERE, "libsgpc.so")

SG_OK, SG_EINVAL, SG_EDEVICE, SG_ENOMEM, SG_NOT_CONVERGED, SG_BREAKDOWN = 0, -1, -2, -3, 1, 2
SG_PC_NONE, SG_PC_MEAN, SG_PC_HSC, SG_PC_BGS = 0, 1, 2, 3
_PC = {"none": SG_PC_NONE, "mean": SG_PC_MEAN, "hsc": SG_PC_HSC, "bgs": SG_PC_BGS}
SG_FAMILY_HERMITE, SG_FAMILY_LEGENDRE = 0, 1


class SgProblem(ctypes.Structure):
    _fields_ = [("n_e", ctypes.c_int32), ("M", ctypes.c_int32), ("p", ctypes.c_int32),
                ("family", ctypes.c_int32), ("theta0", ctypes.c_double), ("sigma", ctypes.c_double),
                ("s", ctypes.POINTER(ctypes.c_double)), ("phi", ctypes.POINTER(ctypes.c_double))]


class SgOpts(ctypes.Structure):
    _fields_ = [("inner_precision", ctypes.c_int32), ("cheb_degree", ctypes.c_int32),
                ("inner_maxit", ctypes.c_int32), ("precond", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("inner_rtol", ctypes.c_double), ("use_graph", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class SgStats(ctypes.Structure):
    _fields_ = [("outer_it", ctypes.c_int32), ("status", ctypes.c_int32),
                ("inner_it_total", ctypes.c_int64), ("n_blockmv", ctypes.c_int64),
                ("n_blocksolve", ctypes.c_int64), ("inner_it_max", ctypes.c_int32 * 16),
                ("relres", ctypes.c_double), ("true_relres", ctypes.c_double),
                ("kappa_est", ctypes.c_double), ("ms", ctypes.c_double),
                ("ms_precond", ctypes.c_double), ("ms_matvec", ctypes.c_double),
                ("ms_inner", ctypes.c_double), ("inner_bytes", ctypes.c_double),
                ("inner_launches", ctypes.c_int64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["inner_it_max"] = list(self.inner_it_max)
        return d


class SgTuneReport(ctypes.Structure):
    _fields_ = [("mv_variant", ctypes.c_int32), ("mv_param", ctypes.c_int32), ("pcg_tile", ctypes.c_int32),
                ("pcg_max_blocks", ctypes.c_int32), ("mv_ms", ctypes.c_double), ("pcg_ms", ctypes.c_double),
                ("candidates", ctypes.c_int32), ("pcg_rows", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P, VP, I32, I64, D = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "sg_workspace_bytes": [P(SgProblem), P(SgOpts), P(ctypes.c_size_t)],
        "sg_setup": [P(SgProblem), P(SgOpts), VP, ctypes.c_size_t, VP, P(VP)],
        "sg_sizes": [VP, P(I64), P(I32), P(I32), P(I32)],
        "sg_set_opts": [VP, P(SgOpts)],
        "sg_matvec": [VP, VP, VP],
        "sg_apply_hsc": [VP, VP, VP],
        "sg_apply_mean": [VP, VP, VP],
        "sg_apply_bgs": [VP, VP, VP],
        "sg_inner_solve": [VP, VP, VP, I32, P(I32)],
        "sg_inner_solve_static": [VP, VP, VP, I32, P(I32)],
        "sg_coupling": [VP, I32, I32, VP, VP],
        "sg_solve": [VP, VP, VP, D, I32, I32, P(SgStats)],
        "sg_solve_reduced": [VP, VP, VP, D, I32, D, P(SgStats)],
        "sg_qoi": [VP, VP, VP, VP, P(D)],
        "sg_adjoint_grad": [VP, VP, VP, VP, D, I32, P(D), P(D), VP, P(SgStats)],
        "sg_autotune": [VP, I32, P(SgTuneReport)],
        "sg_batch_workspace_bytes": [I32, P(SgProblem), P(SgOpts), P(ctypes.c_size_t)],
        "sg_batch_setup": [I32, P(SgProblem), P(SgOpts), VP, ctypes.c_size_t, VP, P(VP)],
        "sg_batch_sizes": [VP, I32, P(I64), P(I32)],
        "sg_batch_solve": [VP, P(VP), P(VP), D, I32, I32, P(SgStats), P(D)],
        "sg_batch_autotune": [VP, I32, P(SgTuneReport)],
        "sg_logn_workspace_bytes": [P(SgProblem), P(ctypes.c_size_t)],
        "sg_logn_setup": [P(SgProblem), VP, ctypes.c_size_t, VP, P(VP)],
        "sg_logn_sizes": [VP, P(I64), P(I32), P(I32)],
        "sg_logn_matvec": [VP, VP, VP],
        "sg_logn_solve": [VP, I32, VP, VP, D, I32, D, I32, P(I32), P(I64), P(D), P(D)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.sg_destroy.argtypes = [VP]
    lib.sg_destroy.restype = None
    lib.sg_batch_destroy.argtypes = [VP]
    lib.sg_batch_destroy.restype = None
    lib.sg_logn_destroy.argtypes = [VP]
    lib.sg_logn_destroy.restype = None
    lib.sg_last_error.argtypes = []
    lib.sg_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


class SGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _check(rc, allow_positive=False):
    if rc < 0 or (rc > 0 and not allow_positive):
        raise SGError(rc, lib.sg_last_error().decode())
    return rc


def last_error() -> str:
    return lib.sg_last_error().decode()


def _release(obj, _finalizing=sys.is_finalizing):
    """Finaliser of the handle classes. Callers close handles explicitly; a
    handle still open when the interpreter shuts down is left to the process
    exit, so that no HIP call runs after the runtime's own teardown began.
    (sys.is_finalizing is bound at definition: module globals may already be
    cleared when a finaliser runs at shutdown.)"""
    if _finalizing():
        return
    try:
        obj.close()
    except Exception:
        pass


@dataclass
class Options:
    inner_precision: int = 64
    cheb_degree: int = 4
    inner_maxit: int = 1000
    precond: str = "hsc"
    tile: int = 0
    inner_rtol: float = 1e-4
    warm_start: bool = False
    use_graph: bool = False

    def to_c(self) -> SgOpts:
        return SgOpts(self.inner_precision, self.cheb_degree, self.inner_maxit, _PC[self.precond],
                      self.tile, int(bool(self.warm_start)), float(self.inner_rtol), int(bool(self.use_graph)), 0)


def _dptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def make_c_problem(problem):
    """(SgProblem, keep-alive arrays) from any object with n_e, M, p, theta0, sigma, s, phi."""
    s = np.ascontiguousarray(np.asarray(problem.s, dtype=np.float64).reshape(-1))
    phi = np.ascontiguousarray(np.asarray(problem.phi, dtype=np.float64).reshape(-1))
    dp = ctypes.POINTER(ctypes.c_double)
    family = {"hermite": SG_FAMILY_HERMITE, "legendre": SG_FAMILY_LEGENDRE}[getattr(problem, "family", "hermite")]
    cp = SgProblem(int(problem.n_e), int(problem.M), int(problem.p), family, float(problem.theta0),
                   float(problem.sigma), s.ctypes.data_as(dp) if s.size else None,
                   phi.ctypes.data_as(dp) if phi.size else None)
    return cp, (s, phi)


def workspace_bytes(problem, opts: Options) -> int:
    cp, keep = make_c_problem(problem)
    co = opts.to_c()
    nb = ctypes.c_size_t(0)
    _check(lib.sg_workspace_bytes(ctypes.byref(cp), ctypes.byref(co), ctypes.byref(nb)))
    return int(nb.value)


class SGSolver:
    """A configured SG problem on one device (a handle plus its workspace)."""

    def __init__(self, problem, opts: Options = None, device="cuda", stream=None):
        self.opts = opts or Options()
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        cp, keep = make_c_problem(problem)
        co = self.opts.to_c()
        nb = ctypes.c_size_t(0)
        _check(lib.sg_workspace_bytes(ctypes.byref(cp), ctypes.byref(co), ctypes.byref(nb)))
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        if stream is None:
            # a captured graph needs a stream of its own
            stream = torch.cuda.Stream(device=self.device) if self.opts.use_graph else \
                torch.cuda.current_stream(self.device)
        self.stream = stream
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        h = ctypes.c_void_p()
        _check(lib.sg_setup(ctypes.byref(cp), ctypes.byref(co), ctypes.c_void_p(self.workspace.data_ptr()),
                            ctypes.c_size_t(int(nb.value)), ctypes.c_void_p(self.stream.cuda_stream),
                            ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int64()
        P = ctypes.c_int32()
        self.M, self.p = int(problem.M), int(problem.p)
        off = (ctypes.c_int32 * (self.p + 2))()
        alpha = (ctypes.c_int32 * max(1, 0))()
        _check(lib.sg_sizes(h, ctypes.byref(n), ctypes.byref(P), off, None))
        self.n, self.P = int(n.value), int(P.value)
        self.level_off = list(off)
        al = (ctypes.c_int32 * max(1, self.P * self.M))()
        _check(lib.sg_sizes(h, None, None, None, al))
        self.alpha = np.array(al[: self.P * self.M], dtype=np.int64).reshape(self.P, self.M)
        del alpha

    # -- helpers ---------------------------------------------------------
    def _block(self, t: torch.Tensor, ncols=None) -> torch.Tensor:
        ncols = self.P if ncols is None else ncols
        if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous() or \
                tuple(t.shape) != (ncols, self.n):
            raise ValueError(f"expected a contiguous float64 ({ncols}, {self.n}) tensor on {self.device}")
        return t

    def _vec(self, t: torch.Tensor) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != self.device or \
                not t.is_contiguous() or tuple(t.shape) != (self.n,):
            raise ValueError(f"expected a contiguous float64 ({self.n},) tensor on {self.device}")
        return t

    def empty(self, ncols=None) -> torch.Tensor:
        return torch.empty((self.P if ncols is None else ncols, self.n), dtype=torch.float64, device=self.device)

    def set_opts(self, opts: Options):
        co = opts.to_c()
        _check(lib.sg_set_opts(self.handle, ctypes.byref(co)))
        self.opts = opts

    # -- entry points (same names as the C interface) ----------------------
    def sg_matvec(self, U, Y=None):
        Y = self.empty() if Y is None else Y
        _check(lib.sg_matvec(self.handle, _dptr(self._block(U)), _dptr(self._block(Y))))
        return Y

    def sg_apply_hsc(self, R, Z=None):
        Z = self.empty() if Z is None else Z
        _check(lib.sg_apply_hsc(self.handle, _dptr(self._block(R)), _dptr(self._block(Z))))
        return Z

    def sg_apply_bgs(self, R, Z=None):
        Z = self.empty() if Z is None else Z
        _check(lib.sg_apply_bgs(self.handle, _dptr(self._block(R)), _dptr(self._block(Z))))
        return Z

    def sg_apply_mean(self, R, Z=None):
        Z = self.empty() if Z is None else Z
        _check(lib.sg_apply_mean(self.handle, _dptr(self._block(R)), _dptr(self._block(Z))))
        return Z

    def sg_inner_solve(self, B, X=None):
        ncols = B.shape[0]
        X = self.empty(ncols) if X is None else X
        its = (ctypes.c_int32 * max(1, ncols))()
        _check(lib.sg_inner_solve(self.handle, _dptr(self._block(B, ncols)), _dptr(self._block(X, ncols)),
                                  ncols, its))
        return X, np.array(its[:ncols])

    def sg_inner_solve_static(self, B, X=None):
        """sg_inner_solve with the solver's scratch in the library's static
        device array (no workspace use beyond the handle's tables)."""
        ncols = B.shape[0]
        X = self.empty(ncols) if X is None else X
        its = (ctypes.c_int32 * max(1, ncols))()
        _check(lib.sg_inner_solve_static(self.handle, _dptr(self._block(B, ncols)), _dptr(self._block(X, ncols)),
                                         ncols, its))
        return X, np.array(its[:ncols])

    def sg_coupling(self, level, direction, R, V):
        _check(lib.sg_coupling(self.handle, int(level), int(direction), _dptr(self._block(R)),
                               _dptr(self._block(V))))
        return R

    def sg_solve(self, F, U=None, rtol=1e-8, maxit=200, use_x0=False):
        U = self.empty() if U is None else U
        st = SgStats()
        caller = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(caller)  # F and U come from the caller's stream
        rc = _check(lib.sg_solve(self.handle, _dptr(self._block(F)), _dptr(self._block(U)), float(rtol),
                                 int(maxit), int(bool(use_x0)), ctypes.byref(st)), allow_positive=True)
        caller.wait_stream(self.stream)
        d = st.as_dict()
        d["rc"] = rc
        return U, d

    def sg_solve_reduced(self, F, U=None, rtol=1e-8, maxit=200, op_rtol=1e-12):
        U = self.empty() if U is None else U
        st = SgStats()
        rc = _check(lib.sg_solve_reduced(self.handle, _dptr(self._block(F)), _dptr(self._block(U)), float(rtol),
                                         int(maxit), float(op_rtol), ctypes.byref(st)), allow_positive=True)
        d = st.as_dict()
        d["rc"] = rc
        return U, d

    def sg_qoi(self, U, w_mean, w_var):
        Q = ctypes.c_double()
        _check(lib.sg_qoi(self.handle, _dptr(self._block(U)), _dptr(self._vec(w_mean)), _dptr(self._vec(w_var)),
                          ctypes.byref(Q)))
        return Q.value

    def sg_adjoint_grad(self, U, w_mean, w_var, rtol=1e-8, maxit=200, Lambda=None):
        Q = ctypes.c_double()
        grad = (ctypes.c_double * (1 + self.M))()
        st = SgStats()
        lam_ptr = _dptr(self._block(Lambda)) if Lambda is not None else None
        rc = _check(lib.sg_adjoint_grad(self.handle, _dptr(self._block(U)), _dptr(self._vec(w_mean)),
                                        _dptr(self._vec(w_var)),
                                        float(rtol), int(maxit), ctypes.byref(Q), grad, lam_ptr,
                                        ctypes.byref(st)), allow_positive=True)
        d = st.as_dict()
        d["rc"] = rc
        return Q.value, np.array(grad[:]), d

    def sg_autotune(self, flags=3):
        rep = SgTuneReport()
        _check(lib.sg_autotune(self.handle, int(flags), ctypes.byref(rep)))
        return rep.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            lib.sg_destroy(self.handle)
            self.handle = None

    def __del__(self, _release=_release):
        _release(self)


class SGBatch:
    """Many independent SG problems solved together (a batch handle plus its workspace).

    All problems share the options; ``precond`` must be "hsc", "bgs" or "mean".
    """

    def __init__(self, problems, opts: Options = None, device="cuda", stream=None):
        self.opts = opts or Options(inner_precision=32)
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.count = len(problems)
        cps, self._keep = [], []
        for pr in problems:
            cp, keep = make_c_problem(pr)
            cps.append(cp)
            self._keep.append(keep)
        self._cps = (SgProblem * self.count)(*cps)
        co = self.opts.to_c()
        nb = ctypes.c_size_t(0)
        _check(lib.sg_batch_workspace_bytes(self.count, self._cps, ctypes.byref(co), ctypes.byref(nb)))
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        # a graph is captured on the batch's stream, which therefore cannot be the default stream
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        h = ctypes.c_void_p()
        _check(lib.sg_batch_setup(self.count, self._cps, ctypes.byref(co),
                                  ctypes.c_void_p(self.workspace.data_ptr()), ctypes.c_size_t(int(nb.value)),
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.sizes = []
        for i in range(self.count):
            n, P = ctypes.c_int64(), ctypes.c_int32()
            _check(lib.sg_batch_sizes(h, i, ctypes.byref(n), ctypes.byref(P)))
            self.sizes.append((int(n.value), int(P.value)))

    def empty(self):
        return [torch.empty((P, n), dtype=torch.float64, device=self.device) for n, P in self.sizes]

    def sg_batch_solve(self, F, U=None, rtol=1e-8, maxit=200, use_graph=True):
        U = self.empty() if U is None else U
        if len(F) != self.count or len(U) != self.count:
            raise ValueError(f"expected {self.count} right-hand sides and solutions")
        for (n, P), f, u in zip(self.sizes, F, U):
            for t in (f, u):
                if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous() or \
                        tuple(t.shape) != (P, n):
                    raise ValueError(f"expected contiguous float64 ({P}, {n}) tensors on {self.device}")
        fp = (ctypes.c_void_p * self.count)(*[f.data_ptr() for f in F])
        up = (ctypes.c_void_p * self.count)(*[u.data_ptr() for u in U])
        st = (SgStats * self.count)()
        ms = ctypes.c_double()
        caller = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(caller)  # F and U were produced on the caller's stream
        rc = _check(lib.sg_batch_solve(self.handle, fp, up, float(rtol), int(maxit), int(bool(use_graph)), st,
                                       ctypes.byref(ms)), allow_positive=True)
        caller.wait_stream(self.stream)
        stats = [s.as_dict() for s in st]
        return U, stats, {"rc": rc, "ms": ms.value}

    def sg_batch_autotune(self, flags=3):
        rep = SgTuneReport()
        _check(lib.sg_batch_autotune(self.handle, int(flags), ctypes.byref(rep)))
        return rep.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            lib.sg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self, _release=_release):
        _release(self)


class LognormalOperator:
    """The lognormal-coefficient SG operator (sg_logn_*): ``mean`` and ``cov``
    of the coefficient, KL data of the Gaussian field from ``problem``."""

    def __init__(self, problem, mean: float, cov: float, device="cuda"):
        dev = torch.device(device)
        self.device = dev if dev.index is not None else torch.device("cuda", torch.cuda.current_device())
        cp, keep = make_c_problem(problem)
        cp.theta0 = float(mean)
        cp.sigma = float(cov)
        nb = ctypes.c_size_t(0)
        _check(lib.sg_logn_workspace_bytes(ctypes.byref(cp), ctypes.byref(nb)))
        self.workspace = torch.empty(max(1, int(nb.value)), dtype=torch.uint8, device=self.device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        h = ctypes.c_void_p()
        _check(lib.sg_logn_setup(ctypes.byref(cp), _dptr(self.workspace), int(nb.value), ctypes.c_void_p(stream),
                                 ctypes.byref(h)))
        self.handle = h
        n, P, nb_ = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.sg_logn_sizes(self.handle, ctypes.byref(n), ctypes.byref(P), ctypes.byref(nb_)))
        self.n, self.P, self.nblocks = int(n.value), int(P.value), int(nb_.value)

    def _block(self, t: torch.Tensor) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous() or \
                tuple(t.shape) != (self.P, self.n) or t.device != self.device:
            raise ValueError(f"expected a contiguous float64 ({self.P}, {self.n}) tensor on {self.device}")
        return t

    def matvec(self, U: torch.Tensor, Y: torch.Tensor = None) -> torch.Tensor:
        Y = torch.empty_like(self._block(U)) if Y is None else Y
        _check(lib.sg_logn_matvec(self.handle, _dptr(self._block(U)), _dptr(self._block(Y))))
        return Y

    def solve(self, F: torch.Tensor, U: torch.Tensor = None, rtol=1e-8, maxit=500, inner_rtol=1e-12,
              inner_maxit=5000, precond="hsc"):
        """A U = F by flexible CG; precond "hsc" (Algorithm 1 over the full level
        blocks), "bgs" or "mean"."""
        pc = {"hsc": SG_PC_HSC, "bgs": SG_PC_BGS, "mean": SG_PC_MEAN}[precond]
        U = torch.empty_like(self._block(F)) if U is None else U
        it, iin, rel, kap = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        rc = _check(lib.sg_logn_solve(self.handle, pc, _dptr(self._block(F)), _dptr(self._block(U)), float(rtol),
                                      int(maxit), float(inner_rtol),
                                      int(inner_maxit), ctypes.byref(it), ctypes.byref(iin), ctypes.byref(rel),
                                      ctypes.byref(kap)), allow_positive=True)
        return U, {"rc": rc, "outer_it": int(it.value), "inner_it": int(iin.value), "relres": float(rel.value),
                   "kappa_est": float(kap.value)}

    def close(self):
        if getattr(self, "handle", None):
            lib.sg_logn_destroy(self.handle)
            self.handle = None

    def __del__(self, _release=_release):
        _release(self)


def to_device_block(A: np.ndarray, device="cuda") -> torch.Tensor:
    """(P, n) numpy array -> contiguous float64 device tensor."""
    return torch.from_numpy(np.ascontiguousarray(A, dtype=np.float64)).to(device)


def to_device_vec(v: np.ndarray, device="cuda") -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(device)
