"""ctypes binding of the PASD C ABI (include/pasd.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Tensors are exchanged as device pointers of torch CUDA tensors (PyTorch
provides the device memory and the stream) or as host numpy arrays.  The
binding raises if the built library is missing; there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpasd.so")

MAX_ORDER = 8
MAX_RANK = 64

OK = 0
NOT_CONVERGED = 1
PRECISION_FLOOR = 2
ERR_INVALID_ARG = -1
ERR_UNSUPPORTED = -2
ERR_OOM = -3
ERR_HIP = -4
ERR_NUMERIC = -5
ERR_STATE = -6

FP64, FP32, BF16_GEMM = 0, 1, 2
FLAG_NO_GRAPH = 1
FLAG_TIEBREAK_KEEP = 2
FLAG_NO_FLOOR_STOP = 4
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16_GEMM}

Q_E, Q_Y, Q_Z, Q_X, Q_U, Q_P, Q_UF, Q_SCALARS, Q_D, Q_WEV, Q_FAC = range(11)

# enum pasd_kernel, in launch order
KERNELS = ("gemm_m", "reduce_m", "qr", "gemm_p", "gram", "eig", "fused", "control")


class Config(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int),
        ("dims", ctypes.c_int64 * MAX_ORDER),
        ("ranks", ctypes.c_int64 * MAX_ORDER),
        ("lambda_", ctypes.c_double * MAX_ORDER),
        ("alpha", ctypes.c_double * MAX_ORDER),
        ("mu0", ctypes.c_double),
        ("mu_max", ctypes.c_double),
        ("rho", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("flags", ctypes.c_int),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("done", ctypes.c_int),
        ("mu", ctypes.c_double),
        ("residual", ctypes.c_double * MAX_ORDER),
        ("rank", ctypes.c_int * MAX_ORDER),
        ("bytes_resident", ctypes.c_size_t),
        ("eig_sweeps", ctypes.c_int * MAX_ORDER),
        ("tol_effective", ctypes.c_double),
        ("merged_modes", ctypes.c_int),
        ("fused_blocks", ctypes.c_int),
        ("gemm_p_pair", ctypes.c_int),
    ]


class PasdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"PASD error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libpasd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; run paper_1712_09999_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        sig = {
            "pasd_config_init": (ctypes.c_int, [P(Config)]),
            "pasd_validate": (ctypes.c_int, [P(Config)]),
            "pasd_footprint": (ctypes.c_int, [P(Config), P(ctypes.c_size_t)]),
            "pasd_create": (ctypes.c_int, [P(Config), vp, ctypes.c_int, P(vp)]),
            "pasd_reset": (ctypes.c_int, [vp]),
            "pasd_step": (ctypes.c_int, [vp, ctypes.c_int]),
            "pasd_solve": (ctypes.c_int, [vp, P(Info)]),
            "pasd_query": (ctypes.c_int, [vp, P(Info)]),
            "pasd_get_result": (ctypes.c_int, [vp, vp, vp, ctypes.c_int]),
            "pasd_export": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int]),
            "pasd_import": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int]),
            "pasd_step_batch": (ctypes.c_int, [P(vp), ctypes.c_int, ctypes.c_int]),
            "pasd_profile": (ctypes.c_int, [vp, ctypes.c_int, P(ctypes.c_double),
                                            P(ctypes.c_int)]),
            "pasd_query_batch": (ctypes.c_int, [P(vp), ctypes.c_int, P(Info)]),
            "pasd_batch_create": (ctypes.c_int, [P(vp), ctypes.c_int, ctypes.c_int, P(vp)]),
            "pasd_batch_step": (ctypes.c_int, [vp]),
            "pasd_batch_destroy": (None, [vp]),
            "pasd_solve_static": (ctypes.c_int, [P(Config), vp, vp, vp, P(Info)]),
            "pasd_static_scratch_bytes": (ctypes.c_size_t, []),
            "pasd_destroy": (None, [vp]),
            "pasd_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().pasd_last_error().decode()


def _check(code: int, allow=(OK,)) -> int:
    if code not in allow:
        raise PasdError(code, last_error())
    return code


def make_config(dims: Sequence[int], ranks: Sequence[int], lam: Optional[Sequence[float]] = None,
                alpha: Optional[Sequence[float]] = None, mu0: float = 1e-4, mu_max: float = 1e10,
                rho: float = 1.1, tol: float = 1e-5, max_iter: int = 1000,
                precision="fp64", device: int = -1, stream: int = 0,
                graphs: bool = True, tiebreak: str = "pre", floor_stop: bool = True) -> Config:
    c = Config()
    lib().pasd_config_init(ctypes.byref(c))
    c.order = len(dims)
    for n, d in enumerate(dims):
        c.dims[n] = int(d)
    for n, r in enumerate(ranks):
        c.ranks[n] = int(r)
    if lam is not None:
        for n, v in enumerate(lam):
            c.lambda_[n] = float(v)
    if alpha is not None:
        for n, v in enumerate(alpha):
            c.alpha[n] = float(v)
    c.mu0, c.mu_max, c.rho, c.tol = float(mu0), float(mu_max), float(rho), float(tol)
    c.max_iter = int(max_iter)
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.device = int(device)
    c.stream = int(stream) if stream else None
    if tiebreak not in ("pre", "keep"):
        raise ValueError("tiebreak must be 'pre' or 'keep'")
    c.flags = ((0 if graphs else FLAG_NO_GRAPH) | (FLAG_TIEBREAK_KEEP if tiebreak == "keep" else 0)
               | (0 if floor_stop else FLAG_NO_FLOOR_STOP))
    return c


def validate(cfg: Config) -> int:
    return lib().pasd_validate(ctypes.byref(cfg))


def footprint(cfg: Config) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().pasd_footprint(ctypes.byref(cfg), ctypes.byref(b)))
    return int(b.value)


def _state_dtype(precision: int):
    return np.float64 if precision == FP64 else np.float32


class Solver:
    """One PASD solve resident on the GPU (wraps a pasd_ctx)."""

    def __init__(self, T, ranks: Sequence[int], *, lam=None, alpha=None, mu0: float = 1e-4,
                 mu_max: float = 1e10, rho: float = 1.1, tol: float = 1e-5, max_iter: int = 1000,
                 precision="fp64", device: Optional[int] = None, stream: int = 0,
                 graphs: bool = True, tiebreak: str = "pre", floor_stop: bool = True):
        import torch
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        sdt = torch.float64 if self.precision == FP64 else torch.float32
        if isinstance(T, np.ndarray):
            T = torch.from_numpy(np.ascontiguousarray(T))
        if not T.is_cuda:
            T = T.to("cuda" if device is None else f"cuda:{device}")
        T = T.to(sdt).contiguous()
        self.device = T.device.index if device is None else int(device)
        self.dims = tuple(int(d) for d in T.shape)
        self.ranks = tuple(int(r) for r in ranks)
        self.numel = int(T.numel())
        self.torch_dtype = sdt
        self.np_dtype = _state_dtype(self.precision)
        self.cfg = make_config(self.dims, ranks, lam, alpha, mu0, mu_max, rho, tol, max_iter,
                               self.precision, self.device, stream, graphs, tiebreak, floor_stop)
        h = ctypes.c_void_p()
        torch.cuda.synchronize(T.device)
        _check(lib().pasd_create(ctypes.byref(self.cfg), ctypes.c_void_p(T.data_ptr()), 1,
                                 ctypes.byref(h)))
        self._h = h

    # -- lifecycle ---------------------------------------------------------
    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise PasdError(ERR_STATE, "solver destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pasd_destroy(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- iteration ---------------------------------------------------------
    def reset(self):
        _check(lib().pasd_reset(self.handle))

    def step(self, n_iters: int = 1):
        _check(lib().pasd_step(self.handle, int(n_iters)))

    def solve(self) -> Info:
        info = Info()
        code = lib().pasd_solve(self.handle, ctypes.byref(info))
        _check(code, allow=(OK, NOT_CONVERGED, PRECISION_FLOOR))
        return info

    def profile(self, n_iters: int):
        """Run n_iters iterations with HIP events around every kernel launch;
        returns {kernel name: (total ms, launches)}."""
        ms = (ctypes.c_double * len(KERNELS))()
        cnt = (ctypes.c_int * len(KERNELS))()
        _check(lib().pasd_profile(self.handle, int(n_iters), ms, cnt))
        return {name: (ms[i], cnt[i]) for i, name in enumerate(KERNELS)}

    def query(self) -> Info:
        info = Info()
        _check(lib().pasd_query(self.handle, ctypes.byref(info)))
        return info

    # -- results -----------------------------------------------------------
    def result(self):
        """(X, E) as torch CUDA tensors of the state dtype."""
        import torch
        X = torch.empty(self.dims, dtype=self.torch_dtype, device=f"cuda:{self.device}")
        E = torch.empty_like(X)
        _check(lib().pasd_get_result(self.handle, ctypes.c_void_p(X.data_ptr()),
                                     ctypes.c_void_p(E.data_ptr()), 1))
        return X, E

    def export(self, quantity: int, index: int = 0) -> np.ndarray:
        """Copy one quantity to a host numpy array (see enum pasd_quantity)."""
        I = self.dims[index]
        J = self.numel // I
        R = self.ranks[index]
        shape, dt = {
            Q_E: (self.dims, self.np_dtype), Q_Y: (self.dims, self.np_dtype),
            Q_Z: (self.dims, self.np_dtype), Q_X: (self.dims, self.np_dtype),
            Q_U: ((I, R), np.float64), Q_P: ((R, J), self.np_dtype),
            Q_UF: ((I, R), np.float64), Q_SCALARS: ((2,), np.float64),
            Q_D: (self.dims, self.np_dtype), Q_WEV: ((R, R), np.float64),
            Q_FAC: ((R,), np.float64),
        }[quantity]
        out = np.empty(shape, dtype=dt)
        _check(lib().pasd_export(self.handle, quantity, index, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def import_(self, quantity: int, index: int, value: np.ndarray):
        dt = np.float64 if quantity in (Q_U, Q_SCALARS, Q_WEV, Q_FAC) else self.np_dtype
        v = np.ascontiguousarray(value, dtype=dt)
        _check(lib().pasd_import(self.handle, quantity, index, v.ctypes.data_as(ctypes.c_void_p), 0))

    def checkpoint(self) -> dict:
        st = {"D": self.export(Q_D), "scalars": self.export(Q_SCALARS)}
        for n in range(len(self.dims)):
            st[f"Y{n}"] = self.export(Q_Y, n)
            st[f"U{n}"] = self.export(Q_U, n)
            st[f"P{n}"] = self.export(Q_P, n)
            st[f"W{n}"] = self.export(Q_WEV, n)
            st[f"F{n}"] = self.export(Q_FAC, n)
        return st

    def restore(self, st: dict):
        self.import_(Q_D, 0, st["D"])
        for n in range(len(self.dims)):
            self.import_(Q_Y, n, st[f"Y{n}"])
            self.import_(Q_U, n, st[f"U{n}"])
            self.import_(Q_P, n, st[f"P{n}"])
            self.import_(Q_WEV, n, st[f"W{n}"])
            if f"F{n}" in st:
                self.import_(Q_FAC, n, st[f"F{n}"])
        self.import_(Q_SCALARS, 0, st["scalars"])


def solve_static(T, ranks: Sequence[int], X=None, E=None, **kw):
    """One solve through pasd_solve_static (no device allocation inside the
    library): T, X and E are torch CUDA tensors of the state dtype, X and E
    preallocated by the caller (either may be None).  Keyword arguments are
    those of make_config.  Returns (status, Info)."""
    import torch
    cfg = make_config(tuple(int(d) for d in T.shape), ranks, device=T.device.index, **kw)
    sdt = torch.float64 if cfg.precision == FP64 else torch.float32
    for t in (T, X, E):
        if t is not None and (t.dtype != sdt or not t.is_contiguous() or not t.is_cuda
                              or tuple(t.shape) != tuple(T.shape)):
            raise ValueError("T, X and E must be contiguous CUDA tensors of the state dtype and shape")
    info = Info()
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
    code = lib().pasd_solve_static(ctypes.byref(cfg), ptr(T), ptr(X), ptr(E), ctypes.byref(info))
    _check(code, allow=(OK, NOT_CONVERGED, PRECISION_FLOOR))
    return code, info


def static_scratch_bytes() -> int:
    return int(lib().pasd_static_scratch_bytes())


def step_batch(solvers: List[Solver], n_iters: int):
    """n_iters iterations of every solver as grouped launches (pasd_step_batch)."""
    arr = (ctypes.c_void_p * len(solvers))(*[s.handle.value for s in solvers])
    _check(lib().pasd_step_batch(arr, len(solvers), int(n_iters)))


class BatchGraph:
    """n_iters iterations of a fixed list of solvers captured once as a HIP
    graph (pasd_batch_create) and replayed by step() (pasd_batch_step).  The
    solvers must stay open while the graph exists."""

    def __init__(self, solvers: List[Solver], n_iters: int):
        arr = (ctypes.c_void_p * len(solvers))(*[s.handle.value for s in solvers])
        h = ctypes.c_void_p()
        _check(lib().pasd_batch_create(arr, len(solvers), int(n_iters), ctypes.byref(h)))
        self._h = h
        self.solvers = list(solvers)

    def step(self):
        if self._h is None:
            raise PasdError(ERR_STATE, "batch graph destroyed")
        _check(lib().pasd_batch_step(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pasd_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def query_batch(solvers: List[Solver]) -> List[Info]:
    """Progress of several solvers with one synchronisation (pasd_query_batch)."""
    arr = (ctypes.c_void_p * len(solvers))(*[s.handle.value for s in solvers])
    infos = (Info * len(solvers))()
    _check(lib().pasd_query_batch(arr, len(solvers), infos))
    return list(infos)

