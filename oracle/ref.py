"""ctypes wrapper of the plain FP64 DROT oracle (drot_ref.c).

Test infrastructure only (see the package docstring).  Follows Algorithm 1
and the stopping criteria of Section 3; see drot_ref.c for the readings.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdrot_ref.so")
_LIB_OMP_PATH = os.path.join(_HERE, "libdrot_ref_omp.so")
_libs = {}

INFO_FIELDS = ["iters", "status", "pobj", "dobj", "r_primal", "r_dual", "gap",
               "eps_p", "eps_d", "eps_g", "alpha", "norm_c", "norm_pq"]
TRACE_FIELDS = ["pobj", "dobj", "r_primal", "r_dual_lag", "gap", "max_eps"]

_dp = ctypes.POINTER(ctypes.c_double)


def _load(parallel: bool = False):
    """The oracle library; parallel=True the OpenMP build of the same source
    (rows of the sweep split over OMP_NUM_THREADS threads)."""
    if parallel in _libs:
        return _libs[parallel]
    path = _LIB_OMP_PATH if parallel else _LIB_PATH
    srcs = [os.path.join(_HERE, f) for f in ("drot_ref.c", "netsimplex.c")]
    if not os.path.exists(path) or (
            os.path.getmtime(path) < max(os.path.getmtime(f) for f in srcs)):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(path)
    lib.drot_ref_solve.restype = ctypes.c_int
    lib.drot_ref_solve.argtypes = [
        ctypes.c_longlong, ctypes.c_longlong, _dp, _dp, _dp, ctypes.c_double,
        ctypes.c_double, ctypes.c_int, ctypes.c_longlong, ctypes.c_int, _dp, _dp,
        _dp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_longlong]
    lib.drot_ref_eval.restype = ctypes.c_int
    lib.drot_ref_eval.argtypes = [ctypes.c_longlong, ctypes.c_longlong, _dp, _dp, _dp,
                                  ctypes.c_double, _dp, _dp, _dp, _dp]
    lib.drot_ref_info_len.restype = ctypes.c_int
    lib.drot_ref_threads.restype = ctypes.c_int
    lib.drot_ref_netsimplex.restype = ctypes.c_int
    lib.drot_ref_netsimplex.argtypes = [
        ctypes.c_longlong, ctypes.c_longlong, _dp, _dp, _dp, ctypes.c_double, ctypes.c_longlong,
        _dp, _dp, _dp, _dp, ctypes.POINTER(ctypes.c_longlong)]
    _libs[parallel] = lib
    return lib


def threads(parallel: bool = False) -> int:
    """Threads the sweep of the given build uses."""
    return int(_load(parallel).drot_ref_threads())


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    out = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and out.shape != shape:
        out = out.reshape(shape)
    return out


@dataclass
class RefResult:
    X: np.ndarray
    phi: np.ndarray
    psi: np.ndarray
    a: np.ndarray
    b: np.ndarray
    info: dict
    trace: np.ndarray | None
    status: int

    @property
    def mu(self):
        return self.phi / self.info["rho"]

    @property
    def nu(self):
        return self.psi / self.info["rho"]


def solve(C, p, q, rho: float, tol: float = 0.0, max_iter: int = 1000, tol_mode: int = 0,
          X0=None, phi0=None, psi0=None, trace: bool = False,
          parallel: bool = False) -> RefResult:
    """Run FP64 DROT (Algorithm 1) until the stopping test or max_iter.

    X0=None starts from X_0 = p q^T.  phi0/psi0 are initial shifts in the
    paper's phi units (phi = rho * mu).  Returns X_K, phi_K, psi_K, a_K, b_K,
    the info dict and (optionally) the per-iteration trace.  parallel=True
    runs the OpenMP build (same steps; the column, cost and r_dual sums are
    combined per row range, so results differ from the one-thread order only
    by rounding).
    """
    lib = _load(parallel)
    C = _f64(C)
    m, n = C.shape
    p = _f64(p, (m,))
    q = _f64(q, (n,))
    X = np.empty((m, n)) if X0 is None else _f64(X0, (m, n)).copy()
    phi = np.empty(m)
    psi = np.empty(n)
    a = np.empty(m)
    b = np.empty(n)
    info = np.zeros(lib.drot_ref_info_len())
    tr = np.zeros((max(1, max_iter), 6)) if trace else None
    phi0 = None if phi0 is None else _f64(phi0, (m,))
    psi0 = None if psi0 is None else _f64(psi0, (n,))
    st = lib.drot_ref_solve(m, n, _ptr(C), _ptr(p), _ptr(q), float(rho), float(tol),
                            int(tol_mode), int(max_iter), 0 if X0 is None else 1,
                            _ptr(phi0), _ptr(psi0), _ptr(X), _ptr(phi), _ptr(psi),
                            _ptr(a), _ptr(b), _ptr(info), _ptr(tr),
                            int(max_iter) if trace else 0)
    if st < 0:
        raise ValueError(f"drot_ref_solve failed with code {st}")
    d = dict(zip(INFO_FIELDS, info.tolist()))
    d["rho"] = float(rho)
    d["iters"] = int(d["iters"])
    if tr is not None:
        tr = tr[:d["iters"]]
    return RefResult(X, phi, psi, a, b, d, tr, st)


def evaluate(C, p, q, rho: float, X, phi, psi) -> dict:
    """Exact residuals and objectives of a primal-dual pair, no lag."""
    lib = _load()
    C = _f64(C)
    m, n = C.shape
    info = np.zeros(lib.drot_ref_info_len())
    st = lib.drot_ref_eval(m, n, _ptr(C), _ptr(_f64(p, (m,))), _ptr(_f64(q, (n,))),
                           float(rho), _ptr(_f64(X, (m, n))), _ptr(_f64(phi, (m,))),
                           _ptr(_f64(psi, (n,))), _ptr(info))
    if st < 0:
        raise ValueError(f"drot_ref_eval failed with code {st}")
    d = dict(zip(INFO_FIELDS, info.tolist()))
    d.pop("iters"); d.pop("status"); d.pop("alpha")
    return d


def solve_instance(inst, max_iter: int = 100000, tol=None, **kw) -> RefResult:
    """Convenience: solve a gen.Instance with its own rho and tol."""
    return solve(inst.C, inst.p, inst.q, inst.rho, inst.tol if tol is None else tol,
                 max_iter=max_iter, **kw)
