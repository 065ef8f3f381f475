"""Python binding of libdrot.so (include/drot.h), argument marshalling only.

Every step of the method runs in the library's HIP kernels; this module only
passes pointers, sizes and the stream.  PyTorch supplies device memory and
the current HIP stream.  If the library is missing the import of this module
still works, but every call raises: there is no CPU fallback.

    from paper_2110_11738_amd import drot
    X, res, mu, nu = drot.solve(C, p, q, rho, tol)      # C, p, q: cuda tensors
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libdrot.so")

OK, MAXITER = 0, 1
EINVAL, EMASS, ENONFINITE, ENOMEM, EDEVICE, EUNSUPPORTED, ESTATE = -1, -2, -3, -4, -5, -6, -7
F32, F64 = 0, 1
TOL_RELATIVE, TOL_ABSOLUTE = 0, 1
X0_PQ, X0_GIVEN = 0, 1
FLAG_NO_GRAPH, FLAG_TIME_SWEEP, FLAG_SKIP_C, FLAG_COMPENSATED = 0x1, 0x2, 0x4, 0x8
CACHE_AUTO, CACHE_CACHED, CACHE_STREAM = 0, 1, 2
COST_DENSE, COST_BF16, COST_COORDS = 0, 1, 2
TRACE_FIELDS = ("pobj", "dobj", "r_primal", "r_dual_lag", "gap", "test", "seconds", "k")

EXPORTED = ("drot_version", "drot_strerror", "drot_last_error", "drot_ctx_create",
            "drot_ctx_destroy", "drot_solve", "drot_bind", "drot_iterate", "drot_poll",
            "drot_finish", "drot_get_trace", "drot_bind_cost", "drot_solve_cost",
            "drot_solve_batched", "drot_mlp_create", "drot_mlp_destroy", "drot_mlp_num_params",
            "drot_mlp_set_weights", "drot_mlp_get_weights", "drot_mlp_forward",
            "drot_mlp_gradients", "drot_mlp_train_step", "drot_mlp_apply_gradients", "drot_tune",
            "drot_checkpoint_size", "drot_checkpoint", "drot_resume", "drot_solve_noalloc",
            "drot_tune_batched")


class Params(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int64), ("tol_mode", ctypes.c_int32),
                ("x0_mode", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("tile_chunks", ctypes.c_int32), ("tile_unroll", ctypes.c_int32),
                ("cache_mode", ctypes.c_int32), ("tile_groups", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("status", ctypes.c_int32),
                ("path", ctypes.c_int32), ("objective", ctypes.c_double),
                ("dual_objective", ctypes.c_double), ("r_primal", ctypes.c_double),
                ("r_dual", ctypes.c_double), ("gap", ctypes.c_double),
                ("eps_primal", ctypes.c_double), ("eps_dual", ctypes.c_double),
                ("eps_gap", ctypes.c_double), ("seconds_to_tol", ctypes.c_double),
                ("seconds_total", ctypes.c_double), ("sweep_ms_total", ctypes.c_double),
                ("sweep_timed", ctypes.c_int64), ("cost_scale", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Cost(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dim", ctypes.c_int32), ("data", ctypes.c_void_p),
                ("ld", ctypes.c_int64), ("xs", ctypes.c_void_p), ("xt", ctypes.c_void_p),
                ("scale", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("C", ctypes.c_void_p),
                ("ldc", ctypes.c_int64), ("p", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("rho", ctypes.c_double),
                ("tol", ctypes.c_double), ("mu", ctypes.c_void_p), ("nu", ctypes.c_void_p),
                ("mu0", ctypes.c_void_p), ("nu0", ctypes.c_void_p)]


class BatchTile(ctypes.Structure):
    _fields_ = [("m_class", ctypes.c_int32), ("n_class", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("blocks_per_item", ctypes.c_int32),
                ("problems", ctypes.c_int32), ("chunks", ctypes.c_int32),
                ("us_per_iter", ctypes.c_double)]


class DrotError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def lib():
    """Load libdrot.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2110_11738_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    L.drot_version.restype = ctypes.c_char_p
    L.drot_strerror.restype = ctypes.c_char_p
    L.drot_strerror.argtypes = [i32]
    L.drot_last_error.restype = ctypes.c_char_p
    L.drot_ctx_create.argtypes = [ctypes.POINTER(vp), i32]
    L.drot_ctx_destroy.argtypes = [vp]
    common = [vp, i64, i64, i32, vp, i64, vp, vp, ctypes.POINTER(Params), vp, i64]
    L.drot_solve.argtypes = common + [vp, vp, vp, vp, ctypes.POINTER(Result), vp]
    L.drot_solve_noalloc.argtypes = common[1:] + [vp, vp, vp, vp, ctypes.POINTER(Result), vp]
    L.drot_bind.argtypes = common + [vp, vp, vp]
    L.drot_iterate.argtypes = [vp, i64, vp]
    L.drot_poll.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int32), vp]
    L.drot_finish.argtypes = [vp, vp, vp, ctypes.POINTER(Result), vp]
    L.drot_get_trace.argtypes = [vp, i64, i64, ctypes.POINTER(ctypes.c_double)]
    cost_common = [vp, i64, i64, i32, ctypes.POINTER(Cost), vp, vp, ctypes.POINTER(Params), vp,
                   i64]
    L.drot_bind_cost.argtypes = cost_common + [vp, vp, vp]
    L.drot_solve_cost.argtypes = cost_common + [vp, vp, vp, vp, ctypes.POINTER(Result), vp]
    L.drot_solve_batched.argtypes = [vp, ctypes.c_int32, i32, ctypes.POINTER(Problem),
                                     ctypes.POINTER(Params), ctypes.POINTER(Result), vp]
    L.drot_tune_batched.argtypes = [vp, ctypes.c_int32, i32, ctypes.POINTER(Problem),
                                    ctypes.POINTER(Params), i64, ctypes.POINTER(BatchTile),
                                    ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), vp]
    fp = ctypes.POINTER(ctypes.c_float)
    dp = ctypes.POINTER(ctypes.c_double)
    L.drot_mlp_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32, i32, ctypes.c_uint64]
    L.drot_mlp_destroy.argtypes = [vp]
    L.drot_mlp_num_params.argtypes = [vp, ctypes.POINTER(i64)]
    L.drot_mlp_set_weights.argtypes = [vp, fp]
    L.drot_mlp_get_weights.argtypes = [vp, fp]
    L.drot_mlp_forward.argtypes = [vp, i32, vp, vp, vp]
    L.drot_mlp_gradients.argtypes = [vp, i32, vp, vp, vp, dp, vp]
    L.drot_mlp_train_step.argtypes = [vp, i32, vp, vp, ctypes.c_float, dp, vp]
    L.drot_mlp_apply_gradients.argtypes = [vp, vp, ctypes.c_float, vp]
    L.drot_tune.argtypes = [vp, i64, ctypes.POINTER(Params), dp, vp]
    L.drot_checkpoint_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.drot_checkpoint.argtypes = [vp, vp, ctypes.c_size_t, vp]
    L.drot_resume.argtypes = [vp, vp, ctypes.c_size_t, vp]
    for name in EXPORTED:
        getattr(L, name).restype = getattr(L, name).restype or i32
    _lib = L
    return L


def last_error() -> str:
    return lib().drot_last_error().decode()


def _check(rc: int, allow=(OK, MAXITER)) -> int:
    if rc not in allow:
        raise DrotError(rc, f"{lib().drot_strerror(rc).decode()}: {last_error()}")
    return rc


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t.dtype} (float32 or float64)")


def _ld(t) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("matrices must be 2-D with unit column stride (row-major)")
    return t.stride(0)


def make_params(rho, tol=0.0, max_iter=100000, tol_mode=TOL_RELATIVE, x0_mode=X0_PQ,
                check_every=0, flags=0, tile_rows=0, tile_chunks=0, tile_unroll=0,
                cache_mode=CACHE_AUTO, tile_groups=0) -> Params:
    return Params(float(rho), float(tol), int(max_iter), int(tol_mode), int(x0_mode),
                  int(check_every), int(flags), int(tile_rows), int(tile_chunks),
                  int(tile_unroll), int(cache_mode), int(tile_groups), 0)


class Context:
    """Owns a drot_ctx (workspace, graphs) on one device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().drot_ctx_create(ctypes.byref(h), int(device)), allow=(OK,))
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().drot_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- step-wise interface --------------------------------------------
    def bind(self, C, p, q, X, params: Params, mu0=None, nu0=None, stream=None):
        self._keep = (C, p, q, X, mu0, nu0)   # the library holds these pointers
        m, n = C.shape
        rc = lib().drot_bind(self.handle, m, n, _dtype_code(C), _ptr(C), _ld(C), _ptr(p),
                             _ptr(q), ctypes.byref(params), _ptr(X), _ld(X), _ptr(mu0),
                             _ptr(nu0), _stream(stream))
        return _check(rc, allow=(OK,))

    def iterate(self, iters: int, stream=None):
        return _check(lib().drot_iterate(self.handle, int(iters), _stream(stream)), allow=(OK,))

    def tune(self, iters: int = 0, stream=None):
        """drot_tune: time the tile variants on the bound problem and bind the
        fastest.  Returns (params, microseconds per iteration)."""
        best = Params()
        us = ctypes.c_double()
        _check(lib().drot_tune(self.handle, int(iters), ctypes.byref(best), ctypes.byref(us),
                               _stream(stream)), allow=(OK,))
        return best, us.value

    def checkpoint(self, stream=None) -> bytes:
        """drot_checkpoint: the iteration state (not X) as bytes."""
        size = ctypes.c_size_t()
        _check(lib().drot_checkpoint_size(self.handle, ctypes.byref(size)), allow=(OK,))
        buf = ctypes.create_string_buffer(size.value)
        _check(lib().drot_checkpoint(self.handle, buf, size, _stream(stream)), allow=(OK,))
        return buf.raw

    def resume(self, blob: bytes, stream=None):
        """drot_resume: continue from a checkpoint (bind the problem first)."""
        buf = ctypes.create_string_buffer(blob, len(blob))
        return _check(lib().drot_resume(self.handle, buf, ctypes.c_size_t(len(blob)),
                                        _stream(stream)), allow=(OK,))

    def poll(self, stream=None):
        k = ctypes.c_int64()
        s = ctypes.c_int32()
        _check(lib().drot_poll(self.handle, ctypes.byref(k), ctypes.byref(s), _stream(stream)),
               allow=(OK,))
        return k.value, bool(s.value)

    def finish(self, mu=None, nu=None, stream=None) -> dict:
        r = Result()
        rc = lib().drot_finish(self.handle, _ptr(mu), _ptr(nu), ctypes.byref(r), _stream(stream))
        _check(rc)
        return r.as_dict()

    def trace(self, first: int, count: int):
        import numpy as np
        out = np.zeros((count, 8), dtype=np.float64)
        rc = lib().drot_get_trace(self.handle, int(first), int(count),
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        _check(rc, allow=(OK,))
        return out

    def bind_cost(self, m, n, cost: "Cost", p, q, X, params: Params, mu0=None, nu0=None,
                  stream=None, keep=()):
        self._keep = (p, q, X, mu0, nu0) + tuple(keep)
        rc = lib().drot_bind_cost(self.handle, m, n, _dtype_code(X), ctypes.byref(cost), _ptr(p),
                                  _ptr(q), ctypes.byref(params), _ptr(X), _ld(X), _ptr(mu0),
                                  _ptr(nu0), _stream(stream))
        return _check(rc, allow=(OK,))

    # -- one-call solve ----------------------------------------------------
    def solve(self, C, p, q, params: Params, X=None, mu=None, nu=None, mu0=None, nu0=None,
              stream=None):
        import torch
        m, n = C.shape
        if X is None:
            X = torch.empty((m, n), dtype=C.dtype, device=C.device)
        r = Result()
        rc = lib().drot_solve(self.handle, m, n, _dtype_code(C), _ptr(C), _ld(C), _ptr(p),
                              _ptr(q), ctypes.byref(params), _ptr(X), _ld(X), _ptr(mu),
                              _ptr(nu), _ptr(mu0), _ptr(nu0), ctypes.byref(r), _stream(stream))
        _check(rc)
        return X, r.as_dict()


def make_cost(kind: int, C=None, xs=None, xt=None, scale: float = 0.0) -> Cost:
    """Cost descriptor: COST_DENSE / COST_BF16 take a 2-D tensor C (float32 or
    float64 / bfloat16), COST_COORDS the float32 point arrays xs (m x d) and
    xt (n x d) and an optional scale (0 = 1/max computed on the device)."""
    if kind == COST_COORDS:
        if xs is None or xt is None or xs.dim() != 2 or xt.dim() != 2 or xs.shape[1] != xt.shape[1]:
            raise ValueError("coordinates need xs (m x d) and xt (n x d)")
        if not (xs.is_contiguous() and xt.is_contiguous()):
            raise ValueError("coordinates must be contiguous")
        return Cost(COST_COORDS, xs.shape[1], None, 0, xs.data_ptr(), xt.data_ptr(), float(scale))
    return Cost(int(kind), 0, C.data_ptr(), _ld(C), None, None, 0.0)


_default_ctx: dict = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def solve_cost(m: int, n: int, p, q, rho: float, kind: int, C=None, xs=None, xt=None,
               scale: float = 0.0, tol: float = 1e-4, max_iter: int = 100000,
               tol_mode: int = TOL_RELATIVE, X0=None, mu0=None, nu0=None, check_every: int = 0,
               flags: int = 0, tile_rows: int = 0, tile_chunks: int = 0, tile_unroll: int = 0,
               cache_mode: int = CACHE_AUTO, tile_groups: int = 0, ctx: Context | None = None,
               stream=None):
    """solve() with a cost descriptor (see make_cost); X and the marginals are
    float32 for the bfloat16 and coordinate costs."""
    import torch
    dev = p.device
    ctx = ctx or default_context(dev.index or 0)
    dt = p.dtype
    X = empty_plan(m, n, dt, dev) if X0 is None else X0
    mu = torch.empty(m, dtype=torch.float64, device=dev)
    nu = torch.empty(n, dtype=torch.float64, device=dev)
    prm = make_params(rho, tol, max_iter, tol_mode, X0_PQ if X0 is None else X0_GIVEN,
                      check_every, flags, tile_rows, tile_chunks, tile_unroll, cache_mode,
                      tile_groups)
    cost = make_cost(kind, C, xs, xt, scale)
    r = Result()
    rc = lib().drot_solve_cost(ctx.handle, m, n, _dtype_code(X), ctypes.byref(cost), _ptr(p),
                               _ptr(q), ctypes.byref(prm), _ptr(X), _ld(X), _ptr(mu), _ptr(nu),
                               _ptr(mu0), _ptr(nu0), ctypes.byref(r), _stream(stream))
    _check(rc)
    return X, r.as_dict(), mu, nu


def row_pitch(n: int, itemsize: int) -> int:
    """Leading dimension (elements) that starts every row on a 128-byte cache
    line: a row that straddles lines makes the sweep fetch the lines shared by
    neighbouring column strips twice (measured 9.5% more bytes read at
    10000 x 15000 float32 with the leading dimension 15000)."""
    mult = max(1, 128 // itemsize)
    return -(-n // mult) * mult


def empty_plan(m: int, n: int, dtype, device):
    """An m x n tensor (a view) whose rows start on 128-byte cache lines."""
    import torch
    ld = row_pitch(n, torch.empty((), dtype=dtype).element_size())
    return torch.empty((m, ld), dtype=dtype, device=device)[:, :n]


def padded(t, mult: int = 0):
    """A 2-D tensor with the same values whose leading dimension is a multiple
    of `mult` elements (a view into a wider buffer); mult = 0 aligns every row
    to a 128-byte cache line (row_pitch)."""
    import torch
    m, n = t.shape
    ld = row_pitch(n, t.element_size()) if mult == 0 else -(-n // mult) * mult
    if ld == n and t.is_contiguous():
        return t
    buf = torch.zeros((m, ld), dtype=t.dtype, device=t.device)
    buf[:, :n] = t
    return buf[:, :n]


def _batch_arrays(problems):
    import torch
    if not problems:
        raise ValueError("no problems")
    C0 = problems[0]["C"]
    arr = (Problem * len(problems))()
    outs = (Result * len(problems))()
    keep = []
    for k, pr in enumerate(problems):
        C = pr["C"]
        m, n = C.shape
        if C.dtype != C0.dtype:
            raise TypeError("all problems of a batch share one dtype")
        X = empty_plan(m, n, C.dtype, C.device)
        mu = torch.empty(m, dtype=torch.float64, device=C.device)
        nu = torch.empty(n, dtype=torch.float64, device=C.device)
        mu0, nu0 = pr.get("mu0"), pr.get("nu0")
        arr[k] = Problem(m, n, C.data_ptr(), _ld(C), pr["p"].data_ptr(), pr["q"].data_ptr(),
                         X.data_ptr(), _ld(X), float(pr["rho"]), float(pr["tol"]),
                         mu.data_ptr(), nu.data_ptr(),
                         None if mu0 is None else mu0.data_ptr(),
                         None if nu0 is None else nu0.data_ptr())
        keep.append((X, mu, nu))
    return C0, arr, outs, keep


def solve_batched(problems, max_iter: int = 100000, tol_mode: int = TOL_RELATIVE,
                  check_every: int = 0, flags: int = 0, tile_rows: int = 0, tile_chunks: int = 0,
                  cache_mode: int = CACHE_AUTO, tile_groups: int = 0, ctx: Context | None = None,
                  stream=None):
    """Solve a list of problems together.  Each item is a dict with C (m x n
    tensor), p, q, rho, tol and optionally mu0, nu0 (float64 warm start); X,
    mu and nu are allocated here (X with rows on 128-byte cache lines).
    Returns (status, [(X, result, mu, nu), ...])."""
    C0, arr, outs, keep = _batch_arrays(problems)
    ctx = ctx or default_context(C0.device.index or 0)
    prm = make_params(1.0, 0.0, max_iter, tol_mode, X0_PQ, check_every, flags, tile_rows,
                      tile_chunks, 0, cache_mode, tile_groups)
    rc = lib().drot_solve_batched(ctx.handle, len(problems), _dtype_code(C0), arr,
                                  ctypes.byref(prm), outs, _stream(stream))
    _check(rc)
    return rc, [(X, outs[k].as_dict(), mu, nu) for k, (X, mu, nu) in enumerate(keep)]


def tune_batched(problems, iters: int = 0, check_every: int = 0, cache_mode: int = CACHE_AUTO,
                 tile_chunks: int = 0, ctx: Context | None = None, stream=None):
    """drot_tune_batched: time the candidate sweep schedules per size class
    of the given problems (their X is overwritten) and keep the fastest in
    the context's tuner cache.  Returns a list of dicts, one per class."""
    C0, arr, outs, keep = _batch_arrays(problems)
    ctx = ctx or default_context(C0.device.index or 0)
    prm = make_params(1.0, 0.0, 10, TOL_RELATIVE, X0_PQ, check_every, 0, 0, tile_chunks, 0,
                      cache_mode)
    table = (BatchTile * 72)()
    n = ctypes.c_int32()
    rc = lib().drot_tune_batched(ctx.handle, len(problems), _dtype_code(C0), arr,
                                 ctypes.byref(prm), int(iters), table, 72, ctypes.byref(n),
                                 _stream(stream))
    _check(rc, allow=(OK,))
    return [{f: getattr(table[k], f) for f, _ in BatchTile._fields_}
            for k in range(min(n.value, 72))]


class MLP:
    """The warm-start network of include/drot.h (drot_mlp_*): marshalling only."""

    def __init__(self, in_dim: int, hidden: int, out_dim: int, max_batch: int, seed: int = 0,
                 device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().drot_mlp_create(ctypes.byref(h), device, in_dim, hidden, out_dim, max_batch,
                                     seed), allow=(OK,))
        self.handle = h
        self.dims = (in_dim, hidden, out_dim)
        k = ctypes.c_int64()
        _check(lib().drot_mlp_num_params(h, ctypes.byref(k)), allow=(OK,))
        self.n_params = k.value

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().drot_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_weights(self):
        import numpy as np
        w = np.empty(self.n_params, dtype=np.float32)
        _check(lib().drot_mlp_get_weights(self.handle, w.ctypes.data_as(
            ctypes.POINTER(ctypes.c_float))), allow=(OK,))
        return w

    def set_weights(self, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(lib().drot_mlp_set_weights(self.handle, w.ctypes.data_as(
            ctypes.POINTER(ctypes.c_float))), allow=(OK,))

    def forward(self, x, stream=None):
        import torch
        y = torch.empty((x.shape[0], self.dims[2]), dtype=torch.float32, device=x.device)
        _check(lib().drot_mlp_forward(self.handle, x.shape[0], _ptr(x), _ptr(y), _stream(stream)),
               allow=(OK,))
        return y

    def gradients(self, x, t, stream=None):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = ctypes.c_double()
        _check(lib().drot_mlp_gradients(self.handle, x.shape[0], _ptr(x), _ptr(t), _ptr(g),
                                        ctypes.byref(loss), _stream(stream)), allow=(OK,))
        return loss.value, g

    def apply_gradients(self, grad, lr: float, stream=None) -> None:
        if grad.numel() != self.n_params or grad.dtype.itemsize != 4 or not grad.is_contiguous():
            raise ValueError("grad must be a contiguous float32 tensor of n_params entries")
        _check(lib().drot_mlp_apply_gradients(self.handle, _ptr(grad), ctypes.c_float(lr),
                                              _stream(stream)), allow=(OK,))

    def train_step(self, x, t, lr: float, stream=None) -> float:
        loss = ctypes.c_double()
        _check(lib().drot_mlp_train_step(self.handle, x.shape[0], _ptr(x), _ptr(t),
                                         ctypes.c_float(lr), ctypes.byref(loss),
                                         _stream(stream)), allow=(OK,))
        return loss.value


@dataclass
class Solution:
    X: object
    mu: object
    nu: object
    result: dict


def solve(C, p, q, rho: float, tol: float = 1e-4, max_iter: int = 100000,
          tol_mode: int = TOL_RELATIVE, X0=None, mu0=None, nu0=None, check_every: int = 0,
          flags: int = 0, tile_rows: int = 0, tile_chunks: int = 0, tile_unroll: int = 0,
          cache_mode: int = CACHE_AUTO, tile_groups: int = 0, ctx: Context | None = None,
          stream=None):
    """solve(C, p, q, rho, tol) -> (X, result, mu, nu) on C's device.

    C (m x n), p (m), q (n): float32 or float64 CUDA tensors.  X0 (optional)
    is the starting plan (default p q^T).  mu0/nu0 (optional, float64) warm
    start the dual shifts.  Returns the plan X_K, the result record (status,
    iterations, objective, residuals, timings) and mu, nu (float64)."""
    import torch
    if not (C.is_cuda and p.is_cuda and q.is_cuda):
        raise ValueError("C, p and q must be device tensors")
    ctx = ctx or default_context(C.device.index or 0)
    m, n = C.shape
    X = empty_plan(m, n, C.dtype, C.device) if X0 is None else X0
    mu = torch.empty(m, dtype=torch.float64, device=C.device)
    nu = torch.empty(n, dtype=torch.float64, device=C.device)
    prm = make_params(rho, tol, max_iter, tol_mode, X0_PQ if X0 is None else X0_GIVEN,
                      check_every, flags, tile_rows, tile_chunks, tile_unroll, cache_mode,
                      tile_groups)
    X, res = ctx.solve(C, p, q, prm, X=X, mu=mu, nu=nu, mu0=mu0, nu0=nu0, stream=stream)
    return X, res, mu, nu


def solve_noalloc(C, p, q, params: Params, X, mu=None, nu=None, mu0=None, nu0=None,
                  stream=None):
    """drot_solve_noalloc: the caller provides X (and optionally mu, nu); the
    library allocates nothing.  Returns (status, result dict)."""
    m, n = C.shape
    r = Result()
    rc = lib().drot_solve_noalloc(m, n, _dtype_code(C), _ptr(C), _ld(C), _ptr(p), _ptr(q),
                                  ctypes.byref(params), _ptr(X), _ld(X), _ptr(mu), _ptr(nu),
                                  _ptr(mu0), _ptr(nu0), ctypes.byref(r), _stream(stream))
    _check(rc)
    return rc, r.as_dict()
