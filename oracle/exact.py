"""Exact optimal values of the OT linear program, by definition.

Test infrastructure only.  The problem is eq. (1) of the paper:
    OPT = min <C, X>  s.t.  X e = p, X^T f = q, X >= 0,
with the dual of eq. (3): max p^T mu + q^T nu s.t. mu_i + nu_j <= C_ij.
Each routine below reaches OPT through a route that does not involve the
Douglas-Rachford iteration:

* brute_force_uniform: for p = q = 1/n the LP is (1/n) times an assignment
  problem, and a vertex optimum is a permutation matrix (Birkhoff-von
  Neumann); enumerate every permutation (n <= 8).
* assignment_uniform: the same through scipy's linear_sum_assignment.
* lp_highs: the LP itself through scipy's HiGHS solver (small m, n).
* line_monotone: points on a line with a cost convex in x - y; the monotone
  (north-west corner on sorted points) coupling is optimal.
* network_simplex: the primal network simplex method on the transportation
  network (netsimplex.c), any m, n and marginals, with an optimality
  certificate (a feasible plan and dual variables whose c-transform bound
  meets its cost).
* single_row / single_col: m = 1 or n = 1 leaves exactly one feasible plan.
* separable: C_ij = g_i + h_j makes every feasible plan cost g.p + h.q.
"""
from __future__ import annotations

import itertools

import numpy as np


def brute_force_uniform(C: np.ndarray) -> float:
    """OPT for m = n <= 8 and p = q = 1/n, by enumerating permutations."""
    C = np.asarray(C, dtype=np.float64)
    n = C.shape[0]
    if C.shape != (n, n) or n > 8:
        raise ValueError("brute force needs a square matrix with n <= 8")
    best = np.inf
    rows = np.arange(n)
    for perm in itertools.permutations(range(n)):
        best = min(best, C[rows, list(perm)].sum())
    return best / n


def assignment_uniform(C: np.ndarray) -> float:
    """OPT for p = q = 1/n via the Hungarian-type solver in scipy."""
    from scipy.optimize import linear_sum_assignment
    C = np.asarray(C, dtype=np.float64)
    r, c = linear_sum_assignment(C)
    return float(C[r, c].sum() / C.shape[0])


def lp_highs(C: np.ndarray, p: np.ndarray, q: np.ndarray):
    """Solve the LP with HiGHS.  Returns (OPT, X, mu, nu)."""
    from scipy.optimize import linprog
    from scipy.sparse import coo_matrix
    C = np.asarray(C, dtype=np.float64)
    m, n = C.shape
    idx = np.arange(m * n)
    rows = np.concatenate([idx // n, m + idx % n])
    cols = np.concatenate([idx, idx])
    A = coo_matrix((np.ones(2 * m * n), (rows, cols)), shape=(m + n, m * n)).tocsr()
    b = np.concatenate([p, q])
    res = linprog(C.reshape(-1), A_eq=A, b_eq=b, bounds=(0, None), method="highs",
                  options={"primal_feasibility_tolerance": 1e-10,
                           "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        raise RuntimeError(f"HiGHS failed: {res.message}")
    duals = res.eqlin.marginals
    return float(res.fun), res.x.reshape(m, n), duals[:m].copy(), duals[m:].copy()


def line_monotone(xs: np.ndarray, xt: np.ndarray, C: np.ndarray, p: np.ndarray,
                  q: np.ndarray):
    """Monotone coupling of two measures on the real line.

    xs, xt: 1-D coordinates of sources and targets; C the cost matrix that
    the solver sees (any cost convex in x - y).  Returns (OPT, X)."""
    xs = np.asarray(xs, dtype=np.float64).reshape(-1)
    xt = np.asarray(xt, dtype=np.float64).reshape(-1)
    m, n = len(xs), len(xt)
    si = np.argsort(xs, kind="stable")
    tj = np.argsort(xt, kind="stable")
    rp = p[si].astype(np.float64).copy()
    rq = q[tj].astype(np.float64).copy()
    X = np.zeros((m, n))
    i = j = 0
    while i < m and j < n:
        f = min(rp[i], rq[j])
        X[si[i], tj[j]] += f
        rp[i] -= f
        rq[j] -= f
        # Advance whichever side is exhausted (relative to its size).
        if rp[i] <= rq[j]:
            i += 1
        else:
            j += 1
    return float((C * X).sum()), X


def single_row(C: np.ndarray, q: np.ndarray) -> float:
    """m = 1: the only feasible plan is X = q^T (p_0 = sum q)."""
    return float(np.asarray(C, dtype=np.float64).reshape(-1) @ q)


def single_col(C: np.ndarray, p: np.ndarray) -> float:
    """n = 1: the only feasible plan is X = p."""
    return float(np.asarray(C, dtype=np.float64).reshape(-1) @ p)


def separable(g: np.ndarray, h: np.ndarray, p: np.ndarray, q: np.ndarray) -> float:
    """C_ij = g_i + h_j: <C, X> = g.(X e) + h.(X^T f) = g.p + h.q."""
    return float(g @ p + h @ q)


def network_simplex(C: np.ndarray, p: np.ndarray, q: np.ndarray, eps: float = 1e-12,
                    max_pivots: int = 50_000_000, want_plan: bool = True) -> dict:
    """Exact optimum of eq. (1) by the primal network simplex (netsimplex.c).

    Returns {"opt", "X" (or None), "u", "v", "pivots", "lb", "ub"}: "ub" is the
    cost of the returned plan (feasible: nonnegative, exact marginals when p
    and q lie on a dyadic grid) and "lb" the dual bound p.u' + q.v' of the
    c-transforms of its duals (feasible by construction, so lb <= OPT <= ub)."""
    import ctypes
    from . import ref
    lib = ref._load()
    C = np.ascontiguousarray(C, dtype=np.float64)
    m, n = C.shape
    p = np.ascontiguousarray(p, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    X = np.empty((m, n)) if want_plan else None
    u = np.empty(m)
    v = np.empty(n)
    obj = np.zeros(1)
    piv = ctypes.c_longlong(0)
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib.drot_ref_netsimplex(m, n, C.ctypes.data_as(dp), p.ctypes.data_as(dp),
                                 q.ctypes.data_as(dp), float(eps), int(max_pivots),
                                 X.ctypes.data_as(dp) if X is not None else None,
                                 u.ctypes.data_as(dp), v.ctypes.data_as(dp),
                                 obj.ctypes.data_as(dp), ctypes.byref(piv))
    if st != 0:
        raise RuntimeError(f"network simplex failed with code {st}")
    # The tree potentials can sit near +-M (artificial arcs left in the basis
    # with zero flow); one common shift (u - t, v + t keeps every u_i + v_j)
    # brings them to the scale of C before the c-transforms
    # v'_j = min_i (C_ij - u_i), u'_i = min_j (C_ij - v'_j).
    t = 0.5 * (u.max() + u.min())
    u = u - t
    v = v + t
    vc = (C - u[:, None]).min(axis=0)
    uc = (C - vc[None, :]).min(axis=1)
    lb = float(p @ uc + q @ vc)
    return {"opt": float(obj[0]), "X": X, "u": u, "v": v, "pivots": int(piv.value),
            "lb": lb, "ub": float(obj[0])}
