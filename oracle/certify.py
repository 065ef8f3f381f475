"""Certified bracket LB <= OPT <= UB for the OT linear program.

Test infrastructure only.  For instances too large for an exact solver, any
dual vector and any approximate plan yield a two-sided certificate:

* Lower bound (weak duality, eq. (3)): for any mu, the c-transform
  nu_j = min_i (C_ij - mu_i) makes (mu, nu) dual feasible, so
  p^T mu + q^T nu <= OPT.  Applying the transform back to mu
  (mu_i = min_j (C_ij - nu_j)) keeps feasibility and can only raise the bound.
* Upper bound: any feasible plan costs at least OPT.  A nearly feasible
  plan is made exactly feasible by the rounding procedure of Altschuler, Weed
  and Rigollet (2017): scale rows down to p, columns down to q, then add the
  rank-one correction err_r err_c^T / |err_r|_1.
"""
from __future__ import annotations

import numpy as np


def lower_bound(C: np.ndarray, p: np.ndarray, q: np.ndarray, mu: np.ndarray,
                nu: np.ndarray | None = None) -> float:
    """Dual-feasible lower bound from mu (and optionally nu as a start)."""
    C = np.asarray(C, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    if nu is not None:
        # Start from the better of the two one-sided transforms.
        mu = np.minimum(mu, (C - np.asarray(nu, dtype=np.float64)[None, :]).min(axis=1))
    nu_c = (C - mu[:, None]).min(axis=0)
    mu_cc = (C - nu_c[None, :]).min(axis=1)
    return float(p @ mu_cc + q @ nu_c)


def round_feasible(X: np.ndarray, p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Altschuler-Weed-Rigollet rounding of a nonnegative X onto
    {X >= 0, X e = p, X^T f = q} (requires sum p == sum q)."""
    F = np.maximum(np.asarray(X, dtype=np.float64), 0.0)
    rs = F.sum(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        sr = np.where(rs > p, p / rs, 1.0)
    F = F * sr[:, None]
    cs = F.sum(axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        sc = np.where(cs > q, q / cs, 1.0)
    F = F * sc[None, :]
    er = p - F.sum(axis=1)
    ec = q - F.sum(axis=0)
    l1 = er.sum()
    if l1 > 0:
        F = F + np.outer(er, ec) / l1
    return F


def upper_bound(C: np.ndarray, X: np.ndarray, p: np.ndarray, q: np.ndarray) -> float:
    return float((np.asarray(C, dtype=np.float64) * round_feasible(X, p, q)).sum())


def bracket(C, p, q, X, mu, nu=None) -> tuple[float, float]:
    """(LB, UB) with LB <= OPT <= UB (up to FP64 rounding)."""
    return lower_bound(C, p, q, mu, nu), upper_bound(C, X, p, q)
