"""Seeded synthetic OT instances.

This module only builds problem data (point clouds, cost matrices, marginals)
and holds none of the solver's arithmetic.  Both the CPU oracle and the GPU
path are fed from here, so that they solve exactly the same problem.

Conventions
-----------
* Every generator takes an integer seed tuple and uses NumPy's PCG64 through
  ``np.random.default_rng(seed_tuple)``; the same tuple always gives the same
  instance on every machine.
* Everything is produced in float64.  ``round_to`` rounds an instance once to
  the GPU dtype; the oracle then receives the rounded arrays upcast exactly.
* Costs are squared Euclidean distances divided by their maximum, so that
  ``max C = 1`` (the normalisation of the paper's experimental section).
* Marginals are quantised to integer multiples of a power of two (chosen so
  that every entry has at most 24 significant bits).  Each marginal is then
  exactly representable in float32 and float64, and ``sum(p) == sum(q) == 1``
  holds exactly, which the one-matrix recursion of the method relies on
  (equal total mass).  The relative change this makes to an entry is at most
  ``2**-24`` of the largest entry.
* The step size follows the paper's experimental section:
  ``rho = rho0 / (m + n)``; ``rho0 = 2`` in its accuracy experiment and
  ``rho0 = 1/log(m)`` in its runtime experiment (natural log).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Instance",
    "quantise_marginal",
    "sq_euclid_cost",
    "uniform_marginals",
    "dirichlet1",
    "uniform_weights",
    "gaussian_mixture_points",
    "config_small_fp64",
    "config_mixture_2d",
    "config_cube_3d",
    "paper_protocol",
    "line_instance",
    "assignment_instance",
    "separable_instance",
    "round_to",
    "rho_runtime",
    "rho_accuracy",
    "config_batch",
    "batch_problem",
    "batch_shape",
    "grid_cost",
    "grid_histogram_pair",
]


@dataclass
class Instance:
    """One OT problem: min <C,X> s.t. X 1 = p, X^T 1 = q, X >= 0."""

    C: np.ndarray          # (m, n) float64, row-major
    p: np.ndarray          # (m,)
    q: np.ndarray          # (n,)
    rho: float             # DR penalty parameter
    tol: float             # relative stopping tolerance
    name: str = ""
    xs: np.ndarray | None = None   # source points (m, d), if geometric
    xt: np.ndarray | None = None   # target points (n, d), if geometric
    cscale: float = 1.0    # C = ||xs_i - xt_j||^2 * cscale (geometric instances)
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.C.shape[0]

    @property
    def n(self) -> int:
        return self.C.shape[1]


def rho_runtime(m: int, n: int) -> float:
    """rho0 = 1/ln(m) divided by (m+n): the runtime-experiment step size.
    (m is clamped to 3 so that degenerate one- and two-row test problems
    still get a finite positive step.)"""
    return (1.0 / math.log(max(m, 3))) / (m + n)


def rho_accuracy(m: int, n: int, rho0: float = 2.0) -> float:
    """rho0 / (m+n) with the accuracy-experiment default rho0 = 2."""
    return rho0 / (m + n)


def quantise_marginal(w: np.ndarray) -> np.ndarray:
    """Nonnegative weights -> probability vector on a dyadic grid, exact sum 1.

    The grid step is 2**-e with e the largest exponent for which the biggest
    entry needs at most 24 bits.  Rounding uses the largest-remainder rule so
    that the integer counts add up to 2**e exactly.
    """
    w = np.asarray(w, dtype=np.float64)
    if w.ndim != 1 or w.size == 0 or np.any(w < 0) or not np.all(np.isfinite(w)):
        raise ValueError("weights must be a nonempty finite nonnegative vector")
    total = w.sum()
    if total <= 0:
        raise ValueError("weights sum to zero")
    w = w / total
    wmax = w.max()
    e = int(math.floor(math.log2((2.0 ** 24 - 1) / wmax)))
    e = min(e, 60)
    scale = 2.0 ** e
    target = int(round(scale))          # == 2**e exactly
    raw = w * scale
    k = np.floor(raw).astype(np.int64)
    short = target - int(k.sum())
    if short > 0:
        order = np.argsort(-(raw - k), kind="stable")
        k[order[:short]] += 1
    out = k.astype(np.float64) / scale
    assert out.sum() == 1.0
    return out


def uniform_marginals(m: int, n: int) -> tuple[np.ndarray, np.ndarray]:
    """p = 1/m, q = 1/n.  For m == n both are the plain constant 1/n (equal
    arrays, hence equal mass); otherwise they are dyadically quantised."""
    if m == n:
        p = np.full(m, 1.0 / m)
        return p, p.copy()
    return quantise_marginal(np.ones(m)), quantise_marginal(np.ones(n))


def sq_euclid_cost(xs: np.ndarray, xt: np.ndarray) -> tuple[np.ndarray, float]:
    """C_ij = ||xs_i - xt_j||^2 / max, built from coordinate differences.

    Returns (C, scale) with C = D * scale, scale = 1/max D.
    """
    xs = np.asarray(xs, dtype=np.float64)
    xt = np.asarray(xt, dtype=np.float64)
    m, n = xs.shape[0], xt.shape[0]
    D = np.zeros((m, n), dtype=np.float64)
    # Row blocks keep the temporaries small for the large instances.
    blk = max(1, (1 << 24) // max(1, n * xs.shape[1]))
    for i0 in range(0, m, blk):
        diff = xs[i0:i0 + blk, None, :] - xt[None, :, :]
        D[i0:i0 + blk] = np.einsum("ijk,ijk->ij", diff, diff)
    dmax = float(D.max())
    scale = 1.0 / dmax if dmax > 0 else 1.0
    D *= scale
    return D, scale


def dirichlet1(rng: np.random.Generator, k: int) -> np.ndarray:
    """Dirichlet(1,...,1) histogram (normalised i.i.d. exponentials)."""
    return quantise_marginal(rng.standard_exponential(k))


def uniform_weights(rng: np.random.Generator, k: int) -> np.ndarray:
    """i.i.d. Uniform(0,1) weights normalised to sum 1."""
    return quantise_marginal(rng.uniform(0.0, 1.0, k))


def gaussian_mixture_points(rng, k: int, d: int, n_comp: int, sigma: float) -> np.ndarray:
    """k points from an equal-weight mixture of isotropic Gaussians.

    Means are uniform in [0,1]^d; sigma is the per-axis standard deviation.
    """
    means = rng.uniform(0.0, 1.0, (n_comp, d))
    comp = rng.integers(0, n_comp, k)
    return means[comp] + sigma * rng.standard_normal((k, d))


def config_small_fp64(i: int = 0, m: int = 100, n: int = 100) -> Instance:
    """Small FP64 case: points U[0,1]^2, U(0,1) marginals, rho0 = 2, tol 1e-6."""
    rng = np.random.default_rng([1, i])
    xs = rng.uniform(0.0, 1.0, (m, 2))
    xt = rng.uniform(0.0, 1.0, (n, 2))
    C, sc = sq_euclid_cost(xs, xt)
    p = uniform_weights(rng, m)
    q = uniform_weights(rng, n)
    return Instance(C, p, q, rho_accuracy(m, n), 1e-6, f"small_fp64[{m}x{n},{i}]",
                    xs, xt, sc)


def config_mixture_2d(i: int = 0, m: int = 4096, n: int = 4096, seed_tag: int = 2) -> Instance:
    """2-D mixtures of 5 Gaussians (sigma 0.1) on each side, Dirichlet(1)
    marginals, rho0 = 1/ln m, tol 1e-4.  Used at 4096^2 and 20000^2."""
    rng = np.random.default_rng([seed_tag, i])
    xs = gaussian_mixture_points(rng, m, 2, 5, 0.1)
    xt = gaussian_mixture_points(rng, n, 2, 5, 0.1)
    C, sc = sq_euclid_cost(xs, xt)
    p = dirichlet1(rng, m)
    q = dirichlet1(rng, n)
    return Instance(C, p, q, rho_runtime(m, n), 1e-4, f"mixture2d[{m}x{n},{i}]",
                    xs, xt, sc)


def config_cube_3d(i: int = 0, m: int = 10000, n: int = 15000, build_cost: bool = True) -> Instance:
    """Points uniform in the unit cube of R^3, Dirichlet(1) marginals."""
    rng = np.random.default_rng([3, i])
    xs = rng.uniform(0.0, 1.0, (m, 3))
    xt = rng.uniform(0.0, 1.0, (n, 3))
    p = dirichlet1(rng, m)
    q = dirichlet1(rng, n)
    if build_cost:
        C, sc = sq_euclid_cost(xs, xt)
    else:
        C = np.zeros((0, 0))
        sc = float("nan")
    return Instance(C, p, q, rho_runtime(m, n), 1e-4, f"cube3d[{m}x{n},{i}]", xs, xt, sc)


def paper_protocol(i: int, m: int = 512, n: int | None = None, sigma_t: float = 5.0,
                   rho0: float = 2.0) -> Instance:
    """The paper's synthetic generator (experimental section).

    Source samples ~ N(mu_s, A_s A_s^T) with mu_s ~ N(0, I) and A_s entries
    uniform in [0,1]; target mean entries ~ N(5, sigma_t) (read as a standard
    deviation), A_t drawn like A_s.  Uniform marginals 1/m and 1/n.
    """
    n = m if n is None else n
    rng = np.random.default_rng([9, 1, i, int(sigma_t * 1000)])
    mu_s = rng.standard_normal(2)
    A_s = rng.uniform(0.0, 1.0, (2, 2))
    mu_t = 5.0 + sigma_t * rng.standard_normal(2)
    A_t = rng.uniform(0.0, 1.0, (2, 2))
    xs = mu_s + rng.standard_normal((m, 2)) @ A_s.T
    xt = mu_t + rng.standard_normal((n, 2)) @ A_t.T
    C, sc = sq_euclid_cost(xs, xt)
    p, q = uniform_marginals(m, n)
    return Instance(C, p, q, rho0 / (m + n), 1e-4, f"paper[{m}x{n},s{sigma_t},{i}]",
                    xs, xt, sc)


def line_instance(i: int, m: int, n: int, rho0: float | None = None) -> Instance:
    """Points on a line, C = (x-y)^2/max, Dirichlet(1) marginals.

    The monotone (north-west corner on sorted points) coupling is optimal for
    any convex cost of x-y on the real line, which gives the exact optimum.
    """
    rng = np.random.default_rng([9, 2, i, m, n])
    xs = rng.uniform(0.0, 1.0, (m, 1))
    xt = rng.uniform(0.0, 1.0, (n, 1)) * 0.8 + 0.1
    C, sc = sq_euclid_cost(xs, xt)
    p = dirichlet1(rng, m)
    q = dirichlet1(rng, n)
    rho = rho_runtime(m, n) if rho0 is None else rho0 / (m + n)
    return Instance(C, p, q, rho, 1e-4, f"line[{m}x{n},{i}]", xs, xt, sc)


def assignment_instance(i: int, n: int, rho0: float = 2.0) -> Instance:
    """Uniform-marginal square problem (an assignment problem up to 1/n).

    Points U[0,1]^2 on both sides; p = q = 1/n (the same array on both sides,
    so the two total masses agree bit for bit).
    """
    rng = np.random.default_rng([9, 3, i, n])
    xs = rng.uniform(0.0, 1.0, (n, 2))
    xt = rng.uniform(0.0, 1.0, (n, 2))
    C, sc = sq_euclid_cost(xs, xt)
    p, q = uniform_marginals(n, n)
    return Instance(C, p, q, rho0 / (2 * n), 1e-6, f"assign[{n},{i}]", xs, xt, sc)


def separable_instance(i: int, m: int, n: int) -> Instance:
    """C_ij = g_i + h_j (every feasible plan has the same cost g.p + h.q)."""
    rng = np.random.default_rng([9, 4, i, m, n])
    g = rng.uniform(0.0, 0.5, m)
    h = rng.uniform(0.0, 0.5, n)
    C = g[:, None] + h[None, :]
    p = dirichlet1(rng, m)
    q = dirichlet1(rng, n)
    inst = Instance(C, p, q, 2.0 / (m + n), 1e-6, f"separable[{m}x{n},{i}]")
    inst.meta["g"] = g
    inst.meta["h"] = h
    return inst


def round_to(inst: Instance, dtype) -> Instance:
    """Round C (and, harmlessly, p and q) once to `dtype`, returning float64
    arrays that hold exactly the rounded values."""
    dt = np.dtype(dtype)
    C = inst.C.astype(dt).astype(np.float64)
    p = inst.p.astype(dt).astype(np.float64)
    q = inst.q.astype(dt).astype(np.float64)
    if p.sum() != q.sum():
        raise ValueError("rounding broke the equal-mass property")
    out = Instance(C, p, q, inst.rho, inst.tol, inst.name + f"@{dt.name}", inst.xs, inst.xt,
                   inst.cscale, dict(inst.meta))
    return out


def batch_problem(b: int, lo: int = 64, hi: int = 2048, seed: int = 0) -> Instance:
    """Problem b of the ragged batch: m and n each uniform in [lo, hi]; each
    side a 2-D cloud of 1-5 Gaussian blobs (sigma 0.1, means uniform in
    [0,1]^2); squared-Euclidean cost normalised to max 1; Dirichlet(1)
    marginals; rho0 = 1/ln m; tol 1e-4.  Every problem has its own seed."""
    rng = np.random.default_rng([4, seed, b])
    m = int(rng.integers(lo, hi + 1))
    n = int(rng.integers(lo, hi + 1))
    xs = gaussian_mixture_points(rng, m, 2, int(rng.integers(1, 6)), 0.1)
    xt = gaussian_mixture_points(rng, n, 2, int(rng.integers(1, 6)), 0.1)
    C, sc = sq_euclid_cost(xs, xt)
    p = dirichlet1(rng, m)
    q = dirichlet1(rng, n)
    return Instance(C, p, q, rho_runtime(m, n), 1e-4, f"batch[{seed},{b}:{m}x{n}]", xs, xt, sc)


def batch_shape(b: int, lo: int = 64, hi: int = 2048, seed: int = 0) -> tuple[int, int]:
    """(m, n) of batch_problem(b) without building it."""
    rng = np.random.default_rng([4, seed, b])
    m = int(rng.integers(lo, hi + 1))
    return m, int(rng.integers(lo, hi + 1))


def config_batch(count: int = 512, lo: int = 64, hi: int = 2048, seed: int = 0) -> list:
    """The ragged batch: batch_problem(b) for b < count."""
    return [batch_problem(b, lo, hi, seed) for b in range(count)]


GRID = 32


def grid_cost(side: int = GRID) -> np.ndarray:
    """Squared distance between the cells of a side x side grid, divided by its
    maximum 2 (side-1)^2 (1922 for the 32 x 32 grid)."""
    ij = np.stack(np.meshgrid(np.arange(side), np.arange(side), indexing="ij"), -1).reshape(-1, 2)
    D = ((ij[:, None, :] - ij[None, :, :]) ** 2).sum(-1).astype(np.float64)
    return D / D.max()


def _bumps(rng, side: int) -> np.ndarray:
    ij = np.stack(np.meshgrid(np.arange(side), np.arange(side), indexing="ij"), -1).reshape(-1, 2)
    h = np.zeros(side * side)
    for _ in range(int(rng.integers(1, 5))):
        c = rng.uniform(0, side, 2)
        w = rng.uniform(1.0, 6.0)
        a = rng.uniform(0.5, 1.5)
        h += a * np.exp(-((ij - c) ** 2).sum(-1) / (2 * w * w))
    return quantise_marginal(h)


def grid_histogram_pair(i: int, split: int = 0, side: int = GRID):
    """(p, q): two histograms on a side x side grid, each a sum of 1-4 Gaussian
    bumps (centres uniform on the grid, standard deviations 1-6 cells,
    amplitudes U(0.5, 1.5)), normalised to 1.  split 0 = training, 1 = held out."""
    rng = np.random.default_rng([5, split, i])
    return _bumps(rng, side), _bumps(rng, side)
