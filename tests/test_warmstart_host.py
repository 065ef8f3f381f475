"""Host-side logic of the learned warm start (no GPU): the gauge fix of the
targets, the double c-transform that makes them learnable, the file format
of the solved training pairs, and the step size of the grid problems.

The c-transform checks are pinned to LP duality, not to the function
itself: on small grid problems the LP's optimal duals (HiGHS) must keep the
optimal dual objective and stay feasible after the transform."""
import math

import numpy as np
import pytest

from gen import grid_cost, grid_histogram_pair
from oracle import exact


def _ws():
    from paper_2110_11738_amd import warmstart
    return warmstart


def test_gauge_fix_removes_the_common_shift():
    ws = _ws()
    rng = np.random.default_rng(3)
    mu, nu = rng.standard_normal((5, 16)), rng.standard_normal((5, 16))
    t = rng.standard_normal((5, 1))
    a, b = ws.gauge_fix(mu, nu), ws.gauge_fix(mu + t, nu - t)
    np.testing.assert_allclose(a, b, atol=1e-6)  # float32 output
    np.testing.assert_allclose(a[:, :16].mean(axis=1), 0.0, atol=1e-6)
    # mu_i + nu_j is unchanged by the fix
    np.testing.assert_allclose(a[:, :16, None] + a[:, None, 16:], mu[:, :, None] + nu[:, None, :],
                               atol=1e-5)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_canonical_keeps_lp_optimal_duals_optimal_and_feasible(k):
    ws = _ws()
    side = 4
    C = grid_cost(side)
    p, q = grid_histogram_pair(k, 0, side)
    opt, X, mu, nu = exact.lp_highs(C, p, q)
    mu2, nu2 = ws.canonical(C, mu[None], nu[None])
    mu2, nu2 = mu2[0], nu2[0]
    assert (mu2[:, None] + nu2[None, :] <= C + 1e-12).all()
    assert abs(p @ mu2 + q @ nu2 - opt) <= 1e-9 * max(1.0, abs(opt))
    # the double c-transform is idempotent
    mu3, nu3 = ws.canonical(C, mu2[None], nu2[None])
    np.testing.assert_allclose(mu3[0], mu2, atol=1e-14)
    np.testing.assert_allclose(nu3[0], nu2, atol=1e-14)


def test_canonical_never_lowers_a_feasible_dual():
    ws = _ws()
    side = 4
    C = grid_cost(side)
    p, q = grid_histogram_pair(7, 0, side)
    opt, X, mu, nu = exact.lp_highs(C, p, q)
    rng = np.random.default_rng(11)
    mu0 = mu - np.abs(rng.standard_normal(mu.shape)) * 0.05  # still feasible
    nu0 = nu - np.abs(rng.standard_normal(nu.shape)) * 0.05
    mu2, nu2 = ws.canonical(C, mu0[None], nu0[None])
    assert (mu2[0] >= mu0 - 1e-15).all() and (nu2[0] >= nu0 - 1e-15).all()
    assert p @ mu2[0] + q @ nu2[0] >= p @ mu0 + q @ nu0 - 1e-15
    assert p @ mu2[0] + q @ nu2[0] <= opt + 1e-12  # weak duality


def _target_file(path, start, count, split=0, side=4):
    N = side * side
    T = (np.arange(count * 2 * N, dtype=np.float64).reshape(count, 2 * N) + 1000 * start)
    np.savez(path, targets=T.astype(np.float16), iters=np.arange(start, start + count),
             status=np.zeros(count, dtype=np.int32), start=start, split=split, tol=1e-4,
             rho0=2.0, side=side)


def test_load_targets_orders_contiguous_ranges_and_rejects_gaps(tmp_path):
    ws = _ws()
    a, b, c = tmp_path / "a.npz", tmp_path / "b.npz", tmp_path / "c.npz"
    _target_file(a, 0, 3)
    _target_file(b, 3, 2)
    T, its, sts = ws.load_targets([str(b), str(a)], side=4)  # any order on input
    assert T.shape == (5, 32) and T.dtype == np.float32
    np.testing.assert_array_equal(its, np.arange(5))
    _target_file(c, 6, 2)  # pairs 5 missing
    with pytest.raises(ValueError):
        ws.load_targets([str(a), str(b), str(c)], side=4)
    _target_file(c, 5, 2, split=1)  # held-out pairs are not training data
    with pytest.raises(ValueError):
        ws.load_targets([str(a), str(b), str(c)], side=4)
    with pytest.raises(ValueError):  # another grid
        ws.load_targets([str(a)], side=8)


def test_step_size_of_the_grid_problems():
    ws = _ws()
    assert ws.rho_grid(2.0, 32) == 2.0 / 2048
    assert ws.rho_grid(None, 32) == pytest.approx(1.0 / math.log(1024) / 2048, rel=1e-15)
    X = ws.features(np.full((2, 16), 1 / 16), np.full((2, 16), 1 / 16))
    assert X.shape == (2, 32) and np.allclose(X, 1.0)
