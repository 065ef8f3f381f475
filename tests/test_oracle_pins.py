"""Pins of the CPU oracle against facts that do not come from the oracle.

Every test here runs on the CPU.  Each pins a part of the oracle to something
fixed by the paper or by mathematics: the generic least-squares projection
(Lemma 2), the literal three-matrix DR iteration (Section 3), exact optima
(brute force, HiGHS, the monotone 1-D coupling, one-row/one-column and
separable problems), the identities of the variational-representation lemma
(Appendix A) and the optimality conditions of Proposition 1.
"""
import json
import os

import numpy as np
import pytest

from gen import (assignment_instance, config_mixture_2d, config_small_fp64,
                 line_instance, paper_protocol, quantise_marginal, round_to,
                 separable_instance)
from oracle import certify, dr3, exact, ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "exact_opt.json")


def _rand_problem(rng, m, n, zeros=False):
    C = rng.uniform(0.0, 1.0, (m, n))
    wp = rng.uniform(0.0, 1.0, m)
    wq = rng.uniform(0.0, 1.0, n)
    if zeros and m > 1:
        wp[rng.integers(0, m)] = 0.0
    if zeros and n > 1:
        wq[rng.integers(0, n)] = 0.0
    return C, quantise_marginal(wp), quantise_marginal(wq)


# --------------------------------------------------------------------------
# Lemma 2: closed-form projection onto {X e = p, X^T f = q}
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,n", [(1, 1), (1, 5), (4, 1), (3, 3), (4, 6), (7, 5)])
def test_lemma2_projection_equals_generic_projection(m, n):
    rng = np.random.default_rng([100, m, n])
    _, p, q = _rand_problem(rng, m, n)
    W = rng.standard_normal((m, n))
    P1 = dr3.project_lemma2(W, p, q)
    P2 = dr3.project_lstsq(W, p, q)
    np.testing.assert_allclose(P1, P2, atol=1e-13)
    # exact marginals, idempotence, and W - P(W) in ran A* (= y e^T + f x^T)
    np.testing.assert_allclose(P1.sum(1), p, atol=1e-14)
    np.testing.assert_allclose(P1.sum(0), q, atol=1e-14)
    np.testing.assert_allclose(dr3.project_lemma2(P1, p, q), P1, atol=1e-14)
    D = W - P1
    np.testing.assert_allclose(D - D[:, :1] - D[:1, :] + D[0, 0], 0.0, atol=1e-13)


# --------------------------------------------------------------------------
# Algorithm 1 == the three-matrix DR of eq. (drot:general:form)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,scale,warm", [(3, 4, 50.0, False), (6, 6, 20.0, False),
                                            (1, 5, 10.0, False), (5, 1, 10.0, False),
                                            (8, 5, 40.0, True), (9, 12, 5.0, True)])
def test_algorithm1_equals_three_matrix_dr(m, n, scale, warm):
    rng = np.random.default_rng([101, m, n])
    C, p, q = _rand_problem(rng, m, n, zeros=True)
    rho = scale / (m + n)
    phi0 = psi0 = None
    Y0 = np.outer(p, q)
    if warm:
        phi0 = 0.01 * rng.standard_normal(m)
        psi0 = 0.01 * rng.standard_normal(n)
        Y0 = Y0 + phi0[:, None] + psi0[None, :]
    K = 40
    Xs, _, Ys = dr3.dr3_iterate(C, p, q, rho, K, Y0=Y0)
    for k in (1, 2, 3, 10, K):
        R = ref.solve(C, p, q, rho, 0.0, max_iter=k, phi0=phi0, psi0=psi0)
        assert R.info["iters"] == k
        np.testing.assert_allclose(R.X, Xs[k - 1], atol=1e-13, rtol=0)
        Y = R.X + R.phi[:, None] + R.psi[None, :]
        np.testing.assert_allclose(Y, Ys[k], atol=1e-13, rtol=0)
        # accumulators: a_k = Y_k e - p, b_k = Y_k^T f - q
        np.testing.assert_allclose(R.a, Ys[k].sum(1) - p, atol=1e-13)
        np.testing.assert_allclose(R.b, Ys[k].sum(0) - q, atol=1e-13)
        # alpha_k = f^T a_k / (m+n)
        assert abs(R.info["alpha"] - R.a.sum() / (m + n)) < 1e-14


def test_shift_sums_agree():
    """f^T phi_k = e^T psi_k for k >= 1 (from the shift updates with equal mass)."""
    inst = config_small_fp64(3, 30, 45)
    for k in (1, 7, 200):
        R = ref.solve(inst.C, inst.p, inst.q, inst.rho, 0.0, max_iter=k)
        assert abs(R.phi.sum() - R.psi.sum()) < 1e-13 * max(1.0, abs(R.phi).sum())


# --------------------------------------------------------------------------
# Exact optima
# --------------------------------------------------------------------------
def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.mark.parametrize("case", _golden()["brute_force"], ids=lambda c: f"n{c['n']}s{c['seed']}")
def test_converges_to_brute_force_assignment(case):
    inst = assignment_instance(case["seed"], case["n"])
    # library solver and brute force agree (pins the golden value itself)
    assert abs(exact.assignment_uniform(inst.C) - case["opt"]) < 1e-14
    R = ref.solve(inst.C, inst.p, inst.q, inst.rho, 1e-9, max_iter=2_000_000)
    assert R.status == 0
    assert abs(R.info["pobj"] - case["opt"]) <= 1e-7 * max(case["opt"], 1e-3)
    assert R.X.min() >= 0.0


@pytest.mark.parametrize("case", _golden()["lp"], ids=lambda c: f"{c['gen']}{c['m']}x{c['n']}s{c['seed']}")
def test_converges_to_lp_optimum(case):
    if case["gen"] == "config_small_fp64":
        inst = config_small_fp64(case["seed"], case["m"], case["n"])
    else:
        inst = paper_protocol(case["seed"], case["m"])
    # The relative stopping test bounds the objective error only up to a
    # modest factor; pin convergence at a tight tolerance.
    tol = 1e-8 if case["m"] * case["n"] <= 2500 else 1e-7
    R = ref.solve(inst.C, inst.p, inst.q, inst.rho, tol, max_iter=5_000_000)
    assert R.status == 0
    assert abs(R.info["pobj"] - case["opt"]) / case["opt"] <= 20 * tol
    # certified bracket from the oracle's own output contains the optimum
    lb, ub = certify.bracket(inst.C, inst.p, inst.q, R.X, R.mu)
    assert lb <= case["opt"] * (1 + 1e-12) and case["opt"] <= ub * (1 + 1e-12)


def test_default_tolerance_objective_error():
    """At its own stopping tolerance (1e-6) the small FP64 case lands within
    a small multiple of the tolerance of the optimum."""
    for seed in (0, 1):
        inst = config_small_fp64(seed)
        case = [c for c in _golden()["lp"] if c["m"] == 100 and c["seed"] == seed][0]
        R = ref.solve_instance(inst, max_iter=2_000_000)
        assert R.status == 0 and R.info["eps_p"] <= 1e-6 and R.info["eps_g"] <= 1e-6
        assert abs(R.info["pobj"] - case["opt"]) / case["opt"] <= 5e-6


@pytest.mark.parametrize("case", _golden()["line"], ids=lambda c: f"{c['m']}x{c['n']}")
def test_converges_to_monotone_coupling_on_a_line(case):
    # Line problems are badly conditioned for DR (slow tail); the larger one
    # is pinned at a looser tolerance to keep the CPU suite short.
    inst = line_instance(case["seed"], case["m"], case["n"], rho0=2.0)
    tol = 1e-8 if case["m"] * case["n"] <= 2400 else 1e-6
    R = ref.solve(inst.C, inst.p, inst.q, inst.rho, tol, max_iter=3_000_000)
    assert R.status == 0
    assert abs(R.info["pobj"] - case["opt"]) / case["opt"] <= 20 * tol


def test_single_row_and_single_column():
    rng = np.random.default_rng(7)
    C, p, q = _rand_problem(rng, 1, 9)
    R = ref.solve(C, p, q, 2.0 / 10, 1e-12, max_iter=200_000)
    np.testing.assert_allclose(R.X[0], q, atol=1e-11)
    assert abs(R.info["pobj"] - exact.single_row(C, q)) < 1e-11
    C, p, q = _rand_problem(rng, 9, 1)
    R = ref.solve(C, p, q, 2.0 / 10, 1e-12, max_iter=200_000)
    np.testing.assert_allclose(R.X[:, 0], p, atol=1e-11)
    assert abs(R.info["pobj"] - exact.single_col(C, p)) < 1e-11


def test_separable_cost():
    inst = separable_instance(0, 30, 20)
    R = ref.solve(inst.C, inst.p, inst.q, inst.rho, 1e-10, max_iter=500_000)
    opt = exact.separable(inst.meta["g"], inst.meta["h"], inst.p, inst.q)
    assert abs(R.info["pobj"] - opt) / opt < 1e-8


# --------------------------------------------------------------------------
# Network simplex (oracle/netsimplex.c): exact optima for large instances
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,zeros", [(1, 1, False), (1, 9, False), (8, 1, False), (2, 2, False),
                                       (7, 5, True), (30, 40, False), (45, 30, True),
                                       (120, 90, False)])
def test_network_simplex_equals_highs(m, n, zeros):
    rng = np.random.default_rng([400, m, n, int(zeros)])
    C, p, q = _rand_problem(rng, m, n, zeros)
    r = exact.network_simplex(C, p, q)
    opt_h = exact.lp_highs(C, p, q)[0]
    X = r["X"]
    assert abs(r["opt"] - opt_h) <= 1e-12 * max(abs(opt_h), 1e-300) + 1e-15
    assert X.min() >= 0.0
    np.testing.assert_array_equal(X.sum(axis=1), p)  # dyadic marginals: exact flows
    np.testing.assert_array_equal(X.sum(axis=0), q)
    assert abs(float((C * X).sum()) - r["opt"]) <= 1e-14
    assert r["lb"] <= r["ub"] + 1e-14 and r["ub"] - r["lb"] <= 1e-12


@pytest.mark.parametrize("n", [3, 6, 8])
def test_network_simplex_equals_brute_force(n):
    for seed in range(3):
        inst = assignment_instance(seed, n)
        r = exact.network_simplex(inst.C, inst.p, inst.q)
        assert abs(r["opt"] - exact.brute_force_uniform(inst.C)) <= 1e-15


def test_network_simplex_closed_forms():
    # points on a line: the monotone coupling (closed form)
    inst = line_instance(3, 700, 900)
    opt_line, _ = exact.line_monotone(inst.xs, inst.xt, inst.C, inst.p, inst.q)
    assert abs(exact.network_simplex(inst.C, inst.p, inst.q)["opt"] - opt_line) <= 1e-13 * opt_line
    # separable costs: every feasible plan costs g.p + h.q
    sep = separable_instance(2, 60, 80)
    opt_sep = exact.separable(sep.meta["g"], sep.meta["h"], sep.p, sep.q)
    assert abs(exact.network_simplex(sep.C, sep.p, sep.q)["opt"] - opt_sep) <= 1e-14
    # one row / one column: the only feasible plan
    rng = np.random.default_rng(401)
    C, p, q = _rand_problem(rng, 1, 13)
    assert abs(exact.network_simplex(C, p, q)["opt"] - exact.single_row(C, q)) <= 1e-15
    C, p, q = _rand_problem(rng, 11, 1)
    assert abs(exact.network_simplex(C, p, q)["opt"] - exact.single_col(C, p)) <= 1e-15


def test_hand_solved_two_by_two():
    """C = [[1,3],[2,5]], p = (0.4,0.6), q = (0.7,0.3).  Feasible plans are
    [[a, .4-a], [.7-a, a-.1]] with a in [.1,.4] and cost a + 2.1, so the
    optimum is a = 0.1, X* = [[.1,.3],[.6,0]], OPT = 2.2."""
    C = np.array([[1.0, 3.0], [2.0, 5.0]])
    p = np.array([0.4, 0.6])
    q = np.array([0.7, 0.3])
    R = ref.solve(C, p, q, 0.5, 1e-12, max_iter=1_000_000)
    assert abs(R.info["pobj"] - 2.2) < 1e-10
    np.testing.assert_allclose(R.X, [[0.1, 0.3], [0.6, 0.0]], atol=1e-9)


# --------------------------------------------------------------------------
# Appendix A (variational representation) and Proposition 1
# --------------------------------------------------------------------------
def test_variational_identities_each_iteration():
    """For every k: <C,X_{k+1}> - p.mu_{k+1} - q.nu_{k+1} = -<Y_{k+1}, Y_{k+1}-Y_k>/rho,
    mu_{k+1} e^T + f nu_{k+1}^T - C <= (Y_{k+1}-Y_k)/rho, and
    ||Y_{k+1}-Y_k|| is non-increasing (T is firmly non-expansive)."""
    inst = config_small_fp64(2, 12, 9)
    C, p, q, rho = inst.C, inst.p, inst.q, inst.rho * 20
    Yprev = np.outer(p, q)
    step_prev = np.inf
    for k in range(1, 60):
        R = ref.solve(C, p, q, rho, 0.0, max_iter=k)
        Y = R.X + R.phi[:, None] + R.psi[None, :]
        mu, nu = R.phi / rho, R.psi / rho
        lhs = (C * R.X).sum() - p @ mu - q @ nu
        rhs = -(Y * (Y - Yprev)).sum() / rho
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(rhs))
        assert np.all(mu[:, None] + nu[None, :] - C <= (Y - Yprev) / rho + 1e-9)
        step = np.linalg.norm(Y - Yprev)
        assert step <= step_prev * (1 + 1e-12) + 1e-15
        step_prev = step
        Yprev = Y


def test_converged_pair_satisfies_proposition_1():
    inst = config_small_fp64(4, 40, 30)
    R = ref.solve(inst.C, inst.p, inst.q, inst.rho, 1e-9, max_iter=2_000_000)
    ev = ref.evaluate(inst.C, inst.p, inst.q, inst.rho, R.X, R.phi, R.psi)
    assert R.X.min() >= 0                                   # (i) X >= 0
    assert ev["eps_p"] < 1e-8                               # (i) marginals
    assert ev["r_dual"] < 1e-7                              # (ii) dual feasibility
    assert ev["gap"] / ev["pobj"] < 1e-8                    # (iii) zero gap
    # Few entries stay positive at a vertex of the transport polytope.
    assert (R.X > 1e-9).sum() <= 2 * (40 + 30)


# --------------------------------------------------------------------------
# Stopping-test bookkeeping
# --------------------------------------------------------------------------
def test_trace_matches_direct_evaluation_with_lagged_dual_residual():
    inst = config_small_fp64(5, 25, 31)
    K = 50
    Rk = ref.solve(inst.C, inst.p, inst.q, inst.rho, 0.0, max_iter=K, trace=True)
    Rk1 = ref.solve(inst.C, inst.p, inst.q, inst.rho, 0.0, max_iter=K - 1)
    ev = ref.evaluate(inst.C, inst.p, inst.q, inst.rho, Rk.X, Rk.phi, Rk.psi)
    ev_prev = ref.evaluate(inst.C, inst.p, inst.q, inst.rho, Rk1.X, Rk1.phi, Rk1.psi)
    last = dict(zip(ref.TRACE_FIELDS, Rk.trace[-1]))
    # r_primal and gap are at iterate K, r_dual at the shifts entering iteration K
    assert abs(last["r_primal"] - np.sqrt(((Rk.X.sum(1) - inst.p) ** 2).sum()
                                          + ((Rk.X.sum(0) - inst.q) ** 2).sum())) < 1e-15
    assert abs(last["r_primal"] - ev["r_primal"]) < 1e-15
    assert abs(last["gap"] - ev["gap"]) < 1e-14
    assert abs(last["r_dual_lag"] - ev_prev["r_dual"]) < 1e-12 * max(1, ev_prev["r_dual"])


def test_stop_is_first_iterate_meeting_tolerance():
    inst = config_small_fp64(6, 20, 20)
    R = ref.solve(inst.C, inst.p, inst.q, inst.rho, 1e-4, max_iter=100_000, trace=True)
    assert R.status == 0
    me = R.trace[:, 5]
    assert me[-1] <= 1e-4 and np.all(me[:-1] > 1e-4)


def test_maxiter_status():
    inst = config_small_fp64(0, 10, 10)
    R = ref.solve(inst.C, inst.p, inst.q, inst.rho, 1e-12, max_iter=3)
    assert R.status == 1 and R.info["iters"] == 3


# --------------------------------------------------------------------------
# FP32-rounded inputs and the certificate on a mid-size instance
# --------------------------------------------------------------------------
@pytest.mark.slow
def test_rounded_midsize_instance_bracket():
    inst = round_to(config_mixture_2d(0, 128, 160), np.float32)
    R = ref.solve(inst.C, inst.p, inst.q, inst.rho, 1e-4, max_iter=400_000)
    assert R.status == 0
    lb, ub = certify.bracket(inst.C, inst.p, inst.q, R.X, R.mu)
    opt = exact.lp_highs(inst.C, inst.p, inst.q)[0]
    assert lb <= opt * (1 + 1e-12) and opt <= ub * (1 + 1e-12)
    assert (ub - lb) / ub < 1e-3
    assert abs(R.info["pobj"] - opt) / opt < 1e-3


def test_paper_protocol_assignment_accuracy():
    """The paper's accuracy experiment: uniform marginals, rho0 = 2, stop on
    constraint violation; objective within 1e-3 of the assignment optimum
    (qualitative check: the paper prints no numbers)."""
    inst = paper_protocol(0, 128)
    opt = exact.assignment_uniform(inst.C)
    R = ref.solve(inst.C, inst.p, inst.q, inst.rho, 1e-4, max_iter=100_000)
    assert R.status == 0
    assert abs(R.info["pobj"] - opt) / opt < 1e-3


# --------------------------------------------------------------------------
# Warm-start MLP reference (not from the paper): pinned by finite differences
# --------------------------------------------------------------------------
def test_mlp_reference_gradient_matches_finite_differences():
    from oracle import mlp_ref
    rng = np.random.default_rng(5)
    dims = (6, 5, 4)
    n_par = 5 * 6 + 5 + 5 * 5 + 5 + 4 * 5 + 4
    theta = rng.standard_normal(n_par) * 0.5
    x = rng.standard_normal((7, 6))
    t = rng.standard_normal((7, 4))
    loss, g = mlp_ref.loss_and_grad(theta, x, t, dims, bf16=False)
    h = 1e-6
    fd = np.empty(n_par)
    for k in range(n_par):
        e = np.zeros(n_par)
        e[k] = h
        fd[k] = (mlp_ref.loss_and_grad(theta + e, x, t, dims, bf16=False)[0]
                 - mlp_ref.loss_and_grad(theta - e, x, t, dims, bf16=False)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)
    assert abs(loss - ((mlp_ref.forward(theta, x, dims, bf16=False) - t) ** 2).mean()) < 1e-15


def test_mlp_bf16_mode_equals_plain_network_on_bfloat16_exact_data():
    """Integer inputs and weights in {-2..2} and {-1, 0, 1}, integer biases
    and targets, batch 2 x 2 outputs (the loss divides by 4): every operand
    that the bfloat16 network rounds (inputs, weights, activations, the
    back-propagated gradients) is a small integer or half-integer, already a
    bfloat16 value, so the bfloat16 mode must equal the plain network exactly
    -- a dropped or misplaced term in either mode breaks this."""
    from oracle import mlp_ref
    rng = np.random.default_rng(8)
    dims = (2, 2, 2)
    n_par = 2 * 2 + 2 + 2 * 2 + 2 + 2 * 2 + 2
    for _ in range(20):
        theta = rng.integers(-1, 2, n_par).astype(np.float64)
        x = rng.integers(-2, 3, (2, 2)).astype(np.float64)
        t = rng.integers(-3, 4, (2, 2)).astype(np.float64)
        l16, g16 = mlp_ref.loss_and_grad(theta, x, t, dims, bf16=True)
        l64, g64 = mlp_ref.loss_and_grad(theta, x, t, dims, bf16=False)
        assert l16 == l64
        np.testing.assert_array_equal(g16, g64)
        np.testing.assert_array_equal(mlp_ref.forward(theta, x, dims, True),
                                      mlp_ref.forward(theta, x, dims, False))


def test_adam_two_steps_by_hand():
    """theta_0 = 1, gradients 1/2 then -1/4, lr 0.1, eps 0.  By hand:
    step 1: m = 1/20, v = 1/4000, m_hat = 1/2, v_hat = 1/4, theta_1 = 0.9;
    step 2: m = 9/10 * 1/20 - 1/40 = 1/50, v = 999/1000 * 1/4000 + 1/16000 =
    1249/4000000, m_hat = (1/50) / (1 - 0.81) = 2/19, v_hat = v / (1 - 0.998001)
    = 1249/7996, theta_2 = 0.9 - 0.1 (2/19) / sqrt(1249/7996) = 0.87336629603..."""
    from oracle import mlp_ref
    th, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    th, m, v = mlp_ref.adam_step(th, [0.5], m, v, 1, 0.1, eps=0.0)
    assert abs(th[0] - 0.9) < 1e-15 and abs(m[0] - 0.05) < 1e-16 and abs(v[0] - 2.5e-4) < 1e-18
    th, m, v = mlp_ref.adam_step(th, [-0.25], m, v, 2, 0.1, eps=0.0)
    assert abs(m[0] - 0.02) < 1e-16 and abs(v[0] - 1249 / 4e6) < 1e-18
    assert abs(th[0] - (0.9 - 0.2 / 19 * np.sqrt(7996 / 1249))) < 1e-15
    assert abs(th[0] - 0.8733662960339598) < 1e-14


def test_adam_constant_gradient_moves_lr_per_step():
    """With eps = 0 and the same gradient at every step, the bias corrections
    make m_hat = g and v_hat = g^2 exactly, so each coordinate moves by lr in
    the direction of -sign(g) per step whatever the gradient's magnitude; and
    the update is invariant to scaling the gradient."""
    from oracle import mlp_ref
    g = np.array([3e-4, -2.0, 50.0, -7e-6])
    th0 = np.array([0.5, -1.0, 2.0, 0.0])
    th, m, v = th0.copy(), np.zeros(4), np.zeros(4)
    ths, ms, vs = th0.copy(), np.zeros(4), np.zeros(4)
    for k in range(1, 11):
        th, m, v = mlp_ref.adam_step(th, g, m, v, k, 0.01, eps=0.0)
        ths, ms, vs = mlp_ref.adam_step(ths, 1000.0 * g, ms, vs, k, 0.01, eps=0.0)
        np.testing.assert_allclose(th, th0 - 0.01 * k * np.sign(g), rtol=0, atol=1e-13)
        np.testing.assert_allclose(ths, th, rtol=0, atol=1e-13)
    # eps bounds the step where the gradient is tiny: |update| <= lr |g| / eps
    th, _, _ = mlp_ref.adam_step(np.zeros(1), [1e-12], np.zeros(1), np.zeros(1), 1, 0.01)
    assert abs(th[0]) <= 0.01 * 1e-12 / 1e-8 * (1 + 1e-12)


def test_bf16_rounding_reference():
    from oracle import mlp_ref
    # exactly representable values stay; ties go to even; 1 + 2^-8 rounds down
    vals = np.array([1.0, 1.0 + 2.0 ** -7, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 0.0])
    out = mlp_ref.bf16_round(vals)
    np.testing.assert_array_equal(out, [1.0, 1.0 + 2.0 ** -7, 1.0, 1.0 + 2.0 ** -6, -2.5, 0.0])


def test_openmp_build_agrees_with_one_thread():
    """The OpenMP build of the oracle (rows split over threads, per-range
    partial sums added in range order) follows the one-thread oracle to
    rounding: 1e-12 relative on X_K, the shifts and every trace entry."""
    from gen import config_mixture_2d
    inst = config_mixture_2d(31, 301, 257)
    K = 60
    A = ref.solve(inst.C, inst.p, inst.q, inst.rho, 0.0, max_iter=K, trace=True)
    B = ref.solve(inst.C, inst.p, inst.q, inst.rho, 0.0, max_iter=K, trace=True, parallel=True)
    assert ref.threads() == 1 and ref.threads(parallel=True) >= 1
    for a, b in ((A.X, B.X), (A.phi, B.phi), (A.psi, B.psi), (A.trace, B.trace)):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    # the stopping iteration is the same
    A = ref.solve(inst.C, inst.p, inst.q, inst.rho, 1e-5, max_iter=200_000)
    B = ref.solve(inst.C, inst.p, inst.q, inst.rho, 1e-5, max_iter=200_000, parallel=True)
    assert A.info["iters"] == B.info["iters"]
