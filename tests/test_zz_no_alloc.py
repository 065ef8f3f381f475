"""drot_solve_noalloc (the entry point that allocates nothing: its workspace
is the library's static device scratch) against drot_solve on the same
inputs: two calls in a row, the second with a smaller problem, then a problem
on the one-workgroup path, each bit for bit equal to drot_solve (the
iterations, the plan, the duals and every reported figure; both paths run
the same kernels in the same order).  Problems whose workspace exceeds the
scratch are refused before any device work."""
import numpy as np
import pytest

from gen import config_mixture_2d, round_to

pytestmark = pytest.mark.gpu

FIELDS = ("iters", "status", "path", "objective", "dual_objective", "r_primal", "r_dual", "gap",
          "eps_primal", "eps_dual", "eps_gap")


def _inputs(seed, m, n, dtype):
    import torch
    inst = round_to(config_mixture_2d(seed, m, n), np.float32) if dtype == "float32" else \
        config_mixture_2d(seed, m, n)
    dt = torch.float32 if dtype == "float32" else torch.float64
    t = lambda a: torch.tensor(a, dtype=dt, device="cuda")
    return inst, t(inst.C), t(inst.p), t(inst.q)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_noalloc_matches_drot_solve(dtype):
    import torch
    from paper_2110_11738_amd import drot
    ctx = drot.Context(0)
    try:
        for seed, (m, n), K, tol in ((1, (700, 900), 60, 0.0), (2, (300, 260), 5000, 1e-4),
                                     (3, (60, 70), 300, 0.0)):
            print(f"[noalloc] {dtype} {m}x{n} K={K} tol={tol}", flush=True)
            inst, C, p, q = _inputs(seed, m, n, dtype)
            prm = drot.make_params(inst.rho, tol, K, check_every=16)
            mu_a = torch.empty(m, dtype=torch.float64, device="cuda")
            nu_a = torch.empty(n, dtype=torch.float64, device="cuda")
            Xa, ra = ctx.solve(C, p, q, prm, mu=mu_a, nu=nu_a)
            Xb = torch.full_like(C, -1.0)
            mu_b = torch.empty(m, dtype=torch.float64, device="cuda")
            nu_b = torch.empty(n, dtype=torch.float64, device="cuda")
            rc, rb = drot.solve_noalloc(C, p, q, prm, Xb, mu_b, nu_b)
            torch.cuda.synchronize()
            print(f"    iters {ra['iters']} / {rb['iters']}, path {rb['path']}, "
                  f"objective {ra['objective']!r} / {rb['objective']!r}", flush=True)
            for f in FIELDS:
                assert ra[f] == rb[f], f
            assert torch.equal(Xa, Xb)
            assert torch.equal(mu_a, mu_b) and torch.equal(nu_a, nu_b)
    finally:
        ctx.close()


def test_noalloc_refuses_oversized_problems():
    import torch
    from paper_2110_11738_amd import drot
    m = n = 11000  # the float32 limit is about 9984 x 9984
    C = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    p = torch.full((m,), 1.0 / m, dtype=torch.float32, device="cuda")
    X = torch.empty_like(C)
    with pytest.raises(drot.DrotError, match="static scratch"):
        drot.solve_noalloc(C, p, p, drot.make_params(1e-5, 0.0, 10), X)
    with pytest.raises(drot.DrotError):
        drot.solve_noalloc(C[:100, :100], p[:100], p[:100],
                           drot.make_params(1e-5, 0.0, 10, flags=drot.FLAG_TIME_SWEEP),
                           X[:100, :100])
