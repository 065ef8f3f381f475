"""Two checks from the paper's own experimental setup and from randomised
tiny inputs.

1. The accuracy experiment (experimental section): 100 problems of 512 x 512
   from the paper's Gaussian generator, uniform marginals, rho0 = 2, at most
   1000 iterations, stop at the 1e-4 test; the total error |<C,X> - OPT| / OPT
   + relative constraint violation against the exact assignment optimum.  The
   paper shows this profile only as a figure, so the test asserts what must
   hold whatever the figure says (finite errors, every run inside the cap,
   float32 within reach of float64) and prints the profile.
2. Tiny random problems (hypothesis): m, n in [1, 9], marginals with zeros,
   any nonnegative cost; the float64 trajectory must match the oracle's."""
import numpy as np
import pytest

from gen import paper_protocol
from oracle import exact, ref

pytestmark = pytest.mark.gpu


def _profile(errs):
    return {eps: float(np.mean(np.asarray(errs) <= eps)) for eps in (1e-2, 1e-3, 1e-4)}


def test_paper_accuracy_protocol():
    import torch
    from paper_2110_11738_amd import drot
    insts = [paper_protocol(i, 512) for i in range(100)]
    opts = np.array([exact.assignment_uniform(I.C) for I in insts])
    prof = {}
    for dtype in (torch.float64, torch.float32):
        probs = [{"C": drot.padded(torch.tensor(I.C, dtype=dtype, device="cuda")),
                  "p": torch.tensor(I.p, dtype=dtype, device="cuda"),
                  "q": torch.tensor(I.q, dtype=dtype, device="cuda"),
                  "rho": I.rho, "tol": 1e-4} for I in insts]
        rc, outs = drot.solve_batched(probs, max_iter=1000, check_every=50)
        torch.cuda.synchronize()
        errs = []
        for (X, r, mu, nu), opt in zip(outs, opts):
            assert r["iters"] <= 1000
            assert bool((X >= 0).all())
            errs.append(abs(r["objective"] - opt) / opt + r["eps_primal"])
        errs = np.array(errs)
        assert np.isfinite(errs).all()
        prof[str(dtype)] = _profile(errs)
        print(f"[protocol] {dtype}: median total error {np.median(errs):.2e}, "
              f"fraction below 1e-2/1e-3/1e-4: {prof[str(dtype)]}", flush=True)
    f64, f32 = prof["torch.float64"], prof["torch.float32"]
    # float32 rounding (2^-24) is far below these thresholds: the two profiles
    # may differ by a few problems near a threshold, not by a different shape.
    for eps in (1e-2, 1e-3):
        assert abs(f64[eps] - f32[eps]) <= 0.1


hyp = pytest.importorskip("hypothesis")
st = hyp.strategies


@hyp.settings(max_examples=40, deadline=None, derandomize=True)
@hyp.given(st.integers(1, 9), st.integers(1, 9), st.integers(0, 2**31 - 1))
def test_tiny_random_problems_match_oracle(m, n, seed):
    import torch
    from paper_2110_11738_amd import drot
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, 1.0, (m, n)) * rng.integers(0, 2, (m, n))  # zeros included
    # integer masses with a common total T: p = k / T, q = l / T (zeros allowed)
    T = 64
    k = rng.multinomial(T, np.ones(m) / m).astype(np.float64)
    l = rng.multinomial(T, np.ones(n) / n).astype(np.float64)
    p, q = k / T, l / T
    rho = 2.0 / (m + n)
    dev = torch.device("cuda:0")
    Ct = torch.tensor(C, dtype=torch.float64, device=dev)
    pt = torch.tensor(p, dtype=torch.float64, device=dev)
    qt = torch.tensor(q, dtype=torch.float64, device=dev)
    X, res, mu, nu = drot.solve(Ct, pt, qt, rho, tol=0.0, max_iter=20)
    torch.cuda.synchronize()
    R = ref.solve(C, p, q, rho, 0.0, max_iter=20)
    Xg = X.cpu().numpy()
    scale = max(np.abs(R.X).max(), 1e-300)
    assert np.abs(Xg - R.X).max() <= 1e-10 * scale
    assert np.abs(mu.cpu().numpy() - R.mu).max() <= 1e-9 * max(np.abs(R.mu).max(), 1.0)
