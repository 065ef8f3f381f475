"""Full-size checks in the launch configuration the benchmark times (default
tiles, float32): 4096 x 4096 and the 20000 x 20000 roofline instance.  The
oracle cannot replay these trajectories, so the checks are (a) sampled
outputs the oracle's arithmetic gives one by one -- rows of X_{K+1} from the
downloaded X_K and duals (Algorithm 1, step 4) -- and (b) properties that hold
at any size: X >= 0, the objective and residuals of the final pass against
float64 sums of the returned plan on the host, sum(phi) = sum(psi)."""
import numpy as np
import pytest

from gen import config_mixture_2d

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("side,tag", [(4096, 2), (20000, 3)])
def test_full_size_sweep_and_final_pass(side, tag):
    import torch
    from paper_2110_11738_amd import drot
    print(f"[full size] {side}x{side}", flush=True)
    inst = config_mixture_2d(0, side, side, seed_tag=tag)
    C32 = inst.C.astype(np.float32)
    p32, q32 = inst.p.astype(np.float32), inst.q.astype(np.float32)
    del inst.C
    dev = torch.device("cuda:0")
    C = torch.from_numpy(C32).to(dev)
    p, q = torch.from_numpy(p32).to(dev), torch.from_numpy(q32).to(dev)
    X = torch.empty_like(C)
    ctx = drot.Context(0)
    try:
        K = 64
        rho = inst.rho
        ctx.bind(C, p, q, X, drot.make_params(rho, 0.0, K + 2, check_every=32))
        ctx.iterate(K)
        mu = torch.empty(side, dtype=torch.float64, device=dev)
        nu = torch.empty(side, dtype=torch.float64, device=dev)
        res = ctx.finish(mu, nu)
        torch.cuda.synchronize()
        rows = np.random.default_rng(side).choice(side, 48, replace=False)
        XK = X[torch.from_numpy(rows).to(dev)].double().cpu().numpy()
        mu_h, nu_h = mu.cpu().numpy(), nu.cpu().numpy()
        Xh = X.cpu().numpy()
        # (b) properties at iterate K
        assert res["iters"] == K
        assert (Xh >= 0).all()
        obj = float(np.einsum("ij,ij->", Xh.astype(np.float64), C32.astype(np.float64)))
        assert abs(res["objective"] - obj) <= 1e-9 * abs(obj)
        r = Xh.sum(axis=1, dtype=np.float64) - p32
        s = Xh.sum(axis=0, dtype=np.float64) - q32
        rp = float(np.sqrt((r * r).sum() + (s * s).sum()))
        assert abs(res["r_primal"] - rp) <= 1e-9 * rp + 1e-15
        assert abs(mu_h.sum() - nu_h.sum()) <= 1e-9 * max(np.abs(mu_h).sum(), 1e-300)
        dobj = float(p32.astype(np.float64) @ mu_h + q32.astype(np.float64) @ nu_h)
        assert abs(res["dual_objective"] - dobj) <= 1e-9 * abs(dobj)
        del Xh
        # (a) one more iteration, sampled rows against the step computed here
        ctx.iterate(1)
        torch.cuda.synchronize()
        XK1 = X[torch.from_numpy(rows).to(dev)].double().cpu().numpy()
        Cr = C32[rows].astype(np.float64)
        t = XK + rho * mu_h[rows][:, None] + rho * nu_h[None, :] - rho * Cr
        want = np.maximum(t, 0.0)
        scale = np.abs(XK) + rho * (np.abs(mu_h[rows])[:, None] + np.abs(nu_h)[None, :] + Cr)
        err = np.abs(XK1 - want)
        print(f"[full size] {side}: max |X_K+1 - step| / scale = {(err / scale).max():.2e}", flush=True)
        # The sweep adds float32 roundings of phi's vector part, of the shared
        # scalar part and of psi (measured: at most 1.3e-7 of the scale, two
        # float32 roundings); 1e-6 leaves room for cancellation between the two
        # parts of phi and still exposes any wrong index, sign or operand,
        # which moves entries by O(1) of the scale.
        assert (err <= 1e-6 * scale + 1e-30).all()
    finally:
        ctx.close()
