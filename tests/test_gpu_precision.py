"""Error of each precision form of the iteration against the exact optimum of
the same float32 problem (HiGHS on the CPU), solved to a tight tolerance:
dense float32 sums, compensated sums and the cost regenerated from float32
coordinates must land within the float32 objective bound (1e-4 relative);
the bfloat16 cost solves a perturbed problem whose optimum can move by at
most 2u/(1-u) relative (u = 2^-8, every c_ij within u of its float32 value),
plus the same float32 bound."""
import numpy as np
import pytest

from gen import config_cube_3d
from oracle import exact

pytestmark = pytest.mark.gpu


def test_precision_forms_error_against_lp():
    import torch
    from paper_2110_11738_amd import drot
    inst = config_cube_3d(5, 120, 180)
    m, n = inst.m, inst.n
    C32 = inst.C.astype(np.float32)
    p32, q32 = inst.p.astype(np.float32), inst.q.astype(np.float32)
    opt = exact.lp_highs(C32.astype(np.float64), p32.astype(np.float64),
                         q32.astype(np.float64))[0]
    dev = torch.device("cuda:0")
    C = torch.from_numpy(C32).to(dev)
    Cb = C.to(torch.bfloat16)
    xs = torch.from_numpy(inst.xs.astype(np.float32)).to(dev)
    xt = torch.from_numpy(inst.xt.astype(np.float32)).to(dev)
    p, q = torch.from_numpy(p32).to(dev), torch.from_numpy(q32).to(dev)
    rho = 2.0 / (m + n)
    u = 2.0 ** -8
    forms = [("dense", drot.COST_DENSE, 0, 1e-4),
             ("compensated", drot.COST_DENSE, drot.FLAG_COMPENSATED, 1e-4),
             ("coords", drot.COST_COORDS, 0, 1e-4),
             ("bf16", drot.COST_BF16, 0, 2 * u / (1 - u) + 1e-4)]
    for name, kind, flags, bound in forms:
        X, res, mu, nu = drot.solve_cost(m, n, p, q, rho, kind, C=C if kind == drot.COST_DENSE
                                         else Cb, xs=xs, xt=xt, scale=float(inst.cscale),
                                         tol=1e-6, max_iter=2_000_000, flags=flags)
        torch.cuda.synchronize()
        # The objective of the returned plan under the float32 cost.
        obj = float((X.double() * C.double()).sum())
        err = abs(obj - opt) / opt
        print(f"[precision] {name}: {res['iters']} iterations, objective error {err:.2e} "
              f"(bound {bound:.1e}), status {res['status']}", flush=True)
        assert res["status"] == drot.OK
        assert err <= bound
