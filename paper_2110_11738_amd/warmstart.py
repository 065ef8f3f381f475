"""Learned warm start for DROT on grid histograms (not part of the paper).

A network maps the marginals (p, q) of a problem on a 32 x 32 grid to initial
dual variables (mu, nu); DROT then starts from phi_0 = rho mu, psi_0 = rho nu
(valid from any start by Lemma 1); cold DROT remains the fallback, and the
warm-started run meets the same stopping test.  Everything numerical runs on the GPU through
libdrot.so: the training targets come from DROT itself (batched solver), and
the network is trained and evaluated with the library's MLP kernels.

    python -m paper_2110_11738_amd.warmstart --train 4096 --test 512

Targets are gauge-fixed: (mu, nu) and (mu + t, nu - t) describe the same
duals, so the pair with mean(mu) = 0 is learned.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from gen import grid_cost, grid_histogram_pair  # noqa: E402

from . import drot  # noqa: E402

SIDE = 32  # grid side of the default experiment (N = SIDE^2 cells per histogram)


def log(msg):
    print(f"[warmstart] {msg}", file=sys.stderr, flush=True)


def rho_grid(rho0: float | None = None, side: int = SIDE) -> float:
    """rho = rho0 / (m + n) with m = n = side^2; rho0 = 1 / ln m unless given."""
    N = side * side
    r0 = 1.0 / math.log(N) if rho0 is None else rho0
    return r0 / (2 * N)


def features(ps: np.ndarray, qs: np.ndarray) -> np.ndarray:
    """Network input: the two histograms scaled by the grid size (mean 1)."""
    N = ps.shape[1]
    return np.concatenate([ps * N, qs * N], axis=1).astype(np.float32)


def gauge_fix(mu: np.ndarray, nu: np.ndarray) -> np.ndarray:
    t = mu.mean(axis=1, keepdims=True)
    return np.concatenate([mu - t, nu + t], axis=1).astype(np.float32)


def make_pairs(count: int, split: int, start: int = 0, side: int = SIDE):
    ps = np.empty((count, side * side))
    qs = np.empty((count, side * side))
    for k in range(count):
        ps[k], qs[k] = grid_histogram_pair(start + k, split, side)
    return ps, qs


def solve_pairs(ctx, C, ps, qs, tol=1e-4, max_iter=500_000, mu0=None, nu0=None, chunk=128,
                rho0=None, quiet=False):
    """Solve every pair with the batched GPU solver (shared cost matrix), in
    chunks of `chunk` problems.  Returns mu, nu (float64, per pair),
    iterations, device seconds, objectives, statuses."""
    import torch
    dev = C.device
    out_mu, out_nu, iters, secs, objs, status = [], [], [], [], [], []
    rho = rho_grid(rho0, int(round(math.sqrt(ps.shape[1]))))
    for s in range(0, len(ps), chunk):
        probs = []
        for k in range(s, min(s + chunk, len(ps))):
            pr = {"C": C, "p": torch.tensor(ps[k], dtype=torch.float32, device=dev),
                  "q": torch.tensor(qs[k], dtype=torch.float32, device=dev),
                  "rho": rho, "tol": tol}
            if mu0 is not None:
                pr["mu0"] = torch.tensor(mu0[k], dtype=torch.float64, device=dev)
                pr["nu0"] = torch.tensor(nu0[k], dtype=torch.float64, device=dev)
            probs.append(pr)
        rc, outs = drot.solve_batched(probs, max_iter=max_iter, check_every=64, ctx=ctx)
        for X, r, mu, nu in outs:
            out_mu.append(mu.cpu().numpy())
            out_nu.append(nu.cpu().numpy())
            iters.append(r["iters"])
            secs.append(r["seconds_to_tol"])
            objs.append(r["objective"])
            status.append(r["status"])
        if not quiet:
            log(f"solved {min(s + chunk, len(ps))}/{len(ps)} (mean iterations {np.mean(iters):.0f})")
    return (np.array(out_mu), np.array(out_nu), np.array(iters), np.array(secs), np.array(objs),
            np.array(status))


def train(net, X, T, epochs: int, batch: int, lr: float, seed: int = 0, quiet: bool = False):
    """Adam over shuffled mini-batches (the last partial batch is dropped)."""
    import torch
    rng = np.random.default_rng(seed)
    Xd = torch.tensor(X, device="cuda")
    Td = torch.tensor(T, device="cuda")
    losses = []
    for ep in range(epochs):
        order = torch.tensor(rng.permutation(len(X)), device="cuda")
        tot = 0.0
        nb = len(X) // batch
        for b in range(nb):
            idx = order[b * batch:(b + 1) * batch]
            tot += net.train_step(Xd[idx].contiguous(), Td[idx].contiguous(), lr)
        losses.append(tot / max(nb, 1))
        if not quiet and (ep % 10 == 0 or ep == epochs - 1):
            log(f"epoch {ep}: loss {losses[-1]:.4e}")
    return losses


def predict(net, X, batch: int):
    """Network outputs for every row of X (padding the last batch)."""
    import torch
    out = []
    for s in range(0, len(X), batch):
        xb = np.zeros((batch, X.shape[1]), dtype=np.float32)
        part = X[s:s + batch]
        xb[:len(part)] = part
        y = net.forward(torch.tensor(xb, device="cuda")).cpu().numpy()
        out.append(y[:len(part)])
    Y = np.concatenate(out).astype(np.float64)
    N = Y.shape[1] // 2
    return Y[:, :N], Y[:, N:]


def canonical(Cn: np.ndarray, mu: np.ndarray, nu: np.ndarray):
    """Double c-transform of each pair: nu' = min_i (C_i. - mu_i), then
    mu' = min_j (C_.j - nu'_j).  The result is dual feasible, no worse than
    (mu, nu) on the LP dual, equal to it where the optimal duals are unique,
    and fixes the values where they are not (cells without mass) to the
    c-concave extension, which is a function of the problem rather than of
    the solver's path."""
    mu2 = np.empty_like(mu)
    nu2 = np.empty_like(nu)
    for k in range(len(mu)):
        nu2[k] = (Cn - mu[k][:, None]).min(axis=0)
        mu2[k] = (Cn - nu2[k][None, :]).min(axis=1)
    return mu2, nu2


def solved_data(ctx, C, ps, qs, tol, rho0, path, tag, quiet=False):
    """solve_pairs, cached in an .npz file (path may be None)."""
    key = f"{tag}_"
    if path and os.path.exists(path):
        z = np.load(path)
        if key + "mu" in z.files and len(z[key + "mu"]) == len(ps):
            log(f"loaded {tag} solutions from {path}")
            return tuple(z[key + f] for f in ("mu", "nu", "it", "sec", "obj", "st"))
    out = solve_pairs(ctx, C, ps, qs, tol, rho0=rho0, quiet=quiet)
    if path:
        old = dict(np.load(path)) if os.path.exists(path) else {}
        for f, v in zip(("mu", "nu", "it", "sec", "obj", "st"), out):
            old[key + f] = v.astype(np.float32) if f in ("mu", "nu") else v
        np.savez(path, **old)
    return out


def run(n_train: int, n_test: int, epochs: int, batch: int, lr: float, tol: float,
        hidden: int = 512, seed: int = 0, rho0: float | None = None, data: str | None = None,
        canon: bool = True, side: int = SIDE, quiet: bool = False,
        train_files: list | None = None) -> dict:
    """Solve (or load, from generate() files) the training pairs, train the
    network, and solve the held-out pairs cold and warm.  The warm time per
    pair includes the network's forward pass (its share of the batched
    inference)."""
    import torch
    N = side * side
    ctx = drot.Context(0)
    Cn = grid_cost(side)
    C = torch.tensor(Cn, dtype=torch.float32, device="cuda")
    t0 = time.time()
    if train_files:
        T, it_train, st_train = load_targets(train_files, side)
        n_train = len(T) if n_train <= 0 else min(n_train, len(T))
        T, it_train, st_train = T[:n_train], it_train[:n_train], st_train[:n_train]
    ps, qs = make_pairs(n_train, 0, side=side)
    pt, qt = make_pairs(n_test, 1, side=side)
    log(f"generated {n_train} + {n_test} pairs in {time.time() - t0:.1f}s")
    t0 = time.time()
    if not train_files:
        mu, nu, it_train, _, _, st_train = solved_data(ctx, C, ps, qs, tol, rho0, data, "train",
                                                       quiet)
        mu, nu = mu.astype(np.float64), nu.astype(np.float64)
        if canon:
            mu, nu = canonical(Cn, mu, nu)
        T = gauge_fix(mu, nu)
    t_data = time.time() - t0
    X = features(ps, qs)
    # Standardised targets (per output: training mean and one global scale).
    t_mean = T.mean(axis=0, keepdims=True)
    t_scale = float(T.std()) or 1.0
    net = drot.MLP(2 * N, hidden, 2 * N, max_batch=max(batch, 64), seed=seed)
    t0 = time.time()
    losses = train(net, X, ((T - t_mean) / t_scale).astype(np.float32), epochs, batch, lr, seed,
                   quiet)
    t_train = time.time() - t0
    log(f"trained {epochs} epochs in {t_train:.1f}s, loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    # held-out: cold vs warm (the warm solve falls back to cold if it fails)
    mu_c, nu_c, it_c, s_c, obj_c, st_c = solved_data(ctx, C, pt, qt, tol, rho0, data, "test",
                                                       quiet)
    mu_c, nu_c = mu_c.astype(np.float64), nu_c.astype(np.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mu_hat, nu_hat = predict(net, features(pt, qt), max(batch, 64))
    t_infer = (time.perf_counter() - t0) / n_test  # host-side features and transfers included
    mu_hat = mu_hat * t_scale + t_mean[0, :N]
    nu_hat = nu_hat * t_scale + t_mean[0, N:]
    mu_w, nu_w, it_w, s_w, obj_w, st_w = solve_pairs(ctx, C, pt, qt, tol, mu0=mu_hat, nu0=nu_hat,
                                                     rho0=rho0, quiet=quiet)
    fallback = st_w != 0
    it_w_eff = np.where(fallback, it_w + it_c, it_w)
    rel_obj = np.abs(obj_w - obj_c) / np.abs(obj_c)
    Tt = gauge_fix(*(canonical(Cn, mu_c, nu_c) if canon else (mu_c, nu_c)))
    pred_err = float(np.sqrt(((np.concatenate([mu_hat, nu_hat], 1) - Tt) ** 2).mean()))
    spread = float(np.sqrt(((Tt - Tt.mean(axis=0)) ** 2).mean()))
    report = {
        "train_pairs": n_train, "test_pairs": n_test, "epochs": epochs, "batch": batch, "lr": lr,
        "tol": tol, "hidden": hidden, "rho0": rho0 if rho0 is not None else 1.0 / math.log(N),
        "side": side, "rho": rho_grid(rho0, side), "canonical_targets": canon, "seconds_data": t_data,
        "seconds_train": t_train,
        "train_iters_mean": float(it_train.mean()), "train_unconverged": int((st_train != 0).sum()),
        "loss_first": losses[0], "loss_last": losses[-1],
        "test_rmse_duals": pred_err, "test_rmse_of_mean_predictor": spread,
        "cold_iters_mean": float(it_c.mean()), "cold_iters_median": float(np.median(it_c)),
        "warm_iters_mean": float(it_w_eff.mean()), "warm_iters_median": float(np.median(it_w_eff)),
        "cold_seconds_mean": float(s_c.mean()), "warm_seconds_mean": float(s_w.mean()),
        "inference_seconds_per_pair": t_infer,
        "warm_seconds_with_inference_mean": float(s_w.mean()) + t_infer,
        "seconds_ratio_with_inference": (float(s_w.mean()) + t_infer) / float(s_c.mean()),
        "warm_fallbacks": int(fallback.sum()),
        "objective_rel_diff_warm_vs_cold_max": float(rel_obj.max()),
        "iteration_ratio_mean": float(it_w_eff.mean() / it_c.mean()),
    }
    net.close()
    ctx.close()
    return report


def generate(out: str, count: int, start: int, split: int, tol: float, rho0: float | None,
             chunk: int = 512, side: int = SIDE, canon: bool = True) -> None:
    """Solve pairs [start, start + count) of a split with the batched solver
    and save their gauge-fixed (double c-transformed) duals as float16 with
    the iteration counts and statuses, `chunk` pairs per batch, the file
    rewritten after every batch.  The histograms are not stored: they are
    regenerated from their seeds."""
    import torch
    ctx = drot.Context(0)
    Cn = grid_cost(side)
    C = torch.tensor(Cn, dtype=torch.float32, device="cuda")
    T, its, sts = [], [], []
    t0 = time.time()
    for s0 in range(start, start + count, chunk):
        n = min(chunk, start + count - s0)
        ps, qs = make_pairs(n, split, start=s0, side=side)
        mu, nu, it, _, _, st = solve_pairs(ctx, C, ps, qs, tol, rho0=rho0, chunk=n, quiet=True)
        if canon:
            mu, nu = canonical(Cn, mu, nu)
        T.append(gauge_fix(mu, nu).astype(np.float16))
        its.append(it)
        sts.append(st)
        np.savez(out, targets=np.concatenate(T), iters=np.concatenate(its),
                 status=np.concatenate(sts), start=start, split=split, tol=tol,
                 rho0=-1.0 if rho0 is None else rho0, side=side)
        log(f"pairs {start}..{s0 + n} of split {split}: mean iterations "
            f"{np.concatenate(its).mean():.0f}, {time.time() - t0:.0f}s")
    ctx.close()


def load_targets(paths, side: int = SIDE):
    """Concatenate generate() files of split 0 (contiguous ranges from 0)."""
    T, its, sts, n = [], [], [], 0
    for path in sorted(paths, key=lambda q: int(np.load(q)["start"])):
        z = np.load(path)
        if int(z["start"]) != n or int(z["split"]) != 0 or int(z["side"]) != side:
            raise ValueError(f"{path}: not the next contiguous range of training pairs")
        T.append(z["targets"].astype(np.float32))
        its.append(z["iters"])
        sts.append(z["status"])
        n += len(z["targets"])
    return np.concatenate(T), np.concatenate(its), np.concatenate(sts)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--test", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--hidden", type=int, default=512)
    ap.add_argument("--rho0", type=float, default=None, help="rho = rho0 / (m + n); default 1 / ln m")
    ap.add_argument("--data", default=None, help=".npz cache of the solved training and test pairs")
    ap.add_argument("--raw-targets", action="store_true", help="learn the solver's duals as returned")
    ap.add_argument("--side", type=int, default=SIDE, help="grid side (histograms of side^2 cells)")
    ap.add_argument("--gen", default=None, help="only solve training pairs into this .npz")
    ap.add_argument("--gen-start", type=int, default=0)
    ap.add_argument("--train-files", default=None,
                    help="comma-separated generate() files with the training targets")
    args = ap.parse_args()
    if args.gen:
        generate(args.gen, args.train, args.gen_start, 0, args.tol, args.rho0, side=args.side)
        return
    rep = run(args.train, args.test, args.epochs, args.batch, args.lr, args.tol, args.hidden,
              rho0=args.rho0, data=args.data, canon=not args.raw_targets, side=args.side,
              train_files=args.train_files.split(",") if args.train_files else None)
    print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
