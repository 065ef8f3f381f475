"""Benchmark of the DROT hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-large] [--no-cpu]
                    [--no-tol] [--tile-rows R] [--tile-chunks H] [--check-every G]

A step is one DROT iteration (Algorithm 1): the fused sweep over the dense
m x n plan plus the O(m+n) dual update and the stopping test.  The timed
workload is the 4096 x 4096 float32 problem (2-D five-Gaussian point clouds,
squared-Euclidean cost normalised to max 1, Dirichlet(1) marginals,
rho = (1/ln m)/(m+n)), resident in HBM before timing starts.  One JSON line
is printed with iterations/s at 4096^2 (`value`: whole graph replays, no
events), the roofline of the sweep kernel on the 20000 x 20000 instance
(3.2 GB, the HBM-bound size; a timed region of eager launches, every sweep
carrying hipExtLaunchKernel start/stop events), the times to the 1e-4
relative stopping test at 4096^2 and 20000^2, the precision forms, the
batched solver and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E peak
BYTES_PER_ENTRY_F32 = 12     # read X, write X, read C (float32)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_instance(m, n, upcast=True):
    """The mixture2d instance rounded to float32 (C kept as float32 when
    `upcast` is False, which the large instance uses to save host memory)."""
    import numpy as np
    from gen import config_mixture_2d, round_to
    t0 = time.time()
    inst = config_mixture_2d(0, m, n, seed_tag=2 if m == n == 4096 else 3)
    if upcast:
        inst = round_to(inst, np.float32)
    else:
        inst.C = inst.C.astype(np.float32)
    log(f"generated {inst.name} in {time.time() - t0:.1f}s")
    return inst


def upload(inst):
    import torch
    dev = torch.device("cuda:0")
    C = torch.from_numpy(inst.C.astype("float32", copy=False)).to(dev)
    p = torch.from_numpy(inst.p.astype("float32")).to(dev)
    q = torch.from_numpy(inst.q.astype("float32")).to(dev)
    return C, p, q


def pmc_summary(m, n):
    return os.path.join(ROOT, "profiles", f"sweep_aux_f32_{m}x{n}.txt")


def source_digest(path):
    """sha256 of a C/HIP source with its comments and blank lines removed, so
    that the recorded counters stay attached to the code they measured and
    survive edits of comments only."""
    import hashlib
    import re
    with open(path, encoding="utf-8") as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    lines = [ln.rstrip() for ln in text.splitlines() if ln.strip()]
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def pmc_traffic(m, n):
    """HBM bytes per sweep launch measured with rocprofv3 FETCH_SIZE and
    WRITE_SIZE (scaled by a plain copy of known size), read from the profile
    summary; None unless it covers this workload and the kernel sources still
    have the code digests (source_digest) recorded with the counters."""
    try:
        lines = open(pmc_summary(m, n)).read().splitlines()
    except OSError:
        return None
    kv, hashes = {}, {}
    for line in lines:
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        if parts[0] == "source_digest" and len(parts) == 3:
            hashes[parts[1]] = parts[2]
        else:
            kv[parts[0]] = " ".join(parts[1:])
    if kv.get("workload") != f"{m}x{n} float32" or not hashes:
        return None
    for rel, h in hashes.items():
        try:
            if source_digest(os.path.join(ROOT, rel)) != h:
                return None
        except OSError:
            return None
    return float(kv["sweep_traffic_bytes"])


def graph_size(steps, check_every):
    """Iterations per captured graph for a timed region of `steps`: the
    largest divisor of `steps` not above `check_every`, so that the timed
    region is whole graph replays."""
    return max(d for d in range(1, max(1, min(steps, check_every)) + 1) if steps % d == 0)


def timed_run(ctx, bind, steps, warmup, flags):
    """Bind with `flags` (bind(flags, max_iter)), capture the graph, run
    `warmup` iterations, then time exactly `steps`.  Returns (seconds,
    average sweep ms or None, sweeps timed)."""
    import torch
    bind(flags, warmup + steps + 1)
    ctx.iterate(0)  # graph capture, outside the timed region
    if warmup:
        ctx.iterate(warmup)
    torch.cuda.synchronize()
    before = ctx.finish()  # read-only final pass: sweep counters so far
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.iterate(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = ctx.finish()
    assert res["iters"] == warmup + steps, res
    cnt = res["sweep_timed"] - before["sweep_timed"]
    avg = (res["sweep_ms_total"] - before["sweep_ms_total"]) / cnt if cnt > 0 else None
    return t1 - t0, avg, cnt


def measure(ctx, bind, steps, warmup, flags=0):
    """Two timed regions of the same workload: graph replays without events
    (the throughput), then eager launches in which every sweep carries
    hipExtLaunchKernel start/stop events (the sweep kernel's own average
    duration, the figure the roofline uses)."""
    from paper_2110_11738_amd import drot
    secs, _, _ = timed_run(ctx, bind, steps, warmup, flags)
    esecs, ms, cnt = timed_run(ctx, bind, steps, warmup,
                               flags | drot.FLAG_NO_GRAPH | drot.FLAG_TIME_SWEEP)
    return {"seconds": secs, "seconds_eager": esecs, "sweep_ms": ms, "sweeps_timed": cnt}


def dense_binder(ctx, C, p, q, rho, args, tile=None):
    """bind(flags, max_iter) for the dense problem; `tile` (rows, chunks,
    groups) overrides the command-line tile options."""
    import torch
    from paper_2110_11738_amd import drot
    X = torch.empty(C.shape, dtype=C.dtype, device=C.device)
    rows, chunks, groups = tile if tile else (args.tile_rows, args.tile_chunks, args.tile_groups)

    def bind(flags, max_iter):
        prm = drot.make_params(rho, 0.0, max_iter, check_every=bind.check_every, flags=flags,
                               tile_rows=rows, tile_chunks=chunks,
                               tile_unroll=args.tile_unroll, cache_mode=args.cache_mode,
                               tile_groups=groups)
        ctx.bind(C, p, q, X, prm)
    bind.X = X
    bind.check_every = args.check_every
    return bind


def tuned_tile(ctx, bind, iters=64):
    """Run drot_tune on the bound problem; returns (rows, chunks, groups)."""
    bind(0, 10)
    best, us = ctx.tune(iters)
    log(f"tuned tile: rows {best.tile_rows}, chunks {best.tile_chunks}, groups "
        f"{best.tile_groups} ({us:.1f} us/iteration while tuning)")
    return best.tile_rows, best.tile_chunks, best.tile_groups


def cost_binder(ctx, m, n, cost, p, q, rho, keep):
    from paper_2110_11738_amd import drot
    import torch
    X = drot.empty_plan(m, n, torch.float32, "cuda")

    def bind(flags, max_iter):
        prm = drot.make_params(rho, 0.0, max_iter, check_every=64, flags=flags)
        ctx.bind_cost(m, n, cost, p, q, X, prm, keep=keep)
    return bind


def precision_section(ctx, steps=200, warmup=20):
    """10000 x 15000, points uniform in the unit cube of R^3: the same
    iteration with C dense float32 (12 B/entry), bfloat16 (10 B/entry) and
    regenerated from float32 coordinates (8 B/entry)."""
    import numpy as np
    import torch
    from gen import config_cube_3d
    from paper_2110_11738_amd import drot
    t0 = time.time()
    inst = config_cube_3d(0)
    m, n = inst.m, inst.n
    log(f"generated {inst.name} in {time.time() - t0:.1f}s")
    # rows of C and X start on 128-byte cache lines (leading dimension 15008)
    C32 = drot.padded(torch.from_numpy(inst.C.astype(np.float32)).cuda())
    Cb = drot.padded(C32.to(torch.bfloat16))
    xs = torch.from_numpy(inst.xs.astype(np.float32)).cuda()
    xt = torch.from_numpy(inst.xt.astype(np.float32)).cuda()
    p = torch.from_numpy(inst.p.astype(np.float32)).cuda()
    q = torch.from_numpy(inst.q.astype(np.float32)).cuda()
    rho = inst.rho
    scale = float(inst.cscale)
    del inst
    out = {"m": m, "n": n, "workload": "cube3d 10000x15000 float32 X",
           "leading_dimension": C32.stride(0)}
    for name, kind, keep, bpe, fl in (
            ("dense_f32", drot.COST_DENSE, (C32,), 12, 0),
            ("dense_f32_compensated", drot.COST_DENSE, (C32,), 12, drot.FLAG_COMPENSATED),
            ("bf16", drot.COST_BF16, (Cb,), 10, 0),
            ("coords", drot.COST_COORDS, (xs, xt), 8, 0)):
        cost = drot.make_cost(kind, C=C32 if kind == drot.COST_DENSE else Cb, xs=xs, xt=xt,
                              scale=scale)
        r = measure(ctx, cost_binder(ctx, m, n, cost, p, q, rho, keep), steps, warmup, fl)
        secs, sw = r["seconds"], r["sweep_ms"]
        ach = bpe * m * n / (sw * 1e-3) / 1e9
        out[name] = {"iter_per_s": steps / secs, "sweep_us": sw * 1e3, "bytes_per_entry": bpe,
                     "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS}
        log(f"precision {name}: {steps / secs:.1f} it/s, sweep {sw * 1e3:.1f} us, "
            f"{ach:.0f} GB/s ({bpe} B/entry)")
    del C32, Cb, xs, xt
    torch.cuda.empty_cache()
    return out


def batch_section(ctx, count=512, iters=100, tol_rho0=2.0, tol=1e-4, n_seq=32, do_tol=True,
                  one_by_one=True):
    """512 ragged problems (m, n uniform in [64, 2048]): the tuner's schedules
    per size class (drot_tune_batched), a fixed number of iterations batched
    against the same problems one by one, and every problem solved to the
    1e-4 relative test batched against the first n_seq of them one by one."""
    import numpy as np
    import torch
    from gen import config_batch
    from paper_2110_11738_amd import drot
    t0 = time.time()
    insts = config_batch(count)
    log(f"generated {count} batch problems in {time.time() - t0:.1f}s")
    probs = []
    entries = 0
    for I in insts:
        probs.append({"C": drot.padded(torch.from_numpy(I.C.astype(np.float32)).cuda()),
                      "p": torch.from_numpy(I.p.astype(np.float32)).cuda(),
                      "q": torch.from_numpy(I.q.astype(np.float32)).cuda(),
                      "rho": I.rho, "tol": 0.0, "m": I.m, "n": I.n})
        entries += I.m * I.n
    del insts
    drot.solve_batched(probs[:8], max_iter=5, ctx=ctx)  # warm-up
    torch.cuda.synchronize()
    # untuned (default schedule: items of about 65 536 entries)
    t0 = time.perf_counter()
    rc, outs = drot.solve_batched(probs, max_iter=iters, check_every=50, ctx=ctx)
    torch.cuda.synchronize()
    t_untuned = time.perf_counter() - t0
    del outs
    t0 = time.perf_counter()
    table = drot.tune_batched(probs, iters=64, check_every=32, ctx=ctx)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    log(f"batch tuner: {len(table)} size classes in {t_tune:.1f}s")
    t0 = time.perf_counter()
    rc, outs = drot.solve_batched(probs, max_iter=iters, check_every=50, ctx=ctx)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    assert all(o[1]["iters"] == iters for o in outs)
    del outs
    # steady state: the difference of two runs (setup, initialisation and the
    # final pass cancel)
    t0 = time.perf_counter()
    rc, outs = drot.solve_batched(probs, max_iter=3 * iters, check_every=50, ctx=ctx)
    torch.cuda.synchronize()
    t_batch3 = time.perf_counter() - t0
    del outs
    per_iter = (t_batch3 - t_batch) / (2 * iters)
    gbs_ss = 12.0 * entries / per_iter / 1e9
    log(f"batched steady state: {per_iter * 1e3:.3f} ms per iteration, {gbs_ss:.0f} GB/s "
        f"({100 * gbs_ss / HBM_PEAK_GBS:.1f}% of peak)")
    # the same with the default schedule (a fresh context has an empty tuner cache)
    ctx_u = drot.Context(ctx.device)
    drot.solve_batched(probs[:8], max_iter=5, ctx=ctx_u)
    tu = []
    for k in (iters, 3 * iters):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, outs = drot.solve_batched(probs, max_iter=k, check_every=50, ctx=ctx_u)
        torch.cuda.synchronize()
        tu.append(time.perf_counter() - t0)
        del outs
    ctx_u.close()
    per_iter_u = (tu[1] - tu[0]) / (2 * iters)
    gbs_su = 12.0 * entries / per_iter_u / 1e9
    log(f"batched steady state, default schedule: {per_iter_u * 1e3:.3f} ms per iteration, "
        f"{gbs_su:.0f} GB/s ({100 * gbs_su / HBM_PEAK_GBS:.1f}% of peak)")
    t0 = time.perf_counter()
    for pr in (probs if one_by_one else []):
        drot.solve(pr["C"], pr["p"], pr["q"], pr["rho"], tol=0.0, max_iter=iters, check_every=50,
                   ctx=ctx)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0 if one_by_one else float("nan")
    gbs = 12.0 * entries * iters / t_batch / 1e9
    log(f"batch of {count} x {iters} iterations: {t_batch:.3f}s batched (tuned; untuned "
        f"{t_untuned:.3f}s) vs {t_seq:.3f}s one by one ({t_seq / t_batch:.1f}x), {gbs:.0f} GB/s "
        f"({100 * gbs / HBM_PEAK_GBS:.1f}% of peak)")
    out = {"problems": count, "iterations": iters, "entries": entries,
           "seconds_batched": t_batch, "seconds_batched_untuned": t_untuned,
           "seconds_one_by_one": t_seq, "speedup": t_seq / t_batch, "achieved_GBs": gbs,
           "frac": gbs / HBM_PEAK_GBS, "steady_ms_per_iter": per_iter * 1e3,
           "steady_GBs": gbs_ss, "steady_frac": gbs_ss / HBM_PEAK_GBS,
           "steady_ms_per_iter_default_schedule": per_iter_u * 1e3,
           "steady_frac_default_schedule": gbs_su / HBM_PEAK_GBS,
           "tuner_seconds": t_tune, "tuned_classes": table,
           "workload": "config_batch: m, n ~ U[64, 2048], 2-D blob clouds, Dirichlet(1), float32"}
    if not do_tol:
        return out
    # every problem to the relative test
    for pr in probs:
        pr["rho"] = tol_rho0 / (pr["m"] + pr["n"])
        pr["tol"] = tol
    t0 = time.perf_counter()
    rc, outs = drot.solve_batched(probs, max_iter=3_000_000, check_every=64, ctx=ctx)
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    its = [o[1]["iters"] for o in outs]
    n_conv = sum(1 for o in outs if o[1]["status"] == 0)
    del outs
    log(f"batched {count} to {tol:g} (rho0 = {tol_rho0:g}): {t_all:.2f}s, {n_conv} converged, "
        f"iterations {min(its)}..{max(its)}")
    t0 = time.perf_counter()
    rc, outs = drot.solve_batched(probs[:n_seq], max_iter=3_000_000, check_every=64, ctx=ctx)
    torch.cuda.synchronize()
    t_sub_b = time.perf_counter() - t0
    del outs
    t0 = time.perf_counter()
    for k, pr in enumerate(probs[:n_seq]):
        drot.solve(pr["C"], pr["p"], pr["q"], pr["rho"], tol=tol, max_iter=3_000_000,
                   check_every=64, ctx=ctx)
        if k % 16 == 15:
            log(f"  one by one: {k + 1}/{n_seq}, {time.perf_counter() - t0:.0f}s")
    torch.cuda.synchronize()
    t_sub_s = time.perf_counter() - t0
    log(f"first {n_seq} to {tol:g}: batched {t_sub_b:.2f}s vs one by one {t_sub_s:.2f}s")
    out["time_to_tol"] = {"tol": tol, "rho0": tol_rho0, "seconds_batched_all": t_all,
                          "converged": n_conv, "iters_min": min(its), "iters_max": max(its),
                          "iters_mean": float(np.mean(its)), "subset": n_seq,
                          "seconds_batched_subset": t_sub_b, "seconds_one_by_one_subset": t_sub_s,
                          "ratio_subset": t_sub_b / t_sub_s}
    return out


def protocol_runs(ctx, bind, runs=10, iters=100):
    """The paper's per-iteration runtime protocol (runtime experiment): `runs`
    independent runs of `iters` iterations (graph replays), each from a fresh
    bind; median iterations/s and a 95% interval of the median (order
    statistics of the runs)."""
    import statistics
    import torch
    rates = []
    for _ in range(runs):
        bind(0, iters + 1)
        ctx.iterate(0)  # captures the graph: the protocol times its replay
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.iterate(iters)
        torch.cuda.synchronize()
        rates.append(iters / (time.perf_counter() - t0))
    r = sorted(rates)
    # Distribution-free confidence interval of the median: for 10 runs the
    # order statistics 2 and 9 (1-based) bracket the population median with
    # probability 1 - 2 P(Binomial(10, 1/2) <= 1) = 1 - 22/1024 = 97.9%
    # (at least the 95% of the paper's protocol).
    lo, hi = (r[1], r[-2]) if runs >= 10 else (r[0], r[-1])
    log(f"protocol {runs}x{iters}: median {statistics.median(r):.1f} it/s [{lo:.1f}, {hi:.1f}]")
    return {"runs": runs, "iterations": iters, "median_iter_per_s": statistics.median(r),
            "interval_iter_per_s": [lo, hi],
            "interval": "distribution-free 97.9% confidence interval of the median: order "
                        "statistics 2 and 9 of 10 (binomial, p = 1/2)"}


def paper_sizes_section(ctx, sizes=(100, 200, 500, 1000, 2000, 5000, 10000, 20000), runs=10,
                        iters=100):
    """The paper's runtime experiment: m = n from 100 to 20000, its 2-D
    Gaussian generator (sigma_t = 5, uniform marginals), rho0 = 1/ln m; per
    size `runs` runs of `iters` iterations from a fresh bind, median
    iterations/s and the interval of order statistics 2 and 9."""
    import math
    import statistics
    import numpy as np
    import torch
    from gen import paper_protocol
    from paper_2110_11738_amd import drot
    out = []
    for m in sizes:
        inst = paper_protocol(0, m, rho0=1.0 / math.log(m))
        # rows on 128-byte cache lines, as the main workload's
        C = drot.padded(torch.from_numpy(inst.C.astype(np.float32)).cuda())
        p = torch.from_numpy(inst.p.astype(np.float32)).cuda()
        q = torch.from_numpy(inst.q.astype(np.float32)).cuda()
        X = drot.empty_plan(m, m, torch.float32, "cuda")
        rho = inst.rho
        del inst
        rates = []
        for _ in range(runs):
            ctx.bind(C, p, q, X, drot.make_params(rho, 0.0, iters + 1, check_every=iters))
            ctx.iterate(0)  # captures the graph: the protocol times its replay
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.iterate(iters)
            torch.cuda.synchronize()
            rates.append(iters / (time.perf_counter() - t0))
        r = sorted(rates)
        lo, hi = (r[1], r[-2]) if runs >= 10 else (r[0], r[-1])
        med = statistics.median(r)
        gbs = 12.0 * m * m * med / 1e9
        log(f"paper sizes {m}x{m}: median {med:.1f} it/s [{lo:.1f}, {hi:.1f}], {gbs:.0f} GB/s")
        out.append({"m": m, "n": m, "median_iter_per_s": med, "interval": [lo, hi],
                    "ms_per_iter": 1e3 / med, "algorithmic_GBs": gbs})
        del C, p, q, X
        torch.cuda.empty_cache()
    return out


def small_section(ctx, sizes=(100, 128), iters=2000, warm=200):
    """Small problems (the paper's generator, float32, rho0 = 1/ln m): the
    one-workgroup path that the default parameters select, against sweep +
    aux forced by a tile parameter, iterations/s over `iters` iterations."""
    import math
    import numpy as np
    import torch
    from gen import paper_protocol
    from paper_2110_11738_amd import drot
    out = []
    for m in sizes:
        inst = paper_protocol(0, m, rho0=1.0 / math.log(m))
        # rows on 128-byte cache lines, as the main workload's
        C = drot.padded(torch.from_numpy(inst.C.astype(np.float32)).cuda())
        p = torch.from_numpy(inst.p.astype(np.float32)).cuda()
        q = torch.from_numpy(inst.q.astype(np.float32)).cuda()
        X = drot.empty_plan(m, m, torch.float32, "cuda")
        row = {"m": m, "n": m}
        for name, tr in (("one_workgroup", 0), ("sweep_aux", 16)):
            ctx.bind(C, p, q, X, drot.make_params(inst.rho, 0.0, warm + iters + 1, tile_rows=tr))
            ctx.iterate(warm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.iterate(iters)
            torch.cuda.synchronize()
            row[name + "_iter_per_s"] = iters / (time.perf_counter() - t0)
        row["speedup"] = row["one_workgroup_iter_per_s"] / row["sweep_aux_iter_per_s"]
        log(f"small {m}x{m}: one workgroup {row['one_workgroup_iter_per_s']:.0f} it/s, "
            f"sweep + aux {row['sweep_aux_iter_per_s']:.0f} it/s ({row['speedup']:.2f}x)")
        out.append(row)
    return out


def mlp_section(dims=(2048, 512, 2048), batch=256, steps=50, warm=5):
    """The warm-start network's kernels (bfloat16 MFMA GEMMs with fused
    epilogues, Adam): a training step and a forward pass on random data,
    milliseconds and dense matrix-core throughput (bfloat16 peak 2.5 PFLOP/s)."""
    import numpy as np
    import torch
    from paper_2110_11738_amd import drot
    i, h, o = dims
    net = drot.MLP(i, h, o, max_batch=batch, seed=0)
    rng = np.random.default_rng(7)
    x = torch.tensor(rng.standard_normal((batch, i)).astype(np.float32), device="cuda")
    t = torch.tensor(rng.standard_normal((batch, o)).astype(np.float32), device="cuda")
    for _ in range(warm):
        net.train_step(x, t, 1e-4)
        net.forward(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        net.forward(x)
    torch.cuda.synchronize()
    ms_fwd = (time.perf_counter() - t0) * 1e3 / steps
    macs = batch * (i * h + h * h + h * o)
    fwd_flop, step_flop = 2 * macs, 2 * macs * 3 - 2 * batch * i * h  # no input gradient
    net.close()
    log(f"mlp {i}->{h}->{h}->{o}, batch {batch}: train step {ms_step:.3f} ms "
        f"({step_flop / ms_step / 1e9:.1f} TFLOP/s), forward {ms_fwd:.3f} ms")
    return {"dims": list(dims), "batch": batch, "train_step_ms": ms_step, "forward_ms": ms_fwd,
            "train_step_TFLOPs": step_flop / ms_step / 1e9, "forward_TFLOPs": fwd_flop / ms_fwd / 1e9,
            "forward_us_per_sample": ms_fwd * 1e3 / batch,
            "note": "host-synchronous steps (the loss is read back every step): launch-bound at "
                    "this size"}


def phase_times(ctx, bind, reps=5):
    """Host wall time of the phases around the iteration: bind (validation,
    initialisation pass X_0 = p q^T with its sums, and the check of the
    marginals, which waits for the device) and the final FP64 evaluation pass
    (drot_finish); median of `reps`."""
    import statistics
    import torch
    b, f = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bind(0, 10)
        b.append(1e3 * (time.perf_counter() - t0))
        ctx.iterate(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.finish()
        f.append(1e3 * (time.perf_counter() - t0))
    res = {"bind_with_init_pass": statistics.median(b), "final_evaluation": statistics.median(f)}
    log(f"phases: bind + initialisation {res['bind_with_init_pass']:.3f} ms, final evaluation "
        f"{res['final_evaluation']:.3f} ms")
    return res


def copy_reference(mib=256, reps=20):
    """Read + write bandwidth of torch's device copy of `mib` MiB (context for
    the sweep's roofline fraction)."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2 * src.numel() * 4 / (ms * 1e-3) / 1e9
    log(f"device copy of {mib} MiB: {ms * 1e3:.1f} us -> {gbs:.0f} GB/s (read + write)")
    del src, dst
    return {"bytes_moved": 2 * (mib << 20), "us": ms * 1e3, "GBs": gbs}


def time_to_tol(ctx, C, p, q, rho, rho0_name, args, tol=1e-4, max_iter=2_000_000, flags=0):
    """Solve to the relative tolerance; device seconds from the start of the
    initialisation to the iteration that met the test."""
    import torch
    from paper_2110_11738_amd import drot
    X = torch.empty(C.shape, dtype=C.dtype, device=C.device)
    prm = drot.make_params(rho, tol, max_iter, check_every=args.check_every, flags=flags,
                           tile_rows=args.tile_rows, tile_chunks=args.tile_chunks,
                           tile_unroll=args.tile_unroll, cache_mode=args.cache_mode,
                           tile_groups=args.tile_groups)
    X, r = ctx.solve(C, p, q, prm, X=X)
    torch.cuda.synchronize()
    log(f"time to {tol:g} (rho0 = {rho0_name}): {r['iters']} iterations, "
        f"{r['seconds_to_tol']:.3f}s device, {r['seconds_total']:.3f}s host, status {r['status']}")
    return {"tol": tol, "rho0": rho0_name, "rho": rho, "status": r["status"], "iters": r["iters"],
            "seconds_device": r["seconds_to_tol"], "seconds_host": r["seconds_total"],
            "objective": r["objective"], "eps_primal": r["eps_primal"],
            "eps_dual": r["eps_dual"], "eps_gap": r["eps_gap"]}


def time_to_tol_logged(ctx, C, p, q, rho0, args, tol=1e-4, max_iter=3_000_000, chunk=16384):
    """time_to_tol for long runs: iterations enqueued in chunks, with a
    progress line per chunk; the device time comes from the state record
    (start of initialisation to the iteration that met the test)."""
    import torch
    from paper_2110_11738_amd import drot
    m, n = C.shape
    rho = rho0 / (m + n)
    X = torch.empty(C.shape, dtype=C.dtype, device=C.device)
    ctx.bind(C, p, q, X, drot.make_params(rho, tol, max_iter, check_every=args.check_every))
    t0 = time.perf_counter()
    while True:
        ctx.iterate(chunk)
        k, stopped = ctx.poll()
        log(f"  {m}x{n} rho0 {rho0:g}: {k} iterations, {time.perf_counter() - t0:.0f}s")
        if stopped:
            break
    r = ctx.finish()
    log(f"time to {tol:g} at {m}x{n} (rho0 = {rho0:g}): {r['iters']} iterations, "
        f"{r['seconds_to_tol']:.2f}s device, status {r['status']}")
    return {"tol": tol, "rho0": rho0, "rho": rho, "status": r["status"], "iters": r["iters"],
            "seconds_device": r["seconds_to_tol"], "seconds_host": time.perf_counter() - t0,
            "objective": r["objective"], "eps_primal": r["eps_primal"],
            "eps_dual": r["eps_dual"], "eps_gap": r["eps_gap"]}


def run_to_tol(ctx, bind, label, tol=1e-4, max_iter=3_000_000, chunk=8192):
    """Bind (bind(flags, max_iter) with the tolerance set by the binder), then
    iterate in chunks with a progress line per chunk until the device stop
    flag is set; returns the final result record."""
    bind(0, max_iter)
    t0 = time.perf_counter()
    while True:
        ctx.iterate(chunk)
        k, stopped = ctx.poll()
        if stopped:
            break
        log(f"  {label}: {k} iterations, {time.perf_counter() - t0:.0f}s")
    r = ctx.finish()
    log(f"{label}: {r['iters']} iterations, {r['seconds_to_tol']:.2f}s device to {tol:g}, "
        f"status {r['status']}, objective {r['objective']:.8e}")
    return {"iters": r["iters"], "seconds_device": r["seconds_to_tol"], "status": r["status"],
            "objective": r["objective"], "eps_primal": r["eps_primal"], "eps_dual": r["eps_dual"],
            "eps_gap": r["eps_gap"]}


def tol_forms_section(ctx, rho0=2.0, tol=1e-4, compensated=True):
    """Time to the 1e-4 relative test of the plain float32 form against the
    reduced-byte forms at 10000 x 15000 (the batched form's is in the batch
    section)."""
    import numpy as np
    import torch
    from gen import config_cube_3d
    from paper_2110_11738_amd import drot
    out = {"tol": tol, "rho0": rho0}
    inst = config_cube_3d(0)
    m, n = inst.m, inst.n
    rho = rho0 / (m + n)
    C32 = drot.padded(torch.from_numpy(inst.C.astype(np.float32)).cuda())
    Cb = drot.padded(C32.to(torch.bfloat16))
    xs = torch.from_numpy(inst.xs.astype(np.float32)).cuda()
    xt = torch.from_numpy(inst.xt.astype(np.float32)).cuda()
    p = torch.from_numpy(inst.p.astype(np.float32)).cuda()
    q = torch.from_numpy(inst.q.astype(np.float32)).cuda()
    scale = float(inst.cscale)
    del inst
    X = drot.empty_plan(m, n, torch.float32, "cuda")
    forms = {}
    for name, kind, keep, fl in (("dense_f32", drot.COST_DENSE, (C32,), 0),
                                 ("dense_f32_compensated", drot.COST_DENSE, (C32,),
                                  drot.FLAG_COMPENSATED),
                                 ("bf16", drot.COST_BF16, (Cb,), 0),
                                 ("coords", drot.COST_COORDS, (xs, xt), 0)):
        if name == "dense_f32_compensated" and not compensated:
            continue
        cost = drot.make_cost(kind, C=C32 if kind == drot.COST_DENSE else Cb, xs=xs, xt=xt,
                              scale=scale)

        def bind(flags, max_iter, cost=cost, keep=keep, fl=fl):
            prm = drot.make_params(rho, tol, max_iter, check_every=64, flags=flags | fl)
            ctx.bind_cost(m, n, cost, p, q, X, prm, keep=keep)
        forms[name] = run_to_tol(ctx, bind, f"{m}x{n} {name}", tol)
    out["precision_10000x15000"] = forms
    d = forms["dense_f32"]["seconds_device"]
    for name, r in forms.items():
        r["ratio_to_dense_f32"] = r["seconds_device"] / d
    del C32, Cb, xs, xt, X
    torch.cuda.empty_cache()
    return out


def _oracle_rate(inst, parallel, budget_s):
    """Iterations/s of the FP64 oracle on `inst` over a bounded sample:
    (1 + k) iterations minus one, the initialisation time subtracted."""
    from oracle import ref
    t0 = time.perf_counter()
    ref.solve(inst.C, inst.p, inst.q, inst.rho, 0.0, max_iter=1, parallel=parallel)
    t_one = time.perf_counter() - t0
    k = max(2, min(1000, int(budget_s / max(t_one / 2, 1e-3))))
    t0 = time.perf_counter()
    ref.solve(inst.C, inst.p, inst.q, inst.rho, 0.0, max_iter=1 + k, parallel=parallel)
    t_k = time.perf_counter() - t0
    return k / (t_k - t_one), k, t_k


def cpu_baseline(inst, budget_s=10.0, gpu_iters_to_tol=None):
    """The FP64 oracle (oracle/drot_ref.c) per iteration on the host cores:
    its OpenMP build on every thread OMP_NUM_THREADS allows (the reported
    value) and its one-thread build, each on a bounded sample."""
    from oracle import ref
    m, n = inst.m, inst.n
    rate, k, t_k = _oracle_rate(inst, True, budget_s)
    rate1, k1, t_k1 = _oracle_rate(inst, False, budget_s)
    threads = ref.threads(parallel=True)
    out = {"value": rate, "unit": "iter/s", "cores": threads, "kind": "oracle",
           "sample": f"oracle/drot_ref.c (FP64; OpenMP build, rows split over {threads} threads) "
                     f"on the same {m}x{n} instance upcast from float32: ({1 + k} - 1) iterations "
                     f"from X0 = p q^T, initialisation time subtracted; {t_k:.1f}s of CPU work",
           "single_thread": {"value": rate1, "unit": "iter/s", "cores": 1,
                             "sample": f"one-thread build, ({1 + k1} - 1) iterations, "
                                       f"{t_k1:.1f}s"},
           "host_cpu": _cpu_model(), "nproc": os.cpu_count(),
           "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
           else None}
    if gpu_iters_to_tol:
        out["projected_time_to_tol_s"] = {
            "value": gpu_iters_to_tol / rate, "label": "projected: GPU iterations to the 1e-4 "
            "test at rho0 = 1/ln m divided by the all-core oracle rate (not run)",
            "iters": gpu_iters_to_tol}
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def calibrate_copy(torch, out):
    """A plain copy of known size: under `rocprofv3 --pmc FETCH_SIZE` (or
    WRITE_SIZE) its counters give the factor that converts the sweep's
    counters into bytes."""
    src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    out["copy_calibration_bytes"] = src.numel() * 4


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--m", type=int, default=4096)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--large", type=int, default=20000, help="side of the roofline instance (0 = skip)")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tol", action="store_true")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--tile-chunks", type=int, default=0)
    ap.add_argument("--tile-unroll", type=int, default=0)
    ap.add_argument("--cache-mode", type=int, default=0, help="0 auto, 1 cached, 2 streaming")
    ap.add_argument("--tile-groups", type=int, default=0)
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-skipc", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuned runs")
    ap.add_argument("--no-tol-large", action="store_true",
                    help="skip timing the large instance to the 1e-4 test (about 3.5 minutes)")
    ap.add_argument("--tol-large-rho0", type=float, default=2.0)
    ap.add_argument("--tol-forms", action="store_true",
                    help="also time the compensated form to 1e-4 (the dense, bfloat16 and "
                         "coordinate forms are timed by default)")
    ap.add_argument("--tol-forms-rho0", type=float, default=2.0)
    ap.add_argument("--paper-sizes", action="store_true",
                    help="the paper's runtime protocol at m = n from 100 to 20000")
    ap.add_argument("--large-only", action="store_true",
                    help="skip every section before the large instance (profiling runs)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched-solver section (profiling runs)")
    ap.add_argument("--no-one-by-one", action="store_true",
                    help="batch section: skip the one-by-one comparison (profiling runs)")
    ap.add_argument("--precision-only", action="store_true",
                    help="only the 10000 x 15000 precision section (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration for profiles)")
    ap.add_argument("--check-every", type=int, default=64)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs each problem on a single "
              "MI355X (sharding rows across GPUs is not implemented). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2110_11738_amd import drot
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    drot.lib()
    ctx = drot.Context(0)

    if args.precision_only:
        out = {"metric": "DROT precision forms at 10000x15000 (profiling run)",
               "precision_only": True, "precision": precision_section(ctx)}
        if args.calibrate_copy:
            calibrate_copy(torch, out)
        ctx.close()
        print(json.dumps(out), flush=True)
        return
    if args.batch_only:
        out = {"metric": "batched DROT (profiling run)", "batch_only": True,
               "batch": batch_section(ctx, do_tol=not args.no_tol,
                                      one_by_one=not args.no_one_by_one)}
        ctx.close()
        print(json.dumps(out), flush=True)
        return
    if args.large_only:
        out = {"metric": "DROT iters/s at 20000^2 (profiling run)", "large_only": True}
        C = p = q = None
    else:
        # ---- main workload: 4096^2 float32 -------------------------------------
        inst = make_instance(args.m, args.n)
        C, p, q = upload(inst)
        m, n = args.m, args.n
        G = graph_size(args.steps, args.check_every)
        log(f"timing {args.steps} iterations ({args.steps // G} replays of a {G}-iteration graph) "
            f"after {args.warmup} warm-up iterations")
        bind = dense_binder(ctx, C, p, q, inst.rho, args)
        bind.check_every = G
        r = measure(ctx, bind, args.steps, args.warmup)
        bind.check_every = args.check_every
        secs, sweep_ms, cnt = r["seconds"], r["sweep_ms"], r["sweeps_timed"]
        value = args.steps / secs
        alg_bytes = BYTES_PER_ENTRY_F32 * m * n
        achieved = alg_bytes / (sweep_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "label": f"{m}x{n}: plan and cost (128 MiB) resident in the 256 MB last-level "
                         f"cache, so not an HBM figure; the HBM roofline is the 20000^2 instance",
                "kernel": "sweep_kernel<float,iter>", "bytes_per_launch": alg_bytes,
                "traffic_bytes_per_launch": None,
                "avg_launch_us": sweep_ms * 1e3, "launches_timed": cnt,
                "timing": "hipExtLaunchKernel start/stop events on every sweep of a second timed "
                          "region (eager launches, same workload and length)",
                "eager_iter_per_s": args.steps / r["seconds_eager"]}
        tb = pmc_traffic(m, n)
        if tb is not None:
            # Counter bytes per launch over the same average launch duration.
            roof["traffic"] = tb / (sweep_ms * 1e-3) / 1e9
            roof["traffic_bytes_per_launch"] = tb
            roof["traffic_source"] = os.path.relpath(pmc_summary(m, n), ROOT)
        log(f"{value:.1f} it/s ({1e3 * secs / args.steps:.4f} ms/it); sweep {sweep_ms * 1e3:.2f} us "
            f"-> {achieved:.0f} GB/s; eager {args.steps / r['seconds_eager']:.1f} it/s")

        out = {
            "metric": "DROT iters/s + time-to-1e-4 residual at 4096^2 and 20000^2; HBM GB/s vs peak",
            "value": value, "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * secs / args.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"DROT mixture2d {m}x{n} float32 (two 2-D 5-Gaussian clouds, "
                                   f"sigma 0.1, sq-Euclidean C / max, Dirichlet(1) marginals, "
                                   f"rho0 = 1/ln m); value = iterations/s at {m}x{n} (graph "
                                   f"replays of {G} iterations); roofline = the sweep at "
                                   f"{args.large}x{args.large} (the HBM instance)",
                       "m": m, "n": n, "rho": inst.rho, "graph_iterations": G,
                       "tile_rows": args.tile_rows, "tile_chunks": args.tile_chunks,
                       "tile_unroll": args.tile_unroll, "cache_mode": args.cache_mode,
                       "tile_groups": args.tile_groups,
                       "check_every": args.check_every, "parallelism": "single GPU"},
            "roofline": roof,
            "roofline_cache_resident": roof,
        }

        # ---- the paper's runtime protocol: 10 runs x 100 iterations -----------------
        out["protocol_10x100"] = protocol_runs(ctx, bind)
        # ---- one-off phases, reported apart from the iteration ----------------------
        out["phases_ms"] = phase_times(ctx, bind)
        # ---- a plain device copy on the same box, for scale ---------------------------
        out["copy_reference"] = copy_reference()

        if not args.no_tune:
            tile = tuned_tile(ctx, bind, 2048)
            rt = measure(ctx, dense_binder(ctx, C, p, q, inst.rho, args, tile), args.steps, args.warmup)
            ach_t = alg_bytes / (rt["sweep_ms"] * 1e-3) / 1e9
            out["tuned"] = {"tile_rows": tile[0], "tile_chunks": tile[1], "tile_groups": tile[2],
                            "iter_per_s": args.steps / rt["seconds"],
                            "avg_launch_us": rt["sweep_ms"] * 1e3, "achieved": ach_t,
                            "frac": ach_t / HBM_PEAK_GBS}
            log(f"tuned: {args.steps / rt['seconds']:.1f} it/s, sweep {rt['sweep_ms'] * 1e3:.2f} us "
                f"-> {ach_t:.0f} GB/s")

        # ---- the paper's skip-C schedule on the same workload ---------------------
        if not args.no_skipc:
            r = measure(ctx, bind, args.steps, args.warmup, drot.FLAG_SKIP_C)
            secs_s, sweep_s = r["seconds"], r["sweep_ms"]
            out["skip_c"] = {"iter_per_s": args.steps / secs_s, "avg_sweep_us": sweep_s * 1e3,
                             "bytes_per_entry_avg": 10,
                             "achieved_GBs": 10 * m * n / (sweep_s * 1e-3) / 1e9}
            log(f"skip-C: {args.steps / secs_s:.1f} it/s, average sweep {sweep_s * 1e3:.2f} us")

        # ---- time to the 1e-4 relative stopping test -----------------------------
        if not args.no_tol:
            out["time_to_tol"] = time_to_tol(ctx, C, p, q, inst.rho, "1/ln m", args)
            # the other step-size constant of the paper's experiments
            rho2 = 2.0 / (m + n)
            out["time_to_tol_rho0_2"] = time_to_tol(ctx, C, p, q, rho2, "2", args)
            # the paper's skip-C schedule (Claim 1), same problem and step size
            out["time_to_tol_skip_c"] = time_to_tol(ctx, C, p, q, inst.rho, "1/ln m, skip-C", args,
                                                    flags=drot.FLAG_SKIP_C)

        # ---- CPU oracle baseline ----------------------------------------------------
        if not args.no_cpu:
            gi = out.get("time_to_tol", {}).get("iters")
            out["cpu_baseline"] = cpu_baseline(inst, gpu_iters_to_tol=gi)
            log(f"cpu oracle {out['cpu_baseline']['value']:.3f} it/s on "
                f"{out['cpu_baseline']['cores']} threads, "
                f"{out['cpu_baseline']['single_thread']['value']:.3f} it/s on one")

    del C, p, q
    torch.cuda.empty_cache()
    if not args.no_precision and not args.large_only:
        out["precision"] = precision_section(ctx)
    if not args.no_batch and not args.large_only:
        out["batch"] = batch_section(ctx, do_tol=not args.no_tol)
    if not args.no_small and not args.large_only:
        out["small"] = small_section(ctx)
        out["mlp"] = mlp_section()

    # ---- 20000^2 roofline instance ----------------------------------------------
    if not args.no_large and args.large > 0:
        L = args.large
        linst = make_instance(L, L, upcast=False)
        C, p, q = upload(linst)
        rho_l = linst.rho
        del linst
        ksteps, kwarm = 40, 5
        ab = BYTES_PER_ENTRY_F32 * L * L
        binder = dense_binder(ctx, C, p, q, rho_l, args)
        binder.check_every = graph_size(ksteps, args.check_every)
        r = measure(ctx, binder, ksteps, kwarm)
        secs_l, sweep_l, cnt_l = r["seconds"], r["sweep_ms"], r["sweeps_timed"]
        ach = ab / (sweep_l * 1e-3) / 1e9
        tb_l = pmc_traffic(L, L)
        roof_l = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                  "traffic": (tb_l / (sweep_l * 1e-3) / 1e9 if tb_l is not None else None),
                  "kernel": "sweep_kernel<float,iter>",
                  "workload": f"mixture2d {L}x{L} float32 (3.2 GB of plan and cost)",
                  "bytes_per_launch": ab, "traffic_bytes_per_launch": tb_l,
                  "avg_launch_us": sweep_l * 1e3, "launches_timed": cnt_l,
                  "timing": "hipExtLaunchKernel start/stop events on every sweep of an eager "
                            f"timed region of {ksteps} iterations",
                  "iteration_GBs": ab / (secs_l / ksteps) / 1e9,
                  "iteration_frac": ab / (secs_l / ksteps) / 1e9 / HBM_PEAK_GBS}
        if tb_l is not None:
            roof_l["traffic_source"] = os.path.relpath(pmc_summary(L, L), ROOT)
        out["large"] = {"m": L, "n": L, "iter_per_s": ksteps / secs_l,
                        "ms_per_iter": 1e3 * secs_l / ksteps, "roofline": roof_l}
        out["roofline"] = roof_l
        log(f"{L}^2: {ksteps / secs_l:.1f} it/s, sweep {sweep_l * 1e3:.1f} us -> {ach:.0f} GB/s "
            f"({100 * ach / HBM_PEAK_GBS:.1f}% of peak)")
        if not args.no_tune:
            tile = tuned_tile(ctx, binder)
            r = measure(ctx, dense_binder(ctx, C, p, q, rho_l, args, tile), ksteps, kwarm)
            ach_t = ab / (r["sweep_ms"] * 1e-3) / 1e9
            out["large"]["tuned"] = {"tile_rows": tile[0], "tile_chunks": tile[1],
                                     "tile_groups": tile[2],
                                     "iter_per_s": ksteps / r["seconds"],
                                     "avg_launch_us": r["sweep_ms"] * 1e3, "achieved": ach_t,
                                     "frac": ach_t / HBM_PEAK_GBS}
            log(f"{L}^2 tuned: {ksteps / r['seconds']:.1f} it/s, sweep {r['sweep_ms'] * 1e3:.1f} us "
                f"-> {ach_t:.0f} GB/s ({100 * ach_t / HBM_PEAK_GBS:.1f}% of peak)")
        if not args.no_tol_large:
            out["large"]["time_to_tol"] = time_to_tol_logged(ctx, C, p, q, args.tol_large_rho0,
                                                             args)

    if args.paper_sizes:
        out["paper_sizes"] = paper_sizes_section(ctx)

    if not args.no_tol and not args.no_precision and not args.large_only:
        out["time_to_tol_forms"] = tol_forms_section(ctx, rho0=args.tol_forms_rho0,
                                                     compensated=args.tol_forms)

    if args.calibrate_copy:
        calibrate_copy(torch, out)

    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
