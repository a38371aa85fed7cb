#!/usr/bin/env python3
"""Throughput of MPR gap filling on one MI355X.

A step is one whole gap fill of the L=4096 workload: angle map, sample
energy and temperature (e(T, L) table cached per grid size, built during the
warmup), R=100 independent chains relaxed with the energy stopping rule plus
K=1 equilibrium state each (M=100 realizations), and the back-transform.
Inputs are synthetic (lognormal Matern field, 66% of sites removed at
random) and resident on the GPU before timing starts.

Prints one JSON line: site-updates/s (gap-site updates summed over chains and
sweeps, divided by wall time), the roofline of the half-sweep kernel (useful
bytes per launch over its event-timed duration, against 8 TB/s HBM), the
time to fill at equal MAE with the learned warm start against the plain
random start (L=2048, random and cloud masks), and the FP64 oracle's rate on
a bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "half_sweep_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1811_01604_amd", "csrc", f) for f in ("mpr.hip", "mpr_device.h")]
METRIC = "site-updates/s at L=4096; time-to-fill at equal MAE, plain vs CNN warm start"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str):
    import synth
    if name == "l4096-random":
        return synth.workload_l4096("random"), "lognormal exp(G), G Matern nu=1.5 kappa=0.02 std 0.5; 4096x4096; 66% uniform random gaps"
    if name == "l4096-cloud":
        return synth.workload_l4096("cloud"), "lognormal exp(G), G Matern nu=1.5 kappa=0.02 std 0.5; 4096x4096; 40% cloud gaps (Matern threshold)"
    if name == "l1024":
        return synth.workload_l1024(), "Gaussian Matern nu=2.5 kappa=0.05 N(50,10); 1024x1024; 50% uniform random gaps"
    raise SystemExit(f"unknown workload {name}")


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, chains: int, key: str):
    """HBM bytes per half-sweep launch from the committed rocprofv3 counter
    runs (FETCH_SIZE + WRITE_SIZE, scaled by the copy-probe calibration), or
    None when they were taken on other kernel sources, another workload or
    another sweep kernel (key: the block shape's tile_rows value, prefixed
    "fp64-" for the double-precision sweep)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_sha() or t.get("workload") != workload or t.get("chains") != chains:
        return None
    return (t.get("by_tile") or {}).get(key, {}).get("traffic_bytes_per_launch")


def measured_valu(workload: str, chains: int, key: str, launch_ms: float):
    """VALU wave-instructions per launch from the committed counter runs
    (SQ_INSTS_VALU) and the issue rate they give at the live launch time and
    the 2.4 GHz peak clock, per SIMD (1024 of them); None as for traffic."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_sha() or t.get("workload") != workload or t.get("chains") != chains:
        return None
    v = (t.get("by_tile") or {}).get(key, {}).get("valu_insts_per_launch")
    if not v:
        return None
    rate = v / (1024 * launch_ms * 1e-3 * 2.4e9)
    # binding: the kernel issues VALU instructions at (or above) the rate of
    # 4-cycle FP32 FMAs, so the VALU, not HBM, sets its time
    return {"wave_insts_per_launch": v, "issue_per_simd_cycle": rate, "fp32_fma_issue_limit_per_simd_cycle": 0.25,
            "binding": rate >= 0.9 * 0.25}


def cpu_baseline(im, T: float, sweeps: int, seed: int) -> dict:
    """The oracle's sweep on one chain of the same workload (bounded sample),
    at a fixed temperature T (an input: the work per sweep does not depend
    on it)."""
    import numpy as np
    import oracle
    z = im.z.astype(np.float32).astype(np.float64)
    phi, _ = oracle.map_to_angles(z, im.mask)
    g = im.mask == 0
    phi[g] = np.random.default_rng(seed).uniform(0.0, 2.0 * np.pi, size=int(g.sum()))
    P = int(g.sum())
    t0 = time.perf_counter()
    for t in range(sweeps):
        for colour in (0, 1):
            phi, _, _ = oracle.half_sweep(phi, im.mask, colour, T, 1.0 + t / 3.0, t, seed=seed)
    dt = time.perf_counter() - t0
    return {"value": sweeps * P / dt, "unit": "site-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} sweeps of 1 chain ({P} gap sites) of the same workload, FP64 oracle, "
                      f"single thread, {dt:.1f} s"}


def _oracle_chain_worker(args):
    """One oracle chain on the image saved at `path` (gaps already drawn
    into phi): `sweeps` sweeps, returns (site-updates, seconds)."""
    path, T, sweeps, seed = args
    import numpy as np
    import oracle
    d = np.load(path)
    phi, mask = d["phi"].copy(), d["mask"]
    P = int((mask == 0).sum())
    t0 = time.perf_counter()
    for t in range(sweeps):
        for colour in (0, 1):
            phi, _, _ = oracle.half_sweep(phi, mask, colour, T, 1.0 + t / 3.0, t, seed=seed)
    return sweeps * P, time.perf_counter() - t0


def cpu_baseline_all_cores(im, T: float, sweeps: int, seed: int, workers: int) -> dict:
    """The same oracle sweep on `workers` independent chains at once, one
    single-threaded oracle process per chain (the chains of a fill are
    independent, so this is how the oracle uses every core): aggregate
    site-updates per second of wall time, from the start of the first sweep
    to the end of the last."""
    import multiprocessing as mp
    import tempfile
    import numpy as np
    import oracle
    z = im.z.astype(np.float32).astype(np.float64)
    phi, _ = oracle.map_to_angles(z, im.mask)
    g = im.mask == 0
    phi[g] = np.random.default_rng(seed).uniform(0.0, 2.0 * np.pi, size=int(g.sum()))
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "chain.npz")
        np.savez(path, phi=phi, mask=im.mask)
        pool = mp.get_context("spawn").Pool(workers)
        try:
            pool.map(_oracle_chain_worker, [(path, T, 0, seed)] * workers)  # start-up and imports, untimed
            t0 = time.perf_counter()
            res = pool.map(_oracle_chain_worker, [(path, T, sweeps, seed + 1 + w) for w in range(workers)])
            dt = time.perf_counter() - t0
        finally:
            pool.close()
            pool.join()
    updates = sum(r[0] for r in res)
    return {"value": updates / dt, "unit": "site-updates/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} independent chains, {sweeps} sweeps each ({int(g.sum())} gap sites) of the same "
                      f"workload, one single-threaded FP64 oracle process per chain, {dt:.1f} s wall"}


def cpu_baseline_scaling(sizes, fractions=(0.33, 0.66), T: float = 0.09, full_fill_max: int = 1024,
                         extra=()):
    """The oracle on the lattice-size study's images (Whittle-Matern nu=0.5,
    kappa=0.2, N(50, 10), a fraction p removed at random; the images the GPU
    study fills), one JSON line per (L, p): every size in `sizes` at every
    fraction in `fractions`, then the (L, p) pairs of `extra` (the gap-fraction
    sweep).  Up to L = full_fill_max a whole fill as the GPU study times it:
    R = 1 chain, the stopping rule, K = 100 states, at a fixed temperature T
    (the GPU study's T_hat for these images lies in 0.08-0.09; the e(T, L)
    table is excluded on both sides).  Larger L: one sweep, timed, as the
    per-sweep cost."""
    import numpy as np
    import oracle
    import synth
    cases = [(L, p) for L in sizes for p in fractions]
    cases += [c for c in extra if c not in cases]
    for L, p in cases:
        im = synth.workload_table2(L, p, 0)
        z = im.z.astype(np.float32).astype(np.float64)
        phi, _ = oracle.map_to_angles(z, im.mask)
        P = int((im.mask == 0).sum())
        row = {"L": L, "p_removed": p, "gap_sites": P, "T": T, "cores": 1, "kind": "oracle"}
        if L <= full_fill_max:
            prm = oracle.default_params(R=1, K=100, seed=7000)
            t0 = time.perf_counter()
            _, st, _, _ = oracle.simulate(phi, im.mask, T, prm)
            dt = time.perf_counter() - t0
            sweeps = st[0]["relax_sweeps"] + 1 + 100
            row.update(fill_s=dt, relax_sweeps=st[0]["relax_sweeps"], sweeps=sweeps,
                       site_updates_per_s=sweeps * P / dt)
        else:
            prm = oracle.default_params(R=1, K=1, fixed_relax=0, seed=7000)
            t0 = time.perf_counter()
            oracle.simulate(phi, im.mask, T, prm)
            dt = time.perf_counter() - t0
            row.update(fill_s=None, sweep_s=dt, site_updates_per_s=P / dt)
        log(f"oracle L={L} p={p}: {json.dumps(row)}")
        print(json.dumps(row), flush=True)


def read_jsonl(path: str) -> list:
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{"):
                rows.append(json.loads(line))
    return rows


def combine_scaling(gpu_path: str, cpu_path: str) -> dict:
    """The GPU study's rows joined with the oracle's rows of the same (L, p).
    The oracle's time to fill is its measured whole fill where it ran one;
    otherwise its measured per-sweep time times the GPU fill's sweep count
    (relaxation sweeps + 1 + K), the sweeps the oracle would run from the same
    stopping rule.  speedup = oracle time to fill / GPU time to fill (both
    without the e(T, L) table)."""
    cpu = {(r["L"], round(r["p_removed"], 6)): r for r in read_jsonl(cpu_path)}
    rows = []
    for g in read_jsonl(gpu_path):
        if "site_updates_per_s" not in g:
            continue
        c = cpu.get((g["L"], round(g["p_removed"], 6)))
        row = dict(g)
        if c is not None:
            if c.get("fill_s") is not None:
                t_cpu, how = c["fill_s"], "measured fill"
            else:
                t_cpu = c["sweep_s"] * (g["relax_sweeps"] + 1 + g["K"])
                how = "measured sweep x GPU sweep count"
            row.update(oracle_time_to_fill_s=t_cpu, oracle_fill_basis=how,
                       oracle_site_updates_per_s=c["site_updates_per_s"], oracle_cores=c["cores"],
                       speedup_time_to_fill=t_cpu / g["time_to_fill_s"],
                       speedup_site_updates=g["site_updates_per_s"] / c["site_updates_per_s"])
        rows.append(row)
    return {"study": "time to fill and sweep throughput against lattice size L and gap fraction p "
                     "(Whittle-Matern nu=0.5 kappa=0.2 N(50,10), random gaps; R=1 chain, stopping rule, K=100)",
            "rows": rows}


def cnn_inference(ctx, model, size: int = 2048, reps: int = 5) -> dict:
    """Event-timed warm-start network inference on one size x size image,
    from the sample angles to the starting gap angles (one mpr_cnn_infer:
    the encoding in the stem's staging, the decoding in the head's
    epilogue).  Algorithmic HBM bytes per pixel: the stem reads the angle and
    the flag (5 B) and writes its activation (64 B); the 8 residual blocks
    (each one kernel, its inner activation kept on chip) read their input
    and write their output (2 x 64 B); the head reads its input and the flag
    and writes the angle (64 + 1 + 4 B): 1162 B (a layer-by-layer pass with
    separate encode and decode would move about 3.4 KB); flops per pixel:
    18 x 2 x 9 x 32 x 32."""
    import numpy as np
    import torch
    rng = np.random.default_rng(5)
    phi = torch.from_numpy(rng.uniform(0, 2 * np.pi, size=(1, size, size)).astype(np.float32)).cuda()
    sm = torch.from_numpy((rng.random((1, size, size)) < 0.5).astype(np.uint8)).cuda()
    init = torch.empty_like(phi)
    ms = []
    for i in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        model(phi, sm, init)
        e1.record()
        torch.cuda.synchronize()
        if i:
            ms.append(e0.elapsed_time(e1))
    t = float(np.median(ms)) * 1e-3
    px = size * size
    nbytes, flops = 1162.0 * px, 18 * 2 * 9 * 32 * 32 * float(px)
    return {"image": f"{size}x{size}", "inference_ms": t * 1e3, "bound": "hbm", "achieved": nbytes / t / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": nbytes / t / 1e9 / HBM_PEAK_GBS,
            "bytes_per_inference": nbytes, "tflops": flops / t / 1e12, "bf16_mfma_peak_tflops": 2500.0,
            "mfma_frac": flops / t / 1e12 / 2500.0}


def cloud_leg(ctx, mpr, prm, steps: int) -> dict:
    """The same fill (R chains, K states, stopping rule) on the L=4096 field
    with the 40% cloud mask, `steps` timed fills; the e(T, L) table of the
    grid size and the tuned block shape are the random mask's, cached in the
    context by the main measurement."""
    import numpy as np
    import torch
    im, desc = make_workload("l4096-cloud")
    imgs = mpr.images([(im.ny, im.nx)])
    z = torch.from_numpy(im.z.astype(np.float32)).cuda()
    mk = torch.from_numpy(im.mask).cuda()
    phi, ps, zh = torch.zeros_like(z), torch.zeros_like(z), torch.zeros_like(z)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    P = int((im.mask == 0).sum())

    def fill():
        zz = ctx.map_to_angles(imgs, z, mk, phi)
        _, T, _ = ctx.estimate_temperature(imgs, phi, mk, prm, ws)
        st = ctx.simulate(imgs, phi, mk, T, prm, ws, ps)
        ctx.predict(imgs, z, mk, ps, zz, prm.R * prm.K, zh)
        return st, float(T[0])

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates, sweeps = 0, []
    for _ in range(steps):
        st, T = fill()
        s = [x["relax_sweeps"] + prm.K for x in st]
        sweeps.extend(s)
        updates += sum(s) * P
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g = im.mask == 0
    mae = float(np.mean(np.abs(zh.cpu().numpy()[g] - im.z.astype(np.float32)[g])))
    log(f"l4096 cloud: {updates / dt:.3e} site-updates/s, {dt / steps:.1f} s per fill, "
        f"{np.mean(sweeps):.0f} sweeps per chain")
    del ws
    return {"workload": desc, "value": updates / dt, "unit": "site-updates/s", "steps": steps,
            "ms_per_step": dt / steps * 1e3, "chains_R": prm.R, "states_per_chain_K": prm.K, "gap_sites": P,
            "mean_sweeps_per_chain": float(np.mean(sweeps)), "T_hat": T, "MAE": mae}


def small_fill_leg(ctx, mpr, steps: int) -> dict:
    """A small fill in the paper's layout: the L=1024 workload, one chain of
    K = 100 states with the stopping rule, `steps` timed fills after one
    untimed fill (which builds the e(T, L) table of the size and tunes the
    sweep shape, both cached).  Reports site-updates/s over whole fills (map,
    temperature, simulate, predict) and the fill's own sweep time per sweep
    (event-timed sweep groups)."""
    import numpy as np
    import torch
    im, desc = make_workload("l1024")
    imgs = mpr.images([(im.ny, im.nx)])
    z = torch.from_numpy(im.z.astype(np.float32)).cuda()
    mk = torch.from_numpy(im.mask).cuda()
    phi, ps, zh = torch.zeros_like(z), torch.zeros_like(z), torch.zeros_like(z)
    prm = mpr.default_params(R=1, K=100)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    P = int((im.mask == 0).sum())

    def fill():
        zz = ctx.map_to_angles(imgs, z, mk, phi)
        _, T, _ = ctx.estimate_temperature(imgs, phi, mk, prm, ws)
        st = ctx.simulate(imgs, phi, mk, T, prm, ws, ps)
        ctx.predict(imgs, z, mk, ps, zz, prm.R * prm.K, zh)
        return st

    fill()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    sweeps = 0
    for _ in range(steps):
        st = fill()
        sweeps += sum(x["relax_sweeps"] + prm.K for x in st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pr = ctx.profile_read()
    ctx.profile_enable(False)
    del ws
    sweep_us = pr["sweep_kernel_ms"] * 1e3 / max(1, pr["chain_sweeps"])
    log(f"small fill l1024 (1,100): {sweeps * P / dt:.3e} site-updates/s, {dt / steps * 1e3:.2f} ms per fill, "
        f"{sweep_us:.1f} us per sweep")
    return {"workload": desc, "value": sweeps * P / dt, "unit": "site-updates/s", "steps": steps,
            "ms_per_step": dt / steps * 1e3, "chains_R": prm.R, "states_per_chain_K": prm.K, "gap_sites": P,
            "sweeps_per_fill": sweeps / steps, "sweep_us": sweep_us, "tile_rows": pr["last_tile"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="l4096-random")
    ap.add_argument("--chains", type=int, default=100)
    ap.add_argument("--K", type=int, default=1)
    ap.add_argument("--fixed-sweeps", type=int, default=-1,
                    help="relax exactly this many sweeps instead of the stopping rule")
    ap.add_argument("--cpu-sweeps", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the all-cores oracle baseline (0 = the host's cores, at most 16; "
                         "1 = skip it)")
    ap.add_argument("--cpu-scaling", default="",
                    help="only the CPU baseline of the lattice-size study: time the oracle on its images "
                         "at these comma-separated sizes L (p = 0.33 and 0.66), one JSON line per case, "
                         "and exit (no GPU work)")
    ap.add_argument("--cpu-p-sweep", default="",
                    help="with --cpu-scaling: also the gap-fraction sweep, as L:p1,p2,... "
                         "(e.g. 2048:0.05,0.2,0.35,0.5,0.65,0.8,0.95)")
    ap.add_argument("--cnn-only", action="store_true",
                    help="only the warm-start network's 2048^2 inference timing (one JSON line), e.g. for a "
                         "kernel trace of the network alone")
    ap.add_argument("--combine", nargs=2, metavar=("GPU_JSONL", "CPU_JSONL"),
                    help="join the GPU scaling study's lines with the oracle's lines of the same (L, p) into "
                         "one JSON document with the oracle's time to fill and the speed-up, and exit")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 1 GiB plain copy first (calibrates HBM byte counters)")
    ap.add_argument("--tile", default="auto",
                    help="sweep block shape: auto (tuned), or rows 1/2/4/8, with a 'c' suffix for the compacted "
                         "shapes 2c/4c/8c, or 8f/12f/16f/24f/32f/48f for the fused tile sweep, or 8p/12p/16p/24p/32p "
                         "for fused sweeps many per cooperative launch (for profiling runs that must see one kernel)")
    ap.add_argument("--fp64", action="store_true",
                    help="run the chains in double precision (the paper's DP variant)")
    ap.add_argument("--warm-seeds", type=int, default=32,
                    help="images per mask type for the warm-start comparison at L=2048 (0 = skip)")
    ap.add_argument("--cloud-steps", type=int, default=1,
                    help="timed steps of the same fill with the 40%% cloud mask, reported as l4096_cloud "
                         "(0 = skip; only with the default workload)")
    ap.add_argument("--small-steps", type=int, default=5,
                    help="timed fills of the L=1024 workload in the (1, 100) layout, reported as small_fill "
                         "(0 = skip; only with the default workload)")
    args = ap.parse_args()
    if args.combine:
        print(json.dumps(combine_scaling(*args.combine), indent=1))
        return
    if args.cpu_scaling:
        extra = ()
        if args.cpu_p_sweep:
            Ls, ps = args.cpu_p_sweep.split(":")
            extra = tuple((int(Ls), float(p)) for p in ps.split(","))
        cpu_baseline_scaling([int(v) for v in args.cpu_scaling.split(",")], extra=extra)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the sweep has no multi-GPU path "
              f"in this library.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1811_01604_amd as mpr
    from paper_1811_01604_amd import warmstart

    if args.cnn_only:
        ctx = mpr.Context(0)
        params, _ = warmstart.load()
        print(json.dumps(cnn_inference(ctx, warmstart.WarmStart(ctx, params))), flush=True)
        ctx.close()
        return

    # CPU-side inputs first, before anything touches the GPU (the evaluation
    # images are made in worker processes)
    warm_fields = None
    if args.warm_seeds > 0 and os.path.exists(warmstart.DEFAULT_WEIGHTS):
        t0 = time.perf_counter()
        warm_fields = warmstart.make_eval_fields(size=2048, seeds=args.warm_seeds, workers=8)
        log(f"warm-start evaluation images: {len(warm_fields)} in {time.perf_counter() - t0:.1f} s")
    log(f"workload {args.workload}: generating")
    im, desc = make_workload(args.workload)
    log(f"  {im.nx}x{im.ny}, {int((im.mask == 0).sum())} gaps")
    ctx = mpr.Context(0)
    shapes = [(im.ny, im.nx)]
    imgs = mpr.images(shapes)
    z = torch.from_numpy(im.z.astype(np.float32)).cuda()
    mk = torch.from_numpy(im.mask).cuda()
    phi = torch.zeros_like(z)
    ps = torch.zeros_like(z)
    zh = torch.zeros_like(z)
    tile = 0
    if args.tile != "auto":
        tile = int(args.tile.rstrip("cfp")) | (mpr.TILE_COMPACT if args.tile.endswith("c") else 0) | \
            (mpr.TILE_FUSED if args.tile.endswith("f") else 0) | \
            (mpr.TILE_FUSED | mpr.TILE_PERSIST if args.tile.endswith("p") else 0)
    prm = mpr.default_params(R=args.chains, K=args.K, fixed_relax=args.fixed_sweeps, tile_rows=tile,
                             fp64=1 if args.fp64 else 0)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    P = int((im.mask == 0).sum())
    M = prm.R * prm.K

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        ctx.diag_copy(src, dst)
        torch.cuda.synchronize()
        log("copy probe: 1 GiB copied")
        del src, dst

    def step():
        zz = ctx.map_to_angles(imgs, z, mk, phi)
        e_s, T, _ = ctx.estimate_temperature(imgs, phi, mk, prm, ws)
        st = ctx.simulate(imgs, phi, mk, T, prm, ws, ps)
        ctx.predict(imgs, z, mk, ps, zz, M, zh)
        return st, float(T[0])

    t0 = time.perf_counter()
    for i in range(args.warmup):
        st, T = step()
        log(f"warmup {i}: T_hat={T:.3e}, relax sweeps mean {np.mean([s['relax_sweeps'] for s in st]):.1f}, "
            f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates = 0
    sweeps = []
    for i in range(args.steps):
        st, T = step()
        s = [x["relax_sweeps"] + prm.K for x in st]
        sweeps.extend(s)
        updates += sum(s) * P
        log(f"step {i}: mean sweeps/chain {np.mean(s):.1f}, {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    zt = im.z.astype(np.float32)
    g = im.mask == 0
    mae = float(np.mean(np.abs(zh.cpu().numpy()[g] - zt[g])))
    assert prof["site_updates"] == updates, (prof["site_updates"], updates)
    launch_ms = prof["sweep_kernel_ms"] / max(prof["sweep_launches"], 1)
    bytes_per_launch = prof["useful_bytes"] / max(prof["sweep_launches"], 1)
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": updates / dt,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.fp64 else "f32",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "chains_R": prm.R, "states_per_chain_K": prm.K, "gap_sites": P,
            "relaxation": "stopping rule" if args.fixed_sweeps < 0 else f"fixed {args.fixed_sweeps} sweeps",
            "mean_sweeps_per_chain": float(np.mean(sweeps)),
            "T_hat": T, "MAE": mae,
            "e_T_table": "cached per grid size, built during warmup",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(args.workload, prm.R,
                                        ("fp64-" if args.fp64 else "") + str(prof["last_tile"])),
            "kernel": ("sweep_tile_persist_kernel" if prof["last_tile"] & mpr.TILE_PERSIST else
                       "sweep_tile_kernel" if prof["last_tile"] & mpr.TILE_FUSED else
                       "half_sweep_" + ("fp64_" if args.fp64 else "") +
                       ("compact_kernel" if prof["last_tile"] & mpr.TILE_COMPACT else "kernel")),
            "launch": ("one fused sweep (both colours) of every running chain, many per cooperative launch"
                       if prof["last_tile"] & mpr.TILE_PERSIST else
                       "one fused sweep (both colours) of every running chain" if prof["last_tile"] & mpr.TILE_FUSED
                       else "one half-sweep (one colour) of every running chain"),
            "tile_rows": prof["last_tile"] & 0xFF,
            "launch_ms": launch_ms, "useful_bytes_per_launch": bytes_per_launch,
            "sweep_kernel_time_share": prof["sweep_kernel_ms"] * 1e-3 / dt,
            "valu": (None if args.fp64 else
                     measured_valu(args.workload, prm.R, str(prof["last_tile"]), launch_ms)),
        },
    }
    if args.cloud_steps > 0 and args.workload == "l4096-random" and not args.fp64:
        out["l4096_cloud"] = cloud_leg(ctx, mpr, prm, args.cloud_steps)
    if args.small_steps > 0 and args.workload == "l4096-random" and not args.fp64:
        out["small_fill"] = small_fill_leg(ctx, mpr, args.small_steps)
    if warm_fields is not None:
        log("warm start vs plain start at L=2048")
        params, info = warmstart.load()
        model = warmstart.WarmStart(ctx, params)
        cnn = cnn_inference(ctx, model)
        log(f"  network inference 2048^2: {cnn['inference_ms']:.2f} ms, {cnn['achieved']:.0f} GB/s, "
            f"{cnn['tflops']:.0f} TFLOP/s")
        layouts = ((1, 100), (4, 25), (100, 1))
        ws_summary = warmstart.evaluate(ctx, model, warm_fields, layouts=layouts)
        out["warm_start"] = {
            "workload": "Gaussian Matern nu=1.5 kappa=0.05 N(50,10); 2048x2048; 50% random and 50% cloud "
                        "gaps; M=100 realizations as (R chains, K states): 1x100 (the paper's layout), 4x25, "
                        "100x1; T_hat shared; time = network inference (warm) + simulate + predict; MAE ratio "
                        "warm/plain paired per image, mean and 95% CI over the images",
            "network": f"8-block residual CNN, 32 channels, bf16 MFMA; trained on {info['samples']} "
                       f"library simulations of {info['size']}^2 images",
            "warm_min_states": mpr.default_params().warm_min_states,
            "layouts": ws_summary,
            "inference_roofline": cnn,
        }
    elif args.warm_seeds > 0:
        out["warm_start"] = None
    ctx.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(im, 1e-4, args.cpu_sweeps, 3002)
        if args.cpu_workers != 1:
            workers = args.cpu_workers if args.cpu_workers > 1 else min(16, len(os.sched_getaffinity(0)))
            log(f"cpu baseline (oracle), {workers} processes")
            out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(im, 1e-4, max(1, args.cpu_sweeps // 2), 3002,
                                                                   workers)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
