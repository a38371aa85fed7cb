"""Single against double precision on one GPU.

The paper runs the method with single- and double-precision angles and
compares the prediction statistics (Section 4, Tables 2 and 3) and the run
times (Fig. 4).  This study does the same with the library's two sweeps
(mpr_params.fp64 = 0 or 1):
  - statistics: Whittle-Matern fields (nu = 0.5, kappa = 0.2, N(50, 10)),
    p = 33% and 66% of the sites removed at random, M = 100 states of one
    chain (R = 1, K = 100) with the stopping rule; both precisions use the
    same T_hat (estimated once) and the same seeds; MAAE, MARE, MAARE and
    MRASE averaged over the fields;
  - time: the time to fill one image (simulate + predict) per precision, and
    the sweep throughput with the GPU full (R chains of 100 relaxation
    sweeps + 1 state), per precision and lattice size.

    python -m paper_1811_01604_amd.precision [--stat-size 256] [--fields 8] [--sizes 256,1024,4096]

prints one JSON line per case and markdown tables at the end.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = dict(table_nT=12, table_burn=100, table_meas=200)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _imports():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import synth
    import torch
    import paper_1811_01604_amd as mpr
    return synth, torch, mpr


def fill_stats(ctx, L: int, p: float, rep: int) -> dict:
    """One field: both precisions from the same angles, T_hat and seed."""
    synth, torch, mpr = _imports()
    im = synth.workload_table2(L, p, rep)
    imgs = mpr.images([(L, L)])
    z = torch.from_numpy(im.z.astype(np.float32)).cuda()
    mk = torch.from_numpy(im.mask).cuda()
    phi = torch.zeros_like(z)
    zz = ctx.map_to_angles(imgs, z, mk, phi)
    out = {"L": L, "p_removed": p, "field": rep}
    T = None
    for name, fp64 in (("sp", 0), ("dp", 1)):
        prm = mpr.default_params(R=1, K=100, seed=7000 + rep, fp64=fp64, **TABLE)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        if T is None:
            _, T, _ = ctx.estimate_temperature(imgs, phi, mk, prm, ws)
        ps, zh = torch.zeros_like(z), torch.zeros_like(z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.simulate(imgs, phi, mk, T, prm, ws, ps)
        ctx.predict(imgs, z, mk, ps, zz, 100, zh)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        m = synth.validation_measures(im.z.astype(np.float32).astype(np.float64),
                                      zh.cpu().numpy().astype(np.float64), im.mask)
        out[name] = {**m, "relax_sweeps": st[0]["relax_sweeps"], "time_to_fill_s": dt}
    out["T_hat"] = float(T[0])
    return out


def sweep_rate(ctx, L: int, fp64: int) -> dict:
    """Gap-site updates per second of sweep-kernel time with the GPU full."""
    synth, torch, mpr = _imports()
    im = synth.workload_table2(L, 0.66, 0)
    imgs = mpr.images([(L, L)])
    z = torch.from_numpy(im.z.astype(np.float32)).cuda()
    mk = torch.from_numpy(im.mask).cuda()
    phi, ps = torch.zeros_like(z), torch.zeros_like(z)
    ctx.map_to_angles(imgs, z, mk, phi)
    R = int(min(100, max(1, (1 << 31) // (L * L))))
    prm = mpr.default_params(R=R, K=1, fixed_relax=100, fp64=fp64, **TABLE)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    _, T, _ = ctx.estimate_temperature(imgs, phi, mk, prm, ws)
    ctx.simulate(imgs, phi, mk, T, prm, ws, ps)  # tunes the block shape
    ctx.profile_enable(True)
    ctx.simulate(imgs, phi, mk, T, prm, ws, ps)
    pr = ctx.profile_read()
    ctx.profile_enable(False)
    launch_ms = pr["sweep_kernel_ms"] / max(pr["sweep_launches"], 1)
    return {"L": L, "precision": "dp" if fp64 else "sp", "chains": R,
            "site_updates_per_s": pr["site_updates"] / (pr["sweep_kernel_ms"] * 1e-3),
            "useful_GBps": pr["useful_bytes"] / (pr["sweep_kernel_ms"] * 1e-3) / 1e9,
            "launch_ms": launch_ms, "tile": pr["last_tile"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stat-size", type=int, default=256)
    ap.add_argument("--fields", type=int, default=8)
    ap.add_argument("--sizes", default="256,1024,4096")
    args = ap.parse_args()
    _, _, mpr = _imports()
    ctx = mpr.Context(0)
    stats = []
    for p in (0.33, 0.66):
        for rep in range(args.fields):
            r = fill_stats(ctx, args.stat_size, p, rep)
            stats.append(r)
            print(json.dumps(r), flush=True)
            log(f"L={args.stat_size} p={p} field {rep}: MAAE sp {r['sp']['MAAE']:.4f} dp {r['dp']['MAAE']:.4f}")
    rates = []
    for L in (int(v) for v in args.sizes.split(",")):
        for fp64 in (0, 1):
            r = sweep_rate(ctx, L, fp64)
            rates.append(r)
            print(json.dumps(r), flush=True)
            log(f"L={L} {r['precision']}: {r['site_updates_per_s']:.3e} site-updates/s ({r['chains']} chains)")
    ctx.close()
    keys = ("MAAE", "MARE", "MAARE", "MRASE")
    print(f"| p | precision | {' | '.join(keys)} | relax sweeps | time to fill (ms) |")
    print("|---|---|" + "---|" * (len(keys) + 2))
    for p in (0.33, 0.66):
        sel = [r for r in stats if r["p_removed"] == p]
        for name in ("sp", "dp"):
            vals = [np.mean([r[name][k] for r in sel]) for k in keys]
            rs = np.mean([r[name]["relax_sweeps"] for r in sel])
            tf = np.mean([r[name]["time_to_fill_s"] for r in sel]) * 1e3
            print(f"| {p:.2f} | {name} | " + " | ".join(f"{v:.4f}" for v in vals) + f" | {rs:.1f} | {tf:.1f} |")
    print("| L | chains | SP site-updates/s | DP site-updates/s | DP time / SP time |")
    print("|---|---|---|---|---|")
    for L in sorted({r["L"] for r in rates}):
        sp = [r for r in rates if r["L"] == L and r["precision"] == "sp"][0]
        dp = [r for r in rates if r["L"] == L and r["precision"] == "dp"][0]
        print(f"| {L} | {sp['chains']} | {sp['site_updates_per_s']:.3e} | {dp['site_updates_per_s']:.3e} | "
              f"{sp['site_updates_per_s'] / dp['site_updates_per_s']:.2f} |")


if __name__ == "__main__":
    main()
