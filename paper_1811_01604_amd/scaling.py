"""Scaling of the gap filling with lattice size and gap fraction on one GPU.

The set-up of the paper's timing study (Section 4, Figs. 3, 5 and 6): square
L x L images of a Whittle-Matern field (nu = 0.5, kappa = 0.2, N(50, 10)),
a fraction p of sites removed at random.  For each (L, p):
  - time to fill one image: map, temperature (e(T, L) table built once per L,
    not timed), R = 1 chain relaxed by the stopping rule plus K = 100
    equilibrium states (M = 100 as in the paper), and the back-transform;
  - the sweep throughput with enough chains to fill the GPU (R chains of
    100 relaxation sweeps + 1 state from random starts, gap-site updates per
    second of sweep time; the first sweeps from random angles carry more
    double-precision re-decisions than later ones).

    python -m paper_1811_01604_amd.scaling [--sizes 32,64,...] [--fractions ...]

prints one JSON line per case and a markdown table at the end.  Defaults: L
from 32 to 8192 at p = 0.33 and 0.66, and p from 0.05 to 0.95 at L = 2048.
The CPU side of the comparison (the oracle on the same images) is timed by
the benchmark script's --cpu-scaling option.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_case(ctx, L: int, p: float, rep: int = 0, K: int = 100, R: int = 1, throughput: bool = True) -> dict:
    import torch
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import synth
    import paper_1811_01604_amd as mpr
    im = synth.workload_table2(L, p, rep)
    imgs = mpr.images([(L, L)])
    z = torch.from_numpy(im.z.astype(np.float32)).cuda()
    mk = torch.from_numpy(im.mask).cuda()
    phi, ps, zh = torch.zeros_like(z), torch.zeros_like(z), torch.zeros_like(z)
    # a shorter e(T, L) table than the library default (12 temperatures,
    # 100 + 200 sweeps): the study times the sweep, not the table
    base = dict(table_nT=12, table_burn=100, table_meas=200, seed=7000 + rep)
    prm = mpr.default_params(R=R, K=K, **base)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    zz = ctx.map_to_angles(imgs, z, mk, phi)
    _, T0, _ = ctx.estimate_temperature(imgs, phi, mk, prm, ws)  # builds and caches the table
    # an untimed fill first: the sweep shape is tuned for this chain set on
    # its first sweeps and cached
    ctx.simulate(imgs, phi, mk, T0, prm, ws, ps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    zz = ctx.map_to_angles(imgs, z, mk, phi)
    _, T, _ = ctx.estimate_temperature(imgs, phi, mk, prm, ws)
    ctx.profile_enable(True)  # the fill's own sweep time (event-timed sweep groups)
    st = ctx.simulate(imgs, phi, mk, T, prm, ws, ps)
    ctx.predict(imgs, z, mk, ps, zz, R * K, zh)
    torch.cuda.synchronize()
    t_fill = time.perf_counter() - t0
    pf = ctx.profile_read()
    ctx.profile_enable(False)
    fill_sweep_us = pf["sweep_kernel_ms"] * 1e3 / max(1, pf["chain_sweeps"] // R)
    gap = im.mask == 0
    zt = im.z.astype(np.float32)
    mae = float(np.mean(np.abs(zh.cpu().numpy()[gap] - zt[gap])))
    if not throughput:
        return {"L": L, "p_removed": p, "rep": rep, "R": R, "K": K, "gap_sites": int(gap.sum()),
                "relax_sweeps_mean": float(np.mean([s["relax_sweeps"] for s in st])), "time_to_fill_s": t_fill,
                "MAE": mae, "fill_sweep_us": fill_sweep_us, "fill_tile": pf["last_tile"]}
    # throughput with the GPU full: R chains, 100 relaxation sweeps + 1 state
    R = int(min(256, max(1, (1 << 27) // (L * L))))
    prm_t = mpr.default_params(R=R, K=1, fixed_relax=100, **base)
    ws_t = torch.empty(ctx.workspace_size(imgs, prm_t), dtype=torch.uint8, device="cuda")
    ctx.simulate(imgs, phi, mk, T, prm_t, ws_t, ps)  # tunes the block shape
    ctx.profile_enable(True)
    ctx.simulate(imgs, phi, mk, T, prm_t, ws_t, ps)
    pr = ctx.profile_read()
    ctx.profile_enable(False)
    return {
        "L": L, "p_removed": p, "gap_sites": int(gap.sum()), "T_hat": float(T[0]),
        "relax_sweeps": st[0]["relax_sweeps"], "K": K, "time_to_fill_s": t_fill, "MAE": mae,
        "fill_sweep_us": fill_sweep_us, "fill_tile": pf["last_tile"],
        "chains_for_throughput": R,
        "site_updates_per_s": pr["site_updates"] / (pr["sweep_kernel_ms"] * 1e-3),
        "sweep_ms_one_chain_equiv": pr["sweep_kernel_ms"] / (101.0 * R),
        "tile": pr["last_tile"],
    }


def layouts(args):
    """Time to fill and MAE of the same M in several (R, K) layouts."""
    import paper_1811_01604_amd as mpr
    ctx = mpr.Context(0)
    lay = [tuple(int(v) for v in t.split("x")) for t in args.layouts.split(",")]
    rows = []
    for L in (int(v) for v in args.sizes.split(",")):
        for p in (float(v) for v in args.size_fractions.split(",")):
            for R, K in lay:
                # an untimed fill of another field first: the block shape is tuned per chain count
                run_case(ctx, L, p, args.reps, K=K, R=R, throughput=False)
                rs = [run_case(ctx, L, p, rep, K=K, R=R, throughput=False) for rep in range(args.reps)]
                r = {"L": L, "p_removed": p, "R": R, "K": K, "reps": args.reps,
                     "time_to_fill_s": float(np.mean([x["time_to_fill_s"] for x in rs])),
                     "MAE": float(np.mean([x["MAE"] for x in rs])),
                     "MAE_per_rep": [x["MAE"] for x in rs],
                     "relax_sweeps_mean": float(np.mean([x["relax_sweeps_mean"] for x in rs]))}
                rows.append(r)
                print(json.dumps(r), flush=True)
                log(f"L={L} p={p} ({R},{K}): fill {r['time_to_fill_s'] * 1e3:.1f} ms, MAE {r['MAE']:.4f}")
    ctx.close()
    print("| L | p | (R, K) | time to fill (ms) | MAE (mean over fields) | relax sweeps |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['L']} | {r['p_removed']:.2f} | ({r['R']}, {r['K']}) | {r['time_to_fill_s'] * 1e3:.1f} | "
              f"{r['MAE']:.4f} | {r['relax_sweeps_mean']:.1f} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="32,64,128,256,512,1024,2048,4096,8192")
    ap.add_argument("--size-fractions", default="0.33,0.66")
    ap.add_argument("--fraction-size", type=int, default=2048)
    ap.add_argument("--fractions", default="0.05,0.2,0.35,0.5,0.65,0.8,0.95")
    ap.add_argument("--layouts", default="",
                    help="instead of the study above: time to fill and MAE of M = R K realizations in each "
                         "layout RxK (e.g. 1x100,4x25,10x10) for every size in --sizes at p = --size-fractions, "
                         "over --reps fields")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    if args.layouts:
        return layouts(args)
    import paper_1811_01604_amd as mpr
    ctx = mpr.Context(0)
    rows = []
    cases = [(int(L), float(p)) for L in args.sizes.split(",") for p in args.size_fractions.split(",")]
    cases += [(args.fraction_size, float(p)) for p in args.fractions.split(",")]
    seen = set()
    for L, p in cases:
        if (L, p) in seen:
            continue
        seen.add((L, p))
        r = run_case(ctx, L, p)
        rows.append(r)
        print(json.dumps(r), flush=True)
        log(f"L={L} p={p}: fill {r['time_to_fill_s'] * 1e3:.1f} ms ({r['relax_sweeps']} + {r['K']} sweeps), "
            f"{r['site_updates_per_s']:.3e} site-updates/s with {r['chains_for_throughput']} chains")
    ctx.close()
    print("| L | p | gap sites | relax sweeps | time to fill (ms) | fill sweep (us) | site-updates/s (GPU full) "
          "| chains |")
    print("|---|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['L']} | {r['p_removed']:.2f} | {r['gap_sites']} | {r['relax_sweeps']} | "
              f"{r['time_to_fill_s'] * 1e3:.1f} | {r['fill_sweep_us']:.1f} | {r['site_updates_per_s']:.3e} | "
              f"{r['chains_for_throughput']} |")


if __name__ == "__main__":
    main()
