"""Cost of the realizations' statistics, of the choice of q and of the
temperature tables, on one GPU.

  - Quantiles: the L=4096 workload (lognormal, 66% random gaps) with its 100
    chains' final states recorded (6.7 GB), then mpr_quantiles for the 5%,
    50% and 95% levels: event-timed, as bytes read and written per second
    (100 states + the mask and data per site, 3 outputs per site).
  - Choice of q: L=256 fields of two kinds (Whittle-Matern nu=0.5 kappa=0.2,
    the paper's rough set-up, and nu=2.5 kappa=0.05, smooth), 50% random
    gaps; mpr_select_q over q in {1/8, 1/4, 3/8, 1/2} with 10% of the
    samples held out and M = 100 as (1, 100); then the fill of the real gaps
    at the chosen q and at q = 1/2, and their mean absolute errors.

    python -m paper_1811_01604_amd.stats_study

prints one JSON line per measurement.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def quantile_cost(ctx, mpr, synth, torch):
    im = synth.workload_l4096("random")
    ny, nx = im.z.shape
    n = ny * nx
    imgs = mpr.images([im.z.shape])
    z = torch.from_numpy(im.z.astype(np.float32)).cuda()
    mk = torch.from_numpy(im.mask).cuda()
    phi = torch.zeros_like(z)
    zz = ctx.map_to_angles(imgs, z, mk, phi)
    prm = mpr.default_params(R=100, K=1, fixed_relax=20)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps = torch.zeros_like(z)
    st = torch.empty((100, n), dtype=torch.float32, device="cuda")
    ctx.simulate(imgs, phi, mk, np.array([6e-5]), prm, ws, ps, phi_states=st)
    del ws
    probs = [0.05, 0.5, 0.95]
    zq = torch.empty((len(probs), n), dtype=torch.float32, device="cuda")
    ctx.quantiles(imgs, z, mk, st, 100, probs, zz, zq)  # warm-up
    ms = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.quantiles(imgs, z, mk, st, 100, probs, zz, zq)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = float(np.median(ms)) * 1e-3
    nbytes = n * (100 * 4 + 1 + 4 + len(probs) * 4)
    return {"measure": "quantiles", "workload": "4096x4096, 100 recorded states, 3 levels", "ms": t * 1e3,
            "bytes": nbytes, "GBps": nbytes / t / 1e9, "hbm_frac": nbytes / t / 8e12,
            "note": "call time incl. argument upload and synchronisation"}


def q_choice(ctx, mpr, synth, torch, nu, kappa, seed):
    L = 256
    z = synth.matern_field(L, L, nu, kappa, 50.0, 10.0, seed)
    m = synth.random_mask(L, L, 0.5, seed + 1)
    img = mpr.images([(L, L)])
    zd = torch.from_numpy(z.astype(np.float32)).cuda()
    mk = torch.from_numpy(m).cuda()
    qs = [0.125, 0.25, 0.375, 0.5]
    prm = mpr.default_params(R=1, K=100, seed=seed + 2, table_nT=16, table_burn=100, table_meas=200)
    ws = torch.empty(ctx.select_q_workspace_size(img, prm, qs), dtype=torch.uint8, device="cuda")
    ctx.select_q(img, zd, mk, prm, qs, 0.1, ws)  # builds the tables
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qb, mae, T = ctx.select_q(img, zd, mk, prm, qs, 0.1, ws)
    torch.cuda.synchronize()
    t_sel = time.perf_counter() - t0
    g = m == 0
    out = {}
    for name, q in (("chosen", qb), ("half", 0.5)):
        p = mpr.default_params(R=1, K=100, seed=seed + 2, table_nT=16, table_burn=100, table_meas=200, q=q,
                               fp64=0 if q == 0.5 else 1)
        phi, ps, zh = torch.zeros_like(zd), torch.zeros_like(zd), torch.zeros_like(zd)
        zz = ctx.map_to_angles(img, zd, mk, phi)
        _, Th, _ = ctx.estimate_temperature(img, phi, mk, p, ws)
        ctx.simulate(img, phi, mk, Th, p, ws, ps)
        ctx.predict(img, zd, mk, ps, zz, 100, zh)
        out[name] = float(np.mean(np.abs(zh.cpu().numpy()[g] - z.astype(np.float32)[g])))
    return {"measure": "select_q", "field": f"WM nu={nu} kappa={kappa}, 256x256, 50% gaps", "q_grid": qs,
            "holdout_mae": [float(v) for v in mae], "T_hat": [float(v) for v in T], "q_best": qb,
            "select_s (tables cached)": t_sel, "gap_MAE_at_q_best": out["chosen"], "gap_MAE_at_half": out["half"]}


def table_cap(mpr, synth, torch):
    im = synth.workload_l4096("random")
    imgs = mpr.images([im.z.shape])
    z = torch.from_numpy(im.z.astype(np.float32)).cuda()
    mk = torch.from_numpy(im.mask).cuda()
    g = im.mask == 0
    rows = []
    for cap in (256, 1024, 0):
        ctx = mpr.Context(0)
        prm = mpr.default_params(R=100, K=1, table_side_cap=cap)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        phi, ps, zh = torch.zeros_like(z), torch.zeros_like(z), torch.zeros_like(z)
        zz = ctx.map_to_angles(imgs, z, mk, phi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e_s, T, cl = ctx.estimate_temperature(imgs, phi, mk, prm, ws)
        torch.cuda.synchronize()
        t_tab = time.perf_counter() - t0
        ctx.simulate(imgs, phi, mk, T, prm, ws, ps)
        ctx.predict(imgs, z, mk, ps, zz, 100, zh)
        mae = float(np.mean(np.abs(zh.cpu().numpy()[g] - im.z.astype(np.float32)[g])))
        rows.append({"table_grid": "4096x4096" if cap == 0 else f"{cap}x{cap}", "build_s": t_tab,
                     "T_hat": float(T[0]), "clamped": bool(cl[0]), "gap_MAE": mae})
        del ws
        ctx.close()
        log(f"table {rows[-1]['table_grid']}: built in {t_tab:.3f} s, T_hat {T[0]:.4e}, MAE {mae:.6f}")
    full = rows[-1]["T_hat"]
    for r in rows:
        r["T_hat_over_full"] = r["T_hat"] / full
    return {"measure": "table_side_cap", "workload": "4096x4096 lognormal, 66% random gaps, R=100, K=1",
            "table": "32 temperatures on [1e-5, 10], 200 + 400 sweeps", "rows": rows}


def main():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import synth
    import torch
    import paper_1811_01604_amd as mpr
    ctx = mpr.Context(0)
    r = quantile_cost(ctx, mpr, synth, torch)
    print(json.dumps(r), flush=True)
    log(f"quantiles: {r['ms']:.2f} ms, {r['GBps']:.0f} GB/s")
    for nu, kappa, seed in ((0.5, 0.2, 5000), (2.5, 0.05, 5100)):
        r = q_choice(ctx, mpr, synth, torch, nu, kappa, seed)
        print(json.dumps(r), flush=True)
        log(f"select_q nu={nu}: q* {r['q_best']}, hold-out MAE {r['holdout_mae']}, gap MAE q* "
            f"{r['gap_MAE_at_q_best']:.4f} vs q=1/2 {r['gap_MAE_at_half']:.4f}, {r['select_s (tables cached)']:.3f} s")
    ctx.close()
    print(json.dumps(table_cap(mpr, synth, torch)), flush=True)


if __name__ == "__main__":
    main()
