"""Learned warm start for the MPR chains.

Training data are the library's own conditional simulations: synthetic
fields (Gaussian Matern and lognormal, random and cloud-like masks) are
mapped to angles, their temperature is estimated, and one chain per image
relaxes and averages K equilibrium states (mpr_simulate); the target at each
gap site is (cos q phi_bar, sin q phi_bar) of that mean angle.  The network
(mpr_cnn_*) is trained on the GPU with the library's own forward, backward
and Adam kernels.  At use, its decoded output replaces the U(0, 2 pi) start
of the gap angles; the chain then runs to the same stopping rule, so the
plain random start stays the reference.

Run as a module to train and write the weights:
    python -m paper_1811_01604_amd.warmstart --samples 20000 --out <file.npz>
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart.npz")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------- training data
def _one_field(args):
    """One training image: field and mask of the requested kind (CPU)."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import synth
    i, size, seed = args
    rng = np.random.default_rng(seed * 100003 + i)
    if i % 2 == 0:
        nu = float(rng.choice([0.5, 1.5, 2.5]))
        kappa = float(math.exp(rng.uniform(math.log(0.01), math.log(0.3))))
        z = synth.matern_field(size, size, nu, kappa, 50.0, 10.0, int(rng.integers(1 << 31)))
    else:
        kappa = float(math.exp(rng.uniform(math.log(0.02), math.log(0.1))))
        z = synth.lognormal_field(size, size, 1.5, kappa, 0.5, int(rng.integers(1 << 31)))
    if (i // 2) % 2 == 0:
        m = synth.random_mask(size, size, float(rng.uniform(0.2, 0.8)), int(rng.integers(1 << 31)))
    else:
        m = synth.cloud_mask(size, size, float(rng.uniform(0.2, 0.6)), int(rng.integers(1 << 31)))
    return z.astype(np.float32), m


def _pool_map(fn, args, workers: int, chunksize: int = 1):
    """fn over args in `workers` fresh processes (closed and joined, not
    terminated), or in this process when workers <= 1.  Call it before the
    process touches the GPU: children of a profiled process inherit the
    profiler."""
    if workers <= 1:
        for a in args:
            yield fn(a)
        return
    pool = mp.get_context("spawn").Pool(workers)
    try:
        for r in pool.imap(fn, args, chunksize=chunksize):
            yield r
        pool.close()
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()


def make_fields(n: int, size: int, seed: int, workers: int = 16):
    """n synthetic images of size x size (fields and masks), in parallel."""
    z = np.empty((n, size, size), dtype=np.float32)
    m = np.empty((n, size, size), dtype=np.uint8)
    for i, (zi, mi) in enumerate(_pool_map(_one_field, [(i, size, seed) for i in range(n)], workers, 8)):
        z[i], m[i] = zi, mi
        if (i + 1) % 1000 == 0:
            log(f"  {i + 1} fields")
    return z, m


def simulate_targets(ctx, z: np.ndarray, mask: np.ndarray, K: int = 16, batch: int = 256, seed: int = 9000):
    """Angles, masks and MPR targets on the GPU for every image.

    Returns device tensors phi (n, s, s), sampled (n, s, s) and target
    (n, s, s, 2), and host arrays of T_hat and relaxation sweeps."""
    import torch
    import paper_1811_01604_amd as mpr
    n, s, _ = z.shape
    phi_all = torch.empty((n, s, s), dtype=torch.float32, device="cuda")
    tgt_all = torch.empty((n, s, s, 2), dtype=torch.float32, device="cuda")
    smp_all = torch.from_numpy(mask).cuda()
    Ts, sweeps = [], []
    prm = mpr.default_params(R=1, K=K, seed=seed)
    for b0 in range(0, n, batch):
        nb = min(batch, n - b0)
        imgs = mpr.images([(s, s)] * nb, ids=list(range(b0, b0 + nb)))
        zd = torch.from_numpy(z[b0:b0 + nb]).cuda().reshape(-1)
        md = smp_all[b0:b0 + nb].reshape(-1)
        phi = phi_all[b0:b0 + nb].reshape(-1)
        ctx.map_to_angles(imgs, zd, md, phi)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        _, T, _ = ctx.estimate_temperature(imgs, phi, md, prm, ws)
        ps = torch.empty_like(phi)
        st = ctx.simulate(imgs, phi, md, T, prm, ws, ps)
        th = 0.5 * ps.reshape(nb, s, s) / K
        tg = tgt_all[b0:b0 + nb]
        tg[..., 0] = torch.cos(th)
        tg[..., 1] = torch.sin(th)
        Ts.extend(T.tolist())
        sweeps.extend(x["relax_sweeps"] for x in st)
        del ws
    return phi_all, smp_all, tgt_all, np.array(Ts), np.array(sweeps)


# ------------------------------------------------------------------ network
def init_params(ctx, seed: int) -> np.ndarray:
    """He-normal weights in the library's layout; residual second convs and
    the head start small; unused stem inputs and head outputs are zero."""
    rng = np.random.default_rng(seed)
    n_layers, C = 18, 32
    out = []
    for k in range(n_layers):
        fan_in = 9 * (3 if k == 0 else C)
        W = rng.normal(0.0, math.sqrt(2.0 / fan_in), size=(9, C, C))
        if k == 0:
            W[:, 3:, :] = 0.0
        if 2 <= k < n_layers - 1 and k % 2 == 0:
            W *= 0.1
        if k == n_layers - 1:
            W *= 0.1
            W[:, :, 2:] = 0.0
        out.append(np.concatenate([W.ravel(), np.zeros(C)]))
    p = np.concatenate(out).astype(np.float32)
    assert p.size == ctx.cnn_param_count()
    return p


def train(ctx, phi, sampled, target, epochs: int = 8, batch: int = 32, lr: float = 2e-3, seed: int = 1,
          val_frac: float = 0.05):
    """Adam with cosine decay on the masked (cos, sin) loss."""
    import torch
    n, h, w = phi.shape
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    n_val = max(1, int(val_frac * n))
    val, trn = perm[:n_val], perm[n_val:]
    p = torch.from_numpy(init_params(ctx, seed)).cuda()
    packed = torch.empty(ctx.cnn_packed_bytes() // 2, dtype=torch.bfloat16, device="cuda")
    m, v, g = torch.zeros_like(p), torch.zeros_like(p), torch.zeros_like(p)
    ws = torch.empty(ctx.cnn_workspace_size(batch, h, w, True), dtype=torch.uint8, device="cuda")
    lw = torch.empty(((batch * h * w + 255) // 256) * 8 + 256, dtype=torch.uint8, device="cuda")
    x = torch.empty((batch, h, w, 32), dtype=torch.bfloat16, device="cuda")
    y, dy = torch.empty_like(x), torch.empty_like(x)
    steps_per_epoch = len(trn) // batch
    total = epochs * steps_per_epoch
    step = 0
    hist = []

    def run_batch(idx, training):
        it = torch.from_numpy(idx).cuda()
        ph = phi.index_select(0, it).contiguous()
        sm = sampled.index_select(0, it).contiguous()
        tg = target.index_select(0, it).contiguous()
        nb = len(idx)
        xb, yb, db = x[:nb], y[:nb], dy[:nb]
        ctx.cnn_encode(ph, sm, xb)
        ctx.cnn_forward(p, packed, xb, ws, yb, training=training)
        ng = int((sm == 0).sum().item())
        return ctx.cnn_loss(yb, tg, sm, ng, db, lw), xb, db

    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(trn)
        run = 0.0
        for k in range(steps_per_epoch):
            step += 1
            lr_t = 0.5 * lr * (1.0 + math.cos(math.pi * (step - 1) / total)) + 1e-5
            ctx.cnn_pack(p, packed)
            L, xb, db = run_batch(order[k * batch:(k + 1) * batch], True)
            ctx.cnn_backward(p, packed, xb, db, ws, g)
            ctx.cnn_opt_step(p, g, m, v, step, lr=lr_t)
            run += L
        ctx.cnn_pack(p, packed)
        vl = [run_batch(val[i:i + batch], False)[0] for i in range(0, len(val), batch)]
        hist.append({"epoch": ep, "train_loss": run / steps_per_epoch, "val_loss": float(np.mean(vl)),
                     "time_s": time.perf_counter() - t0})
        log(f"epoch {ep}: train {run / steps_per_epoch:.5f} val {np.mean(vl):.5f} ({time.perf_counter() - t0:.1f} s)")
    return p.cpu().numpy(), hist


def save(params: np.ndarray, path: str, info: dict):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez_compressed(path, params=params.astype(np.float32), info=np.array(json.dumps(info)))


def load(path: str = DEFAULT_WEIGHTS):
    with np.load(path, allow_pickle=False) as f:
        return f["params"].astype(np.float32), json.loads(str(f["info"]))


class WarmStart:
    """Starting gap angles from the trained network (inference on the GPU)."""

    def __init__(self, ctx, params: np.ndarray):
        import torch
        self.ctx = ctx
        self.p = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).cuda()
        self.packed = torch.empty(ctx.cnn_packed_bytes() // 2, dtype=torch.bfloat16, device="cuda")
        ctx.cnn_pack(self.p, self.packed)
        self._ws = None

    def __call__(self, phi, sampled, phi_init):
        """phi, sampled, phi_init: device tensors of shape (n, h, w); one
        library call (encode, inference and decode fused)."""
        import torch
        n, h, w = phi.shape
        need = self.ctx.cnn_workspace_size(n, h, w, False)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        self.ctx.cnn_infer(self.p, self.packed, phi, sampled, self._ws, phi_init)


def _eval_field(args):
    """One evaluation image (CPU): Gaussian Matern nu=1.5 kappa=0.05 N(50, 10)
    with a 50% random or 50th-percentile cloud mask."""
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import synth
    kind, size, seed = args
    z = synth.matern_field(size, size, 1.5, 0.05, 50.0, 10.0, 7000 + seed)
    if kind == "random":
        m = synth.random_mask(size, size, 0.5, 8000 + seed)
    else:
        m = synth.cloud_mask(size, size, 0.5, 8500 + seed)
    return z.astype(np.float32), m


def make_eval_fields(size: int = 2048, seeds: int = 32, workers: int = 8):
    """The evaluation images, both mask kinds per seed (CPU; before the GPU
    is touched when workers > 1): a list of (kind, seed, z, mask)."""
    cases = [(kind, size, s) for kind in ("random", "cloud") for s in range(seeds)]
    return [(kind, s, z, m) for (kind, _, s), (z, m) in zip(cases, _pool_map(_eval_field, cases, workers))]


def _t95(n: int) -> float:
    """Two-sided 95% quantile of Student's t with n - 1 degrees of freedom."""
    import scipy.stats
    return float(scipy.stats.t.ppf(0.975, max(n - 1, 1)))


def evaluate(ctx, model, fields, layouts=((1, 100),), min_states=None):
    """Plain random start vs warm start on fresh images, for each (R, K)
    layout of the M = R K realizations: sweeps to stop (mean over the R
    chains), time to fill (warm start inference + simulate + predict, T_hat
    estimated once per image and shared) and MAE of the prediction at the
    gaps, for random and cloud masks.  The MAE comparison is paired (same
    image, temperature and random numbers): per image the ratio warm/plain,
    its mean and 95% confidence interval over the images.  A layout with
    K below the library's warm_min_states gets the plain fill only (the
    library refuses that warm start)."""
    import torch
    import paper_1811_01604_amd as mpr
    if min_states is None:
        min_states = mpr.default_params().warm_min_states
    out = {lay: {} for lay in layouts}
    # one untimed pass over the first image first: the e(T, L) table, the
    # block-shape tuning and the caches are not part of a fill's time
    for warmup, (kind, s, z, m) in [(True, fields[0])] + [(False, f) for f in fields]:
        size = z.shape[0]
        imgs = mpr.images([(size, size)])
        zd = torch.from_numpy(z).cuda()
        md = torch.from_numpy(m).cuda()
        phi = torch.empty_like(zd)
        zz = ctx.map_to_angles(imgs, zd, md, phi)
        g = m == 0
        T = None
        for R, K in layouts:
            prm = mpr.default_params(R=R, K=K, seed=4242, warm_min_states=min_states)
            ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
            if T is None:
                _, T, _ = ctx.estimate_temperature(imgs, phi, md, prm, ws)
            res = {}
            for mode in ("plain", "warm"):
                if mode == "warm" and K < min_states:
                    continue
                ps, zh = torch.empty_like(phi), torch.empty_like(phi)
                init = torch.empty_like(phi) if mode == "warm" else None
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode == "warm":
                    model(phi.view(1, size, size), md.view(1, size, size), init.view(1, size, size))
                st = ctx.simulate(imgs, phi, md, T, prm, ws, ps, phi_init=init)
                ctx.predict(imgs, zd, md, ps, zz, R * K, zh)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                mae = float(np.mean(np.abs(zh.cpu().numpy()[g] - z[g])))
                res[mode] = {"sweeps": float(np.mean([c["relax_sweeps"] for c in st])), "time_s": dt, "mae": mae}
            del ws
            if warmup:
                continue
            out[(R, K)].setdefault(kind, []).append(res)
            w = res.get("warm")
            log(f"  ({R},{K}) {kind} seed {s}: plain {res['plain']['sweeps']:.1f} sweeps "
                f"{res['plain']['time_s'] * 1e3:.0f} ms MAE {res['plain']['mae']:.4f}" +
                (f" | warm {w['sweeps']:.1f} sweeps {w['time_s'] * 1e3:.0f} ms MAE {w['mae']:.4f}" if w else
                 " | warm start refused (K < warm_min_states)"))
    summary = {}
    for (R, K), by_kind in out.items():
        lay = {}
        for kind, rows in by_kind.items():
            f = lambda mode, key: float(np.mean([r[mode][key] for r in rows]))  # noqa: E731
            d = {"seeds": len(rows), "sweeps_plain": f("plain", "sweeps"),
                 "time_to_fill_plain_s": f("plain", "time_s"), "mae_plain": f("plain", "mae"),
                 "mae_seed_spread_plain": float(np.std([r["plain"]["mae"] for r in rows]))}
            if all("warm" in r for r in rows):
                ratio = np.array([r["warm"]["mae"] / r["plain"]["mae"] for r in rows])
                half = _t95(len(rows)) * float(np.std(ratio, ddof=1)) / np.sqrt(len(rows)) if len(rows) > 1 else 0.0
                lo, hi = float(ratio.mean()) - half, float(ratio.mean()) + half
                d.update({"sweeps_warm": f("warm", "sweeps"), "time_to_fill_warm_s": f("warm", "time_s"),
                          "mae_warm": f("warm", "mae"), "mae_warm_over_plain": float(ratio.mean()),
                          "mae_ratio_ci95": [lo, hi],
                          # the target: warm MAE within 1% of plain, with 95% confidence
                          "within_1pct": bool(lo >= 0.99 and hi <= 1.01),
                          "time_speedup": f("plain", "time_s") / f("warm", "time_s")})
            else:
                d["warm"] = f"refused: K = {K} < warm_min_states = {min_states}"
            lay[kind] = d
        summary[f"{R}x{K}"] = lay
    return summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=20000)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--K", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--evaluate", default="",
                    help="instead of training: compare the committed network's warm start with the plain start "
                         "in these layouts RxK (e.g. 1x100,2x50,4x25) on --eval-seeds images of --eval-size^2 "
                         "per mask kind, with the library's warm-start check set to --min-states; one JSON line")
    ap.add_argument("--eval-size", type=int, default=2048)
    ap.add_argument("--eval-seeds", type=int, default=32)
    ap.add_argument("--min-states", type=int, default=-1, help="-1: the library default")
    args = ap.parse_args()
    if args.evaluate:
        layouts = tuple(tuple(int(v) for v in t.split("x")) for t in args.evaluate.split(","))
        fields = make_eval_fields(size=args.eval_size, seeds=args.eval_seeds, workers=min(args.workers, 8))
        if ROOT not in sys.path:
            sys.path.insert(0, ROOT)
        import paper_1811_01604_amd as mpr
        ctx = mpr.Context(0)
        params, info = load()
        res = evaluate(ctx, WarmStart(ctx, params), fields, layouts=layouts,
                       min_states=None if args.min_states < 0 else args.min_states)
        print(json.dumps({"layouts": res, "size": args.eval_size, "seeds": args.eval_seeds,
                          "min_states": args.min_states}), flush=True)
        ctx.close()
        return
    t0 = time.perf_counter()
    log(f"generating {args.samples} fields of {args.size}^2 on {args.workers} workers")
    z, mask = make_fields(args.samples, args.size, args.seed, args.workers)
    t_fields = time.perf_counter() - t0
    log(f"  {t_fields:.1f} s")
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import paper_1811_01604_amd as mpr
    ctx = mpr.Context(0)
    t1 = time.perf_counter()
    phi, sampled, target, T, sweeps = simulate_targets(ctx, z, mask, K=args.K)
    t_sim = time.perf_counter() - t1
    log(f"targets: {t_sim:.1f} s, T_hat median {np.median(T):.2e}, relax sweeps mean {sweeps.mean():.1f}")
    del z
    params, hist = train(ctx, phi, sampled, target, epochs=args.epochs, batch=args.batch, lr=args.lr,
                         seed=args.seed)
    info = {"samples": args.samples, "size": args.size, "K": args.K, "epochs": args.epochs, "batch": args.batch,
            "lr": args.lr, "seed": args.seed, "history": hist, "fields_s": t_fields, "targets_s": t_sim,
            "T_hat_median": float(np.median(T)), "relax_sweeps_mean": float(sweeps.mean())}
    save(params, args.out, info)
    log(f"wrote {args.out}")
    ctx.close()


if __name__ == "__main__":
    main()
