"""The ragged batch at its full size: 256 images with sides log-uniform in
[128, 2048] (Matern fields, nu in {0.5, 1.5, 2.5}, kappa log-uniform in
[0.01, 0.3], 20-80% of the sites removed at random), R = 16 chains each
(M = 16), filled by one call each of map, temperature, simulate and predict.

At this size the oracle cannot follow the whole batch, so the checks are
properties that hold at any size and per-image comparisons the oracle can
afford: samples copied bit for bit, predictions inside each image's data
range, every chain stopped by the stopping rule's own test, each image's
sums bit-identical to those of the image run alone (smallest, median and
largest), and the smallest image's prediction against the oracle's at a
fixed temperature.  The e(T, L) tables use 12 temperatures and 100 + 200
sweeps (a shorter table than the library default, to keep the test short).
"""
import sys
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_1811_01604_amd as mpr  # noqa: E402

pytestmark = pytest.mark.gpu
R = 16
TABLE = dict(table_nT=12, table_burn=100, table_meas=200)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mpr.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def batch():
    t0 = time.perf_counter()
    ims = synth.ragged_batch(256, workers=8)
    say(f"batch: 256 images, {sum(im.z.size for im in ims)} sites, made in {time.perf_counter() - t0:.1f} s")
    return ims


def pack(ims, sel):
    shapes = [ims[i].z.shape for i in sel]
    imgs = mpr.images(shapes, ids=list(sel))
    z = np.concatenate([ims[i].z.astype(np.float32).ravel() for i in sel])
    m = np.concatenate([ims[i].mask.ravel() for i in sel])
    return imgs, z, m


@pytest.fixture(scope="module")
def filled(ctx, batch):
    sel = list(range(len(batch)))
    imgs, z, m = pack(batch, sel)
    zd = torch.from_numpy(z).cuda()
    mk = torch.from_numpy(m).cuda()
    phi, ps, zh = torch.zeros_like(zd), torch.zeros_like(zd), torch.zeros_like(zd)
    prm = mpr.default_params(R=R, K=1, **TABLE)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    say(f"  workspace {ws.numel() / 2**30:.2f} GiB")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    zz = ctx.map_to_angles(imgs, zd, mk, phi)
    e_s, T, cl = ctx.estimate_temperature(imgs, phi, mk, prm, ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = ctx.simulate(imgs, phi, mk, T, prm, ws, ps)
    ctx.predict(imgs, zd, mk, ps, zz, R, zh)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sweeps = np.array([s["relax_sweeps"] for s in st]) + 1
    say(f"  map + 256 tables {t1 - t0:.2f} s; simulate + predict {t2 - t1:.2f} s, "
        f"sweeps per chain {sweeps.mean():.1f} (max {sweeps.max()})")
    del ws
    return dict(imgs=imgs, z=z, m=m, zz=zz, T=T, clamped=cl, stats=st, phi_sum=ps.cpu().numpy(),
                z_hat=zh.cpu().numpy(), prm=prm)


def test_batch_outputs_hold_their_invariants(batch, filled):
    z, m, zh, ps = filled["z"], filled["m"], filled["z_hat"], filled["phi_sum"]
    s = m == 1
    assert np.array_equal(zh[s].view(np.uint32), z[s].view(np.uint32))
    assert np.all(ps[s] == 0)
    g = ~s
    assert np.all((ps[g] >= 0) & (ps[g] < 2 * np.pi * R))
    off = 0
    for b, im in enumerate(batch):
        n = im.z.size
        lo, hi = filled["zz"][2 * b], filled["zz"][2 * b + 1]
        zg = zh[off:off + n][m[off:off + n] == 0].astype(np.float64)
        assert zg.size == 0 or (zg.min() >= np.float32(lo) and zg.max() <= np.float32(hi)), b
        off += n
    prm = filled["prm"]
    for c, st in enumerate(filled["stats"]):
        t = st["relax_sweeps"] - 1
        assert t >= prm.n_fit and t % prm.n_f == 0 and st["k_last"] >= 0 and not st["not_converged"], (c, st)
    assert np.all(np.isfinite(filled["T"])) and np.all(filled["T"] > 0)


def test_batch_images_equal_their_runs_alone(ctx, batch, filled):
    sizes = [im.z.size for im in batch]
    order = np.argsort(sizes)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    prm = filled["prm"]
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        imgs, z, m = pack(batch, [i])
        zd = torch.from_numpy(z).cuda()
        mk = torch.from_numpy(m).cuda()
        phi, ps = torch.zeros_like(zd), torch.zeros_like(zd)
        ctx.map_to_angles(imgs, zd, mk, phi)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        st = ctx.simulate(imgs, phi, mk, filled["T"][i:i + 1], prm, ws, ps)
        alone = ps.cpu().numpy()
        assert np.array_equal(alone.view(np.uint32), filled["phi_sum"][offs[i]:offs[i + 1]].view(np.uint32)), i
        assert [s["relax_sweeps"] for s in st] == [s["relax_sweeps"] for s in filled["stats"][R * i:R * (i + 1)]]
        say(f"  image {i} ({batch[i].z.shape}): identical alone and in the batch")


def test_batch_smallest_image_against_oracle(ctx, batch):
    """The smallest image at a fixed temperature (an input of both sides):
    the prediction's mean absolute error matches the oracle's within 3%."""
    i = int(np.argmin([im.z.size for im in batch]))
    im = batch[i]
    T = 0.05
    imgs, z, m = pack(batch, [i])
    zd = torch.from_numpy(z).cuda()
    mk = torch.from_numpy(m).cuda()
    phi, ps, zh = torch.zeros_like(zd), torch.zeros_like(zd), torch.zeros_like(zd)
    zz = ctx.map_to_angles(imgs, zd, mk, phi)
    prm = mpr.default_params(R=R, K=1, seed=21)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ctx.simulate(imgs, phi, mk, np.array([T]), prm, ws, ps)
    ctx.predict(imgs, zd, mk, ps, zz, R, zh)
    zt = im.z.astype(np.float32).astype(np.float64)
    po, zzo = oracle.map_to_angles(zt, im.mask)
    t0 = time.perf_counter()
    pso, sto, _, _ = oracle.simulate(po.astype(np.float32).astype(np.float64), im.mask, T,
                                     oracle.default_params(R=R, K=1, seed=21, stream=i))
    zo = oracle.predict(zt, im.mask, pso, R, zzo)
    g = im.mask == 0
    mae_g = float(np.mean(np.abs(zh.cpu().numpy().reshape(im.z.shape)[g] - zt[g])))
    mae_o = float(np.mean(np.abs(zo[g] - zt[g])))
    say(f"  image {i} {im.z.shape}: MAE gpu {mae_g:.4f} oracle {mae_o:.4f} (oracle {time.perf_counter() - t0:.1f} s)")
    assert abs(mae_g / mae_o - 1.0) < 0.03
