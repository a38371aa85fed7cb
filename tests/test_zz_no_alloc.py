"""The allocation-free simulate (mpr_simulate_noalloc, the library's static
per-device workspace) against mpr_simulate with a caller's workspace, called
through the C ABI: the same kernels, random numbers and stopping rule, so
the outputs must be equal bit for bit.  Two calls in a row, the second on a
smaller batch (the static workspace keeps the first call's contents), a third
in the persistent sweep shape, then a batch too large for the static
workspace, which is refused before any work.
"""
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1811_01604_amd as mpr  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mpr.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def batch(shapes, seed):
    zs, ms = [], []
    for b, (ny, nx) in enumerate(shapes):
        zs.append(synth.matern_field(nx, ny, 1.5, 0.1, 50.0, 10.0, seed + b).astype(np.float32))
        ms.append(synth.random_mask(nx, ny, 0.4 + 0.1 * b, seed + 50 + b))
    imgs = mpr.images(shapes)
    z = dev(np.concatenate([a.ravel() for a in zs]))
    mk = dev(np.concatenate([a.ravel() for a in ms]), torch.uint8)
    return imgs, z, mk


def outputs(ps, m2, states, st):
    return (ps.cpu().numpy().tobytes(), m2.cpu().numpy().tobytes(),
            None if states is None else states.cpu().numpy().tobytes(),
            [(s["relax_sweeps"], s["not_converged"], s["k_last"], s["a_final"], s["A_last"]) for s in st])


def both(ctx, shapes, seed, T, record, **kw):
    imgs, z, mk = batch(shapes, seed)
    phi = torch.zeros_like(z)
    ctx.map_to_angles(imgs, z, mk, phi)
    prm = mpr.default_params(seed=seed, **kw)
    Ts = np.full(len(shapes), T)
    ns = phi.numel()
    res = []
    for noalloc in (False, True):
        ps = torch.full_like(phi, -1.0)
        m2 = torch.full_like(phi, -1.0)
        states = torch.zeros(prm.R * prm.K * ns, device="cuda") if record else None
        if noalloc:
            st = ctx.simulate_noalloc(imgs, phi, mk, Ts, prm, ps, phi_m2=m2, phi_states=states)
        else:
            ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
            st = ctx.simulate(imgs, phi, mk, Ts, prm, ws, ps, phi_m2=m2, phi_states=states)
            del ws
        torch.cuda.synchronize()
        res.append(outputs(ps, m2, states, st))
    return prm, imgs, res


def test_noalloc_equals_simulate_on_two_calls_the_second_smaller(ctx):
    say("  call 1: 2 images (96x130, 64x64), R=3, K=4, spread, recorded states")
    prm, imgs, (a, b) = both(ctx, [(96, 130), (64, 64)], 900, 0.05, True, R=3, K=4, spread=1)
    need = mpr.load().mpr_workspace_size(imgs, len(imgs), prm)
    assert 0 < need <= mpr.load().mpr_simulate_noalloc_max_bytes()
    assert a == b
    say(f"  call 1 equal ({need} workspace bytes); call 2: 1 image (40x50), R=2, K=3")
    _, _, (a, b) = both(ctx, [(40, 50)], 901, 0.02, False, R=2, K=3, spread=1)
    assert a == b
    say("  call 2 equal; call 3: the same image in the persistent sweep shape (no graph either way)")
    tile = 32 | mpr.TILE_FUSED | mpr.TILE_PERSIST
    _, _, (a, b) = both(ctx, [(40, 50)], 901, 0.02, False, R=2, K=3, spread=1, tile_rows=tile)
    assert a == b
    say("  call 3 equal")


def test_noalloc_refuses_a_batch_beyond_its_static_workspace(ctx):
    imgs, z, mk = batch([(1024, 1024)], 7)
    phi = torch.zeros_like(z)
    prm = mpr.default_params(R=16, K=2)
    need = mpr.load().mpr_workspace_size(imgs, 1, prm)
    assert need > mpr.load().mpr_simulate_noalloc_max_bytes()
    ps = torch.full_like(phi, -1.0)
    with pytest.raises(mpr.MprError) as e:
        ctx.simulate_noalloc(imgs, phi, mk, np.array([0.05]), prm, ps)
    assert e.value.code == mpr.MPR_ERR_WORKSPACE
    assert "static workspace" in str(e.value)
    torch.cuda.synchronize()
    assert bool((ps == -1.0).all())
