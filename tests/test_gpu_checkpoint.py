"""Checkpoint and resume of mpr_simulate (determinism: an interrupted run
continues bit for bit).

A run stopped at params.sweep_limit leaves its whole state in the
workspace; the workspace bytes are copied to the host (the checkpoint) and
back into another workspace at another address, and a call with
params.resume = 1 continues the run.  Random numbers are keyed by (site,
sweep, chain, image) and energies are summed in fixed point, so the resumed
run must give the uninterrupted run's sums, spreads, recorded states and
per-chain statistics exactly, whatever block shapes the calls use (the
fused tile sweep exchanges its buffers every sweep, which the resumed
descriptors must follow).  Resuming what is not a stopped run of the same
images, parameters and temperatures is refused.
"""
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1811_01604_amd as mpr  # noqa: E402

pytestmark = pytest.mark.gpu

SHAPES = [(3, 5), (130, 257), (70, 600), (33, 129)]
FUSED32 = 32 | mpr.TILE_FUSED
FUSED16 = 16 | mpr.TILE_FUSED
COMPACT4 = 4 | mpr.TILE_COMPACT


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


@pytest.fixture(scope="module")
def data(ctx):
    zs, ms = [], []
    for b, (ny, nx) in enumerate(SHAPES):
        z = synth.matern_field(nx, max(ny, 2), 1.5, 0.1, 50.0, 10.0, 80 + b)[:ny]
        zs.append(z.astype(np.float32))
        ms.append(synth.random_mask(nx, ny, 0.35 + 0.1 * b, 90 + b))
    imgs = mpr.images(SHAPES)
    z = dev(np.concatenate([a.ravel() for a in zs]))
    mk = dev(np.concatenate([a.ravel() for a in ms]), torch.uint8)
    phi = torch.zeros_like(z)
    ctx.map_to_angles(imgs, z, mk, phi)
    return imgs, phi, mk, np.full(len(SHAPES), 0.03)


PRM = dict(R=3, K=6, spread=1, seed=4242)


def outputs(ps, m2, states, st):
    return {"sum": ps.cpu().numpy().tobytes(), "m2": m2.cpu().numpy().tobytes(),
            "states": states.cpu().numpy().tobytes(),
            "stats": [(s["relax_sweeps"], s["not_converged"], s["k_last"], s["a_final"], s["A_last"]) for s in st]}


def buffers(phi, prm):
    return (torch.full_like(phi, -1.0), torch.full_like(phi, -1.0),
            torch.zeros(prm.R * prm.K * phi.numel(), device="cuda"))


def uninterrupted(ctx, data, tile):
    imgs, phi, mk, Ts = data
    prm = mpr.default_params(tile_rows=tile, sweeps_per_launch=5, **PRM)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps, m2, states = buffers(phi, prm)
    st = ctx.simulate(imgs, phi, mk, Ts, prm, ws, ps, phi_m2=m2, phi_states=states)
    return outputs(ps, m2, states, st)


def moved(ws):
    """The workspace bytes through the host into a new buffer at another
    address (512 bytes into a larger allocation, keeping 256-byte alignment)."""
    host = ws.cpu().numpy().copy()
    big = torch.zeros(ws.numel() + 1024, dtype=torch.uint8, device="cuda")
    out = big[512:512 + ws.numel()]
    out.copy_(torch.from_numpy(host).cuda())
    assert out.data_ptr() != ws.data_ptr()
    return big, out


def test_resumed_run_equals_the_uninterrupted_run(ctx, data):
    imgs, phi, mk, Ts = data
    ref = uninterrupted(ctx, data, FUSED32)
    say(f"  uninterrupted: relax sweeps {[s[0] for s in ref['stats']]}")
    assert ref == uninterrupted(ctx, data, COMPACT4)
    # stop after 17 sweeps, checkpoint to the host, resume elsewhere with another shape
    prm = mpr.default_params(tile_rows=FUSED32, sweeps_per_launch=5, sweep_limit=17, **PRM)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps, m2, states = buffers(phi, prm)
    done, st = ctx.simulate(imgs, phi, mk, Ts, prm, ws, ps, phi_m2=m2, phi_states=states, allow_incomplete=True)
    assert not done
    assert bool((ps == -1.0).all()) and bool((m2 == -1.0).all())  # nothing finalized yet
    _keep, ws2 = moved(ws)
    del ws
    prm.sweep_limit, prm.resume, prm.tile_rows = 0, 1, COMPACT4
    done, st = ctx.simulate(imgs, phi, mk, Ts, prm, ws2, ps, phi_m2=m2, phi_states=states, allow_incomplete=True)
    assert done
    assert outputs(ps, m2, states, st) == ref
    # a finished run is not resumable
    with pytest.raises(mpr.MprError) as e:
        ctx.simulate(imgs, phi, mk, Ts, prm, ws2, ps, phi_m2=m2, phi_states=states)
    assert e.value.code == mpr.MPR_ERR_ARG


def test_many_short_calls_with_changing_shapes(ctx, data):
    """Calls of 7 sweeps each, alternating fused and two-pass shapes, on
    the same workspace, until the run is done."""
    imgs, phi, mk, Ts = data
    ref = uninterrupted(ctx, data, FUSED16)
    prm = mpr.default_params(sweeps_per_launch=3, sweep_limit=7, **PRM)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps, m2, states = buffers(phi, prm)
    shapes = [FUSED16, COMPACT4, FUSED32, 2, FUSED32]
    calls, done = 0, False
    while not done:
        prm.tile_rows = shapes[calls % len(shapes)]
        prm.resume = 1 if calls else 0
        done, st = ctx.simulate(imgs, phi, mk, Ts, prm, ws, ps, phi_m2=m2, phi_states=states,
                                allow_incomplete=True)
        calls += 1
        assert calls < 200
    say(f"  {calls} calls of at most 7 sweeps")
    assert calls > 3
    assert outputs(ps, m2, states, st) == ref


def test_resume_is_refused_without_a_matching_stopped_run(ctx, data):
    imgs, phi, mk, Ts = data
    prm = mpr.default_params(sweep_limit=5, **PRM)
    ws = torch.zeros(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps = torch.zeros_like(phi)
    prm.resume = 1
    with pytest.raises(mpr.MprError) as e:  # a zeroed workspace holds no run
        ctx.simulate(imgs, phi, mk, Ts, prm, ws, ps)
    assert e.value.code == mpr.MPR_ERR_ARG
    prm.resume = 0
    done, _ = ctx.simulate(imgs, phi, mk, Ts, prm, ws, ps, allow_incomplete=True)
    assert not done
    for change in (dict(seed=4243), dict(K=5), dict(n_f=4)):  # the same workspace size, another run
        q = mpr.default_params(sweep_limit=5, resume=1, **{**PRM, **change})
        assert ctx.workspace_size(imgs, q) == ws.numel()
        with pytest.raises(mpr.MprError) as e:
            ctx.simulate(imgs, phi, mk, Ts, q, ws, ps)
        assert e.value.code == mpr.MPR_ERR_ARG, change
    q = mpr.default_params(sweep_limit=5, resume=1, **PRM)
    with pytest.raises(mpr.MprError) as e:  # other temperatures
        ctx.simulate(imgs, phi, mk, Ts * 1.5, q, ws, ps)
    assert e.value.code == mpr.MPR_ERR_ARG
    # the stopped run itself resumes
    done, _ = ctx.simulate(imgs, phi, mk, Ts, q, ws, ps, allow_incomplete=True)
    assert not done
