"""The fused tile sweep (one launch per sweep on LDS tiles with a halo)
against the two half-sweep launches per sweep.

Both compute Algorithm 1 on colour 0 and then colour 1 of every chain with
the same per-site arithmetic and random numbers, so every output must be
bit-identical: sums of the states, their squared deviations, recorded
states, stopping decisions and the final a.  The batch mixes images smaller
than a tile, a single row, ragged tile edges and several tiles, and starts
from random angles, where weak local fields send many decisions to the
double-precision path.  Parity with the oracle is in test_gpu_parity.py
(teacher-forced half-sweeps in every shape, the fused one included).
"""
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1811_01604_amd as mpr  # noqa: E402

pytestmark = pytest.mark.gpu
FUSED_TILES = [16 | mpr.TILE_FUSED, 24 | mpr.TILE_FUSED, 32 | mpr.TILE_FUSED, 48 | mpr.TILE_FUSED,
               8 | mpr.TILE_FUSED, 12 | mpr.TILE_FUSED]
PERSIST_TILES = [r | mpr.TILE_FUSED | mpr.TILE_PERSIST for r in (8, 12, 16, 24, 32)]


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


SHAPES = [(3, 5), (1, 300), (130, 257), (70, 600), (33, 129)]


def batch():
    zs, ms = [], []
    for b, (ny, nx) in enumerate(SHAPES):
        z = synth.matern_field(nx, max(ny, 2), 1.5, 0.1, 50.0, 10.0, 60 + b)[:ny]
        zs.append(z.astype(np.float32))
        ms.append(synth.random_mask(nx, ny, 0.3 + 0.1 * b, 70 + b))
    imgs = mpr.images(SHAPES)
    z = dev(np.concatenate([a.ravel() for a in zs]))
    mk = dev(np.concatenate([a.ravel() for a in ms]), torch.uint8)
    return imgs, z, mk


def run(ctx, imgs, phi, mk, T, tile, spl=0, record=False, **kw):
    prm = mpr.default_params(tile_rows=tile, sweeps_per_launch=spl, **kw)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps = torch.zeros_like(phi)
    m2 = torch.zeros_like(phi) if (prm.K <= 1 or prm.spread) else None
    states = torch.zeros(prm.R * prm.K * phi.numel(), device="cuda") if record else None
    st = ctx.simulate(imgs, phi, mk, T, prm, ws, ps, phi_m2=m2, phi_states=states)
    out = {"sum": ps.cpu().numpy().tobytes(),
           "stats": [(s["relax_sweeps"], s["not_converged"], s["k_last"], s["a_final"], s["A_last"]) for s in st]}
    if m2 is not None:
        out["m2"] = m2.cpu().numpy().tobytes()
    if record:
        out["states"] = states.cpu().numpy().tobytes()
    return out


@pytest.mark.parametrize("T", [2e-3, 0.05])
def test_fused_sweep_equals_half_sweeps_on_a_ragged_batch(ctx, T):
    """Stopping rule, R = 3 chains x K = 5 states with their spread: every
    fused tile height and graph size equals the plain 4-row half-sweeps."""
    imgs, z, mk = batch()
    phi = torch.zeros_like(z)
    ctx.map_to_angles(imgs, z, mk, phi)
    Ts = np.full(len(SHAPES), T)
    ref = run(ctx, imgs, phi, mk, Ts, 4, 5, R=3, K=5, spread=1)
    say(f"  T={T}: relax sweeps {[s[0] for s in ref['stats']]}")
    for tile, spl in [(FUSED_TILES[0], 5), (FUSED_TILES[1], 1), (FUSED_TILES[2], 64), (FUSED_TILES[2], 3),
                      (FUSED_TILES[3], 4), (FUSED_TILES[4], 2), (FUSED_TILES[5], 7),
                      (PERSIST_TILES[0], 3), (PERSIST_TILES[1], 64), (PERSIST_TILES[2], 1), (PERSIST_TILES[3], 0),
                      (PERSIST_TILES[4], 9)]:
        got = run(ctx, imgs, phi, mk, Ts, tile, spl, R=3, K=5, spread=1)
        for key in ref:
            assert got[key] == ref[key], (tile, spl, key)


def test_fused_sweep_with_recorded_states_and_one_state_chains(ctx):
    """The recorded states (read between the sweep and the control, after
    the fused sweep has swapped its buffers) and the K = 1 layout, whose sums
    are the final states, equal those of the half-sweeps; so does a call
    that starts from given gap angles."""
    imgs, z, mk = batch()
    phi = torch.zeros_like(z)
    ctx.map_to_angles(imgs, z, mk, phi)
    Ts = np.full(len(SHAPES), 0.01)
    for kw in (dict(R=2, K=4, fixed_relax=7), dict(R=5, K=1)):
        rec = kw["K"] > 1
        ref = run(ctx, imgs, phi, mk, Ts, 2 | mpr.TILE_COMPACT, 5, record=rec, **kw)
        for tile in FUSED_TILES + PERSIST_TILES:
            got = run(ctx, imgs, phi, mk, Ts, tile, 5, record=rec, **kw)
            for key in ref:
                assert got[key] == ref[key], (kw, tile, key)


def test_tuner_may_pick_any_shape_with_identical_results(ctx):
    """An autotuned run (which times every shape, fused ones included, on
    its first sweeps) equals a run fixed to one shape."""
    imgs, z, mk = batch()
    phi = torch.zeros_like(z)
    ctx.map_to_angles(imgs, z, mk, phi)
    Ts = np.full(len(SHAPES), 0.02)
    a = run(ctx, imgs, phi, mk, Ts, 0, 0, R=4, K=3)
    b = run(ctx, imgs, phi, mk, Ts, 32 | mpr.TILE_FUSED, 0, R=4, K=3)
    assert a == b
    say(f"  tuned shape {ctx.profile_read()['last_tile']:#x}")


def test_persistent_sweeps_of_a_1024_fill(ctx):
    """A 1024 x 1024 fill in the paper's layout (one chain, 100 states, the
    stopping rule): the persistent launches (many sweeps each, a grid
    barrier between sweeps) give the one-launch-per-sweep results bit for
    bit, whatever the launch length; so do runs cut by the sweep limit and
    resumed."""
    im = synth.workload_l1024()
    imgs = mpr.images([im.z.shape])
    z = dev(im.z.astype(np.float32))
    mk = dev(im.mask, torch.uint8)
    phi = torch.zeros_like(z)
    ctx.map_to_angles(imgs, z, mk, phi)
    Ts = np.array([0.09])
    ref = run(ctx, imgs, phi, mk, Ts, 24 | mpr.TILE_FUSED, 8, R=1, K=100)
    say(f"  relax sweeps {ref['stats'][0][0]}")
    for tile in PERSIST_TILES:
        for spl in (0, 37):
            got = run(ctx, imgs, phi, mk, Ts, tile, spl, R=1, K=100)
            for key in ref:
                assert got[key] == ref[key], (tile, spl, key)
    # cut after 50 and 40 more sweeps (of about 140), resumed with the same workspace
    tile = 16 | mpr.TILE_FUSED | mpr.TILE_PERSIST
    prm = mpr.default_params(R=1, K=100, tile_rows=tile, sweeps_per_launch=0)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps = torch.zeros_like(phi)
    done, st = False, None
    for limit, resume in ((50, 0), (40, 1), (100000, 1)):
        prm = mpr.default_params(R=1, K=100, tile_rows=tile, sweeps_per_launch=0, sweep_limit=limit, resume=resume)
        done, st = ctx.simulate(imgs, phi, mk, Ts, prm, ws, ps, allow_incomplete=True)
        say(f"  limit {limit}: done {done}")
        assert done == (limit > 1000)
    assert ps.cpu().numpy().tobytes() == ref["sum"]
    assert [(s["relax_sweeps"], s["not_converged"], s["k_last"], s["a_final"], s["A_last"]) for s in st] == ref["stats"]


def test_persistent_fill_longer_than_one_launch(ctx):
    """The same 1024 x 1024 chain with 300 equilibrium states: with the
    default launch groups (256 sweeps) the fill takes two persistent
    launches, whose results equal one fused launch per sweep bit for bit."""
    im = synth.workload_l1024()
    imgs = mpr.images([im.z.shape])
    z = dev(im.z.astype(np.float32))
    mk = dev(im.mask, torch.uint8)
    phi = torch.zeros_like(z)
    ctx.map_to_angles(imgs, z, mk, phi)
    Ts = np.array([0.09])
    ref = run(ctx, imgs, phi, mk, Ts, 32 | mpr.TILE_FUSED, 8, R=1, K=300)
    assert ref["stats"][0][0] + 300 > 256  # more sweeps than one launch group
    got = run(ctx, imgs, phi, mk, Ts, 32 | mpr.TILE_FUSED | mpr.TILE_PERSIST, 0, R=1, K=300)
    for key in ref:
        assert got[key] == ref[key], key


def test_persistent_barrier_timeout_is_an_error_and_the_context_recovers(ctx):
    """A barrier wait bound of 1 us (params.barrier_timeout_us), which the
    early blocks of a 256-block persistent launch exceed at the first
    barrier: every block leaves at its next barrier and the call returns
    MPR_ERR_HIP (no hang); the next call on the same context, with the
    default bound, gives the results of one launch per sweep."""
    im = synth.workload_l1024()
    imgs = mpr.images([im.z.shape])
    z = dev(im.z.astype(np.float32))
    mk = dev(im.mask, torch.uint8)
    phi = torch.zeros_like(z)
    ctx.map_to_angles(imgs, z, mk, phi)
    Ts = np.array([0.09])
    tile = 32 | mpr.TILE_FUSED | mpr.TILE_PERSIST
    prm = mpr.default_params(R=1, K=5, fixed_relax=20, tile_rows=tile, barrier_timeout_us=1)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    with pytest.raises(mpr.MprError) as e:
        ctx.simulate(imgs, phi, mk, Ts, prm, ws, torch.zeros_like(phi))
    assert e.value.code == mpr.MPR_ERR_HIP and "barrier" in str(e.value)
    say(f"  refused: {e.value}")
    ref = run(ctx, imgs, phi, mk, Ts, 32 | mpr.TILE_FUSED, 4, R=1, K=5, fixed_relax=20)
    got = run(ctx, imgs, phi, mk, Ts, tile, 0, R=1, K=5, fixed_relax=20)
    assert got == ref
