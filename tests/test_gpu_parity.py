"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Inputs are seeded and synthetic, and the oracle only ever sees inputs made
by the test or by itself: both sides start each step from the same float32
state, and a chain of half-sweeps continues from the oracle's result rounded
to float32 (teacher forcing), so per-site comparisons are meaningful.
Sample angles for the oracle come from its own map (the GPU's map equals it
bit for bit); temperatures are fixed inputs.  Bars (from the method's precision targets): over-relaxation-only
angles within 1e-5 rad; fewer than 1e-6 of Metropolis decisions flipped;
per-sweep specific energy within 1e-6; identical stopping slopes on identical
energy series; integer and byte outputs bit-exact.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_1811_01604_amd as mpr  # noqa: E402

pytestmark = pytest.mark.gpu
TWO_PI = 2.0 * math.pi


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


def colour_mask(ny, nx, colour):
    return (np.add.outer(np.arange(ny), np.arange(nx)) % 2) == colour


# ------------------------------------------------------------------ Philox
def test_philox_bit_exact(ctx):
    """The library's Philox4x32-10 equals the oracle's numpy implementation on
    10^6 counters (two keys), and the oracle's C one on 600 of them."""
    n = 1_000_000
    say(f"philox: {n} counters x 2 keys")
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    ctr[1] = 0xFFFFFFFF
    for seed in (0xDEADBEEF12345678, 3000):
        key = [seed & 0xFFFFFFFF, seed >> 32]
        out = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
        ctx.diag_philox(dev(ctr.view(np.int32), torch.int32), seed, out)
        got = out.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, oracle.philox4x32_10_np(ctr, key))
        for i in list(range(300)) + list(range(n - 300, n)):
            assert np.array_equal(got[i], oracle.philox4x32_10(ctr[i], key)), i


# ---------------------------------------------------------------- data map
@pytest.mark.parametrize("shape", [(64, 64), (37, 129), (1, 2), (300, 1)])
def test_map_bit_exact(ctx, shape):
    ny, nx = shape
    say("map", shape)
    rng = np.random.default_rng(ny * 1000 + nx)
    z = rng.normal(50, 10, size=shape).astype(np.float32)
    m = (rng.random(shape) < 0.6).astype(np.uint8)
    m.flat[:2] = 1
    phi = torch.zeros(shape, device="cuda")
    zz = ctx.map_to_angles(mpr.images([shape]), dev(z), dev(m, torch.uint8), phi)
    po, zo = oracle.map_to_angles(z.astype(np.float64), m)
    assert np.array_equal(zz, zo)
    assert np.array_equal(phi.cpu().numpy().view(np.uint32), po.astype(np.float32).view(np.uint32))


def test_binding_checks_dtype_and_extent(ctx):
    """Tensors of the wrong dtype or shorter than the batch's packed sites are
    refused before the call; the right ones go through."""
    imgs = mpr.images([(8, 8), (4, 6)])
    z = torch.linspace(0.0, 1.0, 88, device="cuda")
    mk = torch.zeros(88, dtype=torch.uint8, device="cuda")
    mk[::3] = 1
    phi = torch.zeros(88, device="cuda")
    with pytest.raises(TypeError, match="z: dtype"):
        ctx.map_to_angles(imgs, z.double(), mk, phi)
    with pytest.raises(TypeError, match="sampled: dtype"):
        ctx.map_to_angles(imgs, z, mk.float(), phi)
    with pytest.raises(ValueError, match="phi: 87 elements, the call needs 88"):
        ctx.map_to_angles(imgs, z, mk, phi[:87])
    with pytest.raises(ValueError, match="must be contiguous"):
        ctx.map_to_angles(imgs, z, mk, torch.zeros(176, device="cuda")[::2])
    ctx.map_to_angles(imgs, z, mk, phi)
    prm = mpr.default_params(R=2, K=3)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps = torch.zeros_like(phi)
    with pytest.raises(ValueError, match="phi_states: 527 elements, the call needs 528"):
        ctx.simulate(imgs, phi, mk, np.array([0.1, 0.1]), prm, ws, ps, phi_states=torch.zeros(527, device="cuda"))
    with pytest.raises(ValueError, match="T_hat: 1 values for 2 images"):
        ctx.simulate(imgs, phi, mk, np.array([0.1]), prm, ws, ps)


def test_library_refuses_host_memory(ctx):
    """The C ABI checks its device pointers itself: pinned host memory passed
    as phi (through the raw C call, past the binding's checks) is refused
    with MPR_ERR_ARG naming the argument.  Pinned memory is readable by a
    kernel, so nothing would fault if the check let it through."""
    imgs = mpr.images([(8, 8)])
    z = torch.linspace(0.0, 1.0, 64, device="cuda")
    mk = torch.zeros(64, dtype=torch.uint8, device="cuda")
    mk[::3] = 1
    host = torch.zeros(64, dtype=torch.float32).pin_memory()
    zz = np.zeros(2)
    import ctypes as C
    rc = ctx.lib.mpr_map_to_angles(ctx._h, imgs, 1, C.c_void_p(z.data_ptr()), C.c_void_p(mk.data_ptr()),
                                   C.c_void_p(host.data_ptr()), zz.ctypes.data_as(C.c_void_p), None)
    assert rc == mpr.MPR_ERR_ARG
    assert ctx.lib.mpr_last_error(ctx._h).decode() == "map_to_angles: phi is not device memory of device 0"
    assert not host.any()
    # an interior pointer of a device allocation is accepted
    big = torch.zeros(64 + 37, device="cuda")
    ctx.map_to_angles(imgs, z, mk, big[37:])
    assert big[37:][mk == 1].max() > 0


def test_map_batch_and_errors(ctx):
    shapes = [(16, 20), (9, 7), (33, 3)]
    rng = np.random.default_rng(5)
    zs = [rng.normal(size=s).astype(np.float32) * (b + 1) for b, s in enumerate(shapes)]
    ms = [(rng.random(s) < 0.5).astype(np.uint8) for s in shapes]
    for m in ms:
        m.flat[:2] = 1
    z = np.concatenate([a.ravel() for a in zs])
    m = np.concatenate([a.ravel() for a in ms])
    phi = torch.zeros(z.size, device="cuda")
    zz = ctx.map_to_angles(mpr.images(shapes), dev(z), dev(m, torch.uint8), phi)
    off = 0
    for b, s in enumerate(shapes):
        po, zo = oracle.map_to_angles(zs[b].astype(np.float64), ms[b])
        n = s[0] * s[1]
        assert np.array_equal(zz[2 * b:2 * b + 2], zo)
        assert np.array_equal(phi[off:off + n].cpu().numpy(), po.astype(np.float32).ravel())
        off += n
    with pytest.raises(mpr.MprError) as e:
        ctx.map_to_angles(mpr.images([(4, 4)]), dev(np.full(16, 3.0, np.float32)),
                          dev(np.ones(16, np.uint8), torch.uint8), torch.zeros(16, device="cuda"))
    assert e.value.code == mpr.MPR_ERR_DEGENERATE
    bad = np.arange(16, dtype=np.float32)
    bad[3] = np.inf
    with pytest.raises(mpr.MprError) as e:
        ctx.map_to_angles(mpr.images([(4, 4)]), dev(bad), dev(np.ones(16, np.uint8), torch.uint8),
                          torch.zeros(16, device="cuda"))
    assert e.value.code == mpr.MPR_ERR_ARG


# ---------------------------------------------------- teacher-forced sweeps
def smooth_state(ny, nx, nu, kappa, p_removed, noise, seed):
    """Sample angles of a smooth field with the gaps near their true values."""
    z = synth.matern_field(nx, ny, nu, kappa, 50.0, 10.0, seed).astype(np.float32)
    m = synth.random_mask(nx, ny, p_removed, seed + 1)
    phi = TWO_PI * (z.astype(np.float64) - z.min()) / (z.max() - z.min())
    rng = np.random.default_rng(seed + 2)
    g = m == 0
    phi[g] = np.mod(phi[g] + rng.normal(0, noise, size=g.sum()), TWO_PI)
    return phi.astype(np.float32), m


PLAIN, COMPACT = 0, 4 | mpr.TILE_COMPACT  # default plain shape; compacted 4-row shape
FUSED = 32 | mpr.TILE_FUSED  # fused tile sweep, 32-row tiles (one colour in the diagnostics)
ALL_TILES = [1, 2, 4, 8, 2 | mpr.TILE_COMPACT, 4 | mpr.TILE_COMPACT, 8 | mpr.TILE_COMPACT,
             16 | mpr.TILE_FUSED, 24 | mpr.TILE_FUSED, 32 | mpr.TILE_FUSED, 48 | mpr.TILE_FUSED,
             8 | mpr.TILE_FUSED, 12 | mpr.TILE_FUSED]


def run_pair(ctx, phi32, m, colour, T, a, sweep, mode=0, chain=0, stream_id=0, seed=3000, tile=PLAIN):
    """One half-sweep on the GPU and in the oracle from the same float32 state."""
    ny, nx = phi32.shape
    g = dev(phi32)
    fl = torch.zeros((ny, nx), dtype=torch.uint8, device="cuda")
    acc_g = ctx.diag_half_sweep(g, dev(m, torch.uint8), colour, T, a, sweep, chain=chain, stream_id=stream_id,
                                seed=seed, mode=mode, flags=fl, tile=tile)
    po, acc_o, fo = oracle.half_sweep(phi32.astype(np.float64), m, colour, T, a, sweep, chain=chain,
                                      stream=stream_id, seed=seed, mode=mode, with_flags=True)
    return g.cpu().numpy(), acc_g, fl.cpu().numpy(), po, acc_o, fo


@pytest.mark.parametrize("tile", [PLAIN, COMPACT, FUSED])
@pytest.mark.parametrize("kind", ["uniform", "smooth"])
@pytest.mark.parametrize("shape", [(64, 64), (97, 131), (1, 40), (40, 1)])
def test_over_relaxation_only_teacher_forced(ctx, kind, shape, tile):
    ny, nx = shape
    say("OR-only", kind, shape, "tile", tile)
    rng = np.random.default_rng(ny + 7 * nx)
    if kind == "uniform":
        phi = rng.uniform(0, TWO_PI, size=shape).astype(np.float32)
        m = (rng.random(shape) < 0.3).astype(np.uint8)
    else:
        phi, m = smooth_state(max(ny, 2), max(nx, 2), 2.5, 0.05, 0.5, 0.01, 21)
        phi, m = phi[:ny, :nx].copy(), m[:ny, :nx].copy()
    keep_flips = 0
    for colour in (0, 1):
        pg, acc_g, fg, po, acc_o, fo = run_pair(ctx, phi, m, colour, 0.1, 1.0, 0, mode=1, tile=tile)
        assert acc_g == 0 and acc_o == 0
        sel = colour_mask(ny, nx, colour) & (m == 0)
        kf = ((fg & 1) != (fo & 1)) & sel
        keep_flips += int(kf.sum())
        ok = sel & ~kf
        if ok.any():
            assert np.max(np.abs(pg[ok].astype(np.float64) - po[ok])) <= 1e-5
        fixed = m == 1
        assert np.array_equal(pg[fixed], phi[fixed])
        phi = po.astype(np.float32)
    assert keep_flips <= 1, keep_flips


LOW_T = [2.6e-4, 1.0e-3, 0.1]


@pytest.mark.parametrize("tile", [PLAIN, COMPACT, FUSED])
@pytest.mark.parametrize("T", LOW_T)
def test_metropolis_decisions_teacher_forced(ctx, T, tile):
    """Chains of half-sweeps; at every step the oracle redoes it from the GPU's state."""
    say("decisions T =", T, "tile", tile)
    ny, nx = 384, 517
    phi, m = smooth_state(ny, nx, 2.5, 0.05, 0.5, 0.02, 31)
    n_dec = n_flip = n_fp64 = 0
    max_err = 0.0
    step = 0
    for a in (1.0, 4.0, 40.0):
        for sweep in range(3):
            for colour in (0, 1):
                pg, acc_g, fg, po, acc_o, fo = run_pair(ctx, phi, m, colour, T, a, 100 * step + sweep, tile=tile)
                sel = colour_mask(ny, nx, colour) & (m == 0)
                flip = (((fg ^ fo) & 3) != 0) & sel
                n_dec += int(sel.sum())
                n_flip += int(flip.sum())
                n_fp64 += int(((fg & 16) != 0).sum())
                ok = sel & ~flip
                max_err = max(max_err, float(np.max(np.abs(pg[ok].astype(np.float64) - po[ok]))))
                phi = po.astype(np.float32)
            step += 1
    say(f"  decisions {n_dec}, flips {n_flip}, double-precision path {n_fp64 / n_dec:.2e}, max |dphi| {max_err:.2e}")
    assert n_flip <= max(0, int(1e-6 * n_dec)), (n_flip, n_dec)
    assert max_err <= 1e-5


@pytest.mark.parametrize("tile", [PLAIN, COMPACT, FUSED])
def test_accept_count_and_energy_teacher_forced(ctx, tile):
    ny, nx = 130, 257
    phi, m = smooth_state(ny, nx, 1.5, 0.1, 0.66, 0.05, 41)
    ngp = oracle.bond_count(nx, ny)
    for T, a in ((2e-3, 3.0), (2.6e-4, 20.0), (0.2, 1.0)):
        for colour in (0, 1):
            pg, acc_g, fg, po, acc_o, fo = run_pair(ctx, phi, m, colour, T, a, 7, tile=tile)
            assert acc_g == int(((fg & 2) != 0).sum())
            assert acc_g == acc_o
            if colour == 1:
                # the sweep's own energy sum (from its update terms) against
                # the oracle's energy of the state the oracle wrote: |de| <= 1e-6
                _, e_fused = ctx.diag_half_sweep(dev(phi), dev(m, torch.uint8), 1, T, a, 7, with_energy=True,
                                                 tile=tile)
                e_o = oracle.energy(po) + ngp
                assert abs(e_fused - e_o) / ngp <= 1e-6, (e_fused, e_o)
            phi = po.astype(np.float32)
    # energy of the resulting state, as the simulation accumulates it
    hp = ctx.diag_energy(dev(phi))
    ngp = oracle.bond_count(nx, ny)
    ho = oracle.energy(phi.astype(np.float64)) + ngp
    assert abs(hp - ho) / ngp <= 1e-6
    assert abs(hp / ho - 1.0) <= 1e-4


@pytest.mark.parametrize("tile", [PLAIN, COMPACT, FUSED])
@pytest.mark.parametrize("shape", [(1, 2), (2, 1), (3, 3), (5, 2), (2, 7), (1, 9)])
def test_degenerate_and_tiny_grids(ctx, shape, tile):
    ny, nx = shape
    rng = np.random.default_rng(nx * 10 + ny)
    phi = rng.uniform(0, TWO_PI, size=shape).astype(np.float32)
    m = np.zeros(shape, np.uint8)
    for colour in (0, 1):
        pg, acc_g, fg, po, acc_o, fo = run_pair(ctx, phi, m, colour, 0.5, 1.0, 3, tile=tile)
        sel = colour_mask(ny, nx, colour)
        assert np.array_equal(fg[sel] & 3, fo[sel] & 3)
        assert np.max(np.abs(pg.astype(np.float64) - po)) <= 1e-5
        phi = po.astype(np.float32)


# -------------------------------------------------------------- SG slope
def test_sg_slope_matches_oracle(ctx):
    rng = np.random.default_rng(3)
    for degree in (1, 2, 3):
        for n in (5, 20, 33, 64):
            e = -0.99 + 1e-4 * np.cumsum(rng.normal(size=n))
            g = ctx.diag_sg_slope(e, degree)
            o = oracle.sg_slope(e, degree)
            assert abs(g - o) <= 1e-9 * max(abs(o), 1e-6)
            assert (g >= 0) == (o >= 0)


# ------------------------------------------------------------- end to end
def pipeline_gpu(ctx, im, prm, T=None):
    shapes = [(im.ny, im.nx)]
    imgs = mpr.images(shapes)
    z = dev(im.z.astype(np.float32))
    mk = dev(im.mask, torch.uint8)
    phi = torch.zeros_like(z)
    zz = ctx.map_to_angles(imgs, z, mk, phi)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    e_s, T_hat, cl = ctx.estimate_temperature(imgs, phi, mk, prm, ws)
    if T is not None:
        T_hat = np.array([T])
    ps = torch.zeros_like(z)
    m2 = torch.zeros_like(z) if (prm.K <= 1 or prm.spread) else None
    st = ctx.simulate(imgs, phi, mk, T_hat, prm, ws, ps, phi_m2=m2)
    zh = torch.zeros_like(z)
    ctx.predict(imgs, z, mk, ps, zz, prm.R * prm.K, zh)
    out = dict(phi=phi.cpu().numpy(), zz=zz, e_s=e_s[0], T=T_hat[0], clamped=cl[0], phi_sum=ps.cpu().numpy(),
               stats=st, z_hat=zh.cpu().numpy())
    if m2 is not None:
        zs = torch.zeros_like(z)
        ctx.spread(imgs, mk, m2, zz, prm.R * prm.K, zs)
        out.update(phi_m2=m2.cpu().numpy(), z_std=zs.cpu().numpy())
    return out


def oracle_angles(im):
    """The oracle's map of the float32 data: sample angles rounded to float32
    (as the GPU stores them) and (z_min, z_max)."""
    po, zz = oracle.map_to_angles(im.z.astype(np.float32).astype(np.float64), im.mask)
    return po.astype(np.float32), zz


def test_temperature_estimate_matches_oracle(ctx):
    im = synth.workload_l64()
    prm = mpr.default_params(table_nT=12, table_T_lo=0.01, table_T_hi=2.0, table_burn=100, table_meas=300, K=1)
    out = pipeline_gpu(ctx, im, prm)
    phi32, zz = oracle_angles(im)
    assert np.array_equal(out["phi"].view(np.uint32), phi32.view(np.uint32)) and np.array_equal(out["zz"], zz)
    e_s_o, _ = oracle.sample_energy(phi32.astype(np.float64), im.mask)
    assert abs(out["e_s"] - e_s_o) <= 1e-12
    Tg = oracle.temperature_grid(12, 0.01, 2.0)
    et = oracle.energy_table(64, 64, Tg, 100, 300, seed=prm.seed)
    T_o, cl = oracle.invert_temperature(Tg, et, e_s_o)
    say(f"T_hat gpu {out['T']:.5f} oracle {T_o:.5f}")
    assert not cl and not out["clamped"]
    assert abs(out["T"] / T_o - 1.0) < 0.03


def test_temperature_table_on_capped_grid(ctx):  # ctx: skips without a GPU; the test uses fresh contexts
    """table_side_cap = 64: the e(T, L) table of a 150 x 200 image (and of a
    90 x 100 one in the same call, which shares it) is the one of a 64 x 64
    grid.  A later uncapped call on a 64 x 64 image in the same context, which
    finds that table cached, gives the T_hat bit for bit that a fresh context
    gives after building the 64 x 64 table itself; the big image's T_hat is
    the oracle's inversion of the 64 x 64 table within 3%."""
    tab = dict(table_nT=12, table_T_lo=0.01, table_T_hi=2.0, table_burn=100, table_meas=300, K=1)
    big = [synth.matern_field(200, 150, 0.5, 0.2, 50.0, 10.0, 31), synth.matern_field(100, 90, 0.5, 0.2, 50.0, 10.0, 32)]
    bmask = [synth.random_mask(200, 150, 0.5, 33), synth.random_mask(100, 90, 0.5, 34)]
    small = synth.workload_l64()

    def estimate(c, zs, ms, prm):
        imgs = mpr.images([z.shape for z in zs])
        z = dev(np.concatenate([a.astype(np.float32).ravel() for a in zs]))
        mk = dev(np.concatenate([a.ravel() for a in ms]), torch.uint8)
        phi = torch.zeros_like(z)
        ctx_zz = c.map_to_angles(imgs, z, mk, phi)
        ws = torch.empty(c.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        return c.estimate_temperature(imgs, phi, mk, prm, ws), ctx_zz

    a, b = mpr.Context(0), mpr.Context(0)
    try:
        (e_big, T_big, cl_big), _ = estimate(a, big, bmask, mpr.default_params(table_side_cap=64, **tab))
        (_, T_a, _), _ = estimate(a, [small.z], [small.mask], mpr.default_params(**tab))
        (_, T_b, _), _ = estimate(b, [small.z], [small.mask], mpr.default_params(**tab))
    finally:
        a.close()
        b.close()
    assert T_a[0] == T_b[0]
    Tg = oracle.temperature_grid(12, 0.01, 2.0)
    et = oracle.energy_table(64, 64, Tg, 100, 300, seed=mpr.default_params().seed)
    for i in range(2):
        po, _ = oracle.map_to_angles(big[i].astype(np.float32).astype(np.float64), bmask[i])
        e_o, _ = oracle.sample_energy(po.astype(np.float32).astype(np.float64), bmask[i])
        assert abs(e_big[i] - e_o) <= 1e-12
        T_o, cl_o = oracle.invert_temperature(Tg, et, e_o)
        say(f"image {i}: T_hat gpu {T_big[i]:.5f}, oracle (64 x 64 table) {T_o:.5f}")
        assert not cl_big[i] and not cl_o
        assert abs(T_big[i] / T_o - 1.0) < 0.03


@pytest.mark.parametrize("ny,nx,seed,tol", [(40, 72, 41, 0.03), (1, 300, 43, 0.05)])
def test_temperature_estimate_on_rectangular_and_line_images(ctx, ny, nx, seed, tol):
    """e(T, L) of a rectangular grid (bonds nx (ny - 1) + ny (nx - 1)) and of a
    single row: T_hat is the oracle's inversion of the oracle's table for the
    same shape, within a few times the seed-to-seed spread of that table
    (0.7% and 1.8%)."""
    tab = dict(table_nT=12, table_T_lo=0.01, table_T_hi=2.0, table_burn=100, table_meas=300, K=1)
    z = synth.matern_field(nx, max(ny, 2), 0.5, 0.2, 50.0, 10.0, seed)[:ny]
    m = synth.random_mask(nx, ny, 0.5, seed + 1)
    imgs = mpr.images([(ny, nx)])
    zd, mk = dev(z.astype(np.float32)), dev(m, torch.uint8)
    phi = torch.zeros_like(zd)
    ctx.map_to_angles(imgs, zd, mk, phi)
    prm = mpr.default_params(**tab)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    e_s, T_hat, cl = ctx.estimate_temperature(imgs, phi, mk, prm, ws)
    po, _ = oracle.map_to_angles(z.astype(np.float32).astype(np.float64), m)
    e_o, _ = oracle.sample_energy(po.astype(np.float32).astype(np.float64), m)
    assert abs(e_s[0] - e_o) <= 1e-12
    Tg = oracle.temperature_grid(12, 0.01, 2.0)
    T_o, cl_o = oracle.invert_temperature(Tg, oracle.energy_table(nx, ny, Tg, 100, 300, seed=prm.seed), e_o)
    say(f"  {ny} x {nx}: T_hat gpu {T_hat[0]:.5f} oracle {T_o:.5f}")
    assert not cl[0] and not cl_o
    assert abs(T_hat[0] / T_o - 1.0) < tol


def test_simulate_free_running_short_chains(ctx):
    """After one sweep GPU and oracle agree per site; divergence grows afterwards."""
    im = synth.workload_l64()
    phi32, _ = oracle_angles(im)
    for n_sweeps in (1, 2, 4, 8):
        prm = mpr.default_params(R=1, K=1, fixed_relax=n_sweeps - 1, seed=77)
        out = pipeline_gpu(ctx, im, prm, T=0.15)
        opr = oracle.default_params(R=1, K=1, fixed_relax=n_sweeps - 1, seed=77)
        ps, st, _, _ = oracle.simulate(phi32.astype(np.float64), im.mask, 0.15, opr)
        g = im.mask == 0
        d = np.abs(out["phi_sum"][g].astype(np.float64) - ps[g])
        frac = float(np.mean(d <= 1e-5))
        say(f"  {n_sweeps} sweep(s): {frac:.5f} of gap sites within 1e-5")
        if n_sweeps == 1:
            assert frac >= 0.999
        assert out["stats"][0]["relax_sweeps"] == st[0]["relax_sweeps"] == n_sweeps - 1


# a fixed temperature near the estimate for the L=64 workload (about 0.18)
T_L64 = 0.18


def test_simulate_stopping_rule_l64(ctx):
    """The L=64 pipeline (map, simulate with the stopping rule, predict) at a
    fixed temperature: stopping decisions, relaxation length and MAE vs the oracle."""
    im = synth.workload_l64()
    prm = mpr.default_params(R=8, K=10, table_nT=12, table_T_lo=0.01, table_T_hi=2.0, table_burn=100,
                             table_meas=300)
    out = pipeline_gpu(ctx, im, prm, T=T_L64)
    phi32, zz = oracle_angles(im)
    opr = oracle.default_params(R=8, K=10, seed=prm.seed)
    ps, st, _, _ = oracle.simulate(phi32.astype(np.float64), im.mask, T_L64, opr)
    zo = oracle.predict(im.z.astype(np.float32).astype(np.float64), im.mask, ps, 80, zz)
    zt = im.z.astype(np.float32).astype(np.float64)
    mg = synth.validation_measures(zt, out["z_hat"].astype(np.float64), im.mask)
    mo = synth.validation_measures(zt, zo, im.mask)
    rs_g = [s["relax_sweeps"] for s in out["stats"]]
    rs_o = [s["relax_sweeps"] for s in st]
    say(f"  MAAE gpu {mg['MAAE']:.4f} oracle {mo['MAAE']:.4f}; relax gpu {rs_g} oracle {rs_o}")
    for s in out["stats"]:
        t = s["relax_sweeps"] - 1
        assert t >= prm.n_fit and t % prm.n_f == 0 and s["k_last"] >= 0 and not s["not_converged"]
    assert abs(np.mean(rs_g) - np.mean(rs_o)) <= 10
    assert abs(mg["MAAE"] / mo["MAAE"] - 1.0) < 0.03
    # samples copied exactly
    s = im.mask == 1
    assert np.array_equal(out["z_hat"][s], im.z.astype(np.float32)[s])


def test_predict_matches_oracle_bit_exact(ctx):
    rng = np.random.default_rng(9)
    shape = (33, 47)
    z = rng.normal(5, 2, size=shape).astype(np.float32)
    m = (rng.random(shape) < 0.5).astype(np.uint8)
    ps = (rng.random(shape) * TWO_PI * 7).astype(np.float32)
    zz = np.array([float(z[m == 1].min()), float(z[m == 1].max())])
    zh = torch.zeros(shape, device="cuda")
    ctx.predict(mpr.images([shape]), dev(z), dev(m, torch.uint8), dev(ps), zz, 7, zh)
    zo = oracle.predict(z.astype(np.float64), m, ps.astype(np.float64), 7, zz)
    assert np.array_equal(zh.cpu().numpy(), zo.astype(np.float32))


def test_no_gap_image_and_batch_independence(ctx):
    """An image's result does not depend on the batch around it (same image id)."""
    a = synth.workload_l64()
    b_z = synth.matern_field(40, 24, 1.5, 0.1, 50, 10, 5)
    b_m = synth.random_mask(40, 24, 0.4, 6)
    full = np.ones((10, 12), np.uint8)
    c_z = synth.matern_field(12, 10, 0.5, 0.2, 50, 10, 7)
    prm = mpr.default_params(R=2, K=3)
    T = np.array([0.15, 0.02, 0.1])
    parts = [(a.z, a.mask), (b_z, b_m), (c_z, full)]
    shapes = [p[0].shape for p in parts]

    def run(sel):
        sh = [shapes[i] for i in sel]
        imgs = mpr.images(sh, ids=list(sel))
        z = dev(np.concatenate([parts[i][0].astype(np.float32).ravel() for i in sel]))
        mk = dev(np.concatenate([parts[i][1].ravel() for i in sel]), torch.uint8)
        phi = torch.zeros_like(z)
        ctx.map_to_angles(imgs, z, mk, phi)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        ps = torch.zeros_like(z)
        ctx.simulate(imgs, phi, mk, T[list(sel)], prm, ws, ps)
        out, off = {}, 0
        for i in sel:
            n = shapes[i][0] * shapes[i][1]
            out[i] = ps[off:off + n].cpu().numpy()
            off += n
        return out

    together = run([0, 1, 2])
    for i in range(3):
        alone = run([i])
        assert np.array_equal(together[i], alone[i]), i
    assert np.all(together[2] == 0.0)


def test_images_at_arbitrary_offsets(ctx):
    """mpr_image.offset places each image anywhere in the per-site buffers:
    two images stored in reverse order with unused elements around them give
    the packed batch's map, sums, spread, prediction and quantiles bit for
    bit, and the unused elements are left as they were."""
    a = synth.workload_l64()
    b_z = synth.matern_field(40, 24, 1.5, 0.1, 50, 10, 5)
    b_m = synth.random_mask(40, 24, 0.4, 6)
    parts = [(a.z, a.mask), (b_z, b_m)]
    prm = mpr.default_params(R=2, K=3, spread=1, seed=23)
    T = np.array([0.15, 0.05])
    M = prm.R * prm.K
    probs = [0.1, 0.5, 0.9]

    def run(offsets, total):
        imgs = (mpr.Image * 2)()
        for i, ((zz_, _), off) in enumerate(zip(parts, offsets)):
            imgs[i].ny, imgs[i].nx = zz_.shape
            imgs[i].offset, imgs[i].id = off, i
        z = np.full(total, -7.0, np.float32)
        m = np.full(total, 1, np.uint8)
        for (zz_, mm), off in zip(parts, offsets):
            z[off:off + zz_.size] = zz_.astype(np.float32).ravel()
            m[off:off + zz_.size] = mm.ravel()
        zd, mk = dev(z), dev(m, torch.uint8)
        sentinel = -3.25
        phi = torch.full_like(zd, sentinel)
        zz = ctx.map_to_angles(imgs, zd, mk, phi)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        ps, m2, zh, zs = (torch.full_like(zd, sentinel) for _ in range(4))
        N = mpr.sites_of(imgs)  # the stride of a recorded state
        st = torch.full((M, N), sentinel, device="cuda")
        ctx.simulate(imgs, phi, mk, T, prm, ws, ps, phi_m2=m2, phi_states=st)
        ctx.predict(imgs, zd, mk, ps, zz, M, zh)
        ctx.spread(imgs, mk, m2, zz, M, zs)
        zq = torch.full((len(probs), N), sentinel, device="cuda")
        ctx.quantiles(imgs, zd, mk, st, M, probs, zz, zq)
        outs = [t.cpu().numpy() for t in (phi, ps, m2, zh, zs)] + [st.cpu().numpy(), zq.cpu().numpy()]
        used = np.zeros(total, bool)
        for (zz_, _), off in zip(parts, offsets):
            used[off:off + zz_.size] = True
        for o in outs:
            assert np.all(o[..., ~used[:o.shape[-1]]] == sentinel)  # unused elements untouched
        per_image = []
        for (zz_, _), off in zip(parts, offsets):
            per_image.append([o[..., off:off + zz_.size].copy() for o in outs])
        return zz, per_image

    n0, n1 = a.z.size, b_z.size
    zz_p, packed = run([0, n0], n0 + n1)
    zz_s, spaced = run([n1 + 777, 129], n0 + n1 + 1500)  # reversed, with gaps
    assert np.array_equal(zz_p, zz_s)
    for i in range(2):
        for k, (x, y) in enumerate(zip(packed[i], spaced[i])):
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), (i, k)


# a fixed temperature near the estimate for the L=1024 workload
T_L1024 = 2.6e-4


def test_l1024_prediction_matches_oracle(ctx):
    """L=1024 Matern nu=2.5 kappa=0.05, 50% random gaps, M=100 as one chain
    (R=1, K=100) at a fixed temperature near its estimate: the GPU's
    prediction MAE is within 0.5% of the oracle's, and on the 256x256 centre
    crop the GPU-oracle per-site difference is no larger than the GPU's own
    seed-to-seed spread."""
    im = synth.workload_l1024()
    say("L=1024 pipeline on the GPU")
    prm = mpr.default_params(R=1, K=100, seed=3001, spread=1)
    g1 = pipeline_gpu(ctx, im, prm, T=T_L1024)
    prm2 = mpr.default_params(R=1, K=100, seed=4001, spread=1)
    g2 = pipeline_gpu(ctx, im, prm2, T=T_L1024)
    say(f"  estimated T_hat {g1['T']:.4e} (run at {T_L1024:.1e}), relax sweeps {g1['stats'][0]['relax_sweeps']}; "
        f"oracle run (about 30 s)")
    zt = im.z.astype(np.float32).astype(np.float64)
    phi32, zz = oracle_angles(im)
    ps, st, _, _, pq = oracle.simulate(phi32.astype(np.float64), im.mask, T_L1024,
                                       oracle.default_params(R=1, K=100, seed=3001), want_sq=True)
    zo = oracle.predict(zt, im.mask, ps, 100, zz)
    # the realizations' spread (standard deviation of the 100 states per site)
    so = oracle.spread(im.mask, ps, pq, 100, zz)
    gap0 = im.mask == 0
    m_g, m_g2, m_o = (float(np.mean(a[gap0])) for a in (g1["z_std"], g2["z_std"], so))
    d_so = float(np.mean(np.abs(g1["z_std"][gap0] - so[gap0])))
    d_ss = float(np.mean(np.abs(g1["z_std"][gap0] - g2["z_std"][gap0])))
    say(f"  spread: mean z_std gpu {m_g:.5f} (seed 2: {m_g2:.5f}) oracle {m_o:.5f}; mean |gpu - oracle| "
        f"{d_so:.3e}, |seed1 - seed2| {d_ss:.3e}")
    assert abs(m_g / m_o - 1.0) <= 0.03
    assert d_so <= 1.5 * d_ss
    gap = im.mask == 0
    mae_g = float(np.mean(np.abs(g1["z_hat"][gap] - zt[gap])))
    mae_g2 = float(np.mean(np.abs(g2["z_hat"][gap] - zt[gap])))
    mae_o = float(np.mean(np.abs(zo[gap] - zt[gap])))
    say(f"  MAE gpu {mae_g:.6f} (seed 2: {mae_g2:.6f}) oracle {mae_o:.6f}; relax gpu "
        f"{g1['stats'][0]['relax_sweeps']} oracle {st[0]['relax_sweeps']}")
    assert abs(mae_g / mae_o - 1.0) <= 0.005
    c = slice(384, 640)
    gc = gap[c, c]
    d_go = np.mean(np.abs(g1["z_hat"][c, c][gc] - zo[c, c][gc]))
    d_gg = np.mean(np.abs(g1["z_hat"][c, c][gc] - g2["z_hat"][c, c][gc]))
    say(f"  crop: mean |gpu - oracle| {d_go:.3e}, mean |gpu seed1 - seed2| {d_gg:.3e}")
    assert d_go <= 1.5 * d_gg


@pytest.mark.parametrize("shape", [(64, 64), (45, 211)])
def test_results_independent_of_block_shape_and_graph_size(ctx, shape):
    """Every block shape (plain rows 1, 2, 4, 8; compacted rows 2, 4, 8;
    fused tile sweeps of 16, 24, 32 rows; autotuned) and graph size gives
    bit-identical sums, statistics and stopping decisions."""
    ny, nx = shape
    z = synth.matern_field(nx, ny, 1.5, 0.1, 50, 10, 17)
    m = synth.random_mask(nx, ny, 0.5, 18)
    imgs = mpr.images([shape])
    zd = dev(z.astype(np.float32))
    mk = dev(m, torch.uint8)
    phi = torch.zeros_like(zd)
    ctx.map_to_angles(imgs, zd, mk, phi)
    ref = None
    for rows, spl in ((4, 5), (1, 5), (2, 7), (8, 1), (0, 0), (4, 64), (2 | mpr.TILE_COMPACT, 5),
                      (4 | mpr.TILE_COMPACT, 3), (8 | mpr.TILE_COMPACT, 64), (16 | mpr.TILE_FUSED, 5),
                      (24 | mpr.TILE_FUSED, 1), (32 | mpr.TILE_FUSED, 64), (32 | mpr.TILE_FUSED, 3)):
        prm = mpr.default_params(R=3, K=4, tile_rows=rows, sweeps_per_launch=spl)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        ps = torch.zeros_like(zd)
        st = ctx.simulate(imgs, phi, mk, np.array([2e-3]), prm, ws, ps)
        out = (ps.cpu().numpy().tobytes(), [(s["relax_sweeps"], s["k_last"], s["a_final"]) for s in st])
        if ref is None:
            ref = out
        else:
            assert out == ref, (rows, spl)


@pytest.mark.parametrize("p_removed", [0.0, 0.33, 0.66, 1.0])
@pytest.mark.parametrize("shape", [(67, 1100), (300, 129)])
def test_half_sweep_identical_for_every_tile(ctx, shape, p_removed):
    """One half-sweep per colour in every block shape: angles, flags,
    accepted counts and the fused energy are bit-identical (the shapes wider
    than the grid and the ragged right and bottom edges included)."""
    ny, nx = shape
    say("tiles", shape, p_removed)
    phi, m = smooth_state(ny, nx, 1.5, 0.1, 0.5, 0.05, 51)
    rng = np.random.default_rng(52)
    m = (rng.random(shape) >= p_removed).astype(np.uint8)
    mk = dev(m, torch.uint8)
    for colour in (0, 1):
        ref = None
        for tile in ALL_TILES:
            g = dev(phi)
            fl = torch.zeros((ny, nx), dtype=torch.uint8, device="cuda")
            acc, e = ctx.diag_half_sweep(g, mk, colour, 1e-3, 4.0, 11, flags=fl, with_energy=True, tile=tile)
            out = (g.cpu().numpy().tobytes(), fl.cpu().numpy().tobytes(), acc, e)
            if ref is None:
                ref = out
            else:
                assert out == ref, (tile, colour)


@pytest.mark.parametrize("R,K", [(2, 3), (4, 1), (1, 5)])
def test_spread_matches_oracle_early_sweeps(ctx, R, K):
    """The realizations' spread after the first sweeps, where GPU and oracle
    chains still agree site by site: the sum of squared deviations (Welford
    per chain for K > 1, two passes over the final states for K = 1) and the
    back-transformed standard deviation match the oracle's plain sums on
    99% of gap sites; sampled sites are 0."""
    im = synth.workload_l64()
    prm = mpr.default_params(R=R, K=K, fixed_relax=0, seed=91, spread=1)
    out = pipeline_gpu(ctx, im, prm, T=0.15)
    phi32, zz = oracle_angles(im)
    opr = oracle.default_params(R=R, K=K, fixed_relax=0, seed=91)
    ps, _, _, _, pq = oracle.simulate(phi32.astype(np.float64), im.mask, 0.15, opr, want_sq=True)
    M = R * K
    m2_o = pq - ps * ps / M
    so = oracle.spread(im.mask, ps, pq, M, zz)
    g = im.mask == 0
    ok_m2 = np.abs(out["phi_m2"][g] - m2_o[g]) <= 1e-4 * np.maximum(1.0, m2_o[g]) + 2e-5
    ok_sd = np.abs(out["z_std"][g] - so[g]) <= 1e-3 * np.maximum(1.0, so[g]) + 1e-3
    say(f"  R={R} K={K}: m2 agrees on {ok_m2.mean():.4f}, z_std on {ok_sd.mean():.4f} of gap sites")
    assert ok_m2.mean() >= 0.99 and ok_sd.mean() >= 0.99
    assert np.all(out["phi_m2"][~g] == 0) and np.all(out["z_std"][~g] == 0)
    if M == 1:
        assert np.all(out["z_std"] == 0)


def test_spread_needs_flag_for_equilibrium_sums(ctx):
    im = synth.workload_l64()
    imgs = mpr.images([(im.ny, im.nx)])
    mk = dev(im.mask, torch.uint8)
    phi = dev(np.where(im.mask == 1, 1.0, 0.0).astype(np.float32))
    prm = mpr.default_params(R=1, K=3)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps, m2 = torch.zeros_like(phi), torch.zeros_like(phi)
    with pytest.raises(mpr.MprError) as e:
        ctx.simulate(imgs, phi, mk, np.array([0.1]), prm, ws, ps, phi_m2=m2)
    assert e.value.code == mpr.MPR_ERR_ARG
