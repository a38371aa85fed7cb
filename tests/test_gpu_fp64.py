"""GPU parity of the double-precision sweep (mpr_params.fp64) against the
FP64 oracle.

Both sides compute in double, so the bars are far tighter than for the
single-precision sweep (the oracle sees only inputs made here or by itself;
chains of half-sweeps continue from the oracle's state): teacher-forced half-sweeps take the same decisions
at every site and agree in angle to rounding; free-running chains track the
oracle's site by site through relaxation and the equilibrium states; the
stopping rule stops at the same sweep.  The GPU's energy sums are fixed
point of 2^-30 per site, so a colour's sum is within (sites) x 2^-31 of the
exact one.
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
PLAIN_TILES = [1, 2, 4, 8]
COMPACT_TILES = [2 | mpr.TILE_COMPACT, 4 | mpr.TILE_COMPACT, 8 | mpr.TILE_COMPACT]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mpr.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def colour_mask(ny, nx, colour):
    return (np.add.outer(np.arange(ny), np.arange(nx)) % 2) == colour


def smooth_state(ny, nx, nu, kappa, p_removed, noise, seed):
    """Double angles of a smooth field, gaps perturbed around their true values."""
    z = synth.matern_field(nx, ny, nu, kappa, 50.0, 10.0, seed)
    m = synth.random_mask(nx, ny, p_removed, seed + 1)
    phi = TWO_PI * (z - z.min()) / (z.max() - z.min())
    rng = np.random.default_rng(seed + 2)
    g = m == 0
    phi[g] = np.mod(phi[g] + rng.normal(0, noise, size=g.sum()), TWO_PI)
    return phi, m


def run_pair(ctx, phi, m, colour, T, a, sweep, mode=0, seed=3000, tile=0):
    """One half-sweep on the GPU (double) and in the oracle from the same state."""
    ny, nx = phi.shape
    g = dev(phi)
    fl = torch.zeros((ny, nx), dtype=torch.uint8, device="cuda")
    acc_g, e_g = ctx.diag_half_sweep_fp64(g, dev(m, torch.uint8), colour, T, a, sweep, seed=seed, mode=mode,
                                          flags=fl, with_energy=True, tile=tile)
    po, acc_o, fo = oracle.half_sweep(phi, m, colour, T, a, sweep, seed=seed, mode=mode, with_flags=True)
    return g.cpu().numpy(), acc_g, e_g, fl.cpu().numpy(), po, acc_o, fo


@pytest.mark.parametrize("tile", [0, 4 | mpr.TILE_COMPACT])
@pytest.mark.parametrize("kind", ["uniform", "smooth"])
@pytest.mark.parametrize("shape", [(64, 64), (97, 131), (1, 40), (40, 1)])
def test_fp64_over_relaxation_only(ctx, kind, shape, tile):
    ny, nx = shape
    say("fp64 OR-only", kind, shape, tile)
    rng = np.random.default_rng(ny + 7 * nx)
    if kind == "uniform":
        phi = rng.uniform(0, TWO_PI, size=shape)
        m = (rng.random(shape) < 0.3).astype(np.uint8)
    else:
        phi, m = smooth_state(max(ny, 2), max(nx, 2), 2.5, 0.05, 0.5, 0.01, 21)
        phi, m = phi[:ny, :nx].copy(), m[:ny, :nx].copy()
    for colour in (0, 1):
        pg, acc_g, _, fg, po, acc_o, fo = run_pair(ctx, phi, m, colour, 0.1, 1.0, 0, mode=1, tile=tile)
        assert acc_g == 0 and acc_o == 0
        sel = colour_mask(ny, nx, colour) & (m == 0)
        assert np.array_equal(fg[sel] & 15, fo[sel] & 15)
        if sel.any():
            assert np.max(np.abs(pg[sel] - po[sel])) <= 1e-11
        fixed = m == 1
        assert np.array_equal(pg[fixed], phi[fixed])
        phi = po


@pytest.mark.parametrize("T,tile", [(2.6e-4, 0), (1.0e-3, 0), (0.1, 0), (2.6e-4, 8 | mpr.TILE_COMPACT),
                                    (0.1, 2 | mpr.TILE_COMPACT)])
def test_fp64_decisions_teacher_forced(ctx, T, tile):
    """Every Metropolis decision equals the oracle's, down to T = 2.6e-4;
    angles agree to 1e-11 rad; accepted counts are equal; the fused energy
    is the oracle's energy of the written state within the fixed-point bound
    (the default plain shape and the compacted ones)."""
    say("fp64 decisions T =", T, "tile", tile)
    ny, nx = 384, 517
    phi, m = smooth_state(ny, nx, 2.5, 0.05, 0.5, 0.02, 31)
    ngp = oracle.bond_count(nx, ny)
    n1 = int(colour_mask(ny, nx, 1).sum())
    n_dec = 0
    max_err = 0.0
    step = 0
    for a in (1.0, 4.0, 40.0):
        for sweep in range(3):
            for colour in (0, 1):
                pg, acc_g, e_g, fg, po, acc_o, fo = run_pair(ctx, phi, m, colour, T, a, 100 * step + sweep, tile=tile)
                sel = colour_mask(ny, nx, colour) & (m == 0)
                n_dec += int(sel.sum())
                assert np.array_equal(fg[sel] & 15, fo[sel] & 15), (a, sweep, colour)
                assert acc_g == acc_o
                max_err = max(max_err, float(np.max(np.abs(pg[sel] - po[sel]))))
                if colour == 1:
                    e_o = oracle.energy(po) + ngp
                    assert abs(e_g - e_o) <= n1 * 2.0 ** -31 + 1e-9 * ngp, (e_g, e_o)
                phi = po
            step += 1
    say(f"  decisions {n_dec}, all equal; max |dphi| {max_err:.2e}")
    assert max_err <= 1e-11


@pytest.mark.parametrize("shape", [(1, 2), (2, 1), (3, 3), (5, 2), (2, 7), (1, 9)])
def test_fp64_degenerate_and_tiny_grids(ctx, shape):
    ny, nx = shape
    rng = np.random.default_rng(nx * 10 + ny)
    phi = rng.uniform(0, TWO_PI, size=shape)
    m = np.zeros(shape, np.uint8)
    for colour in (0, 1):
        pg, acc_g, _, fg, po, acc_o, fo = run_pair(ctx, phi, m, colour, 0.5, 1.0, 3)
        sel = colour_mask(ny, nx, colour)
        assert np.array_equal(fg[sel] & 15, fo[sel] & 15)
        assert acc_g == acc_o
        assert np.max(np.abs(pg - po)) <= 1e-11
        phi = po


@pytest.mark.parametrize("p_removed", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("shape", [(67, 1100), (300, 129)])
def test_fp64_half_sweep_identical_for_every_tile(ctx, shape, p_removed):
    ny, nx = shape
    phi, _ = smooth_state(ny, nx, 1.5, 0.1, 0.5, 0.05, 51)
    m = (np.random.default_rng(52).random(shape) >= p_removed).astype(np.uint8)
    mk = dev(m, torch.uint8)
    for colour in (0, 1):
        ref = None
        for tile in PLAIN_TILES + COMPACT_TILES:
            g = dev(phi)
            fl = torch.zeros((ny, nx), dtype=torch.uint8, device="cuda")
            acc, e = ctx.diag_half_sweep_fp64(g, mk, colour, 1e-3, 4.0, 11, flags=fl, with_energy=True, tile=tile)
            out = (g.cpu().numpy().tobytes(), fl.cpu().numpy().tobytes(), acc, e)
            if ref is None:
                ref = out
            else:
                assert out == ref, (tile, colour)


def simulate_gpu(ctx, phi32, mask, T, prm):
    """mpr_simulate on one image from float sample angles; float outputs."""
    ny, nx = phi32.shape
    imgs = mpr.images([(ny, nx)])
    ph = dev(phi32, torch.float32)
    mk = dev(mask, torch.uint8)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps = torch.zeros_like(ph)
    m2 = torch.zeros_like(ph) if (prm.K <= 1 or prm.spread) else None
    st = ctx.simulate(imgs, ph, mk, np.array([T]), prm, ws, ps, phi_m2=m2)
    return ps.cpu().numpy(), (m2.cpu().numpy() if m2 is not None else None), st


def l64_angles():
    im = synth.workload_l64()
    po, zz = oracle.map_to_angles(im.z.astype(np.float32).astype(np.float64), im.mask)
    return im, po.astype(np.float32)


@pytest.mark.parametrize("n_relax", [1, 10, 40])
def test_fp64_free_running_chains_track_oracle(ctx, n_relax):
    """R = 2 chains, n_relax relaxation sweeps and K = 3 states at T = 0.15,
    from the same float sample angles: the sums of the states agree with the
    oracle's at every gap site to the float rounding of the output."""
    im, phi32 = l64_angles()
    prm = mpr.default_params(R=2, K=3, fixed_relax=n_relax, seed=77, fp64=1)
    ps, _, st = simulate_gpu(ctx, phi32, im.mask, 0.15, prm)
    opr = oracle.default_params(R=2, K=3, fixed_relax=n_relax, seed=77)
    po, sto, _, _ = oracle.simulate(phi32.astype(np.float64), im.mask, 0.15, opr)
    g = im.mask == 0
    d = np.abs(ps[g].astype(np.float64) - po[g])
    say(f"  fp64, {n_relax} relaxation sweeps: max |phi_sum gpu - oracle| {d.max():.2e}")
    assert d.max() <= 4e-6  # sums below 6 pi, float rounding of the output
    assert [s["relax_sweeps"] for s in st] == [s["relax_sweeps"] for s in sto] == [n_relax] * 2
    assert [s["a_final"] for s in st] == [s["a_final"] for s in sto]


@pytest.mark.parametrize("fp64", [1, 0])
def test_simulate_from_given_starting_angles(ctx, fp64):
    """phi_init, the entry the warm start uses: the chains start from given
    gap angles (made here) instead of Philox draws.  From the same float
    starting angles, double-precision chains run by the stopping rule track
    the oracle's (sums to the float rounding of the output, the same stopping
    sweeps); single-precision chains agree at 99.9% of the gap sites after
    one sweep.  Without phi_init the result differs (the given angles are
    used)."""
    im, phi32 = l64_angles()
    ny, nx = phi32.shape
    g = im.mask == 0
    init = np.zeros_like(phi32)
    init[g] = np.random.default_rng(5).uniform(0, TWO_PI, size=int(g.sum())).astype(np.float32)
    T = 0.15
    kw = dict(R=2, K=3, seed=21) if fp64 else dict(R=1, K=1, fixed_relax=0, seed=21)
    # warm_min_states = 0: the start here is the parity input, not a warm
    # start whose realizations must average it out
    prm = mpr.default_params(fp64=fp64, warm_min_states=0, **kw)
    imgs = mpr.images([(ny, nx)])
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ph, mk = dev(phi32, torch.float32), dev(im.mask, torch.uint8)
    ps, ps0 = torch.zeros_like(ph), torch.zeros_like(ph)
    with pytest.raises(mpr.MprError) as e:  # the default refuses a warm start with K < 25
        ctx.simulate(imgs, ph, mk, np.array([T]), mpr.default_params(fp64=fp64, **kw), ws, ps,
                     phi_init=dev(init, torch.float32))
    assert e.value.code == mpr.MPR_ERR_ARG
    st = ctx.simulate(imgs, ph, mk, np.array([T]), prm, ws, ps, phi_init=dev(init, torch.float32))
    ctx.simulate(imgs, ph, mk, np.array([T]), prm, ws, ps0)
    ps, ps0 = ps.cpu().numpy(), ps0.cpu().numpy()
    po, sto, _, _ = oracle.simulate(phi32.astype(np.float64), im.mask, T, oracle.default_params(**kw),
                                    phi_init=init.astype(np.float64))
    d = np.abs(ps[g].astype(np.float64) - po[g])
    assert np.abs(ps0[g].astype(np.float64) - po[g]).max() > 1e-2
    if fp64:
        say(f"  fp64 from phi_init: max |phi_sum gpu - oracle| {d.max():.2e}, relax {[s['relax_sweeps'] for s in st]}")
        assert d.max() <= 8e-6  # sums of 6 states below 12 pi
        assert [s["relax_sweeps"] for s in st] == [s["relax_sweeps"] for s in sto]
    else:
        frac = float(np.mean(d <= 1e-5))
        say(f"  fp32 from phi_init, one sweep: {frac:.5f} of gap sites within 1e-5")
        assert frac >= 0.999


def test_given_start_is_reduced_into_range(ctx):
    """phi_init values outside [0, 2 pi) are reduced into it, and -0.0 is
    +0.0 (a set sign bit would mark the site as sampled and freeze it):
    single-precision chains from -0.0 equal those from +0.0 bit for bit, and
    double-precision chains from angles shifted by +-2 pi equal those from
    the host's reduction of the same shifted values."""
    im, phi32 = l64_angles()
    ny, nx = phi32.shape
    g = im.mask == 0
    ng = int(g.sum())
    rng = np.random.default_rng(9)
    base = np.zeros_like(phi32)
    base[g] = rng.uniform(0, TWO_PI, size=ng).astype(np.float32)
    base[g] = np.where(np.arange(ng) % 7 == 0, 0.0, base[g]).astype(np.float32)
    imgs = mpr.images([(ny, nx)])
    ph, mk = dev(phi32, torch.float32), dev(im.mask, torch.uint8)

    def fill(init, fp64):
        prm = mpr.default_params(R=2, K=1, fixed_relax=1, fp64=fp64, warm_min_states=0, seed=31)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        ps = torch.zeros_like(ph)
        ctx.simulate(imgs, ph, mk, np.array([0.12]), prm, ws, ps, phi_init=dev(init, torch.float32))
        return ps.cpu().numpy()

    neg0 = base.copy()
    neg0[g & (base == 0)] = -0.0
    assert np.signbit(neg0[g]).sum() == int((base[g] == 0).sum()) > 0
    assert fill(neg0, 0).tobytes() == fill(base, 0).tobytes()
    shifted = base.copy()
    shifted[g] = (base[g].astype(np.float64) + np.where(np.arange(ng) % 2 == 0, TWO_PI, -TWO_PI)).astype(np.float32)
    v = shifted.astype(np.float64)
    reduced = np.abs(v - TWO_PI * np.floor(v / TWO_PI)).astype(np.float32)
    reduced[~g] = 0.0
    assert np.all((reduced[g] >= 0) & (reduced[g] < TWO_PI))
    d = np.abs(fill(shifted, 1).astype(np.float64) - fill(reduced, 1))
    say(f"  start shifted by +-2 pi: max |phi_sum - phi_sum(reduced)| {d.max():.2e}")
    assert d.max() <= 1e-5


@pytest.mark.parametrize("sg_degree,n_fit,n_f,eq_a_mode", [(2, 12, 3, 0), (1, 20, 5, 1), (3, 30, 4, 1)])
def test_fp64_stopping_rule_options_match_oracle(ctx, sg_degree, n_fit, n_f, eq_a_mode):
    """Other settings of the stopping rule (degree of the Savitzky-Golay fit,
    its window, the check interval) and eq_a_mode = 1 (the equilibrium states
    keep the final relaxation a): double-precision chains stop at the
    oracle's sweeps with its a, and the sums of their states agree."""
    im, phi32 = l64_angles()
    kw = dict(R=2, K=4, seed=9, sg_degree=sg_degree, n_fit=n_fit, n_f=n_f, eq_a_mode=eq_a_mode)
    ps, _, st = simulate_gpu(ctx, phi32, im.mask, 0.05, mpr.default_params(fp64=1, **kw))
    po, sto, _, _ = oracle.simulate(phi32.astype(np.float64), im.mask, 0.05, oracle.default_params(**kw))
    g = im.mask == 0
    d = np.abs(ps[g].astype(np.float64) - po[g])
    rs = [s["relax_sweeps"] for s in st]
    say(f"  degree {sg_degree}, n_fit {n_fit}, n_f {n_f}, eq_a_mode {eq_a_mode}: relax {rs}, max |dsum| {d.max():.2e}")
    assert rs == [s["relax_sweeps"] for s in sto]
    assert [s["a_final"] for s in st] == [s["a_final"] for s in sto]
    assert d.max() <= 8e-6  # sums of 8 states below 16 pi


def test_fp64_stopping_rule_and_spread_match_oracle(ctx):
    """The whole simulation with the stopping rule (R = 4, K = 10, spread on):
    each chain stops at the oracle's sweep with its slope, and the sums of
    the states and of their squared deviations agree site by site."""
    im, phi32 = l64_angles()
    T = 0.05
    prm = mpr.default_params(R=4, K=10, seed=5, fp64=1, spread=1)
    ps, m2, st = simulate_gpu(ctx, phi32, im.mask, T, prm)
    opr = oracle.default_params(R=4, K=10, seed=5)
    po, sto, _, _, pq = oracle.simulate(phi32.astype(np.float64), im.mask, T, opr, want_sq=True)
    rs_g = [s["relax_sweeps"] for s in st]
    rs_o = [s["relax_sweeps"] for s in sto]
    say(f"  fp64 stopping: gpu {rs_g} oracle {rs_o}")
    assert rs_g == rs_o
    # the slope is sum_j w_j e_j with the least-squares weights w_j = (j - c) /
    # sum (j - c)^2 over the last n_fit energies; each GPU e_j is within
    # (colour-1 sites) x 2^-31 / N_GP of the exact one (fixed-point rounding)
    j = np.arange(prm.n_fit) - 0.5 * (prm.n_fit - 1)
    w_abs = float(np.sum(np.abs(j)) / np.sum(j * j))
    ngp = oracle.bond_count(64, 64)
    tol_k = w_abs * int(colour_mask(64, 64, 1).sum()) * 2.0 ** -31 / ngp
    for a, b in zip(st, sto):
        assert abs(a["k_last"] - b["k_last"]) <= tol_k + 1e-12 * abs(b["k_last"]), (a["k_last"], b["k_last"])
        assert a["a_final"] == b["a_final"]
    g = im.mask == 0
    d = np.abs(ps[g].astype(np.float64) - po[g])
    m2_o = pq - po * po / 40.0
    dm = np.abs(m2[g].astype(np.float64) - m2_o[g])
    say(f"  max |phi_sum diff| {d.max():.2e}, max |m2 diff| {dm.max():.2e}")
    assert d.max() <= 4e-5  # sums below 80 pi
    assert np.all(dm <= 1e-6 * np.maximum(1.0, m2_o[g]) + 1e-7)
    assert np.all(ps[~g] == 0) and np.all(m2[~g] == 0)


@pytest.mark.parametrize("fp64", [1, 0])
def test_relaxation_only_runs_zero_states(ctx, fp64):
    """K = 0: the chains relax to the stopping rule and record no state, so
    the sums are zero everywhere (sampled sites included) and the spread too.
    Double-precision chains stop at the oracle's sweeps with its final a;
    single-precision ones relax for as many sweeps as with K = 10, the same
    chains before their equilibrium phase."""
    im, phi32 = l64_angles()
    T = 0.15
    prm = mpr.default_params(R=2, K=0, seed=5, fp64=fp64)
    ps, m2, st = simulate_gpu(ctx, phi32, im.mask, T, prm)
    assert not ps.any() and not m2.any()
    if fp64:
        _, sto, _, _ = oracle.simulate(phi32.astype(np.float64), im.mask, T, oracle.default_params(R=2, K=0, seed=5))
        ref = [(s["relax_sweeps"], s["a_final"]) for s in sto]
    else:
        _, _, st10 = simulate_gpu(ctx, phi32, im.mask, T, mpr.default_params(R=2, K=10, seed=5, spread=1))
        ref = [(s["relax_sweeps"], s["a_final"]) for s in st10]
    got = [(s["relax_sweeps"], s["a_final"]) for s in st]
    say(f"  K=0 fp64={fp64}: {got} against {ref}")
    assert got == ref
    assert all(s["relax_sweeps"] > 0 and not s["not_converged"] for s in st)


def test_fp64_batch_matches_single_and_compact_shapes(ctx):
    """A ragged batch in double precision gives each image the result it
    gets alone, and the compacted block shapes give the plain shape's sums
    bit for bit."""
    im = synth.workload_l64()
    shapes = [(64, 64), (24, 40)]
    zs = [im.z, synth.matern_field(40, 24, 1.5, 0.1, 50, 10, 5)]
    ms = [im.mask, synth.random_mask(40, 24, 0.4, 6)]
    prm = mpr.default_params(R=2, K=3, fp64=1)
    T = np.array([0.15, 0.02])

    def run(sel, prm=prm):
        imgs = mpr.images([shapes[i] for i in sel], ids=list(sel))
        z = dev(np.concatenate([zs[i].astype(np.float32).ravel() for i in sel]), torch.float32)
        mk = dev(np.concatenate([ms[i].ravel() for i in sel]), torch.uint8)
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

    both = run([0, 1])
    for i in range(2):
        assert np.array_equal(both[i], run([i])[i]), i
    for tile in COMPACT_TILES:
        c = run([0, 1], mpr.default_params(R=2, K=3, fp64=1, tile_rows=tile))
        for i in range(2):
            assert np.array_equal(c[i].view(np.uint32), both[i].view(np.uint32)), (tile, i)


def test_affine_change_of_the_data_transforms_the_prediction(ctx):
    """z -> a z + b leaves the angles unchanged up to rounding (equation
    map), so the prediction becomes a z_hat + b; with double-precision chains
    the rounding of the transformed inputs does not send the chains apart."""
    im = synth.workload_l64()
    shape = im.z.shape
    imgs = mpr.images([shape])
    mk = dev(im.mask, torch.uint8)
    out = []
    for a, b in ((1.0, 0.0), (3.0, 7.0), (0.25, -40.0)):
        z32 = (a * im.z + b).astype(np.float32)
        z = dev(z32, torch.float32)
        phi = torch.zeros_like(z)
        zz = ctx.map_to_angles(imgs, z, mk, phi)
        prm = mpr.default_params(R=2, K=5, fixed_relax=20, seed=3, fp64=1)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        ps, zh = torch.zeros_like(z), torch.zeros_like(z)
        ctx.simulate(imgs, phi, mk, np.array([0.1]), prm, ws, ps)
        ctx.predict(imgs, z, mk, ps, zz, 10, zh)
        out.append((a, b, zh.cpu().numpy().astype(np.float64), z32))
    _, _, ref, _ = out[0]
    g = im.mask == 0
    for a, b, zh, z32 in out[1:]:
        assert np.array_equal(zh[~g], z32[~g].astype(np.float64))
        err = np.max(np.abs((zh[g] - b) / a - ref[g]))
        assert err <= 1e-3, (a, b, err)  # float rounding of the transformed data and outputs
