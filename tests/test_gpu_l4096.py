"""The L=4096 workload at its full size (lognormal exp(G), G Matern nu=1.5
kappa=0.02 std 0.5; 66% random gaps or 40% cloud gaps).

  - Teacher-forced half-sweeps over the whole 4096 x 4096 grid in the block
    shapes the autotuner picks on this workload (compacted 4 and 8 half-rows)
    and the default plain shape, against the oracle at every site: fewer
    than 1e-6 of the decisions flipped, angles within 1e-5 rad elsewhere,
    accepted counts equal up to the flips, the fused energy within 1e-6 per
    bond.  The random-mask case starts from U(0, 2 pi) gaps with a = 1 (the
    first sweeps), the cloud case from the true angles plus noise with
    a = 20 (late relaxation), both at T = 6e-5 (near this workload's
    estimate).
  - The recorded realizations at full size and their quantiles at sampled
    sites against the oracle.
  - The launch configuration the benchmark times (R = 100 chains, K = 1,
    stopping rule) gives each chain the relaxation it gets in a 2-chain
    launch, and the same sums in the plain and both compacted shapes (the
    launch list shrinking as chains stop).
"""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_1811_01604_amd as mpr  # noqa: E402

pytestmark = pytest.mark.gpu
TWO_PI = 2.0 * np.pi
T = 6e-5
TILES = [4 | mpr.TILE_COMPACT, 8 | mpr.TILE_COMPACT, 0, 32 | mpr.TILE_FUSED]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mpr.Context(0)
    yield c
    c.close()


def start_state(im, kind):
    """Sample angles from the oracle's map (rounded to float32) and gap
    angles made here: uniform, or the true angles plus noise."""
    po, _ = oracle.map_to_angles(im.z.astype(np.float32).astype(np.float64), im.mask)
    phi = po.astype(np.float32)
    g = im.mask == 0
    rng = np.random.default_rng(17)
    if kind == "uniform":
        phi[g] = rng.uniform(0, TWO_PI, size=int(g.sum())).astype(np.float32)
    else:
        zt = im.z.astype(np.float64)
        true = TWO_PI * (zt - zt[~g].min()) / (zt[~g].max() - zt[~g].min())
        phi[g] = np.mod(true[g] + rng.normal(0, 0.05, size=int(g.sum())), TWO_PI).astype(np.float32)
    return phi


@pytest.mark.parametrize("mask,kind,a", [("random", "uniform", 1.0), ("cloud", "noisy", 20.0)])
def test_l4096_teacher_forced_half_sweeps(ctx, mask, kind, a):
    im = synth.workload_l4096(mask)
    phi = start_state(im, kind)
    ny, nx = phi.shape
    m = im.mask
    mk = torch.from_numpy(m).cuda()
    ngp = oracle.bond_count(nx, ny)
    col = np.add.outer(np.arange(ny), np.arange(nx)) % 2
    for colour in (0, 1):
        po, acc_o, fo = oracle.half_sweep(phi.astype(np.float64), m, colour, T, a, 9, with_flags=True)
        e_o = oracle.energy(po) + ngp if colour == 1 else None
        sel = (col == colour) & (m == 0)
        n_dec = int(sel.sum())
        for tile in TILES:
            g = torch.from_numpy(phi).cuda()
            fl = torch.zeros((ny, nx), dtype=torch.uint8, device="cuda")
            acc_g, e_g = ctx.diag_half_sweep(g, mk, colour, T, a, 9, flags=fl, with_energy=True, tile=tile)
            pg, fg = g.cpu().numpy(), fl.cpu().numpy()
            flip = (((fg ^ fo) & 3) != 0) & sel
            n_flip = int(flip.sum())
            ok = sel & ~flip
            err = float(np.max(np.abs(pg[ok].astype(np.float64) - po[ok])))
            say(f"  {mask} colour {colour} tile {tile}: {n_dec} decisions, {n_flip} flipped, "
                f"double-precision path {int(((fg & 16) != 0).sum())}, max |dphi| {err:.2e}")
            assert n_flip <= int(1e-6 * n_dec)
            assert err <= 1e-5
            assert abs(acc_g - acc_o) <= n_flip
            assert np.array_equal(pg[m == 1].view(np.uint32), phi[m == 1].view(np.uint32))
            if colour == 1:
                assert abs(e_g - e_o) / ngp <= 1e-6, (e_g, e_o)
        phi = po.astype(np.float32)


def test_l4096_benchmark_launch_matches_smaller_launches(ctx):
    im = synth.workload_l4096("random")
    imgs = mpr.images([im.z.shape])
    z = torch.from_numpy(im.z.astype(np.float32)).cuda()
    mk = torch.from_numpy(im.mask).cuda()
    phi = torch.zeros_like(z)
    ctx.map_to_angles(imgs, z, mk, phi)
    Tn = np.array([T])
    runs = {}
    for R, tile in ((100, 0), (100, 4 | mpr.TILE_COMPACT), (100, 8 | mpr.TILE_COMPACT), (100, 32 | mpr.TILE_FUSED),
                    (2, 0)):
        # the stopping rule: chains stop at different sweeps, so the launch
        # list shrinks as they finish
        prm = mpr.default_params(R=R, K=1, tile_rows=tile)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        ps = torch.zeros_like(z)
        st = ctx.simulate(imgs, phi, mk, Tn, prm, ws, ps)
        runs[(R, tile)] = (ps.cpu().numpy(), st)
        del ws
        say(f"  R={R} tile {tile}: relax sweeps {sorted(set(s['relax_sweeps'] for s in st))}")
    ref_ps, ref_st = runs[(100, 0)]
    for key in ((100, 4 | mpr.TILE_COMPACT), (100, 8 | mpr.TILE_COMPACT), (100, 32 | mpr.TILE_FUSED)):
        ps, st = runs[key]
        assert np.array_equal(ps.view(np.uint32), ref_ps.view(np.uint32)), key
        assert st == ref_st, key
    _, st2 = runs[(2, 0)]
    assert st2 == ref_st[:2]
    g = im.mask == 0
    assert np.all(ref_ps[~g] == 0) and np.all((ref_ps[g] >= 0) & (ref_ps[g] < TWO_PI * 100))


def test_l4096_recorded_states_and_quantiles(ctx):
    """The benchmark's launch (100 chains, K = 1, stopping rule) with every
    realization recorded (6.7 GB): the states sum to phi_sum, samples are
    recorded with their angle, and the quantiles at 2000 sampled gap sites
    equal the oracle's quantiles of those sites' 100 recorded values."""
    im = synth.workload_l4096("random")
    ny, nx = im.z.shape
    imgs = mpr.images([im.z.shape])
    z = torch.from_numpy(im.z.astype(np.float32)).cuda()
    mk = torch.from_numpy(im.mask).cuda()
    phi = torch.zeros_like(z)
    zz = ctx.map_to_angles(imgs, z, mk, phi)
    prm = mpr.default_params(R=100, K=1)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps = torch.zeros_like(z)
    st = torch.empty((100, ny * nx), dtype=torch.float32, device="cuda")
    ctx.simulate(imgs, phi, mk, np.array([T]), prm, ws, ps, phi_states=st)
    del ws
    probs = [0.05, 0.5, 0.95]
    zq = torch.empty((len(probs), ny * nx), dtype=torch.float32, device="cuda")
    ctx.quantiles(imgs, z, mk, st, 100, probs, zz, zq)
    g = (im.mask == 0).ravel()
    tot = st.double().sum(0)
    d = (tot - ps.view(-1).double()).abs()[torch.from_numpy(g).cuda()]
    # phi_sum adds the 100 float states in float: 99 roundings of partial sums
    # below 200 pi, each at most half an ulp of 512..1024 (2^-15)
    assert float(d.max()) <= 99 * 2.0 ** -15
    s_idx = torch.from_numpy(np.flatnonzero(~g)[:1000]).cuda()
    assert torch.equal(st[:, s_idx], phi.view(-1)[s_idx].unsqueeze(0).expand(100, -1))
    rng = np.random.default_rng(3)
    sites = np.sort(rng.choice(np.flatnonzero(g), size=2000, replace=False))
    vals = st[:, torch.from_numpy(sites).cuda()].cpu().numpy().astype(np.float64)  # 100 x 2000
    # the oracle on a 1 x 2000 "image" of those sites (all gaps)
    qo = oracle.quantiles(np.zeros((1, 2000)), np.zeros((1, 2000), np.uint8), vals.reshape(100, 1, 2000), probs, zz)
    got = zq[:, torch.from_numpy(sites).cuda()].cpu().numpy()
    assert np.array_equal(got.view(np.uint32), qo.reshape(len(probs), 2000).astype(np.float32).view(np.uint32))
