"""GPU parity of the recorded realizations and their per-site quantiles.

  - The quantile kernel on states made here (ragged images, ties, M from 1
    to 256) equals the oracle's quantiles bit for bit after rounding to
    float (both interpolate and back-transform in double).
  - The states mpr_simulate records equal the oracle's recorded states on
    early sweeps, where the single-precision chains still follow the
    oracle's site by site (99% of gap sites within 1e-5 rad), and at every
    site for double-precision chains; they sum to phi_sum.
"""
import math

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_1811_01604_amd as mpr  # noqa: E402

pytestmark = pytest.mark.gpu
TWO_PI = 2.0 * math.pi
PROBS = [0.0, 0.025, 0.25, 0.5, 0.75, 0.975, 1.0]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mpr.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("M", [1, 2, 7, 100, 256])
def test_quantile_kernel_matches_oracle(ctx, M):
    rng = np.random.default_rng(M)
    shapes = [(33, 47), (20, 9)]
    zs = [rng.normal(50, 10, size=s).astype(np.float32) for s in shapes]
    ms = [(rng.random(s) < 0.4).astype(np.uint8) for s in shapes]
    for m in ms:
        m.flat[:2] = 1
    n_total = sum(a * b for a, b in shapes)
    st = rng.uniform(0, TWO_PI, size=(M, n_total)).astype(np.float32)
    st[M // 2:, ::7] = st[0, ::7]  # ties
    zz = np.concatenate([[float(z[m == 1].min()), float(z[m == 1].max())] for z, m in zip(zs, ms)])
    z = np.concatenate([a.ravel() for a in zs])
    mk = np.concatenate([a.ravel() for a in ms])
    out = torch.zeros((len(PROBS), n_total), device="cuda")
    ctx.quantiles(mpr.images(shapes), dev(z), dev(mk, torch.uint8), dev(st), M, PROBS, zz, out)
    got = out.cpu().numpy()
    off = 0
    for b, (ny, nx) in enumerate(shapes):
        n = ny * nx
        want = oracle.quantiles(zs[b].astype(np.float64), ms[b], st[:, off:off + n].astype(np.float64).reshape(M, ny, nx),
                                PROBS, zz[2 * b:2 * b + 2])
        g = got[:, off:off + n].reshape(len(PROBS), ny, nx)
        assert np.array_equal(g.view(np.uint32), want.astype(np.float32).view(np.uint32)), b
        off += n


def test_quantile_arguments_are_checked(ctx):
    shapes = [(4, 4)]
    z = dev(np.ones(16, np.float32))
    mk = dev(np.zeros(16, np.uint8), torch.uint8)
    out = torch.zeros((1, 16), device="cuda")
    for M, probs in ((257, [0.5]), (4, [1.5]), (4, [-0.1])):
        st = torch.zeros((M, 16), device="cuda")
        with pytest.raises(mpr.MprError) as e:
            ctx.quantiles(mpr.images(shapes), z, mk, st, M, probs, [0.0, 1.0], out)
        assert e.value.code == mpr.MPR_ERR_ARG


def run_states(ctx, im, prm, T):
    ny, nx = im.z.shape
    po, zz = oracle.map_to_angles(im.z.astype(np.float32).astype(np.float64), im.mask)
    phi32 = po.astype(np.float32)
    imgs = mpr.images([(ny, nx)])
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    ps = torch.zeros(ny * nx, device="cuda")
    M = prm.R * prm.K
    st = torch.zeros((M, ny * nx), device="cuda")
    ctx.simulate(imgs, dev(phi32.ravel()), dev(im.mask.ravel(), torch.uint8), np.array([T]), prm, ws, ps,
                 phi_states=st)
    zq = torch.zeros((len(PROBS), ny * nx), device="cuda")
    ctx.quantiles(imgs, dev(im.z.astype(np.float32).ravel()), dev(im.mask.ravel(), torch.uint8), st, M, PROBS, zz,
                  zq)
    return phi32, zz, ps.cpu().numpy().reshape(ny, nx), st.cpu().numpy().reshape(M, ny, nx), \
        zq.cpu().numpy().reshape(len(PROBS), ny, nx)


@pytest.mark.parametrize("R,K", [(2, 3), (5, 1)])
def test_recorded_states_match_oracle_early_sweeps(ctx, R, K):
    im = synth.workload_l64()
    prm = mpr.default_params(R=R, K=K, fixed_relax=0, seed=91)
    phi32, zz, ps, st, zq = run_states(ctx, im, prm, 0.15)
    opr = oracle.default_params(R=R, K=K, fixed_relax=0, seed=91)
    pso, _, _, _, sto = oracle.simulate(phi32.astype(np.float64), im.mask, 0.15, opr, want_states=True)
    g = im.mask == 0
    ok = np.abs(st[:, g].astype(np.float64) - sto[:, g]) <= 1e-5
    assert ok.mean() >= 0.99, ok.mean()
    # samples recorded with their angle; the states sum to phi_sum
    assert np.all(st[:, ~g] == phi32[~g][None, :])
    assert np.allclose(st.astype(np.float64).sum(0)[g], ps[g], rtol=2e-6, atol=1e-5)
    qo = oracle.quantiles(im.z.astype(np.float32).astype(np.float64), im.mask, sto, PROBS, zz)
    okq = np.abs(zq[:, g] - qo[:, g]) <= 1e-3
    assert okq.mean() >= 0.99, okq.mean()


def test_recorded_states_of_double_precision_chains(ctx):
    im = synth.workload_l64()
    prm = mpr.default_params(R=2, K=3, fixed_relax=6, seed=17, fp64=1)
    phi32, zz, ps, st, zq = run_states(ctx, im, prm, 0.15)
    opr = oracle.default_params(R=2, K=3, fixed_relax=6, seed=17)
    _, _, _, _, sto = oracle.simulate(phi32.astype(np.float64), im.mask, 0.15, opr, want_states=True)
    g = im.mask == 0
    # double chains follow the oracle at every site; the record rounds to float
    assert np.max(np.abs(st[:, g].astype(np.float64) - sto[:, g])) <= 1e-6
    qo = oracle.quantiles(im.z.astype(np.float32).astype(np.float64), im.mask, sto, PROBS, zz)
    assert np.max(np.abs(zq[:, g] - qo[:, g])) <= 1e-4


def test_recorded_states_of_a_ragged_batch_equal_the_images_alone(ctx):
    """Two images of different sizes in one call: each image's recorded
    states (and quantiles) equal those of the image run alone, bit for bit."""
    shapes = [(64, 64), (24, 40)]
    zs = [synth.workload_l64().z, synth.matern_field(40, 24, 1.5, 0.1, 50, 10, 5)]
    ms = [synth.workload_l64().mask, synth.random_mask(40, 24, 0.4, 6)]
    prm = mpr.default_params(R=2, K=3, fixed_relax=4, seed=19)
    T = np.array([0.15, 0.05])
    M = prm.R * prm.K

    def run(sel):
        imgs = mpr.images([shapes[i] for i in sel], ids=list(sel))
        z = dev(np.concatenate([zs[i].astype(np.float32).ravel() for i in sel]))
        mk = dev(np.concatenate([ms[i].ravel() for i in sel]), torch.uint8)
        phi = torch.zeros_like(z)
        zz = ctx.map_to_angles(imgs, z, mk, phi)
        ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
        ps = torch.zeros_like(z)
        st = torch.zeros((M, z.numel()), device="cuda")
        ctx.simulate(imgs, phi, mk, T[list(sel)], prm, ws, ps, phi_states=st)
        zq = torch.zeros((len(PROBS), z.numel()), device="cuda")
        ctx.quantiles(imgs, z, mk, st, M, PROBS, zz, zq)
        out, off = {}, 0
        for i in sel:
            n = shapes[i][0] * shapes[i][1]
            out[i] = (st[:, off:off + n].cpu().numpy(), zq[:, off:off + n].cpu().numpy())
            off += n
        return out

    both = run([0, 1])
    for i in range(2):
        alone = run([i])[i]
        assert np.array_equal(both[i][0].view(np.uint32), alone[0].view(np.uint32)), i
        assert np.array_equal(both[i][1].view(np.uint32), alone[1].view(np.uint32)), i
