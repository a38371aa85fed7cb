"""Coupling exponents q < 1/2 (double-precision chains) and the hold-out
choice of q, against the FP64 oracle.

  - Teacher-forced half-sweeps at q = 0.3 and 0.125: every decision equals
    the oracle's, angles within 1e-11 rad (as for q = 1/2).
  - Free-running chains at q = 0.3 follow the oracle's to the float rounding
    of the sums; the temperature from the double-precision e(T, L) tables is
    the oracle's within 3%.
  - q < 1/2 on single-precision chains is refused.
  - mpr_select_q: per-candidate temperatures and hold-out errors within 5% of
    the oracle's rule, and the same choice when the oracle's two errors are
    more than 15% apart.
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


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


@pytest.mark.parametrize("q", [0.3, 0.125])
@pytest.mark.parametrize("kind", ["uniform", "smooth"])
def test_q_teacher_forced_half_sweeps(ctx, q, kind):
    ny, nx = 97, 131
    rng = np.random.default_rng(3)
    if kind == "uniform":
        phi = rng.uniform(0, TWO_PI, size=(ny, nx))
        m = (rng.random((ny, nx)) < 0.3).astype(np.uint8)
    else:
        z = synth.matern_field(nx, ny, 2.5, 0.05, 50.0, 10.0, 21)
        m = synth.random_mask(nx, ny, 0.5, 22)
        phi = TWO_PI * (z - z.min()) / (z.max() - z.min())
        g = m == 0
        phi[g] = np.mod(phi[g] + rng.normal(0, 0.02, size=g.sum()), TWO_PI)
    col = np.add.outer(np.arange(ny), np.arange(nx)) % 2
    n_dec = 0
    for T, a in ((1e-3, 1.0), (0.1, 10.0), (2.6e-4, 40.0)):
        for colour in (0, 1):
            for mode in (1, 0):
                g = dev(phi)
                fl = torch.zeros((ny, nx), dtype=torch.uint8, device="cuda")
                acc_g = ctx.diag_half_sweep_fp64(g, dev(m, torch.uint8), colour, T, a, 5, q=q, mode=mode, flags=fl)
                po, acc_o, fo = oracle.half_sweep(phi, m, colour, T, a, 5, q=q, mode=mode, with_flags=True)
                pg, fg = g.cpu().numpy(), fl.cpu().numpy()
                sel = (col == colour) & (m == 0)
                n_dec += int(sel.sum())
                assert np.array_equal(fg[sel] & 15, fo[sel] & 15), (T, a, colour, mode)
                assert acc_g == acc_o
                assert np.max(np.abs(pg - po)) <= 1e-11
            phi = po
    say(f"  q={q} {kind}: {n_dec} updates, all decisions equal")


def l64_angles():
    im = synth.workload_l64()
    po, zz = oracle.map_to_angles(im.z.astype(np.float32).astype(np.float64), im.mask)
    return im, po.astype(np.float32), zz


def test_q_free_running_chains_and_temperature(ctx):
    q = 0.3
    im, phi32, _ = l64_angles()
    imgs = mpr.images([im.z.shape])
    mk = dev(im.mask, torch.uint8)
    ph = dev(phi32, torch.float32)
    prm = mpr.default_params(q=q, fp64=1, R=2, K=3, fixed_relax=10, seed=13, table_nT=12, table_T_lo=0.01,
                             table_T_hi=2.0, table_burn=100, table_meas=300)
    ws = torch.empty(ctx.workspace_size(imgs, prm), dtype=torch.uint8, device="cuda")
    e_s, T_hat, cl = ctx.estimate_temperature(imgs, ph, mk, prm, ws)
    ps = torch.zeros_like(ph)
    st = ctx.simulate(imgs, ph, mk, np.array([0.15]), prm, ws, ps)
    opr = oracle.default_params(q=q, R=2, K=3, fixed_relax=10, seed=13)
    po, sto, _, _ = oracle.simulate(phi32.astype(np.float64), im.mask, 0.15, opr)
    g = im.mask == 0
    d = np.abs(ps.cpu().numpy()[g].astype(np.float64) - po[g])
    say(f"  q={q}: max |phi_sum gpu - oracle| {d.max():.2e}")
    assert d.max() <= 4e-6
    assert [s["a_final"] for s in st] == [s["a_final"] for s in sto]
    e_o, _ = oracle.sample_energy(phi32.astype(np.float64), im.mask, q)
    assert abs(e_s[0] - e_o) <= 1e-12
    Tg = oracle.temperature_grid(12, 0.01, 2.0)
    T_o, cl_o = oracle.invert_temperature(Tg, oracle.energy_table(64, 64, Tg, 100, 300, seed=prm.seed, q=q), e_o)
    say(f"  q={q}: T_hat gpu {T_hat[0]:.5f} oracle {T_o:.5f}")
    assert not cl[0] and not cl_o
    assert abs(T_hat[0] / T_o - 1.0) < 0.03


def test_q_below_half_needs_double_chains(ctx):
    imgs = mpr.images([(8, 8)])
    assert ctx.workspace_size(imgs, mpr.default_params(q=0.3, fp64=0)) < 0
    assert ctx.workspace_size(imgs, mpr.default_params(q=0.6, fp64=1)) < 0
    assert ctx.workspace_size(imgs, mpr.default_params(q=0.3, fp64=1)) > 0


def test_select_q_matches_oracle_rule(ctx):
    ny, nx = 40, 48
    z = synth.matern_field(nx, ny, 1.5, 0.2, 50.0, 10.0, 61)
    m = synth.random_mask(nx, ny, 0.4, 62)
    qs = [0.25, 0.5]
    tab = dict(table_nT=10, table_T_lo=1e-3, table_T_hi=2.0, table_burn=50, table_meas=100)
    prm = mpr.default_params(R=4, K=10, seed=71, **tab)
    img = mpr.images([(ny, nx)])
    ws = torch.empty(ctx.select_q_workspace_size(img, prm, qs), dtype=torch.uint8, device="cuda")
    qb, mae, T = ctx.select_q(img, dev(z.astype(np.float32), torch.float32), dev(m, torch.uint8), prm, qs, 0.3, ws)
    opr = oracle.default_params(R=4, K=10, seed=71)
    qb_o, mae_o, T_o = oracle.select_q(z.astype(np.float32).astype(np.float64), m, opr, qs, 0.3, 10, 1e-3, 2.0,
                                       50, 100)
    say(f"  gpu q* {qb} errors {mae} T {T}; oracle q* {qb_o} errors {mae_o} T {T_o}")
    assert np.all(np.abs(T / T_o - 1.0) < 0.05)
    assert np.all(np.abs(mae / mae_o - 1.0) < 0.05)
    if abs(mae_o[0] / mae_o[1] - 1.0) > 0.15:
        assert qb == qb_o
