"""Decision flips over more than 10^8 teacher-forced Metropolis decisions.

The L=4096 workload (lognormal exp(G), 66% random gaps) from uniform gap
angles, then chained: each half-sweep starts from the oracle's result of the
previous one (rounded to float32), in the tuned block shape (the fused tile
sweep, one colour in place) and at temperatures, a values and sweep counters
that cover the relaxation (T from 6e-5, this workload's estimate, to 0.1;
a from 1 to 40; fresh Philox streams each time).  Every decision is compared
with the oracle's at the same site: fewer than 1e-6 of them may differ (the
bound on decision flips), and the angles elsewhere agree within 1e-5 rad.
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
# (T, a, sweep counter) per sweep; two half-sweeps each
SETTINGS = [(6e-5, 1.0, 0), (6e-5, 4.0, 1), (6e-5, 20.0, 2), (1e-4, 40.0, 3), (2.6e-4, 8.0, 4),
            (1e-3, 2.0, 5), (1e-3, 12.0, 6), (0.01, 1.0, 7), (0.1, 1.0, 8), (6e-5, 30.0, 9)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_decision_flips_below_1e6_over_1e8_decisions():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = mpr.Context(0)
    try:
        im = synth.workload_l4096("random")
        po, _ = oracle.map_to_angles(im.z.astype(np.float32).astype(np.float64), im.mask)
        phi = po.astype(np.float32)
        m = im.mask
        g = m == 0
        phi[g] = np.random.default_rng(23).uniform(0, TWO_PI, size=int(g.sum())).astype(np.float32)
        ny, nx = phi.shape
        mk = torch.from_numpy(m).cuda()
        col = np.add.outer(np.arange(ny), np.arange(nx)) % 2
        tile = 48 | mpr.TILE_FUSED
        total = flips = 0
        for T, a, sweep in SETTINGS:
            for colour in (0, 1):
                ref, _, fo = oracle.half_sweep(phi.astype(np.float64), m, colour, T, a, sweep, with_flags=True)
                dev = torch.from_numpy(phi).cuda()
                fl = torch.zeros((ny, nx), dtype=torch.uint8, device="cuda")
                ctx.diag_half_sweep(dev, mk, colour, T, a, sweep, flags=fl, tile=tile)
                pg, fg = dev.cpu().numpy(), fl.cpu().numpy()
                sel = (col == colour) & g
                flip = (((fg ^ fo) & 3) != 0) & sel
                n_dec, n_flip = int(sel.sum()), int(flip.sum())
                ok = sel & ~flip
                err = float(np.max(np.abs(pg[ok].astype(np.float64) - ref[ok])))
                total += n_dec
                flips += n_flip
                say(f"  T={T:g} a={a:g} sweep {sweep} colour {colour}: {n_dec} decisions, {n_flip} flipped, "
                    f"max |dphi| {err:.1e}; {total} so far, {flips} flipped")
                assert err <= 1e-5
                phi = ref.astype(np.float32)
        assert total >= 100_000_000
        assert flips < 1e-6 * total, (flips, total)
    finally:
        ctx.close()
