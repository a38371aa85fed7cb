"""The largest image the library accepts: 46000 x 46000 sites (2.1e9), whose
single-precision half-grid (46000 rows of 23040 floats, 3.95 GiB) is just
under the 4 GiB that the sweep kernels' 32-bit byte offsets address.

Over-relaxation only (no random numbers: a gap site's new angle depends on
its four neighbours alone), so each updated site can be checked against the
oracle's half-sweep of the 3 x 3 crop around it.  Gap sites are placed at
both ends of the grid, around the half-grid byte offset 2^31 and at random;
every other site is sampled.  For each colour and for the default plain and
the compacted 4-row block shape: the sites that change are updated gap sites
of that colour, and each gap site of the colour equals the oracle's value
within 1e-5 rad.
"""
import sys

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
import paper_1811_01604_amd as mpr  # noqa: E402

pytestmark = pytest.mark.gpu
N = 46000
TWO_PI = 2.0 * np.pi


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mpr.Context(0)
    yield c
    c.close()


SCALE = np.float32(TWO_PI / 65536)


def angles(y0, y1, x0=0, x1=N):
    """The test's angle field on rows y0..y1-1, columns x0..x1-1 (float32):
    a 16-bit integer hash of the site times 2 pi / 65536, one rounding."""
    x = np.arange(x0, x1, dtype=np.int64)[None, :]
    y = np.arange(y0, y1, dtype=np.int64)[:, None]
    return ((x * 40503 + y * 9973) & 0xFFFF).astype(np.float32) * SCALE


def angles_dev(y0, y1):
    """The same field built on the GPU (integer ops and one float multiply,
    so it equals angles() bit for bit)."""
    x = torch.arange(N, dtype=torch.int64, device="cuda")[None, :]
    y = torch.arange(y0, y1, dtype=torch.int64, device="cuda")[:, None]
    return ((x * 40503 + y * 9973) & 0xFFFF).to(torch.float32) * float(SCALE)


def gap_sites():
    S = (N // 2 + 63) // 64 * 64
    i = (1 << 29)  # element at byte offset 2^31 of a half-grid
    ym, hm = i // S, i % S
    pts = {(0, 0), (1, 0), (0, 1), (1, 1), (2, 1), (N - 1, N - 1), (N - 2, N - 1), (N - 1, N - 2), (N - 2, N - 2),
           (N - 3, N - 1), (0, N - 1), (N - 1, 0)}
    for dy in (-1, 0, 1):
        for dx in range(-3, 4):
            pts.add((2 * hm + dx, ym + dy))
    rng = np.random.default_rng(11)
    for x, y in zip(rng.integers(0, N, 200), rng.integers(0, N, 200)):
        pts.add((int(x), int(y)))
    return sorted(pts)


def oracle_site(x, y, gaps, colour):
    """The oracle's over-relaxed angle of gap site (x, y) from its 3 x 3 crop."""
    ya, yb = max(0, y - 1), min(N - 1, y + 1)
    xa, xb = max(0, x - 1), min(N - 1, x + 1)
    crop = angles(ya, yb + 1, xa, xb + 1).astype(np.float64)
    m = np.ones(crop.shape, np.uint8)
    for gx, gy in gaps:
        if xa <= gx <= xb and ya <= gy <= yb:
            m[gy - ya, gx - xa] = 0
    # the crop keeps the site's colour when its origin has an even x + y
    c = ((x - xa) + (y - ya)) & 1
    assert c == colour ^ ((xa + ya) & 1)
    po, _, _ = oracle.half_sweep(crop, m, c, 0.1, 1.0, 0, mode=oracle.MODE_OR_ONLY)
    return po[y - ya, x - xa]


def test_largest_image_over_relaxation_against_oracle(ctx):
    # the host checks accept this size (and refuse 46340 x 46340, a CPU test)
    assert ctx.workspace_size(mpr.images([(N, N)]), mpr.default_params(R=1, K=1)) > 0
    say(f"  {N} x {N}: building the angles")
    phi0 = torch.empty((N, N), dtype=torch.float32, device="cuda")
    for y0 in range(0, N, 4000):
        y1 = min(N, y0 + 4000)
        phi0[y0:y1] = angles_dev(y0, y1)
    gaps = gap_sites()
    for x, y in gaps[:: 7]:  # the device field is the host formula's
        assert phi0[y - 1 if y else y: y + 2, x].cpu().numpy().tobytes() == \
            angles(y - 1 if y else y, min(N, y + 2), x, x + 1).ravel().tobytes()
    sampled = torch.ones((N, N), dtype=torch.uint8, device="cuda")
    gx = torch.tensor([g[0] for g in gaps], device="cuda")
    gy = torch.tensor([g[1] for g in gaps], device="cuda")
    sampled[gy, gx] = 0
    phi = torch.empty_like(phi0)
    for tile in (0, 4 | mpr.TILE_COMPACT, 32 | mpr.TILE_FUSED):
        for colour in (0, 1):
            phi.copy_(phi0)
            ctx.diag_half_sweep(phi, sampled, colour, 0.1, 1.0, 0, mode=1, tile=tile)
            changed = (phi.view(torch.int32) != phi0.view(torch.int32)).nonzero().cpu().numpy()
            mine = {(x, y) for x, y in gaps if ((x + y) & 1) == colour}
            assert {(int(x), int(y)) for y, x in changed} <= mine, (tile, colour)
            assert len(changed) >= len(mine) // 2  # about 3 in 4 reflections stay in range here
            got = phi[gy, gx].cpu().numpy()
            worst = 0.0
            for k, (x, y) in enumerate(gaps):
                if (x, y) not in mine:
                    continue
                err = abs(float(got[k]) - oracle_site(x, y, gaps, colour))
                worst = max(worst, err)
                assert err <= 1e-5, (tile, colour, x, y, float(got[k]))
            say(f"  tile {tile} colour {colour}: {len(changed)} sites changed of {len(mine)} gaps, "
                f"max |dphi| {worst:.2e}")
