"""What the trained warm start gains over the plain random start.

The committed network (trained on the library's own simulations of 256^2
images) is applied to fresh 1024^2 images; the chains with the learned start
must stop in fewer sweeps and reach the same prediction MAE (within 1% on
random masks, where the seed-to-seed spread is small).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_1811_01604_amd as mpr  # noqa: E402
from paper_1811_01604_amd import warmstart  # noqa: E402

pytestmark = pytest.mark.gpu


def test_warm_start_gain():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    params, info = warmstart.load()
    ctx = mpr.Context(0)
    model = warmstart.WarmStart(ctx, params)
    s = warmstart.evaluate(ctx, model, size=1024, seeds=2, workers=4)
    ctx.close()
    print(s)
    for kind in ("random", "cloud"):
        assert s[kind]["sweeps_warm"] < s[kind]["sweeps_plain"]
        assert s[kind]["time_to_fill_warm_s"] < s[kind]["time_to_fill_plain_s"] * 1.05
    assert abs(s["random"]["mae_warm_over_plain"] - 1.0) < 0.01
    assert abs(s["cloud"]["mae_warm_over_plain"] - 1.0) < 0.05
