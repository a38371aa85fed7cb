"""The seeded input generators (CPU)."""
import numpy as np

import synth


def test_ragged_batch_is_the_same_with_worker_processes():
    a = synth.ragged_batch(6, lo=16, hi=64, workers=1)
    b = synth.ragged_batch(6, lo=16, hi=64, workers=2)
    assert [x.name for x in a] == [x.name for x in b]
    for x, y in zip(a, b):
        assert np.array_equal(x.z, y.z) and np.array_equal(x.mask, y.mask)
