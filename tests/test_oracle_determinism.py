"""Order independence of the oracle: the patches of a level listed in another
order, and a run repeated, give bit-identical states and counts."""
import numpy as np

import oracle
from paper_1803_01450_amd import inputs

BOXES = [(16, 16, 32, 32), (48, 16, 16, 32), (24, 48, 72, 16), (96, 40, 20, 30), (116, 40, 10, 30)]


def run(boxes):
    c = inputs.fixed_small()
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(2,), r=c["r"])
    H.set_bathymetry(c["Bf"]); H.set_state(0, c["q"])
    H.set_patches(1, boxes)
    rc, dts = H.advance(5)
    assert rc == 0
    return [H.state(l) for l in range(2)], dts, H.counters()


def same(a, b):
    na, nb = np.isnan(a), np.isnan(b)
    return np.array_equal(na, nb) and np.array_equal(a[~na], b[~nb])


def test_patch_order_and_repeat():
    s0, d0, c0 = run(BOXES)
    for order in ([4, 3, 2, 1, 0], [2, 0, 4, 1, 3]):
        s1, d1, c1 = run([BOXES[k] for k in order])
        assert np.array_equal(d0, d1)
        assert all(same(a, b) for a, b in zip(s0, s1))
        assert c0 == c1
    s2, d2, c2 = run(BOXES)
    assert np.array_equal(d0, d2) and all(same(a, b) for a, b in zip(s0, s2)) and c0 == c2
