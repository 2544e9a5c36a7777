"""The shelf demonstration inputs (plane wave onto a discontinuous shelf) and
the oracle on them: the hierarchy's level-0 bathymetry is the block mean of the
finest samples with the break on a level-0 cell boundary, the interface sits at
-0.125 everywhere, the wave's layers move at eta1 sqrt(g), and without the wave the oracle keeps
the layers exactly at rest across the break (well-balanced over a
discontinuous bottom)."""
import numpy as np

import oracle
from paper_1803_01450_amd import inputs

G = 9.81


def test_shelf_inputs_are_consistent():
    c = inputs.shelf_wave(n0=32, width=0.05)
    r = int(np.prod(c["ratios"]))
    assert np.array_equal(c["B0"], inputs.block_mean(c["Bf"], r))
    assert set(np.unique(c["B0"])) == {-1.0, -0.25}
    for B, q in ((c["Bf"], c["qf"]), (c["B0"], c["q0"])):
        assert np.all(B + q[3] == -0.125)
        eta1 = B + q[3] + q[0]
        assert np.allclose(q[1], q[0] * eta1 * np.sqrt(G), rtol=0, atol=1e-15)
        assert np.allclose(q[4], q[3] * eta1 * np.sqrt(G), rtol=0, atol=1e-15)
        assert np.all(q[2] == 0) and np.all(q[5] == 0)


def test_oracle_rest_across_the_break():
    """Without the wave the two layers rest over the discontinuous shelf: 20
    steps leave every depth and momentum bit for bit as they were."""
    c = inputs.shelf_wave(n0=16, amp=0.0)
    nx, ny, dx = c["nfx"], c["nfy"], c["dxf"]
    H = oracle.Hierarchy(nx, ny, dx, dx, r=c["r"])
    H.set_bathymetry(c["Bf"])
    H.set_state(0, c["qf"])
    rc, dts = H.advance(20)
    assert rc == 0 and dts.min() > 0
    q = H.state(0)
    for f in range(6):
        assert np.array_equal(q[f], c["qf"][f]), f
