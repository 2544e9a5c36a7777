"""Checkpoint and resume of the oracle's level hierarchy: a run of N coarse steps
(three levels, shorelines, regrid every 4) equals, bit for bit, a run of k steps
whose patches, states and time-stepping state (t, speeds of the last step) are
copied into a new hierarchy that then runs the remaining N - k steps (k a
multiple of the regrid interval).  Restoring states and patches alone is not
enough: the first resumed step then takes its dt from the state, and the runs
part."""
import numpy as np

import oracle
from paper_1803_01450_amd import inputs

N, K, EVERY, TAU = 8, 4, 4, (4e-6, 8e-6)


def fresh(c):
    H = oracle.Hierarchy(c["n0"], c["n0"], c["dx0"], c["dx0"], ratios=c["ratios"], r=c["r"])
    H.set_bathymetry(c["Bf"])
    return H


def same(a, b):
    na, nb = np.isnan(a), np.isnan(b)
    return np.array_equal(na, nb) and np.array_equal(a[~na], b[~nb])


def checkpoint(H, nlev):
    return ([H.patches(l) for l in range(nlev)], [H.state(l) for l in range(nlev)], H.step_state())


def restore(c, ck, with_clock=True):
    patches, states, clock = ck
    H = fresh(c)
    for l in range(len(states)):
        if l > 0:
            H.set_patches(l, patches[l])
        H.set_state(l, np.nan_to_num(states[l]))
    if with_clock:
        H.set_step_state(clock)
    return H


def test_resume_is_bitwise():
    c = inputs.amr_shoreline(n0=32, L=50e3, ratios=(2, 4))
    A = fresh(c)
    A.set_state(0, c["q0"])
    rc, dA = A.advance(N, EVERY, TAU)
    assert rc == 0
    B = fresh(c)
    B.set_state(0, c["q0"])
    rc, d1 = B.advance(K, EVERY, TAU)
    assert rc == 0
    ck = checkpoint(B, 3)
    assert ck[2][0] == B.counters()["t"] and ck[2][1] == 1.0 and np.all(ck[2][2:] > 0)
    C = restore(c, ck)
    rc, d2 = C.advance(N - K, EVERY, TAU)
    assert rc == 0
    assert np.array_equal(np.concatenate([d1, d2]), dA)
    assert C.counters()["t"] == A.counters()["t"]
    for l in range(3):
        assert np.array_equal(C.patches(l), A.patches(l)), l
        assert same(C.state(l), A.state(l)), l
    assert len(A.patches(2)) > 0
    # without the time-stepping state the first resumed dt comes from the state
    D = restore(c, ck, with_clock=False)
    rc, d3 = D.advance(N - K, EVERY, TAU)
    assert rc == 0 and d3[0] != d2[0]
