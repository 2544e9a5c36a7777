"""Order independence on the GPU: a level's patches listed in another order,
the problems of a batch defined in reverse order, and a repeated run with the
launch shape chosen by the autotuner all give bit-identical states, dts and
counts."""
import sys

import numpy as np
import pytest

from paper_1803_01450_amd import inputs

pytestmark = pytest.mark.gpu

BOXES = [(16, 16, 32, 32), (48, 16, 16, 32), (24, 48, 72, 16), (96, 40, 20, 30), (116, 40, 10, 30)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b):
    na, nb = np.isnan(a), np.isnan(b)
    return np.array_equal(na, nb) and np.array_equal(a[~na], b[~nb])


def run_patches(boxes, mode):
    from paper_1803_01450_amd.binding import Solver
    c = inputs.fixed_small()
    S = Solver()
    p = S.define(64, 64, c["dx"], c["dx"], c["r"], (2,))
    S.set_bathymetry(p, c["Bf"]); S.set_state(p, 0, c["q"])
    S.refine(p, 1, boxes)
    dts = S.advance(5, mode=mode, want_dts=True)[0]
    out = ([S.state(p, l) for l in range(2)], dts, S.counters(p))
    S.close()
    return out


@pytest.mark.parametrize("mode", [0, 1])
def test_patch_order(mode):
    say("case: patch order, mode", mode)
    s0, d0, c0 = run_patches(BOXES, mode)
    for order in ([4, 3, 2, 1, 0], [2, 0, 4, 1, 3]):
        s1, d1, c1 = run_patches([BOXES[k] for k in order], mode)
        assert np.array_equal(d0, d1)
        assert all(same(a, b) for a, b in zip(s0, s1))
        for k in ("hyp", "nclip", "repair", "updates"):
            assert c0[k] == c1[k], k


def run_batch(order, tune):
    from paper_1803_01450_amd.binding import Solver, BATCHED
    sizes = inputs.batch_sizes(512)[:8]
    S = Solver()
    ids = {}
    for k in order:
        c = inputs.batch_problem(k, int(sizes[k]))
        p = S.define(c["n"], c["n"], c["dx"], c["dx"], c["r"], (2,))
        S.set_bathymetry(p, np.kron(c["B"], np.ones((2, 2))))
        S.set_state(p, 0, c["q"])
        ids[k] = p
    if tune:
        S.autotune(None, reps=1)
    tau = np.tile([2e-5, 0.0], (len(order), 1))
    S.advance(6, 3, tau, mode=BATCHED)
    out = {k: ([S.state(ids[k], l) for l in range(2)], [S.patches(ids[k], l) for l in range(2)],
               S.counters(ids[k])) for k in order}
    S.close()
    return out


def test_batch_order_and_repeat():
    say("case: 8 batch problems, forward and reverse definition order, autotuned repeat")
    a = run_batch(list(range(8)), False)
    b = run_batch(list(range(7, -1, -1)), False)
    t = run_batch(list(range(8)), True)
    for k in range(8):
        for other in (b, t):
            assert all(same(x, y) for x, y in zip(a[k][0], other[k][0])), k
            assert all(np.array_equal(x, y) for x, y in zip(a[k][1], other[k][1])), k
            assert a[k][2]["updates"] == other[k][2]["updates"]
            assert a[k][2]["t"] == other[k][2]["t"]
