"""Parity at the full sizes of the measured workloads, in the launch
configuration `bench.py` times (one launch per level substep over all problems,
union tiles, tile heights chosen per level):

* the batch of 512 uneven two-level problems, a few coarse steps with a regrid,
  sampled problems (smallest, median, largest) each against the oracle run on
  that problem alone;
* the three-level shoreline AMR run (256^2, ratios 2 and 4), a few coarse
  steps with a regrid, every level against the oracle.

Bars: patch layouts and update counts exact, dts within 1e-12 relative, states
within 1e-9 relative."""
import sys

import numpy as np
import pytest

import oracle
from paper_1803_01450_amd import inputs

pytestmark = pytest.mark.gpu

G = 9.81


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(a, b, H=4000.0):
    a = np.asarray(a); b = np.asarray(b)
    na, nb = np.isnan(a), np.isnan(b)
    assert np.array_equal(na, nb), "coverage differs"
    out = []
    for f in range(6):
        m = ~na[f]
        if not m.any():
            out.append(0.0)
            continue
        floor = 1.0 if f in (0, 3) else 1e-6 * H * np.sqrt(G * H)
        sc = max(np.abs(b[f][m]).max(), floor)
        out.append(np.abs(a[f][m] - b[f][m]).max() / sc)
    return np.array(out)


def test_full_batch_sampled_problems():
    from paper_1803_01450_amd.binding import Solver, BATCHED
    sizes = inputs.batch_sizes(512)
    nsteps, every, tau = 4, 10, 2e-5
    say("case: full batch, 512 problems, %d coarse steps (regrid at the first), batched" % nsteps)
    S = Solver()
    probs = []
    for k, n in enumerate(sizes):
        c = inputs.batch_problem(k, int(n))
        p = S.define(c["n"], c["n"], c["dx"], c["dx"], c["r"], (2,))
        S.set_bathymetry(p, np.kron(c["B"], np.ones((2, 2))))
        S.set_state(p, 0, c["q"])
        probs.append(c)
    dts = S.advance(nsteps, every, np.tile([tau, 0.0], (512, 1)), mode=BATCHED, want_dts=True)
    order = np.argsort(sizes, kind="stable")
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    for k in picks:
        c = probs[k]
        n = c["n"]
        say("problem", k, "size", n)
        H = oracle.Hierarchy(n, n, c["dx"], c["dx"], ratios=(2,), r=c["r"])
        H.set_bathymetry(np.kron(c["B"], np.ones((2, 2))))
        H.set_state(0, c["q"])
        rc, rdts = H.advance(nsteps, every, [tau])
        assert rc == 0
        assert np.abs(dts[k] - rdts).max() <= 1e-12 * rdts.max()
        for l in range(2):
            assert np.array_equal(S.patches(k, l), H.patches(l)), (k, l)
            err = rel_err(S.state(k, l), H.state(l))
            say("  level", l, "patches", len(S.patches(k, l)), "rel err", err.max())
            assert err.max() <= 1e-9
        assert S.counters(k)["updates"] == H.counters()["updates"]
    S.close()


def test_full_amr_shoreline():
    from paper_1803_01450_amd.binding import Solver, BATCHED
    c = inputs.amr_shoreline()
    nsteps, every, tau = 4, 4, [2e-6, 4e-6]
    say("case: full AMR shoreline, 256^2, ratios 2 and 4, %d coarse steps, batched" % nsteps)
    S = Solver()
    p = S.define(c["n0"], c["n0"], c["dx0"], c["dx0"], c["r"], c["ratios"])
    S.set_bathymetry(p, c["Bf"])
    S.set_patches(p, 0, c["level0_boxes"])
    S.set_state(p, 0, c["q0"])
    dts = S.advance(nsteps, every, [tau], mode=BATCHED, want_dts=True)
    H = oracle.Hierarchy(c["n0"], c["n0"], c["dx0"], c["dx0"], ratios=c["ratios"], r=c["r"])
    H.set_bathymetry(c["Bf"])
    H.set_patches(0, c["level0_boxes"])
    H.set_state(0, c["q0"])
    rc, rdts = H.advance(nsteps, every, tau)
    assert rc == 0
    assert np.abs(dts[0] - rdts).max() <= 1e-12 * rdts.max()
    for l in range(3):
        assert np.array_equal(S.patches(p, l), H.patches(l)), l
        err = rel_err(S.state(p, l), H.state(l))
        say("level", l, "patches", len(S.patches(p, l)), "rel err", err.max())
        assert err.max() <= 1e-9
    assert len(S.patches(p, 2)) > 50
    assert S.counters(p)["updates"] == H.counters()["updates"]
    S.close()


def test_amr_shoreline_at_stated_size():
    """The shoreline run at its stated size of about 1.5M finest cells: eight
    pulses (the same bathymetry and first pulse, seven more drawn after it), so
    that the first regrid at tau (2e-7, 4e-7), the benchmark's thresholds,
    already refines ~1.67M finest cells in ~870 patches; then four coarse
    steps (8 substeps of the finest level each), batched launches in the
    benchmark's configuration, every level against the oracle."""
    from paper_1803_01450_amd.binding import Solver, BATCHED
    c = inputs.amr_shoreline(pulses=8)
    nsteps, every, tau = 4, 4, [2e-7, 4e-7]
    say("case: AMR shoreline at stated size, 256^2 + 8 pulses, %d coarse steps, batched" % nsteps)
    S = Solver()
    p = S.define(c["n0"], c["n0"], c["dx0"], c["dx0"], c["r"], c["ratios"])
    S.set_bathymetry(p, c["Bf"])
    S.set_patches(p, 0, c["level0_boxes"])
    S.set_state(p, 0, c["q0"])
    dts = S.advance(nsteps, every, [tau], mode=BATCHED, want_dts=True)
    fine = sum(int(b[2]) * int(b[3]) for b in S.patches(p, 2))
    say("finest cells", fine, "patches", len(S.patches(p, 2)))
    assert fine >= 1_200_000
    H = oracle.Hierarchy(c["n0"], c["n0"], c["dx0"], c["dx0"], ratios=c["ratios"], r=c["r"])
    H.set_bathymetry(c["Bf"])
    H.set_patches(0, c["level0_boxes"])
    H.set_state(0, c["q0"])
    rc, rdts = H.advance(nsteps, every, tau)
    assert rc == 0
    assert np.abs(dts[0] - rdts).max() <= 1e-12 * rdts.max()
    for l in range(3):
        assert np.array_equal(S.patches(p, l), H.patches(l)), l
        err = rel_err(S.state(p, l), H.state(l))
        say("level", l, "patches", len(S.patches(p, l)), "rel err", err.max())
        assert err.max() <= 1e-9
    assert S.counters(p)["updates"] == H.counters()["updates"]
    S.close()
