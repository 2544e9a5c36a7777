"""The demonstration workload of the paper's Sec. 3 (plane wave from deep water
onto a discontinuous shelf, scaled units, invented parameters) at a small size:
three levels (ratios 2 and 4), regrid every 4 coarse steps, against the oracle
(patch layouts and update counts exact, dts within 1e-12, states within 1e-9),
and the uniform finest grid against the oracle."""
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


def rel_err(a, b, H=1.0):
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


@pytest.mark.parametrize("mode", [1, 2])
def test_shelf_amr_matches_oracle(mode):
    from paper_1803_01450_amd.binding import Solver
    c = inputs.shelf_wave(n0=32, width=0.05)
    say("case: shelf wave, level 0 %dx%d, ratios %s, 12 coarse steps, mode %d" % (c["n0x"], c["n0y"], c["ratios"], mode))
    S = Solver()
    p = S.define(c["n0x"], c["n0y"], c["dx0"], c["dx0"], c["r"], c["ratios"])
    S.set_bathymetry(p, c["Bf"])
    S.set_state(p, 0, c["q0"])
    dts = S.advance(12, 4, [c["tau"]], mode=mode, want_dts=True)
    H = oracle.Hierarchy(c["n0x"], c["n0y"], c["dx0"], c["dx0"], ratios=c["ratios"], r=c["r"])
    H.set_bathymetry(c["Bf"]); H.set_state(0, c["q0"])
    rc, rdts = H.advance(12, 4, c["tau"])
    assert rc == 0
    assert np.abs(dts[0] - rdts).max() <= 1e-12 * rdts.max()
    for l in range(3):
        pg, po = S.patches(p, l), H.patches(l)
        say("level", l, "patches", len(pg))
        assert np.array_equal(pg, po)
        err = rel_err(S.state(p, l), H.state(l))
        say("level", l, "rel err", err.max())
        assert err.max() <= 1e-9
    assert len(S.patches(p, 2)) > 0
    assert S.counters(p)["updates"] == H.counters()["updates"]
    S.close()


def test_shelf_uniform_matches_oracle():
    from paper_1803_01450_amd.binding import Solver
    c = inputs.shelf_wave(n0=16)
    say("case: shelf wave, uniform %dx%d, 40 steps" % (c["nfx"], c["nfy"]))
    S = Solver()
    p = S.define(c["nfx"], c["nfy"], c["dxf"], c["dxf"], c["r"])
    S.set_bathymetry(p, c["Bf"])
    S.set_state(p, 0, c["qf"])
    dts = S.advance(40, want_dts=True)
    H = oracle.Hierarchy(c["nfx"], c["nfy"], c["dxf"], c["dxf"], r=c["r"])
    H.set_bathymetry(c["Bf"]); H.set_state(0, c["qf"])
    rc, rdts = H.advance(40)
    assert rc == 0
    err = rel_err(S.state(p, 0), H.state(0))
    say("rel err", err.max())
    assert err.max() <= 1e-9
    assert np.abs(dts[0] - rdts).max() <= 1e-12 * rdts.max()
    S.close()
