"""Dynamic time-refinement ratios (config dynamic_rt) on the GPU against the
oracle's choice: a ratio-4 fine patch over shallow water takes 3 substeps per
coarse step once speeds are known, with and without the flux correction, in
every launch mode: ratios, dts, states (bit for bit) and update counts equal
the oracle's; a three-level shoreline run with regrids matches as well; and in
a context of several problems (one level ratio for all, the largest any
problem needs) batched and plain launches agree bit for bit."""
import sys

import numpy as np
import pytest

import oracle
from paper_1803_01450_amd import inputs

pytestmark = pytest.mark.gpu

BOX = (208, 32, 32, 64)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_run(reflux, steps=4):
    c = inputs.fixed_small()
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(4,), r=c["r"])
    H.set_dynamic_rt(True); H.set_reflux(reflux)
    H.set_bathymetry(np.kron(c["B"], np.ones((4, 4)))); H.set_state(0, c["q"])
    H.set_patches(1, [BOX])
    rts, dts = [], []
    for _ in range(steps):
        rc, d = H.advance(1)
        assert rc == 0
        rts.append(int(H.time_ratios()[0])); dts.append(d[0])
    return rts, np.array(dts), [H.state(l) for l in range(2)], H.counters()


@pytest.mark.parametrize("reflux", [False, True])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_shallow_patch_matches_oracle(mode, reflux):
    from paper_1803_01450_amd.binding import Solver
    say("case: dynamic time ratio, shallow ratio-4 patch, mode %d, reflux %s" % (mode, reflux))
    c = inputs.fixed_small()
    S = Solver(dynamic_rt=True, reflux=reflux)
    p = S.define(64, 64, c["dx"], c["dx"], c["r"], (4,))
    S.set_bathymetry(p, np.kron(c["B"], np.ones((4, 4)))); S.set_state(p, 0, c["q"])
    S.refine(p, 1, [BOX])
    rts, dts = [], []
    for _ in range(4):
        dts.append(S.advance(1, mode=mode, want_dts=True)[0][0])
        rts.append(int(S.time_ratios(p)[0]))
    ro, do, so, co = oracle_run(reflux)
    say("ratios", rts, ro)
    assert rts == ro == [4, 3, 3, 3]
    assert np.array_equal(np.array(dts), do)
    for l in range(2):
        assert np.array_equal(S.state(p, l), so[l], equal_nan=True), l
    assert S.counters(p)["updates"] == co["updates"]
    S.close()


def test_shoreline_three_levels_matches_oracle():
    from paper_1803_01450_amd.binding import Solver, BATCHED
    say("case: dynamic time ratio, 3-level shoreline 64^2, batched")
    c = inputs.amr_shoreline(n0=64, L=100e3, ratios=(2, 4))
    tau = [4e-6, 8e-6]
    S = Solver(dynamic_rt=True)
    p = S.define(c["n0"], c["n0"], c["dx0"], c["dx0"], c["r"], c["ratios"])
    S.set_bathymetry(p, c["Bf"]); S.set_state(p, 0, c["q0"])
    d = S.advance(8, 4, [tau], mode=BATCHED, want_dts=True)[0]
    H = oracle.Hierarchy(c["n0"], c["n0"], c["dx0"], c["dx0"], ratios=c["ratios"], r=c["r"])
    H.set_dynamic_rt(True)
    H.set_bathymetry(c["Bf"]); H.set_state(0, c["q0"])
    rc, rd = H.advance(8, 4, tau)
    assert rc == 0
    assert np.array_equal(d, rd)
    assert np.array_equal(S.time_ratios(p), H.time_ratios())
    for l in range(3):
        assert np.array_equal(S.patches(p, l), H.patches(l)), l
        assert np.array_equal(S.state(p, l), H.state(l), equal_nan=True), l
    S.close()


def test_several_problems_batched_equals_plain():
    from paper_1803_01450_amd.binding import Solver
    say("case: dynamic time ratio, 3 problems, batched vs plain")
    c = inputs.fixed_small()
    out = []
    for mode in (0, 1):
        S = Solver(dynamic_rt=True)
        ps = []
        for k, box in enumerate([BOX, (16, 32, 32, 64), (120, 120, 48, 32)]):
            p = S.define(64, 64, c["dx"], c["dx"], c["r"], (4,))
            S.set_bathymetry(p, np.kron(c["B"], np.ones((4, 4)))); S.set_state(p, 0, c["q"])
            S.refine(p, 1, [box])
            ps.append(p)
        S.advance(4, mode=mode)
        out.append(([S.state(p, l) for p in ps for l in range(2)], [list(S.time_ratios(p)) for p in ps]))
        S.close()
    (a, ra), (b, rb) = out
    assert ra == rb
    assert all(np.array_equal(x, y, equal_nan=True) for x, y in zip(a, b))


@pytest.mark.parametrize("mode", [1, 2])
def test_rejection_with_flux_correction_and_dynamic_ratio(mode):
    """The batch problem whose wet/dry front forces a coarse-step retake, with
    the flux correction and dynamic time ratios on: the retake keeps the
    step's time ratios and recomputes the face fluxes; dts, rejections, ratios
    and states equal the oracle's."""
    from paper_1803_01450_amd.binding import Solver
    say("case: rejection + flux correction + dynamic ratio, batch problem 301, mode %d" % mode)
    c = inputs.batch_problem(301, 152)
    n = 152
    Bf = np.kron(c["B"], np.ones((2, 2)))
    S = Solver(reflux=True, dynamic_rt=True)
    p = S.define(n, n, c["dx"], c["dx"], c["r"], (2,))
    S.set_bathymetry(p, Bf); S.set_state(p, 0, c["q"])
    S.advance(2, 10, [[2e-5, 0.0]], mode=mode)
    dts = S.advance(20, 10, [[2e-5, 0.0]], mode=mode, want_dts=True)[0]
    H = oracle.Hierarchy(n, n, c["dx"], c["dx"], ratios=(2,), r=c["r"])
    H.set_reflux(True); H.set_dynamic_rt(True)
    H.set_bathymetry(Bf); H.set_state(0, c["q"])
    H.advance(2, 10, [2e-5])
    rc, rdts = H.advance(20, 10, [2e-5])
    assert rc == 0
    cg, co = S.counters(p), H.counters()
    say("rejected", cg["rejected"], co["rejected"], "ratios", S.time_ratios(p), H.time_ratios())
    assert cg["rejected"] == co["rejected"] >= 1
    assert np.array_equal(dts, rdts)
    assert np.array_equal(S.time_ratios(p), H.time_ratios())
    for l in range(2):
        assert np.array_equal(S.state(p, l), H.state(l), equal_nan=True), l
    assert cg["nclip"] == co["nclip"] and cg["repair"] == co["repair"] and cg["updates"] == co["updates"]
    S.close()


def test_batch_of_problems_with_both_options_all_modes_agree():
    """64 uneven two-level problems with regrids, the flux correction and
    dynamic time ratios on: plain, batched and graph launches give the same
    states, layouts and ratios bit for bit (union tiles, patch tiles and graph
    replays all carry the correction the same way)."""
    from paper_1803_01450_amd.binding import Solver
    say("case: 64 batch problems, flux correction + dynamic ratio, plain/batched/graph")
    sizes = inputs.batch_sizes(512)[:64]
    tau = np.tile([2e-5, 0.0], (64, 1))
    out = []
    for mode in (0, 1, 2):
        S = Solver(reflux=True, dynamic_rt=True)
        ps = []
        for k, nn in enumerate(sizes):
            cc = inputs.batch_problem(k, int(nn))
            p = S.define(cc["n"], cc["n"], cc["dx"], cc["dx"], cc["r"], (2,))
            S.set_bathymetry(p, np.kron(cc["B"], np.ones((2, 2))))
            S.set_state(p, 0, cc["q"])
            ps.append(p)
        d = S.advance(6, 3, tau, mode=mode, want_dts=True)
        out.append((d, [(S.state(p, 1), S.state(p, 0), S.patches(p, 1)) for p in ps],
                    [list(S.time_ratios(p)) for p in ps]))
        S.close()
    for m in (1, 2):
        assert np.array_equal(out[0][0], out[m][0])
        assert out[0][2] == out[m][2]
        for a, b in zip(out[0][1], out[m][1]):
            assert np.array_equal(a[0], b[0], equal_nan=True) and np.array_equal(a[1], b[1], equal_nan=True)
            assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_newly_populated_level_takes_the_space_ratio(mode):
    """A fine level that gets its first patches after two coarse steps (deep
    water: one substep per coarse step would give a fine Courant number near
    3.6) keeps the space ratio on its first step, with no retake allowed: no
    rejection, no error, ratios, dts and states equal to the oracle's."""
    from paper_1803_01450_amd.binding import Solver
    say("case: dynamic time ratio, level populated mid-run, mode %d" % mode)
    c = inputs.fixed_small()
    box = (16, 64, 32, 64)
    S = Solver(dynamic_rt=True, max_retries=-1)
    p = S.define(64, 64, c["dx"], c["dx"], c["r"], (4,))
    S.set_bathymetry(p, np.kron(c["B"], np.ones((4, 4)))); S.set_state(p, 0, c["q"])
    S.set_patches(p, 1, [])
    S.advance(2, mode=mode)
    S.refine(p, 1, [box])
    rts, dts = [], []
    for _ in range(3):
        dts.append(S.advance(1, mode=mode, want_dts=True)[0][0])
        rts.append(int(S.time_ratios(p)[0]))
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(4,), r=c["r"])
    H.set_dynamic_rt(True); H.set_retries(0)
    H.set_bathymetry(np.kron(c["B"], np.ones((4, 4)))); H.set_state(0, c["q"])
    H.set_patches(1, [])
    assert H.advance(2)[0] == 0
    H.set_patches(1, [box])
    ro, do = [], []
    for _ in range(3):
        rc, d = H.advance(1)
        assert rc == 0
        ro.append(int(H.time_ratios()[0])); do.append(d[0])
    say("ratios", rts, ro)
    assert rts == ro and rts[0] == 4
    assert np.array_equal(np.array(dts), np.array(do))
    assert S.counters(p)["rejected"] == 0
    for l in range(2):
        assert np.array_equal(S.state(p, l), H.state(l), equal_nan=True), l
