"""The mass flux correction at coarse-fine edges (config reflux = 1) on the GPU
against the oracle with the same correction: two and three levels, all cells
wet, regrids every 4 coarse steps, in every launch mode: patch layouts and
dts equal, every level's state equal bit for bit, and each layer's mass on the
composite grid conserved to rounding (without the correction it drifts by
about 1e-8 per coarse step)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1803_01450_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def composite_mass(states, ratios, dx0):
    out = np.zeros(2)
    dx = dx0
    for l, q in enumerate(states):
        cov = ~np.isnan(q[0])
        if l + 1 < len(states):
            r = ratios[l]
            fine = ~np.isnan(states[l + 1][0])
            cov &= ~fine.reshape(fine.shape[0] // r, r, fine.shape[1] // r, r).any(axis=(1, 3))
        out += [np.where(cov, q[0], 0.0).sum() * dx * dx, np.where(cov, q[3], 0.0).sum() * dx * dx]
        if l + 1 < len(states):
            dx /= ratios[l]
    return out


CASES = [((2,), [2e-6]), ((2, 4), [2e-6, 4e-6])]
_ORACLE = {}


def oracle_run(ratios, tau, c, Bf, nsteps):
    key = ratios
    if key not in _ORACLE:
        H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=ratios, r=c["r"])
        H.set_reflux(True)
        H.set_bathymetry(Bf); H.set_state(0, c["q"])
        rc, d = H.advance(nsteps, 4, tau)
        assert rc == 0
        nl = len(ratios) + 1
        _ORACLE[key] = (d, [H.patches(l) for l in range(nl)], [H.state(l) for l in range(nl)])
    return _ORACLE[key]


@pytest.mark.parametrize("case", [0, 1])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_reflux_matches_oracle_and_conserves(case, mode):
    from paper_1803_01450_amd.binding import Solver
    ratios, tau = CASES[case]
    nl, nf = len(ratios) + 1, 64 * int(np.prod(ratios))
    say("case: flux correction, ratios %s, mode %d" % (ratios, mode))
    c = inputs.fixed_small()
    Bf = np.kron(c["B"], np.ones((nf // 64, nf // 64)))
    S = Solver(reflux=True)
    p = S.define(64, 64, c["dx"], c["dx"], c["r"], ratios)
    S.set_bathymetry(p, Bf); S.set_state(p, 0, c["q"])
    m0 = composite_mass([S.state(p, 0)], ratios, c["dx"])
    nsteps = 9
    d = S.advance(nsteps, 4, [tau], mode=mode, want_dts=True)[0]
    rd, rp, rs = oracle_run(ratios, tau, c, Bf, nsteps)
    assert np.array_equal(d, rd)
    states = [S.state(p, l) for l in range(nl)]
    for l in range(nl):
        assert np.array_equal(S.patches(p, l), rp[l]), l
        same = np.array_equal(states[l], rs[l], equal_nan=True)
        if not same:
            m = ~np.isnan(rs[l])
            say("level", l, "max abs diff", np.abs(states[l][m] - rs[l][m]).max())
        assert same, l
    assert S.counters(p)["nclip"] == 0 and len(S.patches(p, nl - 1)) > 0
    drift = np.abs(composite_mass(states, ratios, c["dx"]) - m0) / m0
    say("drift", drift)
    assert np.all(drift <= 1e-14)
    S.close()


def test_reflux_flag_validated():
    from paper_1803_01450_amd import binding
    cfg = binding.Config(9.81, 1e-3, 1e-6, 0.9, 1.0, 0, 0, 0, 0, 2)
    import ctypes
    h = ctypes.c_void_p()
    assert binding.lib().mlswe_create(ctypes.byref(cfg), None, ctypes.byref(h)) == binding.EINVAL
