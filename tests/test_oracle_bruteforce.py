"""Brute-force pin of the oracle's fixed-grid step: the same method restated
from its definitions in 50-digit arithmetic (tests/mp_twolayer.py: coupled
4x4 solve by LU, single-layer edges over the effective bottom, MC-limited
corrections from the upwind neighbour edge, x then y sweeps with walls)
agrees with the FP64 oracle to rounding on small grids over three steps.

The grids are chosen so that every part of the step contributes: rough data
(limiter ratios well spread over negative values, (0, 1/3), [1/3, 3] and
above), waves in both directions, a lower layer that is dry over part of the
domain (single-layer edges, walls of the lower layer), and a shore where the
top layer meets land (walls and overtopping, clipping).  A slip in the oracle
(a dropped term, a wrong sign, the downwind edge in the limiter, another
limiter) moves some field by far more than rounding.

Surfaces, effective bottom and wet ordering: Sec. 2.1, Eqs. 4-9 of the paper.
The solver the paper cites (Sec. 1) is restated in the module's docstring."""
import numpy as np
import pytest

import oracle
import mp_twolayer as M

TOL = 1e-13


def grid(kind, nx, ny, seed):
    """Seeded small grid: bathymetry, state [6][ny][nx], dx."""
    rng = np.random.default_rng(seed)
    dx = 1000.0
    X = np.broadcast_to((np.arange(nx) + 0.5)[None, :] / nx, (ny, nx))
    if kind == "wet":
        B = -2000.0 + 300.0 * rng.uniform(-1, 1, (ny, nx))
        eta2 = -300.0 + 20.0 * rng.uniform(-1, 1, (ny, nx))
        eta1 = 0.5 * rng.uniform(-1, 1, (ny, nx))
    elif kind == "lower_dry":
        B = -600.0 + 500.0 * X + 40.0 * rng.uniform(-1, 1, (ny, nx))
        eta2 = -250.0 + 5.0 * rng.uniform(-1, 1, (ny, nx))
        eta1 = 0.5 * rng.uniform(-1, 1, (ny, nx))
    else:  # shore: land towards +x
        B = -300.0 + 340.0 * X + 10.0 * rng.uniform(-1, 1, (ny, nx))
        eta2 = -120.0 + 3.0 * rng.uniform(-1, 1, (ny, nx))
        eta1 = 0.8 * rng.uniform(-1, 1, (ny, nx))
    h2 = np.maximum(eta2 - B, 0.0)
    h2[h2 < oracle.HDRY] = 0.0
    h1 = np.maximum(eta1 - np.maximum(eta2, B), 0.0)
    h1[h1 < oracle.HDRY] = 0.0
    h2[h1 == 0.0] = 0.0
    q = np.zeros((6, ny, nx))
    q[0], q[3] = h1, h2
    for f, h in ((1, h1), (2, h1), (4, h2), (5, h2)):
        q[f] = h * rng.uniform(-0.5, 0.5, (ny, nx))
    return B, q, dx


CASES = [("wet", 6, 5, 1), ("lower_dry", 7, 6, 2), ("shore", 8, 6, 3)]


def compare(kind, nx, ny, seed, r=0.95):
    """(per-field relative error, speed error, oracle counters, brute-force
    counts) of three steps: relative to max(max |field|, floor) with floor 1 m
    for depths and 1e-6 H sqrt(g H) for momenta."""
    B, q, dx = grid(kind, nx, ny, seed)
    H = float((q[0] + q[3]).max())
    dt = 0.5 * dx / (np.sqrt(oracle.G * H) + 2.0)
    dts = [dt, 0.9 * dt, 1.1 * dt]
    qo, so, co = oracle.fixed_steps(B, q, dx, dx, dts, r=r)
    qm, sm, st = M.run(B.tolist(), q.tolist(), dx, dx, dts, r)
    qm = np.array(qm)
    err = []
    for f in range(6):
        floor = 1.0 if f in (0, 3) else 1e-6 * H * np.sqrt(oracle.G * H)
        err.append(np.abs(qo[f] - qm[f]).max() / max(np.abs(qm[f]).max(), floor))
    serr = np.abs(np.array(sm) - so).max() / np.abs(np.array(sm)).max()
    return np.array(err), serr, co, st


@pytest.mark.parametrize("kind,nx,ny,seed", CASES)
def test_oracle_matches_50_digit_step(kind, nx, ny, seed):
    err, serr, co, st = compare(kind, nx, ny, seed)
    assert np.all(err <= TOL), (kind, err)
    assert serr <= TOL, (kind, serr)
    assert int(co[1]) == st["nclip"] and int(co[2]) == st["repair"]


def test_cases_reach_every_branch():
    """The inputs exercise what they are meant to: limiter ratios in each MC
    regime, a lower layer dry in part, dry land, and clipping on the shore."""
    B, q, dx = grid("wet", 6, 5, 1)
    with M.mp.workdps(M.DPS):
        ths = []
        for j in range(5):
            line = [[M.mp.mpf(float(q[c][j][i])) for c in range(6)] for i in range(6)]
            Bl = [M.mp.mpf(float(B[j][i])) for i in range(6)]
            cells = [M.Cell(v, b) for v, b in zip(line, Bl)]
            E = [M.edge(cells[k], cells[k + 1], 0.95) for k in range(len(cells) - 1)]
            for k in range(1, len(E) - 1):
                for p in range(4):
                    zz = M._dot(E[k].Z[p], E[k].Z[p])
                    up = E[k - 1] if E[k].s[p] > 0 else E[k + 1]
                    ths.append(float(M._dot(up.Z[p], E[k].Z[p]) / zz))
    ths = np.array(ths)
    assert (ths < 0).any() and ((ths > 0) & (ths < 1 / 3)).any()
    assert ((ths > 1 / 3) & (ths < 3)).any() and (ths > 3).any()
    _, q2, _ = grid("lower_dry", 7, 6, 2)
    assert (q2[3] == 0).any() and (q2[3] > 0).any() and (q2[0] > 0).all()
    _, q3, _ = grid("shore", 8, 6, 3)
    assert (q3[0] == 0).any()
    _, _, co, _ = compare("shore", 8, 6, 3)
    assert co[1] > 0
