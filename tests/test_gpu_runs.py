"""Run tiles: a batched substep sweeps the union of a level's patches in fixed
blocks (60 or 64 columns by a row chunk) instead of patch by patch.  Inside a
level every patch's frame cells that lie in a neighbouring patch hold that
patch's values, so the union gives the patch-by-patch results bit for bit; the
counts must follow the oracle's patch-by-patch rule as well: an edge counts once
for each patch holding one of its two cells (twice where two patches meet), a
fix-up once per interior cell.

The layout has patches side by side, stacked, staggered and one wider than a
60-column strip, and the internal-wave floor is raised to 1 so that the
hyperbolicity clamp fires at almost every edge with a velocity shear: the
clamp count then measures the edge multiplicities directly."""
import sys

import numpy as np
import pytest

import oracle
from paper_1803_01450_amd import inputs

pytestmark = pytest.mark.gpu

G = 9.81
# level-1 boxes (ilo, jlo, nx, ny) on the 128 x 128 fine grid
BOXES = [(16, 16, 32, 32), (48, 16, 16, 32), (24, 48, 72, 16), (96, 40, 20, 30), (116, 40, 10, 30)]
KMIN = 1.0
NSTEPS = 6


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


def gpu_run(mode, boxes=BOXES, **tun):
    from paper_1803_01450_amd.binding import Solver
    c = inputs.fixed_small()
    S = Solver(kmin=KMIN)
    if tun:
        S.set_tuning(**tun)
    p = S.define(64, 64, c["dx"], c["dx"], c["r"], (2,))
    S.set_bathymetry(p, c["Bf"])
    S.set_state(p, 0, c["q"])
    S.refine(p, 1, boxes)
    dts = S.advance(NSTEPS, 0, None, mode=mode, want_dts=True)
    out = dict(states=[S.state(p, l) for l in range(2)], counters=S.counters(p), dts=dts[0])
    S.close()
    return out


def same_states(a, b):
    for l in range(2):
        x, y = a[l], b[l]
        assert np.array_equal(np.isnan(x), np.isnan(y))
        m = ~np.isnan(x)
        assert np.array_equal(x[m], y[m]), l


def test_run_tiles_equal_patch_tiles_bitwise():
    say("case: run tiles (batched) vs patch tiles (plain), 5 fine patches, kmin 1")
    plain = gpu_run(0)
    batched = gpu_run(1)
    graph = gpu_run(2)
    same_states(plain["states"], batched["states"])
    same_states(plain["states"], graph["states"])
    assert np.array_equal(plain["dts"], batched["dts"])
    for k in ("hyp", "nclip", "repair", "updates"):
        say(k, plain["counters"][k], batched["counters"][k], graph["counters"][k])
        assert plain["counters"][k] == batched["counters"][k] == graph["counters"][k], k
    assert plain["counters"]["hyp"] > 0


@pytest.mark.parametrize("rows", [(0, 0), (4, 8), (8, 16), (32, 256)])
def test_run_tiles_match_oracle_counts(rows):
    """Against the oracle: patch layout and updates exact, clamp and fix-up
    counts exact, dts within 1e-12, states within 1e-9, over run tiles of
    several row chunk heights (blocks that cut patches at every height)."""
    xr, yr = rows
    say("case: run tiles vs oracle, rows", rows)
    g = gpu_run(1, x_rows=xr, y_rows=yr)
    c = inputs.fixed_small()
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(2,), r=c["r"], kmin=KMIN)
    H.set_bathymetry(c["Bf"]); H.set_state(0, c["q"])
    H.set_patches(1, BOXES)
    rc, rdts = H.advance(NSTEPS)
    assert rc == 0
    co, cg = H.counters(), g["counters"]
    say("hyp gpu", cg["hyp"], "oracle", co["hyp"], "nclip", cg["nclip"], co["nclip"])
    assert cg["hyp"] == co["hyp"] > 0
    assert cg["nclip"] == co["nclip"] and cg["repair"] == co["repair"]
    assert cg["updates"] == co["updates"]
    assert np.abs(g["dts"] - rdts).max() <= 1e-12 * rdts.max()
    for l in range(2):
        err = rel_err(g["states"][l], H.state(l))
        say("level", l, "rel err", err.max())
        assert err.max() <= 1e-9


def test_single_patch_levels_keep_patch_tiles():
    """One patch per level: the union is the patch, and the patch tiles serve
    (same results as the plain launches)."""
    say("case: one fine patch, batched vs plain")
    box = [(24, 24, 64, 40)]
    a, b = gpu_run(0, boxes=box), gpu_run(1, boxes=box)
    same_states(a["states"], b["states"])
    assert a["counters"]["hyp"] == b["counters"]["hyp"]


def test_odd_first_columns_through_registers():
    """Level-0 patches with an odd first column: their patch tiles (plain
    launches) take the rows through registers, the union tiles (batched) through
    LDS copies; both match each other bit for bit and the oracle."""
    from paper_1803_01450_amd.binding import Solver
    say("case: level-0 patches at columns 0 and 33, plain vs batched vs oracle")
    c = inputs.fixed_small()
    boxes = [(0, 0, 33, 40), (33, 0, 31, 40), (0, 40, 17, 24), (17, 40, 47, 24)]
    out = []
    for mode in (0, 1):
        S = Solver()
        p = S.define(64, 64, c["dx"], c["dx"], c["r"])
        S.set_bathymetry(p, c["B"])
        S.set_patches(p, 0, boxes)
        S.set_state(p, 0, c["q"])
        dts = S.advance(20, want_dts=True, mode=mode)
        out.append((S.state(p, 0), S.counters(p), dts[0]))
        S.close()
    (a, ca, da), (b, cb, db) = out
    assert np.array_equal(a, b) and np.array_equal(da, db)
    assert ca["nclip"] == cb["nclip"] and ca["hyp"] == cb["hyp"]
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], r=c["r"])
    H.set_bathymetry(c["B"])
    H.set_patches(0, boxes)
    H.set_state(0, c["q"])
    rc, rdts = H.advance(20)
    assert rc == 0
    err = rel_err(a, H.state(0))
    say("rel err", err.max(), "dt diff", np.abs(da - rdts).max())
    assert err.max() <= 1e-9
    assert np.abs(da - rdts).max() <= 1e-12 * rdts.max()
    assert ca["hyp"] == H.counters()["hyp"] and ca["nclip"] == H.counters()["nclip"]
