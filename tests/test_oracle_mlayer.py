"""Pins of the M-layer refine and coarsen oracle (Sec. 2.1, Eqs. 4-5 and 10;
Sec. 2.2, Eq. 11):

* M = 2 equals the two-layer C oracle cell by cell (stencils with dry layers,
  domain edges, every child of ratios 2 and 4), and its coarsening equals the
  C oracle's level coarsening;
* M = 1 is the single-layer rule: a linear surface is reproduced at the fine
  cell centres;
* a lake at rest with three layers stays at rest with flat surfaces over any
  fine bathymetry below the bottom surface;
* each layer's mass and momenta are conserved by refining where all layers
  are wet (the children's mean equals the coarse value), so coarsening a
  refinement gives the coarse state back;
* refined surfaces create no new extrema over the five-point stencil;
* the wet ordering: a thin top layer is dried and every layer below it too,
  counted as repairs.

Each pin fails for a plausible slip in the oracle: a surface summed over the
wrong layers, the fine bathymetry in place of the effective one, a flipped
child fraction, a minmod that keeps opposite signs, a wet test on the wrong
layer, a missing 1/r^2."""
import numpy as np
import pytest

import oracle
from oracle import mlayer

HD = oracle.HDRY


def rand_state(rng, M, nx, ny, wet=True):
    """Coarse state [3M][ny][nx] and bathymetry from random smooth surfaces:
    bottom at about -1000 m, interfaces at -100 m steps, momenta random."""
    x = np.linspace(0, 1, nx)[None, :]
    y = np.linspace(0, 1, ny)[:, None]
    B = -1000.0 + 50.0 * np.sin(3 * x + 2 * y) + rng.uniform(-5, 5, (ny, nx))
    q = np.zeros((3 * M, ny, nx))
    below = B.copy()
    for m in range(M, 0, -1):
        top = -100.0 * (m - 1) + 3.0 * np.cos(4 * x - 3 * y + m) + rng.uniform(-0.5, 0.5, (ny, nx))
        h = top - below
        if not wet:
            h = np.where(rng.uniform(size=h.shape) < 0.15, rng.choice([0.0, 0.5 * HD, 2 * HD], h.shape), h)
        q[3 * (m - 1)] = h
        q[3 * (m - 1) + 1] = rng.uniform(-50, 50, (ny, nx))
        q[3 * (m - 1) + 2] = rng.uniform(-50, 50, (ny, nx))
        below = below + h
    return q, B


def fine_bathymetry(rng, Bc, r, amp=20.0):
    """Fine bathymetry whose r x r block means are the coarse values up to
    rounding (zero-mean offsets inside each block)."""
    nyc, nxc = Bc.shape
    d = rng.uniform(-amp, amp, (nyc, r, nxc, r))
    d -= d.mean(axis=(1, 3), keepdims=True)
    return (Bc[:, None, :, None] + d).reshape(nyc * r, nxc * r)


@pytest.mark.parametrize("seed", range(4))
def test_two_layers_equal_c_oracle(seed):
    rng = np.random.default_rng(seed)
    for r in (2, 4):
        for trial in range(12):
            nx = 3 if trial % 3 else 1
            ny = 3 if trial % 4 else 1
            q, B = rand_state(rng, 2, 3, 3, wet=(trial % 2 == 0))
            if trial % 5 == 1:  # top layer dry in one neighbour, bottom wet
                q[0, 1, 0] = 0.0
            q, B = q[:, :ny, :nx], B[:ny, :nx]
            I, J = nx // 2, ny // 2
            for a in range(r):
                for b in range(r):
                    Bf = float(B[J, I]) + float(rng.uniform(-30, 30))
                    got, rep = mlayer.refine_cell(q, B, r, r * I + a, r * J + b, Bf)
                    q5 = np.zeros((5, 7))
                    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
                    for k, (di, dj) in enumerate(offs):
                        i, j = I + di, J + dj
                        if 0 <= i < nx and 0 <= j < ny:
                            q5[k, :6] = q[:, j, i]
                            q5[k, 6] = B[j, i]
                    ref, rrep = oracle.refine_point(q5, r, a, b, Bf, inx=nx == 3, iny=ny == 3)
                    assert np.array_equal(got, ref), (r, trial, a, b, got, ref)
                    assert rep == rrep


def test_two_layer_coarsen_equals_c_oracle():
    rng = np.random.default_rng(5)
    for r in (2, 4):
        nxc, nyc = 6, 5
        H = oracle.Hierarchy(nxc, nyc, 100.0, 100.0, ratios=(r,))
        Bc = rng.uniform(-1000, -900, (nyc, nxc))
        H.set_bathymetry(fine_bathymetry(rng, Bc, r))
        qf, _ = rand_state(rng, 2, nxc * r, nyc * r, wet=False)
        H.set_patches(1, [(0, 0, nxc * r, nyc * r)])
        H.set_state(1, qf)
        H.coarsen(1)
        assert np.array_equal(mlayer.coarsen(qf, r), H.state(0))


def test_one_layer_linear_surface_reproduced():
    """eta = 0.5 + 0.25 I - 0.125 J (coarse index units, exact in binary) over
    a 3x3 stencil: every child gets eta at its own centre, I + fa, J + fb."""
    for r in (2, 4):
        B = np.full((3, 3), -64.0)
        eta = np.array([[0.5 + 0.25 * I - 0.125 * J for I in range(3)] for J in range(3)])
        q = np.zeros((3, 3, 3))
        q[0] = eta - B
        for a in range(r):
            for b in range(r):
                out, _ = mlayer.refine_cell(q, B, r, r + a, r + b, -60.0)
                fa, fb = (2 * a + 1 - r) / (2 * r), (2 * b + 1 - r) / (2 * r)
                assert out[0] + -60.0 == 0.5 + 0.25 * (1 + fa) - 0.125 * (1 + fb)


def test_lake_at_rest_three_layers():
    """Flat surfaces at 0, -64, -256 over a bathymetry below -300: every fine
    surface is flat and the momenta stay zero, whatever the fine bathymetry
    (a rule that subtracted the fine bathymetry from every layer's surface
    would put the bathymetry's roughness into the upper interfaces)."""
    rng = np.random.default_rng(3)
    r = 4
    Bc = -512.0 + np.round(rng.uniform(-100, 100, (4, 5)))
    Bf = fine_bathymetry(rng, Bc, r, amp=16.0)
    Bf = np.round(Bf * 8) / 8
    levels = [0.0, -64.0, -256.0]
    q = np.zeros((9, 4, 5))
    q[6] = levels[2] - Bc
    q[3] = levels[1] - levels[2]
    q[0] = levels[0] - levels[1]
    qf, rep = mlayer.refine(q, Bc, Bf, r)
    assert rep == 0
    eta3 = Bf + qf[6]
    eta2 = eta3 + qf[3]
    eta1 = eta2 + qf[0]
    assert np.all(eta3 == levels[2]) and np.all(eta2 == levels[1]) and np.all(eta1 == levels[0])
    assert not qf[[1, 2, 4, 5, 7, 8]].any()


@pytest.mark.parametrize("M", [1, 3, 4])
def test_mass_and_momentum_conserved(M):
    """All layers wet: the mean over each coarse cell's children of every depth
    and momentum equals the coarse value (to rounding), so coarsening the
    refinement returns the coarse state."""
    rng = np.random.default_rng(10 + M)
    for r in (2, 4):
        q, Bc = rand_state(rng, M, 7, 6)
        Bf = fine_bathymetry(rng, Bc, r)
        qf, rep = mlayer.refine(q, Bc, Bf, r)
        assert rep == 0 and np.all(qf[0::3] > 0)
        back = mlayer.coarsen(qf, r)
        for f in range(3 * M):
            sc = np.abs(q[f]).max()
            assert np.abs(back[f] - q[f]).max() <= 1e-13 * sc, (r, f)


def test_no_new_extrema():
    """Each refined surface lies within the extremes of its coarse surface over
    the five-point stencil (minmod slopes; children fractions below 1/2)."""
    rng = np.random.default_rng(21)
    M, r = 3, 4
    q, Bc = rand_state(rng, M, 6, 6)
    for m in range(1, M + 1):  # rough surfaces: many slope sign changes
        q[3 * (m - 1)] += rng.uniform(0, 2.0, q[0].shape)
    Bf = fine_bathymetry(rng, Bc, r)
    qf, _ = mlayer.refine(q, Bc, Bf, r)
    etac = np.zeros((M + 1, 6, 6))
    etaf = np.zeros((M + 1, 24, 24))
    etac[M], etaf[M] = Bc + q[3 * (M - 1)], Bf + qf[3 * (M - 1)]
    for m in range(M - 1, 0, -1):
        etac[m] = etac[m + 1] + q[3 * (m - 1)]
        etaf[m] = etaf[m + 1] + qf[3 * (m - 1)]
    for m in range(1, M + 1):
        for j in range(24):
            for i in range(24):
                I, J = i // r, j // r
                nb = [etac[m, J, I]] + [etac[m, J + dj, I + di] for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1))
                                        if 0 <= I + di < 6 and 0 <= J + dj < 6]
                tol = 1e-12 * 1000
                assert min(nb) - tol <= etaf[m, j, i] <= max(nb) + tol, (m, i, j)


def test_wet_ordering_and_repairs():
    """Three layers along x (one row): the top surface falls by 3 hdry per
    cell over a centre cell whose top layer is 1.5 hdry deep, towards a shore
    cell where only the top layer is wet.  The centre's right-hand children get
    a top layer of 0.75 hdry: it is dried and the two wet layers below it are
    dried too (two repairs per child); the left-hand children stay wet, and
    the dry lower layers of the shore cell stay dry."""
    M, r = 3, 2
    hd = HD
    B = np.array([[-300.0, -300.0, -100.0 - 3.5 * hd]])
    q = np.zeros((9, 1, 3))
    q[6, 0, :2] = 100.0
    q[3, 0, :2] = 100.0
    q[0, 0] = [4.5 * hd, 1.5 * hd, 2.0 * hd]
    q[1, 0] = [1.0, 2.0, 3.0]
    Bf = np.repeat(np.repeat(B, 2, axis=0), 2, axis=1)
    qf, rep = mlayer.refine(q, B, Bf, r)
    wet = qf[0::3] > 0
    for m in range(1, M):
        assert np.all(wet[m] <= wet[m - 1]), "a wet layer under a dry one"
    assert rep == 4
    assert not wet[:, :, 3].any()          # centre, right-hand children: all dry
    assert wet[:, :, 2].all()              # centre, left-hand children: all wet
    assert np.all(qf[0, :, 2] > 2.0 * hd)  # the top layer there thickened
    assert wet[0, :, 4:].all() and not wet[1:, :, 4:].any()
    assert np.all(qf[1][~wet[0]] == 0.0)


def test_fixup_rules():
    v = [0.5 * HD, 3.0, 4.0, 10.0, 1.0, 2.0, 5.0, 1.0, 1.0]
    rep = mlayer.fixup(v)
    assert v == [0.0] * 9 and rep == 2
    v = [2.0, 1.0, 1.0, 0.5 * HD, 9.0, 9.0, 3.0, 1.0, 1.0]
    rep = mlayer.fixup(v)
    assert v == [2.0, 1.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0] and rep == 1
