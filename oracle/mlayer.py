"""Reference oracle for the general M-layer refine and coarsen -- TEST INFRASTRUCTURE.

Plain FP64 Python (one fine or coarse cell at a time, numpy arrays only as
containers), written from the paper's general multilayer formulation
(Schwarzschild & Mandli, arXiv 1803.01450):

* layer surfaces over the bathymetry and the layers below (Sec. 2.1, Eq. 4),
* the effective bathymetry of a layer, the bathymetry plus every layer below
  it (Sec. 2.1, Eq. 5),
* minmod-limited linear interpolation of each surface (Sec. 2.1, Eq. 10),
  bottom layer first, then upwards through the effective bathymetry (Sec. 2.1,
  last paragraph),
* a layer is wet only where every layer above it is (Sec. 2.1, first
  paragraph),
* coarsening as the mean of the children of every quantity (Sec. 2.2, Eq. 11,
  in two dimensions).

Layer 1 is the top layer.  Arrays are field-major: q[3(m-1) + k] for layer m
and k = 0 (depth h_m), 1 (h_m u_m), 2 (h_m v_m), rows with x fastest.  For
M = 2 these are the two-layer rules of the C oracle in this folder (the tests
hold the two against each other cell by cell).  The choices the paper leaves
open (fractions of the children, dry tolerance, treatment of dry coarse
layers and of the domain edge) are the two-layer ones.

It shares no code with the HIP library; only ``tests/`` may use it.
"""
from __future__ import annotations

import numpy as np

HDRY = 1.0e-3


def minmod(a, b):
    """Zero unless both arguments are strictly of one sign, else the one of
    smaller modulus (Sec. 2.1, Eq. 10 and the sentence after it)."""
    if a > 0.0 and b > 0.0:
        return a if a < b else b
    if a < 0.0 and b < 0.0:
        return a if a > b else b
    return 0.0


def surfaces(qc, Bc, I, J, M):
    """Surfaces eta_1..eta_M of coarse cell (I, J) (Eq. 4), summed from the
    bathymetry upwards: eta_M = B + h_M, eta_m = eta_{m+1} + h_m."""
    eta = [0.0] * (M + 1)
    s = float(Bc[J, I])
    for m in range(M, 0, -1):
        s = s + float(qc[3 * (m - 1), J, I])
        eta[m] = s
    return eta


def refine_cell(qc, Bc, r, i, j, Bf, hdry=HDRY):
    """All 3M values of fine cell (i, j) (fine index space, ratio r) and the
    number of wet-order repairs, from the coarse state qc [3M][nyc][nxc] and
    coarse bathymetry Bc [nyc][nxc]; Bf is the fine cell's bathymetry.

    Slopes are zero across the domain edge and for a layer dry in any of the
    three cells of a direction; a dry coarse layer gives a dry fine layer."""
    M = qc.shape[0] // 3
    nyc, nxc = Bc.shape
    I, J, a, b = i // r, j // r, i % r, j % r
    fa = (2 * a + 1 - r) / (2 * r)
    fb = (2 * b + 1 - r) / (2 * r)
    inx = I - 1 >= 0 and I + 1 < nxc
    iny = J - 1 >= 0 and J + 1 < nyc
    cells = {"c": (I, J)}
    if inx:
        cells["xl"], cells["xr"] = (I - 1, J), (I + 1, J)
    if iny:
        cells["yd"], cells["yu"] = (I, J - 1), (I, J + 1)
    eta = {k: surfaces(qc, Bc, ci, cj, M) for k, (ci, cj) in cells.items()}

    def wet(k, m):
        ci, cj = cells[k]
        return float(qc[3 * (m - 1), cj, ci]) >= hdry

    def val(k, f):
        ci, cj = cells[k]
        return float(qc[f, cj, ci])

    sxok = [False] * (M + 1)
    syok = [False] * (M + 1)
    etaf = [0.0] * (M + 1)
    for m in range(M, 0, -1):
        sxok[m] = inx and wet("xl", m) and wet("c", m) and wet("xr", m)
        syok[m] = iny and wet("yd", m) and wet("c", m) and wet("yu", m)
        e = eta["c"][m]
        sx = minmod(e - eta["xl"][m], eta["xr"][m] - e) if sxok[m] else 0.0
        sy = minmod(e - eta["yd"][m], eta["yu"][m] - e) if syok[m] else 0.0
        etaf[m] = (e + sx * fa) + sy * fb
    # depths from the bottom up through the effective bathymetry (Eq. 5)
    h = [0.0] * (M + 1)
    Bhat = float(Bf)
    for m in range(M, 0, -1):
        hm = etaf[m] - Bhat if wet("c", m) else 0.0
        if hm < hdry:
            hm = 0.0
        h[m] = hm
        Bhat = Bhat + hm
    # wet ordering: below a dry layer every layer is dry
    repairs = 0
    dry_above = False
    for m in range(1, M + 1):
        if dry_above and h[m] > 0.0:
            h[m] = 0.0
            repairs += 1
        if h[m] == 0.0:
            dry_above = True

    def mom(f, m):
        v = val("c", f)
        sx = minmod(v - val("xl", f), val("xr", f) - v) if sxok[m] else 0.0
        sy = minmod(v - val("yd", f), val("yu", f) - v) if syok[m] else 0.0
        return (v + sx * fa) + sy * fb

    out = np.zeros(3 * M)
    for m in range(1, M + 1):
        f = 3 * (m - 1)
        out[f] = h[m]
        out[f + 1] = mom(f + 1, m) if h[m] > 0.0 else 0.0
        out[f + 2] = mom(f + 2, m) if h[m] > 0.0 else 0.0
    return out, repairs


def refine(qc, Bc, Bf, r, box=None, hdry=HDRY):
    """Fine cells of box (fi0, fj0, fnx, fny) (default: the whole fine grid of
    r*nxc x r*nyc cells) refined from the coarse grid.  Bf is the box's fine
    bathymetry [fny][fnx].  Returns (qf [3M][fny][fnx], repairs)."""
    qc = np.asarray(qc, dtype=np.float64)
    Bc = np.asarray(Bc, dtype=np.float64)
    nyc, nxc = Bc.shape
    if box is None:
        box = (0, 0, r * nxc, r * nyc)
    fi0, fj0, fnx, fny = box
    M = qc.shape[0] // 3
    qf = np.zeros((3 * M, fny, fnx))
    rep = 0
    for jj in range(fny):
        for ii in range(fnx):
            v, n = refine_cell(qc, Bc, r, fi0 + ii, fj0 + jj, Bf[jj, ii], hdry)
            qf[:, jj, ii] = v
            rep += n
    return qf, rep


def fixup(v, hdry=HDRY):
    """Dry-state fix-up of one cell's 3M values (in place): thin layers to dry
    with zero momenta, then every layer below a dry one dry.  Returns the
    number of layers made dry by the wet ordering."""
    M = len(v) // 3
    for m in range(M, 0, -1):
        f = 3 * (m - 1)
        if v[f] < hdry:
            v[f] = v[f + 1] = v[f + 2] = 0.0
    rep = 0
    dry_above = False
    for m in range(1, M + 1):
        f = 3 * (m - 1)
        if dry_above and v[f] > 0.0:
            v[f] = v[f + 1] = v[f + 2] = 0.0
            rep += 1
        if v[f] == 0.0:
            dry_above = True
    return rep


def coarsen(qf, r, hdry=HDRY):
    """Coarse cells from their r x r children (Eq. 11 in two dimensions): the
    row-major sum of the children of every quantity times 1/r^2, then the
    fix-up.  qf: [3M][r*cny][r*cnx] -> [3M][cny][cnx]."""
    qf = np.asarray(qf, dtype=np.float64)
    nf, nyf, nxf = qf.shape
    cny, cnx = nyf // r, nxf // r
    inv = 1.0 / float(r * r)
    out = np.zeros((nf, cny, cnx))
    for J in range(cny):
        for I in range(cnx):
            v = [0.0] * nf
            for f in range(nf):
                s = 0.0
                for bb in range(r):
                    for aa in range(r):
                        s = s + float(qf[f, r * J + bb, r * I + aa])
                v[f] = s * inv
            fixup(v, hdry)
            out[:, J, I] = v
    return out
