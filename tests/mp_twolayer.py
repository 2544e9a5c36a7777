"""Brute-force two-layer step in 50-digit arithmetic -- TEST INFRASTRUCTURE.

A second, independent statement of the fixed-grid step the oracle computes,
written from the method's definitions rather than from the oracle's code, and
evaluated with mpmath at 50 significant digits.  It pins the FP64 oracle: on
small grids the two must agree to rounding (about 1e-13 relative), so a dropped
term, a wrong sign, a swapped neighbour or a different limiter in the oracle
shows up as an O(1) relative difference in some field.

Where the paper is explicit it is followed directly: surfaces eta2 = B + h2 and
eta1 = eta2 + h1 and the effective bottom B + h2 of the upper layer (Sec. 2.1,
Eqs. 4-9), a layer wet only where the layers above it are (Sec. 2.1).  The
solver itself is one the paper cites but does not write (Sec. 1); this module
restates the readings used for it:

* edge solve with both layers wet on both sides: f-wave split of the jump in
  (flux - integrated source) into four coupled waves with eigenvectors
  (1, s, alpha, alpha s), alpha = ((s - u1)^2 - g h1) / (g h1), at Roe averages,
  speeds to first order in (1 - r): U -+ sqrt(g H) and Uc -+ sqrt(g' h1 h2 / H *
  kappa); the 4x4 system is solved by mpmath's LU solver (not by the oracle's
  hand elimination); transverse momenta ride on the waves with the Roe
  transverse velocity, the remainder on a shear wave at the layer's Roe speed;
* otherwise each layer alone over its effective bottom with Einfeldt speeds; a
  dry neighbour is a reflecting wall (only the fluctuation into the wet cell,
  no correction) when the wet surface does not reach the dry cell's bottom of
  that layer (and always for the lower layer under a dry upper layer), else the
  water spills onto a dry state;
* fluctuations split by the sign of the speed (half each way at zero);
* MC-limited second-order correction with theta from the six-component dot
  product with the upwind neighbour edge's wave of the same slot;
* Godunov splitting x then y, the x-sweep also applied to the two frame rows on
  each side, walls mirrored before the step, dry-state fix-up after each sweep.
"""
from __future__ import annotations

import mpmath as mp

DPS = 50
G = 9.81
HDRY = 1e-3
KMIN = 1e-6


def _m(x):
    return mp.mpf(x)


class Cell:
    """One cell seen from a sweep: h, normal momentum m, transverse t per layer."""

    def __init__(self, q, B):
        self.h = [q[0], q[3]]
        self.m = [q[1], q[4]]
        self.t = [q[2], q[5]]
        self.B = B
        self.wet = [self.h[0] >= HDRY, self.h[1] >= HDRY]
        self.u = [self.m[k] / self.h[k] if self.wet[k] else _m(0) for k in range(2)]
        self.w = [self.t[k] / self.h[k] if self.wet[k] else _m(0) for k in range(2)]
        self.eta2 = B + self.h[1]
        self.eta1 = self.eta2 + self.h[0]


class Edge:
    """Waves of one edge: slot p has speed s[p], six-vector Z[p], mode[p]
    (0 both ways, 1 only into the left cell, 2 only into the right)."""

    def __init__(self):
        self.s = [_m(0)] * 6
        self.Z = [[_m(0)] * 6 for _ in range(6)]
        self.mode = [0] * 6


def _roe(hL, hR, vL, vR):
    a, b = mp.sqrt(hL), mp.sqrt(hR)
    return (a * vL + b * vR) / (a + b)


def _coupled(L, R, r, E):
    g = _m(G)
    gp = (1 - _m(r)) * g
    hb = [(L.h[k] + R.h[k]) / 2 for k in range(2)]
    ub = [_roe(L.h[k], R.h[k], L.u[k], R.u[k]) for k in range(2)]
    vb = [_roe(L.h[k], R.h[k], L.w[k], R.w[k]) for k in range(2)]
    # flux minus source, the hydrostatic parts through the surfaces
    d = [R.m[0] - L.m[0],
         (R.m[0] * R.u[0] - L.m[0] * L.u[0]) + g * hb[0] * (R.eta1 - L.eta1),
         R.m[1] - L.m[1],
         (R.m[1] * R.u[1] - L.m[1] * L.u[1]) + g * hb[1] * ((R.eta2 - L.eta2) + _m(r) * (R.h[0] - L.h[0]))]
    dt = [R.t[k] * R.u[k] - L.t[k] * L.u[k] for k in range(2)]
    H = hb[0] + hb[1]
    U = (hb[0] * ub[0] + hb[1] * ub[1]) / H
    Uc = (hb[0] * ub[1] + hb[1] * ub[0]) / H
    kap = 1 - (ub[0] - ub[1]) ** 2 / (gp * H)
    if kap < KMIN:
        kap = _m(KMIN)
    ce = mp.sqrt(g * H)
    ci = mp.sqrt(gp * hb[0] * hb[1] / H * kap)
    s = [U - ce, Uc - ci, Uc + ci, U + ce]
    al = [((sp - ub[0]) ** 2 - g * hb[0]) / (g * hb[0]) for sp in s]
    Rm = mp.matrix(4, 4)
    for p in range(4):
        Rm[0, p] = 1
        Rm[1, p] = s[p]
        Rm[2, p] = al[p]
        Rm[3, p] = al[p] * s[p]
    beta = mp.lu_solve(Rm, mp.matrix(d))
    for p in range(4):
        b = beta[p]
        E.s[p] = s[p]
        E.Z[p] = [b, b * s[p], b * vb[0], b * al[p], b * al[p] * s[p], b * al[p] * vb[1]]
    E.s[4] = ub[0]
    E.Z[4] = [_m(0), _m(0), dt[0] - vb[0] * d[0], _m(0), _m(0), _m(0)]
    E.s[5] = ub[1]
    E.Z[5] = [_m(0), _m(0), _m(0), _m(0), _m(0), dt[1] - vb[1] * d[2]]


def _single(k, L, R, r, E):
    """Layer k (0 upper, 1 lower) alone over its effective bottom."""
    g = _m(G)
    wl, wr = L.wet[k], R.wet[k]
    if not wl and not wr:
        return
    J = (R.eta1 - L.eta1) if k == 0 else (R.eta2 - L.eta2) + _m(r) * (R.h[0] - L.h[0])
    hL, mL, tL, uL, vL = L.h[k], L.m[k], L.t[k], L.u[k], L.w[k]
    hR, mR, tR, uR, vR = R.h[k], R.m[k], R.t[k], R.u[k], R.w[k]
    mode = 0

    def bottom(c):  # geometric bottom of layer k in cell c
        return c.eta2 if k == 0 else c.B

    def surface(c):
        return c.eta1 if k == 0 else c.eta2

    if wl and not wr:
        wall = (k == 1 and not R.wet[0]) or surface(L) <= bottom(R)
        if wall:
            hR, mR, tR, uR, vR, J, mode = hL, -mL, tL, -uL, vL, _m(0), 1
        else:
            hR = mR = tR = uR = vR = _m(0)
    elif wr and not wl:
        wall = (k == 1 and not L.wet[0]) or surface(R) <= bottom(L)
        if wall:
            hL, mL, tL, uL, vL, J, mode = hR, -mR, tR, -uR, vR, _m(0), 2
        else:
            hL = mL = tL = uL = vL = _m(0)
    hb = (hL + hR) / 2
    uh = _roe(hL, hR, uL, uR)
    vh = _roe(hL, hR, vL, vR)
    dA = mR - mL
    dB = (mR * uR - mL * uL) + g * hb * J
    dT = tR * uR - tL * uL
    ch = mp.sqrt(g * hb)
    sa = min(uL - mp.sqrt(g * hL), uh - ch) if hL > 0 else uR - 2 * mp.sqrt(g * hR)
    sb = max(uR + mp.sqrt(g * hR), uh + ch) if hR > 0 else uL + 2 * mp.sqrt(g * hL)
    bA = (sb * dA - dB) / (sb - sa)
    bB = (dB - sa * dA) / (sb - sa)
    o = 3 * k
    slots = (0, 3, 4) if k == 0 else (1, 2, 5)
    for slot, sp, b in ((slots[0], sa, bA), (slots[1], sb, bB)):
        z = [_m(0)] * 6
        z[o], z[o + 1], z[o + 2] = b, b * sp, b * vh
        E.s[slot], E.Z[slot], E.mode[slot] = sp, z, mode
    z = [_m(0)] * 6
    z[o + 2] = dT - vh * dA
    E.s[slots[2]], E.Z[slots[2]], E.mode[slots[2]] = uh, z, mode


def edge(L, R, r):
    E = Edge()
    if L.wet[0] and L.wet[1] and R.wet[0] and R.wet[1]:
        _coupled(L, R, r, E)
    else:
        _single(0, L, R, r, E)
        _single(1, L, R, r, E)
    return E


def _dot(a, b):
    return mp.fsum(x * y for x, y in zip(a, b))


def mc(theta):
    return max(_m(0), min((1 + theta) / 2, _m(2), 2 * theta))


def _fluct(E):
    am = [_m(0)] * 6
    ap = [_m(0)] * 6
    for p in range(6):
        s = E.s[p]
        wl = 0 if E.mode[p] == 2 else (1 if s < 0 else (mp.mpf("0.5") if s == 0 else 0))
        wr = 0 if E.mode[p] == 1 else (1 if s > 0 else (mp.mpf("0.5") if s == 0 else 0))
        for c in range(6):
            am[c] += wl * E.Z[p][c]
            ap[c] += wr * E.Z[p][c]
    return am, ap


def _corr(El, E, Er, nu):
    F = [_m(0)] * 6
    for p in range(6):
        s = E.s[p]
        if E.mode[p] != 0 or s == 0:
            continue
        zz = _dot(E.Z[p], E.Z[p])
        if zz == 0:
            continue
        up = El if s > 0 else Er
        phi = mc(_dot(up.Z[p], E.Z[p]) / zz)
        coef = (mp.mpf("0.5") if s > 0 else mp.mpf("-0.5")) * (1 - nu * abs(s)) * phi
        for c in range(6):
            F[c] += coef * E.Z[p][c]
    return F


def fixup(q, stats):
    if q[3] < HDRY:
        if q[3] != 0:
            stats["nclip"] += 1
        q[3] = q[4] = q[5] = _m(0)
    if q[0] < HDRY:
        if q[0] != 0:
            stats["nclip"] += 1
        q[0] = q[1] = q[2] = _m(0)
    if q[0] == 0 and q[3] > 0:
        stats["repair"] += 1
        q[3] = q[4] = q[5] = _m(0)


def sweep(line, Bl, nu, r, stats, count):
    """line: n + 4 cells (two ghosts each side) in local order h1 m1 t1 h2 m2 t2;
    returns the n updated interior cells and the largest speed of edges 0..n."""
    n = len(line) - 4
    cells = [Cell(q, b) for q, b in zip(line, Bl)]
    # edge e (between cells e-1 and e) for e = -1 .. n+1
    E = {e: edge(cells[e + 1], cells[e + 2], r) for e in range(-1, n + 2)}
    smax = max(abs(E[e].s[p]) for e in range(0, n + 1) for p in range(6))
    fl = {e: _fluct(E[e]) for e in range(0, n + 1)}
    F = {e: _corr(E[e - 1], E[e], E[e + 1], nu) for e in range(0, n + 1)}
    out = []
    for i in range(n):
        q = line[i + 2]
        left = [fl[i][1][c] - F[i][c] for c in range(6)]        # A+dQ - F at the left edge
        right = [fl[i + 1][0][c] + F[i + 1][c] for c in range(6)]  # A-dQ + F at the right edge
        o = [q[c] - nu * (left[c] + right[c]) for c in range(6)]
        fixup(o, stats if count else {"nclip": 0, "repair": 0})
        out.append(o)
    return out, smax


def wall_frame(q, B, nx, ny):
    """Padded copies (two-cell frame) of the state [6][ny][nx] and B with the
    frame mirrored across reflecting walls (normal momentum negated)."""
    def src(i, j):
        fx = fy = False
        si, sj = i, j
        if i < 0:
            si, fx = -1 - i, True
        elif i >= nx:
            si, fx = 2 * nx - 1 - i, True
        if j < 0:
            sj, fy = -1 - j, True
        elif j >= ny:
            sj, fy = 2 * ny - 1 - j, True
        return si, sj, fx, fy

    Q = {}
    Bp = {}
    for j in range(-2, ny + 2):
        for i in range(-2, nx + 2):
            si, sj, fx, fy = src(i, j)
            v = [q[c][sj][si] for c in range(6)]
            if fx:
                v[1], v[4] = -v[1], -v[4]
            if fy:
                v[2], v[5] = -v[2], -v[5]
            Q[i, j] = v
            Bp[i, j] = B[sj][si]
    return Q, Bp


def step(q, B, dx, dy, dt, r, stats):
    """One wall-bounded split step of the grid q [6][ny][nx] (lists of mpf).
    Returns (new state, (smax_x, smax_y))."""
    ny, nx = len(B), len(B[0])
    Q, Bp = wall_frame(q, B, nx, ny)
    nux, nuy = dt / _m(dx), dt / _m(dy)
    qs = {}
    sx = _m(0)
    for j in range(-2, ny + 2):
        line = [Q[i, j] for i in range(-2, nx + 2)]
        out, s = sweep(line, [Bp[i, j] for i in range(-2, nx + 2)], nux, r, stats, 0 <= j < ny)
        if 0 <= j < ny:
            sx = max(sx, s)
        for i in range(nx):
            qs[i, j] = out[i]
    new = [[[None] * nx for _ in range(ny)] for _ in range(6)]
    sy = _m(0)
    ymap = (0, 2, 1, 3, 5, 4)  # y orientation: normal momentum hv, transverse hu
    for i in range(nx):
        line = [[qs[i, j][ymap[c]] for c in range(6)] for j in range(-2, ny + 2)]
        out, s = sweep(line, [Bp[i, j] for j in range(-2, ny + 2)], nuy, r, stats, True)
        sy = max(sy, s)
        for j in range(ny):
            for c in range(6):
                new[ymap[c]][j][i] = out[j][c]
    return new, (sx, sy)


def run(B, q, dx, dy, dts, r):
    """Wall-bounded run with the given dt sequence; B [ny][nx], q [6][ny][nx]
    (FP64 values, converted exactly).  Returns (q as floats, smax per step,
    stats)."""
    with mp.workdps(DPS):
        ny, nx = len(B), len(B[0])
        Bm = [[_m(float(B[j][i])) for i in range(nx)] for j in range(ny)]
        qm = [[[_m(float(q[c][j][i])) for i in range(nx)] for j in range(ny)] for c in range(6)]
        stats = {"nclip": 0, "repair": 0}
        sm = []
        for dt in dts:
            qm, s = step(qm, Bm, dx, dy, _m(float(dt)), r, stats)
            sm.append((float(s[0]), float(s[1])))
        out = [[[float(qm[c][j][i]) for i in range(nx)] for j in range(ny)] for c in range(6)]
        return out, sm, stats
