"""Seeded synthetic inputs for the two-layer workloads.

This module holds data generation only (bathymetry fields, initial surfaces,
patch layouts, problem sizes) and none of the method's arithmetic.  It is the one
module that both the HIP path's callers and the oracle's tests use, so both sides
see identical inputs.  Everything is drawn from ``numpy.random.default_rng(seed)``
in a fixed order; coordinates are cell centres.

The paper's own demonstration (Sec. 3) is not reproducible (its set-ups are not
part of the text), so the workloads are synthetic stand-ins; each generator
below states its shapes, sizes and value ranges.
"""
from __future__ import annotations

import numpy as np

SEED0 = 180301450
G = 9.81
HDRY = 1.0e-3


def centres(n, L):
    dx = L / n
    return (np.arange(n) + 0.5) * dx


def smooth_field(rng, n, L, k, lo, hi, ny=None, Ly=None):
    """Sum of k Gaussians with amplitudes U(-1,1), centres uniform in the domain and
    widths U(0.03, 0.15) L, mapped affinely onto [lo, hi] over the samples."""
    ny = n if ny is None else ny
    Ly = L if Ly is None else Ly
    x = centres(n, L)
    y = centres(ny, Ly)
    a = rng.uniform(-1.0, 1.0, k)
    cx = rng.uniform(0.0, L, k)
    cy = rng.uniform(0.0, Ly, k)
    s = rng.uniform(0.03, 0.15, k) * min(L, Ly)
    S = np.zeros((ny, n))
    for i in range(k):
        gx = np.exp(-((x - cx[i]) ** 2) / (2 * s[i] ** 2))
        gy = np.exp(-((y - cy[i]) ** 2) / (2 * s[i] ** 2))
        S += a[i] * np.outer(gy, gx)
    smin, smax = S.min(), S.max()
    return lo + (S - smin) * ((hi - lo) / (smax - smin))


def gaussian(n, L, c, sigma, amp, ny=None, Ly=None):
    ny = n if ny is None else ny
    Ly = L if Ly is None else Ly
    x = centres(n, L)
    y = centres(ny, Ly)
    gx = np.exp(-((x - c[0]) ** 2) / (2 * sigma ** 2))
    gy = np.exp(-((y - c[1]) ** 2) / (2 * sigma ** 2))
    return amp * np.outer(gy, gx)


def block_mean(F, r):
    ny, nx = F.shape
    return F.reshape(ny // r, r, nx // r, r).mean(axis=(1, 3))


def state_from_surfaces(eta1, eta2, B, hdry=HDRY):
    """Depths from surfaces at rest: h2 = max(eta2 - B, 0), h1 = max(eta1 - B - h2, 0),
    thin layers set dry.  Returns q[6][ny][nx]."""
    h2 = np.maximum(eta2 - B, 0.0)
    h1 = np.maximum(eta1 - (B + h2), 0.0)
    h2 = np.where(h2 < hdry, 0.0, h2)
    h1 = np.where(h1 < hdry, 0.0, h1)
    h2 = np.where(h1 == 0.0, 0.0, h2)
    q = np.zeros((6,) + B.shape)
    q[0] = h1
    q[3] = h2
    return q


# ------------------------------------------------------------------ workloads
def fixed_small(n=64, L=100e3, seed=SEED0 + 1, fine_ratio=2):
    """64x64 over 100 km: linear slope -4000..-1000 m plus 16 bumps of 100 m,
    interface at -200 m with a -10 m Gaussian, 1 m Gaussian hump on eta1, at rest.
    The bathymetry is sampled on the ratio-2 grid and block-averaged."""
    rng = np.random.default_rng(seed)
    nf = n * fine_ratio
    xf = centres(nf, L)
    Bf = np.tile(-4000.0 + 3000.0 * xf / L, (nf, 1))
    ck = rng.uniform(0.0, L, (16, 2))
    sk = rng.uniform(3e3, 8e3, 16)
    ak = rng.uniform(-1.0, 1.0, 16) * 100.0
    for k in range(16):
        Bf += gaussian(nf, L, ck[k], sk[k], ak[k])
    c1 = rng.uniform(20e3, 80e3, 2)
    c2 = rng.uniform(20e3, 80e3, 2)
    B = block_mean(Bf, fine_ratio)
    eta1 = gaussian(n, L, c1, 10e3, 1.0)
    eta2 = -200.0 + gaussian(n, L, c2, 10e3, -10.0)
    q = state_from_surfaces(eta1, eta2, B)
    return dict(n=n, L=L, dx=L / n, B=B, Bf=Bf, q=q, r=0.95, nsteps=100,
                refine_box=(24, 24, 16, 16))


def roofline_grid(n=4096, L=409.6e3, seed=SEED0 + 3):
    """Single-level n x n grid (dx = 100 m at n = 4096): bathymetry from 64
    Gaussians mapped to [-4000, -50] m, eta1 = 16 Gaussians of 0.5 m, eta2 = -150 m
    plus 16 Gaussians of +-5 m, r = 0.97, at rest.  Where the bottom rises above
    the interface the lower layer is dry."""
    rng = np.random.default_rng(seed)
    B = smooth_field(rng, n, L, 64, -4000.0, -50.0)
    eta1 = np.zeros((n, n))
    eta2 = np.full((n, n), -150.0)
    c = rng.uniform(0.0, L, (16, 2))
    d = rng.uniform(0.0, L, (16, 2))
    eps = rng.choice([-1.0, 1.0], 16)
    w = 10e3 * (L / 409.6e3)
    for k in range(16):
        eta1 += gaussian(n, L, c[k], w, 0.5)
        eta2 += gaussian(n, L, d[k], w, 5.0 * eps[k])
    q = state_from_surfaces(eta1, eta2, B)
    return dict(n=n, L=L, dx=L / n, B=B, q=q, r=0.97, nsteps=500)


def amr_shoreline(n0=256, L=400e3, ratios=(2, 4), seed=SEED0 + 2, pulses=1):
    """Three levels (ratios 2 and 4) over 400 km: bathymetry from 64 Gaussians
    mapped to [-4000, +200] m at the finest samples, interface at -100 m, a 2 m
    pulse on eta1 (sigma 15 km) centred where B < -2000 m.  Level 0 is 16
    patches of 64x64.  pulses > 1 adds further such pulses, drawn after the
    first (the first pulse and everything before it are unchanged), so that the
    refined region is large from the first regrid on."""
    rng = np.random.default_rng(seed)
    nf = n0 * int(np.prod(ratios))
    Bf = smooth_field(rng, nf, L, 64, -4000.0, 200.0)
    B0 = block_mean(Bf, int(np.prod(ratios)))
    eta1 = np.zeros((n0, n0))
    for _ in range(pulses):
        while True:
            c = rng.uniform(0.1 * L, 0.9 * L, 2)
            i = int(c[0] / (L / n0)); j = int(c[1] / (L / n0))
            if B0[j, i] < -2000.0:
                break
        eta1 = eta1 + gaussian(n0, L, c, 15e3, 2.0)
    eta2 = np.full((n0, n0), -100.0)
    q = state_from_surfaces(eta1, eta2, B0)
    ps = 64
    boxes = [(i, j, ps, ps) for j in range(0, n0, ps) for i in range(0, n0, ps)]
    return dict(n0=n0, L=L, dx0=L / n0, ratios=tuple(ratios), Bf=Bf, B0=B0, q0=q, r=0.95,
                level0_boxes=boxes, regrid_every=4, nsteps=200)


def shelf_wave(n0=256, ratios=(2, 4), Lx=2.0, Ly=1.0, amp=0.02, width=0.01, g=9.81):
    """The paper's demonstration workload (Sec. 3) in scaled units, with invented
    parameters (its set-up is not in the text): sea level 0, deep floor -1, a
    shelf at -0.25 from x = 0.625 Lx on (a discontinuous jump), the internal
    interface at -0.125 (depths that averaging keeps exact), and a right-going
    plane wave on eta1 (Gaussian in x,
    uniform in y, amplitude `amp`, width `width` Lx, centre 0.25 Lx) whose layers
    move at eta1 sqrt(g / 1), the long-wave speed over unit depth.  Returns the
    finest-grid bathymetry and state (the uniform run) and the level-0 state of
    the AMR run; level 0 is n0 x n0 / 2 cells."""
    nfac = int(np.prod(ratios))
    n0y = int(round(n0 * Ly / Lx))
    nfx, nfy = n0 * nfac, n0y * nfac
    dxf = Lx / nfx
    xs = 0.625 * Lx  # on a level-0 cell boundary

    def state(x, B):
        eta1 = np.tile(amp * np.exp(-((x - 0.25 * Lx) ** 2) / (2.0 * (width * Lx) ** 2)), (B.shape[0], 1))
        q = state_from_surfaces(eta1, np.full(B.shape, -0.125), B)
        u = eta1 * np.sqrt(g / 1.0)
        q[1] = q[0] * u
        q[4] = q[3] * u
        return q

    xf = centres(nfx, Lx)
    Bf = np.tile(np.where(xf < xs, -1.0, -0.25), (nfy, 1))
    qf = state(xf, Bf)
    B0 = block_mean(Bf, nfac)  # the hierarchy's level-0 bathymetry
    q0 = state(centres(n0, Lx), B0)
    # time for the wave to reach the break and run 0.15 Lx onto the shelf
    T = float((xs - 0.25 * Lx) / np.sqrt(g) + 0.15 * Lx / np.sqrt(0.25 * g))
    return dict(n0x=n0, n0y=n0y, nfx=nfx, nfy=nfy, dx0=Lx / n0, dxf=dxf, ratios=tuple(ratios), Bf=Bf, qf=qf,
                B0=B0, q0=q0, r=0.95, T=T, tau=[0.05, 0.05], regrid_every=4)


def batch_sizes(nprob=512, seed=SEED0 + 4):
    rng = np.random.default_rng(seed)
    n = np.exp(rng.uniform(np.log(48), np.log(512), nprob))
    return (8 * np.round(n / 8)).astype(int)


def batch_problem(p, n, seed0=SEED0 * 10):
    """Problem p of the batch: n x n cells of 500 m, bathymetry from 16 Gaussians
    mapped to [-4000, top] with top = +100 m (shoreline) for about half the
    problems and -100 m otherwise, interface at -200 m, a pulse of 0.2..3 m and
    sigma 0.08 n dx, density ratio U(0.9, 0.99)."""
    rng = np.random.default_rng(seed0 + p)
    dx = 500.0
    L = n * dx
    top = 100.0 if rng.uniform() < 0.5 else -100.0
    B = smooth_field(rng, n, L, 16, -4000.0, top)
    amp = rng.uniform(0.2, 3.0)
    r = rng.uniform(0.9, 0.99)
    while True:
        c = rng.uniform(0.2 * L, 0.8 * L, 2)
        i = int(c[0] / dx); j = int(c[1] / dx)
        if B[j, i] < -1000.0:
            break
    eta1 = gaussian(n, L, c, 0.08 * L, amp)
    eta2 = np.full((n, n), -200.0)
    q = state_from_surfaces(eta1, eta2, B)
    return dict(n=n, L=L, dx=dx, B=B, q=q, r=float(r))


def adjoint_problem(n=1024, L=102.4e3, seed=SEED0 + 5):
    """n x n grid over 102.4 km: bathymetry from 64 Gaussians mapped to
    [-4000, -100] m, interface held at -50 m, 1 m Gaussian (sigma 5 km) on eta1,
    r = 0.95.  The target series at the gauge is seeded synthetic data (a slow
    oscillation of 5 cm plus 1 cm noise, one frame per sample); the 32x32 gauge
    region (physical size kept when n changes) sits 10-25 km from the pulse
    centre."""
    rng = np.random.default_rng(seed)
    B = smooth_field(rng, n, L, 64, -4000.0, -100.0)
    c = rng.uniform(0.35 * L, 0.65 * L, 2)
    ang = rng.uniform(0, 2 * np.pi)
    dist = rng.uniform(10e3, 25e3)
    g = c + dist * np.array([np.cos(ang), np.sin(ang)])
    dx = L / n
    gsize = 32 * 100.0  # physical extent of the gauge region
    gn = max(1, int(round(gsize / dx)))
    gi0 = int(np.clip(round(g[0] / dx - gn / 2), 0, n - gn))
    gj0 = int(np.clip(round(g[1] / dx - gn / 2), 0, n - gn))
    eta1 = gaussian(n, L, c, 5e3, 1.0)
    # seeded target series at the gauge: a slow oscillation plus small noise
    nsamp = 400 // 10
    tk = np.arange(1, nsamp + 1)[:, None, None]
    tg = 0.05 * np.sin(2 * np.pi * tk / 23.0) + 0.01 * rng.standard_normal((nsamp, gn, gn))
    return dict(n=n, L=L, dx=dx, B=B, eta1=eta1, eta2=-50.0, r=0.95,
                gauge=(gi0, gj0, gn), nsteps=400, every=10, ckpt=20, targets=tg)


def layered_problem(M, nxc, nyc, r, seed=SEED0 + 6, L=100e3):
    """M-layer coarse grid (nxc x nyc) with a shore: the fine bathymetry (ratio
    r) rises along x from -1000 m to +40 m with smooth bumps of +-40 m; the
    coarse bathymetry is its r x r block mean.  Layer surfaces sit at
    -900 (m - 1) / M m plus smooth +-2 m perturbations (layer 1 on top), so the
    lower layers end one after another towards the shore.  Depths from the
    bottom up (thin ones dry, every layer below a dry one dry), momenta smooth
    random in +-2 m^2/s per metre of depth.  Returns dict(qc [3M][nyc][nxc], Bc,
    Bf [r nyc][r nxc])."""
    rng = np.random.default_rng(seed + 97 * M + r)
    nxf, nyf = r * nxc, r * nyc
    x = centres(nxf, L)
    ramp = -1000.0 + 1040.0 * (x / L)
    Bf = ramp[None, :] + smooth_field(rng, nxf, L, 8, -40.0, 40.0, ny=nyf, Ly=L * nyc / nxc)
    Bc = block_mean(Bf, r)
    h = np.zeros((M + 1, nyc, nxc))
    eta = [None] + [(-900.0 * (m - 1) / M) + smooth_field(rng, nxc, L, 6, -2.0, 2.0, ny=nyc, Ly=L * nyc / nxc)
                    for m in range(1, M + 1)]
    below = Bc.copy()
    for m in range(M, 0, -1):
        hm = np.maximum(eta[m] - below, 0.0)
        hm = np.where(hm < HDRY, 0.0, hm)
        h[m] = hm
        below = below + hm
    dry = np.zeros((nyc, nxc), dtype=bool)
    for m in range(1, M + 1):
        h[m] = np.where(dry, 0.0, h[m])
        dry |= h[m] == 0.0
    qc = np.zeros((3 * M, nyc, nxc))
    for m in range(1, M + 1):
        qc[3 * (m - 1)] = h[m]
        qc[3 * (m - 1) + 1] = h[m] * smooth_field(rng, nxc, L, 4, -2.0, 2.0, ny=nyc, Ly=L * nyc / nxc)
        qc[3 * (m - 1) + 2] = h[m] * smooth_field(rng, nxc, L, 4, -2.0, 2.0, ny=nyc, Ly=L * nyc / nxc)
    return dict(qc=qc, Bc=Bc, Bf=Bf)
