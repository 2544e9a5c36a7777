"""Pins of the oracle's limiter and of the coarse-to-fine ghost cells in time.

* MC limiter: phi(theta) = max(0, min((1 + theta)/2, 2, 2 theta)) against a
  table worked out by hand (each of its three pieces and both clips).
* Ghost cells of a fine level at time fraction theta of the coarser level's
  step (Sec. 2: fine grids take their boundary values from the coarse grid,
  interpolated in time between the coarse grid's old and new states): every
  frame cell inside the domain and outside every sibling equals the refine
  operator (Sec. 2.1) applied to (1 - theta) Q_old + theta Q_new formed here in
  numpy from the coarse level's two buffers; cells covered by a sibling keep the
  sibling's value; cells outside the domain mirror the fine in-domain values.
* The subcycled advance uses the fraction k / r_t for the k-th fine substep
  (the fine level's time t + k dt / r_t within the coarse step, Sec. 2): one
  coarse step of advance() equals, bit for bit, the recursion written out here
  with those fractions through the oracle's own step, ghost fill and coarsen.
"""
import numpy as np
import pytest

import oracle
from paper_1803_01450_amd import inputs

# hand-worked MC values: theta -> phi
MC_TABLE = [
    (-3.0, 0.0), (-0.5, 0.0), (0.0, 0.0),          # upwind wave opposes: no correction
    (0.1, 0.2), (0.25, 0.5),                        # 2 theta below 1/3
    (1.0 / 3.0, 2.0 / 3.0),                         # corner of 2 theta and (1 + theta)/2
    (0.5, 0.75), (1.0, 1.0), (2.0, 1.5),            # (1 + theta)/2 between 1/3 and 3
    (3.0, 2.0), (7.5, 2.0), (1e6, 2.0),             # clipped at 2
]


def test_mc_limiter_table():
    for th, phi in MC_TABLE:
        assert abs(oracle.mc_limiter(th) - phi) <= 2.3e-16 * max(1.0, phi), (th, oracle.mc_limiter(th), phi)


def mc_table_mismatch():
    return any(abs(oracle.mc_limiter(th) - phi) > 2.3e-16 * max(1.0, phi) for th, phi in MC_TABLE)


def _two_levels(r=2, seed=3):
    """64 x 64 coarse level with a shore on the right, ratio r, three fine
    patches: two siblings side by side and one against the lower wall."""
    c = inputs.fixed_small()
    rng = np.random.default_rng(seed)
    n = 64
    H = oracle.Hierarchy(n, n, c["dx"], c["dx"], ratios=(r,), r=c["r"])
    x = (np.arange(n * r) + 0.5) / (n * r)
    Bf = np.kron(c["B"], np.ones((r, r))) + np.broadcast_to(5200.0 * np.clip(x - 0.55, 0, None)[None, :], (n * r, n * r))
    Bf = Bf + rng.uniform(-20, 20, Bf.shape)
    H.set_bathymetry(Bf)
    B0 = H.bathymetry(0)
    eta1 = inputs.gaussian(n, c["L"], (60e3, 50e3), 8e3, 2.0)
    eta2 = np.full((n, n), -200.0)
    q = inputs.state_from_surfaces(eta1, eta2, B0)
    for f, h in ((1, 0), (2, 0), (4, 3), (5, 3)):
        q[f] = q[h] * rng.uniform(-0.3, 0.3, (n, n))
    H.set_state(0, q)
    s = 16 * r // 2
    boxes = [(s * 2, s * 2, s * 2, s * 2), (s * 4, s * 2, s * 2, s * 3), (s * 5, 0, s * 2, s)]
    H.set_patches(1, [tuple(int(v) for v in b) for b in boxes])
    return H, c, r


def ghost_fill_mismatch(thetas=(0.0, 0.25, 0.5, 0.75)):
    """Largest |oracle ghost - expected| over the frame cells of all patches,
    and the number of cells compared, after one coarse step."""
    H, c, r = _two_levels()
    dt = H.next_dt()
    H.step_level(0, dt, 0.0)
    q_old = H.level_raw(0, which=1)[:, 2:-2, 2:-2]
    q_new = H.level_raw(0, which=0)[:, 2:-2, 2:-2]
    B0 = H.bathymetry(0)
    Bf = H.bathymetry(1)
    nxc, nyc = B0.shape[1], B0.shape[0]
    nxf, nyf = Bf.shape[1], Bf.shape[0]
    boxes = H.patches(1)
    cover = np.zeros((nyf, nxf), dtype=bool)
    for (i0, j0, bw, bh) in boxes:
        cover[j0:j0 + bh, i0:i0 + bw] = True
    worst, count = 0.0, 0
    for th in thetas:
        H.ghost_fill(1, th)
        raw = H.level_raw(1)
        qc = (1.0 - th) * q_old + th * q_new       # coarse data at the fraction
        exp = raw.copy()                             # interiors are the patches' own values
        for (i0, j0, bw, bh) in boxes:
            for j in range(j0 - 2, j0 + bh + 2):
                for i in range(i0 - 2, i0 + bw + 2):
                    if not (0 <= i < nxf and 0 <= j < nyf) or cover[j, i]:
                        continue
                    I, J = i // r, j // r
                    inx, iny = 0 < I < nxc - 1, 0 < J < nyc - 1
                    st = np.zeros((5, 7))
                    for k, (di, dj) in enumerate(((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1))):
                        ii, jj = I + di, J + dj
                        if 0 <= ii < nxc and 0 <= jj < nyc:
                            st[k, :6] = qc[:, jj, ii]
                            st[k, 6] = B0[jj, ii]
                    v, _ = oracle.refine_point(st, r, i % r, j % r, Bf[j, i], inx, iny)
                    exp[:, j + 2, i + 2] = v
        for (i0, j0, bw, bh) in boxes:                # walls: mirror the in-domain values
            for j in range(j0 - 2, j0 + bh + 2):
                for i in range(i0 - 2, i0 + bw + 2):
                    if 0 <= i < nxf and 0 <= j < nyf:
                        continue
                    si = -1 - i if i < 0 else (2 * nxf - 1 - i if i >= nxf else i)
                    sj = -1 - j if j < 0 else (2 * nyf - 1 - j if j >= nyf else j)
                    v = exp[:, sj + 2, si + 2].copy()
                    if si != i:
                        v[[1, 4]] = -v[[1, 4]]
                    if sj != j:
                        v[[2, 5]] = -v[[2, 5]]
                    exp[:, j + 2, i + 2] = v
        for (i0, j0, bw, bh) in boxes:
            sl = np.s_[:, j0:j0 + bh + 4, i0:i0 + bw + 4]
            worst = max(worst, float(np.abs(raw[sl] - exp[sl]).max()))
            count += (bw + 4) * (bh + 4) - bw * bh
    return worst, count


def test_ghost_cells_interpolate_coarse_data_in_time():
    worst, count = ghost_fill_mismatch()
    assert count > 1000 and worst == 0.0, worst


def test_ghost_fill_setup_reaches_shore_and_walls():
    """The coarse step changes the data the ghosts see (so the fraction
    matters), part of the coarse stencils are dry, and one patch's frame leaves
    the domain."""
    H, c, r = _two_levels()
    dt = H.next_dt()
    H.step_level(0, dt, 0.0)
    d = np.abs(H.level_raw(0, 1) - H.level_raw(0, 0))[:, 2:-2, 2:-2]
    assert d[0].max() > 1e-3
    q = H.state(0)
    assert (q[0] == 0).any() and (q[0] > 0).any()
    assert any(b[1] == 0 for b in H.patches(1))


def _subcycled(ratios, manual):
    c = inputs.fixed_small()
    n = 64
    H = oracle.Hierarchy(n, n, c["dx"], c["dx"], ratios=ratios, r=c["r"])
    f = int(np.prod(ratios))
    H.set_bathymetry(np.kron(c["B"], np.ones((f, f))))
    H.set_state(0, c["q"])
    H.set_patches(1, [(16 * ratios[0] // 2, 16 * ratios[0] // 2, 48 * ratios[0] // 2, 32 * ratios[0] // 2)])
    if len(ratios) > 1:
        b = H.patches(1)[0]
        H.set_patches(2, [(b[0] * ratios[1] + 16, b[1] * ratios[1] + 16, 64, 48)])
    if not manual:
        rc, dts = H.advance(1)
        assert rc == 0
        return H, dts[0]
    dt = H.next_dt()

    def adv(l, dtl, th):
        rc, _ = H.step_level(l, dtl, th)
        assert rc == 0
        if l + 1 < len(ratios) + 1:
            rt = ratios[l]
            for k in range(rt):
                adv(l + 1, dtl / rt, k / rt)
            H.coarsen(l + 1)

    adv(0, dt, 0.0)
    return H, dt


def subcycle_mismatch(ratios=(2, 4)):
    """Largest difference between advance(1) and the written-out recursion."""
    Ha, da = _subcycled(ratios, False)
    Hm, dm = _subcycled(ratios, True)
    worst = abs(da - dm)
    for l in range(len(ratios) + 1):
        a, m = Ha.state(l), Hm.state(l)
        ok = ~np.isnan(m)
        worst = max(worst, float(np.abs(a[ok] - m[ok]).max()))
    return worst


@pytest.mark.parametrize("ratios", [(2,), (4,), (2, 4)])
def test_subcycled_substeps_use_fraction_k_over_rt(ratios):
    assert subcycle_mismatch(ratios) == 0.0
