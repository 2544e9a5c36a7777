"""Pins of the oracle's multilayer AMR operators (Sec. 2-2.2 of the paper):
refine-then-coarsen identity, no new extrema in the refined surfaces, linear
reproduction, the bathymetry hierarchy, wet ordering, clustering (exhaustive),
well-balancing and subcycling of the level hierarchy."""
import itertools

import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from paper_1803_01450_amd import inputs

HD = oracle.HDRY


def wet_level0(c, H, seed=0):
    rng = np.random.default_rng(seed)
    B0 = H.bathymetry(0)
    eta1 = inputs.gaussian(64, c["L"], (50e3, 50e3), 10e3, 1.0)
    eta2 = -200.0 + inputs.gaussian(64, c["L"], (40e3, 60e3), 10e3, -10.0)
    q = inputs.state_from_surfaces(eta1, eta2, B0)
    q[1] = rng.uniform(-20, 20, q[1].shape)
    q[2] = rng.uniform(-20, 20, q[1].shape)
    q[4] = rng.uniform(-200, 200, q[1].shape)
    q[5] = rng.uniform(-200, 200, q[1].shape)
    return q


def test_bathymetry_hierarchy_is_block_mean():
    c = inputs.fixed_small()
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(2,), r=0.95)
    H.set_bathymetry(c["Bf"])
    B0 = H.bathymetry(0)
    ref = c["Bf"].reshape(64, 2, 64, 2).mean(axis=(1, 3))
    assert np.abs(B0 - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(H.bathymetry(1), c["Bf"])


def test_refine_then_coarsen_identity():
    """Away from shore (all wet) coarsen(refine(Q)) = Q to 1e-14 max|q| for all six
    fields, for ratios 2 and 4 (the fine offsets have zero mean and the
    bathymetry hierarchy is conservative)."""
    c = inputs.fixed_small()
    for ratio in (2, 4):
        H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(ratio,), r=0.95)
        Bf = np.kron(c["B"], np.ones((ratio, ratio))) + \
            np.random.default_rng(1).uniform(-30, 30, (64 * ratio, 64 * ratio))
        H.set_bathymetry(Bf)
        q = wet_level0(c, H)
        H.set_state(0, q)
        box = (8 * ratio, 8 * ratio, 48 * ratio, 48 * ratio)
        H.set_patches(1, [box])
        qf = H.state(1)
        assert not np.isnan(qf[:, box[1]:box[1] + box[3], box[0]:box[0] + box[2]]).any()
        H.coarsen(1)
        q2 = H.state(0)
        for f in range(6):
            sc = np.abs(q[f]).max()
            assert np.abs(q2[f] - q[f]).max() <= 1e-14 * sc * 4, (ratio, f)


def test_refine_reproduces_linear_surfaces():
    """A surface linear in x and y over the stencil is reproduced exactly at the
    fine cell centres (minmod picks the common slope)."""
    for r in (2, 4):
        for a in range(r):
            for b in range(r):
                q5 = np.zeros((5, 7))
                offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
                for k, (di, dj) in enumerate(offs):
                    B = -2000.0
                    eta2 = -200.0 + 3.0 * di - 2.0 * dj
                    eta1 = 0.5 + 0.25 * di + 0.125 * dj
                    q5[k] = [eta1 - eta2, 0, 0, eta2 - B, 0, 0, B]
                out, rep = oracle.refine_point(q5, r, a, b, -2000.0)
                fa = (2 * a + 1 - r) / (2 * r); fb = (2 * b + 1 - r) / (2 * r)
                eta2f = -200.0 + 3.0 * fa - 2.0 * fb
                eta1f = 0.5 + 0.25 * fa + 0.125 * fb
                assert np.isclose(out[3] - 2000.0, eta2f, rtol=0, atol=1e-12)
                assert np.isclose(out[0] + out[3] - 2000.0, eta1f, rtol=0, atol=1e-12)


def test_refine_at_extremum_is_flat():
    """At a local extremum minmod gives zero slope: every child equals the parent."""
    q5 = np.zeros((5, 7))
    for k, e in enumerate([1.0, 0.2, 0.3, 0.1, 0.4]):
        q5[k] = [e + 200.0, 5.0, 0, 1800.0, 0, 0, -2000.0]
    for a in range(2):
        for b in range(2):
            out, _ = oracle.refine_point(q5, 2, a, b, -2000.0)
            assert out[0] == 201.0 and out[3] == 1800.0 and out[1] == 5.0


stencil_vals = st.floats(min_value=-3.0, max_value=3.0, allow_nan=False)


@settings(max_examples=300, deadline=None)
@given(st.lists(stencil_vals, min_size=5, max_size=5), st.lists(stencil_vals, min_size=5, max_size=5),
       st.lists(st.floats(min_value=-50, max_value=50), min_size=6, max_size=6),
       st.sampled_from([2, 4]), st.integers(0, 3), st.integers(0, 3))
def test_no_new_extrema(e1, e2, db, r, a, b):
    """Each refined surface eta_m lies within [min, max] of the coarse 5-point
    stencil's eta_m (to rounding), for all-wet stencils over varying bathymetry."""
    a %= r; b %= r
    q5 = np.zeros((5, 7))
    for k in range(5):
        B = -3000.0 + db[k]
        eta2 = -200.0 + 10.0 * e2[k]
        eta1 = e1[k]
        q5[k] = [eta1 - eta2, 0, 0, eta2 - B, 0, 0, B]
    Bf = -3000.0 + db[5]
    out, rep = oracle.refine_point(q5, r, a, b, Bf)
    eta2f = Bf + out[3]
    eta1f = eta2f + out[0]
    E2 = q5[:, 6] + q5[:, 3]
    E1 = E2 + q5[:, 0]
    tol = 8 * np.spacing(4000.0)
    assert E2.min() - tol <= eta2f <= E2.max() + tol
    assert E1.min() - tol <= eta1f <= E1.max() + tol
    assert rep == 0


@settings(max_examples=300, deadline=None)
@given(st.lists(st.floats(min_value=-150, max_value=50), min_size=6, max_size=6),
       st.lists(st.floats(min_value=-1, max_value=1), min_size=5, max_size=5),
       st.integers(0, 1), st.integers(0, 1))
def test_refine_near_shore_keeps_wet_ordering(Bs, e1, a, b):
    """Near shore (bottom layer and land partly dry) the refined cell never has a
    dry top layer over a wet bottom layer, and depths are zero or >= h_dry."""
    q5 = np.zeros((5, 7))
    for k in range(5):
        B = Bs[k]
        q = inputs.state_from_surfaces(np.array([[e1[k]]]), np.array([[-100.0]]), np.array([[B]]))
        q5[k] = [q[0, 0, 0], 0, 0, q[3, 0, 0], 0, 0, B]
    out, rep = oracle.refine_point(q5, 2, a, b, Bs[5])
    h1, h2 = out[0], out[3]
    assert not (h1 == 0.0 and h2 > 0.0)
    assert h1 == 0.0 or h1 >= HD
    assert h2 == 0.0 or h2 >= HD


def test_cluster_exhaustive_4x4_tiles():
    """All 2^16 flag patterns on a 4x4 lattice of 16x16 fine tiles: every marked
    tile is covered exactly once, only marked tiles are covered, patch sides are
    16..64, and the output is a deterministic function of the flags."""
    H = oracle.Hierarchy(32, 32, 1.0, 1.0, ratios=(2,), r=0.95)
    for pattern in range(1 << 16):
        marked = np.array([(pattern >> k) & 1 for k in range(16)], dtype=bool).reshape(4, 4)
        flags = np.kron(marked.astype(np.uint8), np.ones((8, 8), dtype=np.uint8))
        boxes = H.cluster(0, flags)
        cover = np.zeros((4, 4), dtype=int)
        for (i, j, nx, ny) in boxes:
            assert i % 16 == 0 and j % 16 == 0 and 16 <= nx <= 64 and 16 <= ny <= 64
            cover[j // 16:(j + ny) // 16, i // 16:(i + nx) // 16] += 1
        assert np.array_equal(cover, marked.astype(int)), pattern
        if pattern % 4099 == 0:
            assert np.array_equal(H.cluster(0, flags), boxes)


def test_cluster_respects_nesting():
    """A fine tile is kept only if its coarse footprint grown by two cells lies in
    the coarse level's coverage."""
    H = oracle.Hierarchy(32, 32, 1.0, 1.0, ratios=(2, 2), r=0.95)
    H.set_bathymetry(np.full((128, 128), -1000.0))
    H.set_patches(1, [(16, 16, 32, 32)])    # level-1 coverage [16,48)^2
    flags = np.zeros((64, 64), dtype=np.uint8)
    flags[16:48, 16:48] = 1
    boxes = H.cluster(1, flags)
    # level-2 tiles cover 8 level-1 cells; only the tiles whose footprint +2 stays
    # inside [16,48) survive: footprints [24,32) and [32,40) in each direction
    cov = np.zeros((128, 128), dtype=int)
    for (i, j, nx, ny) in boxes:
        cov[j:j + ny, i:i + nx] += 1
    expect = np.zeros((128, 128), dtype=int)
    expect[48:80, 48:80] = 1
    assert np.array_equal(cov, expect)


def test_flag_planar_surface():
    """eta1 with a known uniform gradient: flagged exactly where the gradient
    exceeds tau, dilated by the buffer, with walls mirrored."""
    n, dx = 32, 1000.0
    H = oracle.Hierarchy(n, n, dx, dx, ratios=(2,), r=0.95)
    H.set_bathymetry(np.full((2 * n, 2 * n), -1000.0))
    x = (np.arange(n) + 0.5) * dx
    eta1 = np.tile(np.where(x < 16e3, 1e-3 * x, 16.0), (n, 1))     # slope 1e-3 for x < 16 km
    q = inputs.state_from_surfaces(eta1, np.full((n, n), -200.0), H.bathymetry(0))
    H.set_state(0, q)
    f = H.flag(0, 5e-4, nbuf=0)
    # centred difference > 5e-4 for cells 1..15 (cell 0 mirrors: (eta(1)-eta(0))/2dx = 5e-4, not >)
    assert np.all(f[:, 1:16] == 1) and np.all(f[:, 0] == 0) and np.all(f[:, 17:] == 0)
    fb = H.flag(0, 5e-4, nbuf=2)
    assert np.all(fb[:, 0:18] == 1) and np.all(fb[:, 18:] == 0)


def test_amr_lake_at_rest_three_levels():
    """Flat surfaces over a bathymetry with shorelines stay at rest through the
    whole subcycled hierarchy: ghost fill (time-interpolated refine), fine steps,
    coarsening and regridding add no motion."""
    c = inputs.amr_shoreline(n0=64, L=100e3, ratios=(2, 4))
    H = oracle.Hierarchy(64, 64, c["dx0"], c["dx0"], ratios=(2, 4), r=0.95)
    H.set_bathymetry(c["Bf"])
    B0 = H.bathymetry(0)
    q = inputs.state_from_surfaces(np.zeros_like(B0), np.full(B0.shape, -100.0), B0)
    H.set_state(0, q)
    H.set_patches(1, [(32, 32, 64, 48), (96, 32, 16, 16)])
    H.set_patches(2, [(160, 160, 64, 64), (224, 160, 32, 64)])
    rc, dts = H.advance(6)
    assert rc == 0
    for l in range(3):
        s = H.state(l)
        m = ~np.isnan(s[0])
        for f in (1, 2, 4, 5):
            assert np.abs(s[f][m]).max() <= 1e-9, (l, f)
        B = H.bathymetry(l)
        eta1 = (B + s[3] + s[0])[m & (s[0] > 0)]
        assert np.abs(eta1).max() <= 1e-9


def test_subcycling_matches_uniform_fine_run():
    """A fine level covering the whole domain gets only wall ghosts, so after each
    coarse step it equals a uniform fine run with dt/r bit for bit."""
    c = inputs.fixed_small(n=32, L=50e3)
    H = oracle.Hierarchy(32, 32, c["dx"], c["dx"], ratios=(2,), r=0.95)
    H.set_bathymetry(c["Bf"])
    H.set_state(0, inputs.state_from_surfaces(np.zeros((32, 32)), np.full((32, 32), -200.0), H.bathymetry(0)))
    qf0 = inputs.state_from_surfaces(
        inputs.gaussian(64, c["L"], (25e3, 25e3), 4e3, 1.0), np.full((64, 64), -200.0), c["Bf"])
    H.set_patches(1, [(0, 0, 64, 64)])
    H.set_state(1, qf0)
    rc, dts = H.advance(5)
    assert rc == 0
    fine_dts = np.repeat(dts / 2.0, 2)
    ref, *_ = oracle.fixed_steps(c["Bf"], qf0, c["dx"] / 2, c["dx"] / 2, fine_dts)
    assert np.array_equal(H.state(1), ref)
    # coarsening put the fine average on level 0
    q0 = H.state(0)
    assert np.abs(q0[0] - ref[0].reshape(32, 2, 32, 2).mean(axis=(1, 3))).max() <= 1e-12 * 300


def test_regrid_follows_the_pulse():
    """Regridding on |grad eta1| puts level-1 patches over the pulse and keeps
    them nested; the layout is deterministic."""
    c = inputs.amr_shoreline(n0=64, L=100e3, ratios=(2, 4))
    runs = []
    for _ in range(2):
        H = oracle.Hierarchy(64, 64, c["dx0"], c["dx0"], ratios=(2, 4), r=0.95)
        H.set_bathymetry(c["Bf"])
        q = inputs.state_from_surfaces(inputs.gaussian(64, c["L"], (50e3, 50e3), 6e3, 2.0),
                                       np.full((64, 64), -100.0), H.bathymetry(0))
        H.set_state(0, q)
        H.regrid([5e-5, 1e-4])
        runs.append((H.patches(1), H.patches(2)))
        assert len(runs[-1][0]) > 0
        qs = H.state(1)
        m = ~np.isnan(qs[0])
        # the pulse centre is refined
        assert m[64, 64]
    assert all(np.array_equal(a, b) for a, b in zip(runs[0], runs[1]))


def test_rejected_step_is_retaken():
    """A thin layer at a wet/dry front can raise the largest speed within one
    step past the Courant limit; the coarse step is then undone and retaken with
    dt scaled by cfl / (largest substep Courant number), and the run goes on."""
    c = inputs.batch_problem(301, 152)
    n = 152
    H = oracle.Hierarchy(n, n, c["dx"], c["dx"], ratios=(2,), r=c["r"])
    H.set_bathymetry(np.kron(c["B"], np.ones((2, 2))))
    H.set_state(0, c["q"])
    rc, d1 = H.advance(2, 10, [2e-5])
    assert rc == 0
    rc, d2 = H.advance(20, 10, [2e-5])
    assert rc == 0
    cn = H.counters()
    assert cn["rejected"] >= 1
    # every accepted substep respected the limit: re-running an accepted step
    # with its dt is what the driver did; the dt sequence shrank at the rejection
    assert np.all(d2 > 0) and d2.min() < d2.max()


def _composite_mass(H, nlev, ratios, dx0):
    """Per-layer mass over the composite grid: each level's cells not covered
    by the next finer level, times the cell area."""
    out = np.zeros(2)
    dx = dx0
    for l in range(nlev):
        q = H.state(l)
        cov = ~np.isnan(q[0])
        if l + 1 < nlev:
            r = ratios[l]
            fine = ~np.isnan(H.state(l + 1)[0])
            cov &= ~fine.reshape(fine.shape[0] // r, r, fine.shape[1] // r, r).any(axis=(1, 3))
            area = dx * dx
            dx = dx / r
        else:
            area = dx * dx
        out += [np.where(cov, q[0], 0.0).sum() * area, np.where(cov, q[3], 0.0).sum() * area]
    return out


def test_amr_mass_drift_without_refluxing():
    """All wet, no clipping: one level conserves each layer's mass to rounding;
    two levels do not, because the coarse cells beside a fine patch keep their
    own fluxes (the paper has no flux correction at coarse-fine edges).  The
    drift is small (about 1e-8 relative per coarse step here) but not zero."""
    c = inputs.fixed_small()
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], r=c["r"])
    H.set_bathymetry(c["B"]); H.set_state(0, c["q"])
    m0 = _composite_mass(H, 1, (), c["dx"])
    rc, _ = H.advance(5)
    assert rc == 0 and H.counters()["nclip"] == 0
    assert np.all(np.abs(_composite_mass(H, 1, (), c["dx"]) - m0) <= 1e-14 * m0)
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(2,), r=c["r"])
    H.set_bathymetry(np.kron(c["B"], np.ones((2, 2)))); H.set_state(0, c["q"])
    rc, _ = H.advance(5, 4, [2e-6])
    assert rc == 0 and H.counters()["nclip"] == 0 and len(H.patches(1)) > 0
    drift = np.abs(_composite_mass(H, 2, (2,), c["dx"]) - m0) / m0
    assert np.all(drift < 1e-6) and drift.max() > 1e-12, drift


def test_flux_correction_conserves_mass():
    """With the mass flux correction at coarse-fine edges on, each layer's mass
    on the composite grid is conserved to rounding through two and three levels
    with regrids (all wet, no clipping), where without it the mass drifts.
    After one coarse step the correction has changed only depths of coarse cells
    beside a fine patch: momenta, finer levels and every other cell are as
    without it."""
    c = inputs.fixed_small()
    for ratios, tau in [((2,), [2e-6]), ((2, 4), [2e-6, 4e-6])]:
        nl, nf = len(ratios) + 1, 64 * int(np.prod(ratios))
        Bf = np.kron(c["B"], np.ones((nf // 64, nf // 64)))
        H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=ratios, r=c["r"])
        H.set_reflux(True)
        H.set_bathymetry(Bf); H.set_state(0, c["q"])
        m0 = _composite_mass(H, 1, ratios, c["dx"])
        rc, _ = H.advance(9, 4, tau)
        assert rc == 0 and H.counters()["nclip"] == 0 and len(H.patches(nl - 1)) > 0
        drift = np.abs(_composite_mass(H, nl, ratios, c["dx"]) - m0) / m0
        assert np.all(drift <= 1e-14), (ratios, drift)
    # one coarse step, with and without
    out = []
    for on in (False, True):
        H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(2,), r=c["r"])
        H.set_reflux(on)
        H.set_bathymetry(np.kron(c["B"], np.ones((2, 2)))); H.set_state(0, c["q"])
        H.set_patches(1, [(32, 32, 48, 32), (80, 32, 16, 16)])
        rc, _ = H.advance(1)
        assert rc == 0
        out.append((H.state(0), H.state(1)))
    (a0, a1), (b0, b1) = out
    assert np.array_equal(a1, b1, equal_nan=True)
    diff = a0 != b0
    assert not diff[[1, 2, 4, 5]].any()
    fine = np.zeros((64, 64), dtype=bool)
    fine[16:32, 16:40] = True
    fine[16:24, 40:48] = True
    ring = np.zeros_like(fine)
    ring[1:, :] |= fine[:-1, :]; ring[:-1, :] |= fine[1:, :]
    ring[:, 1:] |= fine[:, :-1]; ring[:, :-1] |= fine[:, 1:]
    ring &= ~fine
    changed = diff[0] | diff[3]
    assert changed.any() and not (changed & ~ring).any()


def _shallow_patch_run(dyn, reflux=False, steps=4):
    """Ratio 4, one fine patch over the shallow end of the slope (about 1000 m
    deep against 4000 m at the deep end)."""
    c = inputs.fixed_small()
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(4,), r=c["r"])
    H.set_dynamic_rt(dyn)
    H.set_reflux(reflux)
    H.set_bathymetry(np.kron(c["B"], np.ones((4, 4)))); H.set_state(0, c["q"])
    H.set_patches(1, [(208, 32, 32, 64)])
    rts, dts, speeds = [], [], []
    for _ in range(steps):
        speeds.append(H.step_state())
        rc, d = H.advance(1)
        assert rc == 0
        rts.append(int(H.time_ratios()[0])); dts.append(d[0])
    return H, rts, np.array(dts), speeds, c


def test_dynamic_time_ratio():
    """Fine patch in shallow water, coarse step set by the deep water: the
    dynamic choice takes 3 fine substeps instead of 4 once speeds are known,
    each the fewest within the Courant limit of the fine level's own last
    speeds; dts, clock and rejections are unchanged, fine updates drop by a
    quarter."""
    Hf, rf, df, _, c = _shallow_patch_run(False)
    Hd, rd, dd, sp, _ = _shallow_patch_run(True)
    assert rf == [4, 4, 4, 4] and rd == [4, 3, 3, 3]
    assert np.array_equal(df, dd)
    assert Hd.counters()["rejected"] == 0 and Hd.counters()["t"] == Hf.counters()["t"]
    assert Hd.counters()["updates"][1] * 4 == Hf.counters()["updates"][1] * 13 // 4
    dxf = c["dx"] / 4
    for n in range(1, 4):
        s = sp[n]  # speeds of the step before step n: [t, flag, sx0, sy0, sx1, sy1]
        lim = 0.9 * min(dxf / s[4], dxf / s[5])
        k = rd[n]
        assert dd[n] / k <= lim and (k == 1 or dd[n] / (k - 1) > lim), (n, k)


def test_dynamic_time_ratio_with_flux_correction_conserves_mass():
    """The flux correction averages the fine fluxes over the substeps actually
    taken (3 of ratio 4 here): composite mass is still conserved to rounding."""
    c = inputs.fixed_small()
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(4,), r=c["r"])
    H.set_dynamic_rt(True); H.set_reflux(True)
    H.set_bathymetry(np.kron(c["B"], np.ones((4, 4)))); H.set_state(0, c["q"])
    m0 = _composite_mass(H, 1, (4,), c["dx"])
    H.set_patches(1, [(208, 32, 32, 64)])
    rc, _ = H.advance(5)
    assert rc == 0 and int(H.time_ratios()[0]) == 3
    drift = np.abs(_composite_mass(H, 2, (4,), c["dx"]) - m0) / m0
    assert np.all(drift <= 1e-14), drift


def test_dynamic_time_ratio_for_a_newly_populated_level():
    """A fine level that receives its first patches mid-run has no speeds of
    the last coarse step: it takes the space ratio (as on a first step), so its
    substeps stay within the Courant limit; with no retakes allowed the run
    neither rejects a step nor fails.  Deep water under the patch: one substep
    per coarse step would give a fine Courant number near 3.6."""
    c = inputs.fixed_small()
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(4,), r=c["r"])
    H.set_dynamic_rt(True)
    H.set_retries(0)
    H.set_bathymetry(np.kron(c["B"], np.ones((4, 4)))); H.set_state(0, c["q"])
    H.set_patches(1, [])
    rc, _ = H.advance(2)
    assert rc == 0
    H.set_patches(1, [(16, 64, 32, 64)])
    rts = []
    for _ in range(3):
        rc, _ = H.advance(1)
        assert rc == 0
        rts.append(int(H.time_ratios()[0]))
    assert rts[0] == 4
    assert H.counters()["rejected"] == 0
