"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: integer/byte outputs (flags, patch layouts, counts) bit-exact; floating
point within 1e-12 relative per step and 1e-9 relative after a full run, per
field f: max|gpu - oracle| / max(max|oracle_f|, floor_f), floor 1 m for depths
and 1e-6 H sqrt(g H) for momenta (H the largest column depth)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1803_01450_amd import inputs

pytestmark = pytest.mark.gpu

G = 9.81


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def solver(**kw):
    from paper_1803_01450_amd.binding import Solver
    return Solver(**kw)


def rel_err(a, b, H=4000.0):
    """Per-field relative error; NaN (uncovered) cells must coincide."""
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


def fixed_setup(c, ratios=()):
    S = solver()
    n = c["B"].shape[1]
    ny = c["B"].shape[0]
    p = S.define(n, ny, c["dx"], c["dx"], c["r"], ratios)
    return S, p


# ---------------------------------------------------------------- fixed grid
def test_one_step_matches_oracle_bitwise():
    say("case: fixed 64x64, one step, dt 7 s")
    c = inputs.fixed_small()
    S, p = fixed_setup(c)
    S.set_bathymetry(p, c["B"])
    S.set_state(p, 0, c["q"])
    sm = S.step_level(0, [7.0])
    g = S.state(p, 0)
    ref, rsm, _ = oracle.fixed_steps(c["B"], c["q"], c["dx"], c["dx"], [7.0], r=c["r"])
    err = rel_err(g, ref)
    say("one-step rel err", err, "smax", sm[0], rsm[0])
    assert err.max() <= 1e-12
    assert np.array_equal(sm[0], rsm[0])
    S.close()


def test_hundred_steps_with_dt_rule():
    say("case: fixed 64x64, 100 steps, dt rule")
    c = inputs.fixed_small()
    S, p = fixed_setup(c)
    S.set_bathymetry(p, c["B"])
    S.set_state(p, 0, c["q"])
    dts = S.advance(100, want_dts=True)
    g = S.state(p, 0)
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], r=c["r"])
    H.set_bathymetry(c["B"]); H.set_state(0, c["q"])
    rc, rdts = H.advance(100)
    assert rc == 0
    err = rel_err(g, H.state(0))
    say("100-step rel err", err, "dt diff", np.abs(dts[0] - rdts).max())
    assert err.max() <= 1e-9
    assert np.abs(dts[0] - rdts).max() <= 1e-12 * rdts.max()
    cg, co = S.counters(p), H.counters()
    assert cg["updates"][0] == co["updates"][0] == 100 * 64 * 64
    assert cg["nclip"] == co["nclip"] and cg["repair"] == co["repair"] and cg["hyp"] == co["hyp"]
    S.close()


@pytest.mark.parametrize("shape", [(61, 37), (2, 5), (130, 3), (67, 129), (2, 2)])
def test_ragged_shapes(shape):
    """Sizes that are not multiples of the 60-column / 64-column strips."""
    nx, ny = shape
    say("case: ragged", shape)
    rng = np.random.default_rng(nx * 1000 + ny)
    L = 200e3
    dx = L / max(nx, ny)
    B = -3000.0 + 500.0 * rng.uniform(-1, 1, (ny, nx))
    eta1 = 0.5 * rng.uniform(-1, 1, (ny, nx))
    q = inputs.state_from_surfaces(eta1, np.full((ny, nx), -200.0), B)
    q[1] = rng.uniform(-5, 5, (ny, nx)); q[2] = rng.uniform(-5, 5, (ny, nx))
    q[4] = rng.uniform(-50, 50, (ny, nx)); q[5] = rng.uniform(-50, 50, (ny, nx))
    S = solver()
    p = S.define(nx, ny, dx, dx, 0.95)
    S.set_bathymetry(p, B)
    S.set_state(p, 0, q)
    dts = [0.5 * dx / 200.0] * 3
    for d in dts:
        S.step_level(0, [d])
    ref, _, _ = oracle.fixed_steps(B, q, dx, dx, dts)
    err = rel_err(S.state(p, 0), ref)
    say("ragged rel err", err)
    assert err.max() <= 1e-12
    S.close()


def test_degenerate_sizes_rejected():
    from paper_1803_01450_amd import binding
    S = solver()
    for nx, ny in [(1, 5), (5, 1), (0, 4)]:
        with pytest.raises(binding.MlsweError) as e:
            S.define(nx, ny, 100.0, 100.0, 0.95)
        assert e.value.code == binding.EINVAL
    with pytest.raises(binding.MlsweError):
        S.define(8, 8, 100.0, 100.0, 1.5)
    with pytest.raises(binding.MlsweError):
        S.define(8, 8, 100.0, 100.0, 0.95, (3,))
    S.close()


def test_wet_dry_shoreline_counters():
    """Land and a dry lower layer: clipping and wall branches; counts bit-exact."""
    say("case: wet/dry 64x64, 150 steps")
    c = inputs.fixed_small()
    B = -300.0 + (c["B"] - c["B"].min()) / (c["B"].max() - c["B"].min()) * 302.0
    eta1 = inputs.gaussian(64, c["L"], (30e3, 50e3), 8e3, 3.0)
    q = inputs.state_from_surfaces(eta1, np.full(B.shape, -100.0), B)
    S = solver()
    p = S.define(64, 64, c["dx"], c["dx"], 0.95)
    S.set_bathymetry(p, B)
    S.set_state(p, 0, q)
    S.advance(150)
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], r=0.95)
    H.set_bathymetry(B); H.set_state(0, q)
    rc, _ = H.advance(150)
    assert rc == 0
    g, o = S.state(p, 0), H.state(0)
    err = rel_err(g, o, H=300.0)
    cg, co = S.counters(p), H.counters()
    say("wet/dry rel err", err, cg, co)
    assert err.max() <= 1e-9
    assert np.array_equal(g[0] > 0, o[0] > 0) and np.array_equal(g[3] > 0, o[3] > 0)
    assert cg["nclip"] == co["nclip"] > 0
    assert cg["repair"] == co["repair"]
    assert abs(cg["clip1"] - co["clip1"]) <= 1e-12 * max(1.0, abs(co["clip1"]))
    S.close()


# ---------------------------------------------------------------- operators
def test_refine_coarsen_round_and_flags():
    """Small workload tail: flag, refine a 16x16 block by 2, coarsen back."""
    say("case: refine/coarsen round 64x64 -> 32x32 fine")
    c = inputs.fixed_small()
    S, p = fixed_setup(c, ratios=(2,))
    S.set_bathymetry(p, c["Bf"])
    H = oracle.Hierarchy(64, 64, c["dx"], c["dx"], ratios=(2,), r=c["r"])
    H.set_bathymetry(c["Bf"])
    B0 = H.bathymetry(0)
    q = inputs.state_from_surfaces(c["q"][0] + c["q"][3] + c["B"], c["q"][3] + c["B"], B0)
    S.set_state(p, 0, q); H.set_state(0, q)
    for _ in range(20):
        S.step_level(0, [7.0]); H.step_level(0, 7.0)
    assert rel_err(S.state(p, 0), H.state(0)).max() <= 1e-12
    for tau in (1e-6, 2e-5, 1e-4):
        fg, fo = S.flag(p, 0, tau, 2), H.flag(0, tau, 2)
        say("flags tau", tau, int(fg.sum()), int(fo.sum()))
        assert np.array_equal(fg, fo)
    box = [(48, 48, 32, 32)]
    S.refine(p, 1, box); H.set_patches(1, box)
    err = rel_err(S.state(p, 1), H.state(1))
    say("refine rel err", err)
    assert err.max() <= 1e-12
    S.coarsen(p, 1); H.coarsen(1)
    err = rel_err(S.state(p, 0), H.state(0))
    say("coarsen rel err", err)
    assert err.max() <= 1e-12
    S.close()


def amr_case(n0=64, L=100e3, nsteps=8, regrid_every=4, tau=(4e-6, 8e-6)):
    c = inputs.amr_shoreline(n0=n0, L=L, ratios=(2, 4))
    return c, nsteps, regrid_every, tau


@pytest.mark.parametrize("mode", [0, 1])
def test_amr_three_levels_with_shoreline(mode):
    """Three levels (ratios 2, 4), shorelines, regrid every 4 steps: patch layouts
    bit-exact, every level within 1e-9 after the run."""
    say("case: AMR 3 levels 64^2 mode", mode)
    c, nsteps, every, tau = amr_case()
    S = solver()
    p = S.define(c["n0"], c["n0"], c["dx0"], c["dx0"], c["r"], c["ratios"])
    S.set_bathymetry(p, c["Bf"])
    S.set_state(p, 0, c["q0"])
    H = oracle.Hierarchy(c["n0"], c["n0"], c["dx0"], c["dx0"], ratios=c["ratios"], r=c["r"])
    H.set_bathymetry(c["Bf"]); H.set_state(0, c["q0"])
    dts = S.advance(nsteps, every, [tau], mode=mode, want_dts=True)
    rc, rdts = H.advance(nsteps, every, tau)
    assert rc == 0
    assert np.abs(dts[0] - rdts).max() <= 1e-12 * rdts.max()
    for l in range(3):
        pg, po = S.patches(p, l), H.patches(l)
        say("level", l, "patches", len(pg), len(po))
        assert np.array_equal(pg, po)
        err = rel_err(S.state(p, l), H.state(l))
        say("level", l, "rel err", err)
        assert err.max() <= 1e-9
    cg, co = S.counters(p), H.counters()
    assert cg["updates"] == co["updates"]
    assert len(S.patches(p, 2)) > 0
    S.close()


def test_batched_problems_equal_plain():
    """Several problems of uneven sizes stepped in one launch per substep give
    the same result (bit for bit) as one problem at a time."""
    say("case: batched vs plain, 6 problems")
    sizes = [48, 64, 104, 56, 72, 48]
    res = {}
    for mode in (0, 1):
        S = solver()
        probs = []
        for k, n in enumerate(sizes):
            c = inputs.batch_problem(k, n)
            p = S.define(n, n, c["dx"], c["dx"], c["r"], (2,))
            S.set_bathymetry(p, np.kron(c["B"], np.ones((2, 2))))
            S.set_state(p, 0, c["q"])
            probs.append(p)
        S.advance(12, 6, np.tile([2e-6, 0.0], (len(sizes), 1)), mode=mode)
        res[mode] = [[S.state(p, l) for l in range(2)] for p in probs]
        S.close()
    for k in range(len(sizes)):
        for l in range(2):
            a, b = res[0][k][l], res[1][k][l]
            assert np.array_equal(np.isnan(a), np.isnan(b))
            m = ~np.isnan(a)
            assert np.array_equal(a[m], b[m]), (k, l)


def test_batched_matches_oracle_per_problem():
    say("case: batched problems vs oracle")
    sizes = [48, 80]
    S = solver()
    cs = []
    for k, n in enumerate(sizes):
        c = inputs.batch_problem(k, n)
        p = S.define(n, n, c["dx"], c["dx"], c["r"], (2,))
        Bf = np.kron(c["B"], np.ones((2, 2)))
        S.set_bathymetry(p, Bf)
        S.set_state(p, 0, c["q"])
        cs.append((c, Bf))
    S.advance(10, 5, np.tile([2e-6, 0.0], (2, 1)), mode=1)
    for k, (c, Bf) in enumerate(cs):
        n = sizes[k]
        H = oracle.Hierarchy(n, n, c["dx"], c["dx"], ratios=(2,), r=c["r"])
        H.set_bathymetry(Bf); H.set_state(0, c["q"])
        rc, _ = H.advance(10, 5, [2e-6])
        assert rc == 0
        for l in range(2):
            assert np.array_equal(S.patches(k, l), H.patches(l))
            err = rel_err(S.state(k, l), H.state(l))
            say("problem", k, "level", l, err)
            assert err.max() <= 1e-9
    S.close()


def test_rejected_step_matches_oracle():
    """A batch problem whose wet/dry front pushes a substep past the Courant
    limit: the library undoes and retakes the coarse step like the oracle (same
    dt sequence, same number of rejections, same states)."""
    say("case: coarse-step rejection, batch problem 301")
    c = inputs.batch_problem(301, 152)
    n = 152
    Bf = np.kron(c["B"], np.ones((2, 2)))
    for mode in (1, 2):
        S = solver()
        p = S.define(n, n, c["dx"], c["dx"], c["r"], (2,))
        S.set_bathymetry(p, Bf)
        S.set_state(p, 0, c["q"])
        S.advance(2, 10, [[2e-5, 0.0]], mode=mode)
        dts = S.advance(20, 10, [[2e-5, 0.0]], mode=mode, want_dts=True)
        H = oracle.Hierarchy(n, n, c["dx"], c["dx"], ratios=(2,), r=c["r"])
        H.set_bathymetry(Bf); H.set_state(0, c["q"])
        H.advance(2, 10, [2e-5])
        rc, rdts = H.advance(20, 10, [2e-5])
        assert rc == 0
        cg, co = S.counters(p), H.counters()
        say("mode", mode, "rejected gpu", cg["rejected"], "oracle", co["rejected"],
            "dt diff", np.abs(dts[0] - rdts).max())
        assert cg["rejected"] == co["rejected"] >= 1
        assert np.array_equal(dts[0], rdts)
        for l in range(2):
            err = rel_err(S.state(p, l), H.state(l))
            assert err.max() <= 1e-9, (l, err)
        assert cg["nclip"] == co["nclip"] and cg["repair"] == co["repair"]
        S.close()


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_deferred_check_retakes_like_per_step_check(mode):
    """Without per-step readbacks the library checks the Courant number once
    per window of coarse steps (the first failing substep halts the window);
    the run must retake the same steps as a run checked after every step
    (dts requested) and as the oracle: same rejections, bit-identical states,
    the same simulated time."""
    say("case: deferred Courant check, batch problem 301, mode", mode)
    c = inputs.batch_problem(301, 152)
    n = 152
    Bf = np.kron(c["B"], np.ones((2, 2)))
    tau = [[2e-5, 0.0]]

    def run(want):
        S = solver()
        p = S.define(n, n, c["dx"], c["dx"], c["r"], (2,))
        S.set_bathymetry(p, Bf)
        S.set_state(p, 0, c["q"])
        S.advance(22, 10, tau, mode=mode, want_dts=want)
        return S, p

    A, pa = run(False)
    B, pb = run(True)
    H = oracle.Hierarchy(n, n, c["dx"], c["dx"], ratios=(2,), r=c["r"])
    H.set_bathymetry(Bf); H.set_state(0, c["q"])
    rc, _ = H.advance(22, 10, [2e-5])
    assert rc == 0
    ca, cb, co = A.counters(pa), B.counters(pb), H.counters()
    say("rejected: deferred", ca["rejected"], "per step", cb["rejected"], "oracle", co["rejected"])
    assert ca["rejected"] == cb["rejected"] == co["rejected"] >= 1
    assert ca["t"] == cb["t"]
    assert ca["updates"] == cb["updates"] == co["updates"]
    for l in range(2):
        x, y = A.state(pa, l), B.state(pb, l)
        assert np.array_equal(np.isnan(x), np.isnan(y))
        m = ~np.isnan(x)
        assert np.array_equal(x[m], y[m]), l
        assert rel_err(x, H.state(l)).max() <= 1e-9
    A.close(); B.close()


@pytest.mark.parametrize("want_dts", [True, False])
def test_retake_takes_only_failing_problems(want_dts):
    """A batch in which one problem's step fails the Courant check: checked
    after every step (want_dts) only that problem is retaken and the others
    keep their step; in deferred windows the halted step is retaken for all.
    Either way every problem ends bit for bit as when run alone, and each
    counts only its own rejections."""
    say("case: per-problem retake, want_dts", want_dts)
    specs = [(301, 152, 2e-5), (400, 96, 2e-5), (401, 96, 2e-5)]

    def build(which):
        S = solver()
        for k in which:
            seed, n, tau = specs[k]
            c = inputs.batch_problem(seed, n)
            p = S.define(n, n, c["dx"], c["dx"], c["r"], (2,))
            S.set_bathymetry(p, np.kron(c["B"], np.ones((2, 2))))
            S.set_state(p, 0, c["q"])
        return S

    taus = [[s[2], 0.0] for s in specs]
    G = build(range(3))
    G.advance(22, 10, taus, mode=1, want_dts=want_dts)
    rej = [G.counters(p)["rejected"] for p in range(3)]
    say("rejected in the batch", rej)
    assert rej[0] >= 1
    for k in range(3):
        A = build([k])
        A.advance(22, 10, [taus[k]], mode=1, want_dts=want_dts)
        assert A.counters(0)["rejected"] == rej[k], k
        assert A.counters(0)["t"] == G.counters(k)["t"], k
        for l in range(2):
            x, y = G.state(k, l), A.state(0, l)
            assert np.array_equal(np.isnan(x), np.isnan(y))
            m = ~np.isnan(x)
            assert np.array_equal(x[m], y[m]), (k, l)
        A.close()
    G.close()


@pytest.mark.parametrize("mode", [1, 2])
def test_coarse_steps_without_host_waits(mode):
    """Between regrids a batched (1) or graph (2) advance with retakes waits for
    the stream once per window of 32 coarse steps plus once at its end (the
    final status): 64 steps of four two-level problems take at most 3 waits,
    no graph is captured after the first window, and every coarse step of the
    graph mode is one replay."""
    say("case: host waits per coarse step, mode", mode)
    S = solver()
    n = 96
    for k in range(4):
        c = inputs.batch_problem(400 + k, n)
        p = S.define(n, n, c["dx"], c["dx"], c["r"], (2,))
        S.set_bathymetry(p, np.kron(c["B"], np.ones((2, 2))))
        S.set_state(p, 0, c["q"])
    S.advance(4, 4, [[2e-5, 0.0]] * 4, mode=mode)  # regrid, launch data, graphs
    rej0 = sum(S.counters(p)["rejected"] for p in range(4))
    w0, c0, g0 = S.sync_counts()
    S.advance(64, 0, None, mode=mode)
    w1, c1, g1 = S.sync_counts()
    rej = sum(S.counters(p)["rejected"] for p in range(4)) - rej0
    say("waits", w1 - w0, "captures", c1 - c0, "replays", g1 - g0, "retakes", rej)
    # a retake (none expected here) re-checks its window's rest step by step
    assert w1 - w0 <= 3 + 40 * rej
    if mode == 2 and rej == 0:
        assert c1 - c0 == 0
        assert g1 - g0 == 64
    S.close()


# ---------------------------------------------------------------- full size
def test_roofline_grid_sampled_windows():
    """The 4096^2 grid in the benchmark's launch configuration: one step, checked
    on sampled windows (corners, edges, interior, strip and tile seams) against
    the oracle computing those windows one by one."""
    say("case: 4096^2 one step, sampled windows")
    c = inputs.roofline_grid()
    n = c["n"]
    S = solver()
    p = S.define(n, n, c["dx"], c["dx"], c["r"])
    S.set_bathymetry(p, c["B"])
    S.set_state(p, 0, c["q"])
    dt = 0.9 * c["dx"] / np.sqrt(G * 4000.0)
    sm = S.step_level(0, [dt])
    g = S.state(p, 0)
    boxes = [(0, 0, 40, 40), (n - 40, 0, 40, 40), (0, n - 40, 40, 40), (n - 40, n - 40, 40, 40),
             (2000, 0, 70, 24), (0, 2000, 24, 70), (56, 120, 70, 20), (3000, 1277, 33, 140),
             (4090, 2100, 6, 10)]
    for b in boxes:
        w, wsm = oracle.step_window(c["B"], c["q"], c["dx"], c["dx"], b, dt, r=c["r"])
        i, j, bx, by = b
        err = rel_err(g[:, j:j + by, i:i + bx], w)
        say("window", b, "rel err", err.max())
        assert err.max() <= 1e-12
    # the largest speeds are a property of the whole grid; they bound the windows'
    for b in boxes:
        _, wsm = oracle.step_window(c["B"], c["q"], c["dx"], c["dx"], b, dt, r=c["r"])
        assert wsm[0] <= sm[0, 0] and wsm[1] <= sm[0, 1]
    S.close()


def test_roofline_grid_ten_steps_full():
    """The 4096^2 grid, ten steps at a fixed dt through the benchmark's kernels
    (one x- and one y-sweep launch per step over the patch's tiles, handed to
    the XCDs in bands), against the oracle's ten steps over the whole grid (on
    the host's threads: row strips stepped as boxes, the one-box arithmetic):
    bit for bit."""
    import os
    say("case: 4096^2 ten steps, whole grid")
    c = inputs.roofline_grid()
    n = c["n"]
    S = solver()
    p = S.define(n, n, c["dx"], c["dx"], c["r"])
    S.set_bathymetry(p, c["B"])
    S.set_state(p, 0, c["q"])
    dt = 0.9 * c["dx"] / np.sqrt(G * 4000.0)
    S.run_fixed(p, np.full(10, dt))
    g = S.state(p, 0)
    S.close()
    threads = min(16, len(os.sched_getaffinity(0)))
    _, sec, ref = oracle.time_fixed_mt(c["B"], c["q"], c["dx"], c["dx"], 10, dt, threads, r=c["r"], want_state=True)
    say("oracle: %d threads, %.1f s" % (threads, sec))
    err = rel_err(g, ref)
    say("rel err", err.max())
    assert np.array_equal(g, ref)
