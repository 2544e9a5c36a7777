"""Adjoint of the fixed-grid two-layer run (gauge misfit w.r.t. the initial
top surface and the bathymetry) on the GPU, through the C ABI and the
torch.autograd.Function, checked against the oracle's forward-mode dual
derivative (a CPU reference on a 64x64 copy) and against FP64 central
differences of the GPU forward on the full 1024x1024 grid."""
import sys

import numpy as np
import pytest

import oracle
from paper_1803_01450_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(n, nsteps):
    import torch
    from paper_1803_01450_amd.binding import Solver
    from paper_1803_01450_amd.adjoint import MisfitProblem
    c = inputs.adjoint_problem(n=n)
    dt = 0.9 * c["dx"] / np.sqrt(9.81 * 4000.0)
    dts = np.full(nsteps, dt)
    tg = c["targets"][: nsteps // c["every"]]
    S = Solver(stream=torch.cuda.current_stream().cuda_stream)
    p = S.define(n, n, c["dx"], c["dx"], c["r"])
    S.set_bathymetry(p, c["B"])
    tgt = torch.from_numpy(np.ascontiguousarray(tg)).cuda()
    prob = MisfitProblem(S, p, c["eta2"], dts, c["every"], c["gauge"], tgt, ckpt=c["ckpt"])
    return c, dts, tg, S, prob


def gradients(c, prob):
    import torch
    from paper_1803_01450_amd.adjoint import GaugeMisfit
    e = torch.from_numpy(c["eta1"].copy()).cuda().requires_grad_(True)
    B = torch.from_numpy(c["B"].copy()).cuda().requires_grad_(True)
    loss = GaugeMisfit.apply(e, B, prob)
    loss.backward()
    torch.cuda.synchronize()
    return float(loss.item()), e.grad.cpu().numpy(), B.grad.cpu().numpy()


def test_adjoint_matches_oracle_dual_64():
    say("case: adjoint 64x64, 100 steps, vs oracle dual numbers")
    n, nsteps = 64, 100
    c, dts, tg, S, prob = make(n, nsteps)
    L, ge, gB = gradients(c, prob)
    Lo = oracle.gauge_loss(c["eta1"], c["B"], c["dx"], c["eta2"], dts, c["every"], c["gauge"], tg, r=c["r"])
    say("loss gpu %.17g oracle %.17g" % (L, Lo))
    assert abs(L - Lo) <= 1e-10 * abs(Lo)
    rng = np.random.default_rng(11)
    dirs = []
    for k in range(3):
        dirs.append((rng.standard_normal((n, n)), None))
        dirs.append((None, rng.standard_normal((n, n))))
    # unit vectors at cells near the gauge and the pulse
    i0, j0, gn = c["gauge"]
    for (i, j) in [(i0, j0), (i0 + 3, j0 - 2), (n // 2, n // 2)]:
        u = np.zeros((n, n)); u[j, i] = 1.0
        dirs.append((u, None)); dirs.append((None, u))
    scale = max(np.abs(ge).max(), np.abs(gB).max())
    for ve, vb in dirs:
        _, d = oracle.gauge_loss(c["eta1"], c["B"], c["dx"], c["eta2"], dts, c["every"], c["gauge"], tg,
                                 v_eta=ve, v_B=vb, r=c["r"])
        g = (ge * ve).sum() if ve is not None else (gB * vb).sum()
        say("directional derivative gpu %.15e oracle %.15e" % (g, d))
        assert abs(g - d) <= 1e-9 * abs(d) + 1e-12 * scale
    S.close()


def test_adjoint_matches_oracle_dual_256_full_run():
    """256^2, the full 400 steps with checkpoints every 20: the gradient's
    directional derivatives along two seeded random directions in eta1 and
    two in B against the oracle's forward-mode (dual number) derivative of the
    same discrete map, within 1e-9 relative.  The five oracle runs go to host
    threads (the oracle releases the interpreter while it runs)."""
    from concurrent.futures import ThreadPoolExecutor
    say("case: adjoint 256x256, 400 steps, vs oracle dual numbers in 4 directions")
    n, nsteps = 256, 400
    c, dts, tg, S, prob = make(n, nsteps)
    L, ge, gB = gradients(c, prob)
    rng = np.random.default_rng(256)
    dirs = [(rng.standard_normal((n, n)), None), (None, rng.standard_normal((n, n))),
            (rng.standard_normal((n, n)), None), (None, rng.standard_normal((n, n)))]

    def loss_only():
        return oracle.gauge_loss(c["eta1"], c["B"], c["dx"], c["eta2"], dts, c["every"], c["gauge"], tg, r=c["r"])

    def dual(v):
        return oracle.gauge_loss(c["eta1"], c["B"], c["dx"], c["eta2"], dts, c["every"], c["gauge"], tg,
                                 v_eta=v[0], v_B=v[1], r=c["r"])[1]

    with ThreadPoolExecutor(max_workers=5) as ex:
        fl = ex.submit(loss_only)
        fd = [ex.submit(dual, v) for v in dirs]
        Lo = fl.result()
        ds = [f.result() for f in fd]
    say("loss gpu %.17g oracle %.17g" % (L, Lo))
    assert abs(L - Lo) <= 1e-10 * abs(Lo)
    scale = max(np.abs(ge).max(), np.abs(gB).max())
    for (ve, vb), d in zip(dirs, ds):
        g = (ge * ve).sum() if ve is not None else (gB * vb).sum()
        say("directional derivative (%s) gpu %.15e oracle %.15e rel %.2e" % (
            "eta1" if ve is not None else "B", g, d, abs(g - d) / abs(d)))
        assert abs(g - d) <= 1e-9 * abs(d) + 1e-12 * scale
    S.close()


def test_adjoint_full_size_central_differences():
    """1024^2, 400 steps, checkpoints every 20: the gradient at 64 seeded cells
    within 3 sigma of the pulse centre against central differences of the GPU
    forward (eps 1e-4 m on eta1; 0.5 m on B, since 1 cm on a 4 km column is below
    the rounding noise of the misfit).  The discrete map is only piecewise
    smooth (MC limiter branches): the branch signature shows how many +-eps runs
    switch a branch somewhere in the 4e8 edge solves (on the MI355X each of the
    64 cells has such a run, so none can be held to a tight bar), and such
    switches bias the differences, so this is a report with a
    statistical bar: over cells whose gradient stands above the noise floor,
    median relative error <= 1e-3 and worst <= 5e-2 (measured: 2.2e-5 and
    2.4e-2, 14 of 40 within 1e-5).  The exact derivative is held to 1e-9
    against the oracle's dual numbers on 256^2 over 400 steps in four
    directions (test_adjoint_matches_oracle_dual_256_full_run)."""
    import torch
    say("case: adjoint 1024^2, 400 steps, FD at 64 cells")
    n, nsteps = 1024, 400
    c, dts, tg, S, prob = make(n, nsteps)
    L, ge, gB = gradients(c, prob)
    say("loss", L, "max|dL/deta1|", np.abs(ge).max(), "max|dL/dB|", np.abs(gB).max())
    e0 = torch.from_numpy(c["eta1"].copy()).cuda()
    B0 = torch.from_numpy(c["B"].copy()).cuda()
    S.branch_signature(prob.p, enable=1)
    base, _ = prob.forward(e0, B0)
    sig0 = S.branch_signature(prob.p)
    assert float(base.item()) == L
    rng = np.random.default_rng(2024)
    cy, cx = np.unravel_index(np.argmax(c["eta1"]), c["eta1"].shape)
    floor = {"eta1": 1e-6 * np.abs(ge).max(), "B": 1e-6 * np.abs(gB).max()}
    rels, switched = [], 0
    for k in range(64):
        i = int(np.clip(cx + rng.integers(-150, 151), 0, n - 1))
        j = int(np.clip(cy + rng.integers(-150, 151), 0, n - 1))
        which = "eta1" if k % 2 == 0 else "B"
        eps = 1e-4 if which == "eta1" else 0.5
        vals, sw = [], False
        for sgn in (1.0, -1.0):
            e = e0.clone(); b = B0.clone()
            if which == "eta1":
                e[j, i] += sgn * eps
            else:
                b[j, i] += sgn * eps
            loss, _ = prob.forward(e, b)
            vals.append(float(loss.item()))
            sw = sw or (S.branch_signature(prob.p) != sig0)
        switched += 1 if sw else 0
        fd = (vals[0] - vals[1]) / (2 * eps)
        g = ge[j, i] if which == "eta1" else gB[j, i]
        rel = abs(fd - g) / max(abs(g), 1e-300)
        informative = abs(g) > 1e3 * floor[which]
        if informative:
            rels.append(rel)
        say("cell %d" % k, (i, j), which, "adjoint %.10e fd %.10e rel %.2e%s%s" % (
            g, fd, rel, "" if informative else " (below noise floor)", " branch switch" if sw else ""))
        if not informative:
            assert abs(fd - g) <= 1e3 * floor[which] * 10
    S.branch_signature(prob.p, enable=0)
    rels = np.array(rels)
    say("informative cells", len(rels), "median rel", np.median(rels), "worst", rels.max(),
        "within 1e-5:", int((rels <= 1e-5).sum()), "runs with a branch switch:", switched)
    assert len(rels) >= 32
    assert np.median(rels) <= 1e-3
    assert rels.max() <= 5e-2
    S.close()


def test_adjoint_reports_a_dry_layer():
    """A bathymetry rising above the flat interface leaves the lower layer dry
    there: the adjoint steps record the non-wet edge without a host wait and the
    chain fails with MLSWE_ESTATE by the time it is closed."""
    import torch
    from paper_1803_01450_amd import binding
    from paper_1803_01450_amd.adjoint import GaugeMisfit
    say("case: adjoint 64x64 with a dry lower layer, error reported")
    n, nsteps = 64, 20
    c, dts, tg, S, prob = make(n, nsteps)
    B = c["B"].copy()
    B[20:30, 20:30] = c["eta2"] + 10.0   # bottom above the interface
    S.set_bathymetry(prob.p, B)
    e = torch.from_numpy(c["eta1"].copy()).cuda().requires_grad_(True)
    Bt = torch.from_numpy(B).cuda().requires_grad_(True)
    loss = GaugeMisfit.apply(e, Bt, prob)
    with pytest.raises(binding.MlsweError) as err:
        loss.backward()
    torch.cuda.synchronize()
    assert err.value.code == binding.ESTATE
    # the context stays usable: a wet problem differentiates afterwards
    S.set_bathymetry(prob.p, c["B"])
    L, ge, gB = gradients(c, prob)
    assert np.isfinite(L) and np.isfinite(ge).all() and np.isfinite(gB).all()
    S.close()
