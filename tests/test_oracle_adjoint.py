"""Pins of the oracle's derivative of the gauge misfit: the forward-mode dual
numbers through the oracle step agree with central finite differences of the
oracle's own double-precision loss, and the dual arithmetic reduces to known
derivatives on closed-form cases."""
import numpy as np

import oracle
from paper_1803_01450_amd import inputs


def small_problem(n=16, nsteps=24, every=4):
    c = inputs.adjoint_problem(n=n, L=16 * 1.6e3)
    dx = c["dx"]
    dts = np.full(nsteps, 0.9 * dx / 200.0)
    i0, j0, gn = 4, 5, 4
    tg = np.random.default_rng(3).uniform(-0.1, 0.1, (nsteps // every, gn, gn))
    return c, dx, dts, (i0, j0, gn), tg, every


def test_dual_matches_central_differences():
    c, dx, dts, gauge, tg, every = small_problem()
    rng = np.random.default_rng(7)
    res = []
    for k in range(3):
        ve = rng.standard_normal(c["eta1"].shape) if k != 1 else None
        vb = rng.standard_normal(c["B"].shape) if k != 0 else None
        L0, dL = oracle.gauge_loss(c["eta1"], c["B"], dx, c["eta2"], dts, every, gauge, tg, v_eta=ve, v_B=vb)
        assert L0 == oracle.gauge_loss(c["eta1"], c["B"], dx, c["eta2"], dts, every, gauge, tg)
        eps = 1e-6  # below the distance to the nearest limiter switch of this case
        pe = c["eta1"] + (eps * ve if ve is not None else 0)
        me = c["eta1"] - (eps * ve if ve is not None else 0)
        pb = c["B"] + (eps * vb if vb is not None else 0)
        mb = c["B"] - (eps * vb if vb is not None else 0)
        Lp = oracle.gauge_loss(pe, pb, dx, c["eta2"], dts, every, gauge, tg)
        Lm = oracle.gauge_loss(me, mb, dx, c["eta2"], dts, every, gauge, tg)
        fd = (Lp - Lm) / (2 * eps)
        res.append((fd, dL))
    # relative 2e-5 plus an absolute floor of 1e-6 of the largest derivative
    # (bathymetry perturbations of 1e-6 m ride on 4000 m depths and round)
    floor = 1e-6 * max(abs(d) for _, d in res)
    for k, (fd, dL) in enumerate(res):
        assert abs(fd - dL) <= 2e-5 * abs(dL) + floor, (k, fd, dL)


def test_dual_on_a_closed_form_case():
    """No steps sampled until the first sample at step `every` with a flat
    bottom at rest and zero target: a uniform eta1 shift e keeps the water at rest
    (walls), so L = N_gauge * n_samples * e^2 and dL/de = 2 N n e."""
    n, gn, every, nsteps = 8, 3, 2, 6
    eta1 = np.full((n, n), 0.3)
    B = np.full((n, n), -1000.0)
    dts = np.full(nsteps, 1.0)
    tg = np.zeros((nsteps // every, gn, gn))
    L, dL = oracle.gauge_loss(eta1, B, 100.0, -50.0, dts, every, (2, 2, gn), tg, v_eta=np.ones((n, n)))
    N = gn * gn * (nsteps // every)
    assert abs(L - N * 0.09) <= 1e-12 * N
    assert abs(dL - 2 * N * 0.3) <= 1e-10 * N
