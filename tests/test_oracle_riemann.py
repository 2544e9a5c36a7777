"""Pins of the oracle's layered edge solve against what the model fixes.

The paper does not write the solver (Sec. 1 cites it); the model it relies on is
the two-layer shallow-water system with layer 1 on top (Sec. 2.1).  These tests
check the oracle's edge solve against properties of that model computed here
from first principles: the jump of flux minus source, the eigen-structure of the
quasi-linear matrix, the linearised wave speeds, lake at rest, walls.
"""
import mpmath as mp
import numpy as np

import oracle

G = 9.81


def jump(qL, qR, r):
    """Flux difference minus integrated source across an edge, in flux form:
    x-fluxes (h1u1, h1u1^2 + g h1^2/2, h1u1v1, h2u2, h2u2^2 + g h2^2/2, h2u2v2),
    sources -g h1 (h2+B)_x and -g h2 (r h1 + B)_x with edge-averaged depths.
    Evaluated in 40-digit arithmetic: the flux form cancels large terms."""
    mp.mp.dps = 40
    g = mp.mpf(G)
    rr = mp.mpf(r)

    def flux(q):
        h1, m1, t1, h2, m2, t2, B = [mp.mpf(float(x)) for x in q]
        u1 = m1 / h1 if h1 > 0 else mp.mpf(0)
        u2 = m2 / h2 if h2 > 0 else mp.mpf(0)
        return [m1, m1 * u1 + g * h1 * h1 / 2, t1 * u1, m2, m2 * u2 + g * h2 * h2 / 2, t2 * u2]
    fL, fR = flux(qL), flux(qR)
    L = [mp.mpf(float(x)) for x in qL]
    R = [mp.mpf(float(x)) for x in qR]
    hb1 = (L[0] + R[0]) / 2
    hb2 = (L[3] + R[3]) / 2
    psi = [mp.mpf(0)] * 6
    psi[1] = -g * hb1 * ((R[3] + R[6]) - (L[3] + L[6]))
    psi[4] = -g * hb2 * ((rr * R[0] + R[6]) - (rr * L[0] + L[6]))
    return np.array([float((fR[c] - fL[c]) - psi[c]) for c in range(6)])


def wet_state(rng):
    B = rng.uniform(-4000, -500)
    eta2 = rng.uniform(-300, -100)
    eta1 = rng.uniform(-2, 2)
    h2 = eta2 - B
    h1 = eta1 - eta2
    u1, v1, u2, v2 = rng.uniform(-1.5, 1.5, 4)
    return np.array([h1, h1 * u1, h1 * v1, h2, h2 * u2, h2 * v2, B])


def test_fwave_sum_equals_jump_all_wet():
    rng = np.random.default_rng(1)
    for _ in range(400):
        r = rng.uniform(0.9, 0.99)
        qL, qR = wet_state(rng), wet_state(rng)
        out = oracle.riemann(qL, qR, r=r)
        d = jump(qL, qR, r)
        s = out["Z"].sum(axis=0)
        scale = np.abs(d).max()
        assert np.abs(s - d).max() <= 1e-11 * scale, (s, d)
        # the fluctuations split the same jump
        assert np.abs(out["amdq"] + out["apdq"] - d).max() <= 1e-11 * scale


def test_4x4_solve_matches_numpy():
    rng = np.random.default_rng(2)
    for _ in range(200):
        r = rng.uniform(0.9, 0.99)
        qL, qR = wet_state(rng), wet_state(rng)
        out = oracle.riemann(qL, qR, r=r)
        s = out["s"][:4]
        beta = out["Z"][:4, 0]
        alpha = out["Z"][:4, 3] / beta
        R = np.vstack([np.ones(4), s, alpha, alpha * s])
        d = jump(qL, qR, r)
        rhs = np.array([d[0], d[1], d[3], d[4]])
        ref = np.linalg.solve(R, rhs)
        assert np.allclose(beta, ref, rtol=1e-9, atol=1e-12 * np.abs(rhs).max())


def test_eigenvectors_of_quasilinear_matrix():
    """For L = R the Roe state is the state itself; the vectors (1, s, alpha,
    alpha s) satisfy the first three rows of A r = s r exactly and the fourth to
    O(eps), eps = (1-r) h1 h2 / (h1+h2)^2, because the speeds are the
    first-order approximations in (1-r)."""
    rng = np.random.default_rng(3)
    for _ in range(100):
        r = rng.uniform(0.9, 0.99)
        q = wet_state(rng)
        q2 = q.copy(); q2[1] *= 1.0000001  # avoid a zero jump; same Roe state to 1e-7
        out = oracle.riemann(q, q2, r=r)
        h1, m1, _, h2, m2, _, _ = q
        u1, u2 = m1 / h1, m2 / h2
        A = np.array([[0, 1, 0, 0],
                      [G * h1 - u1 ** 2, 2 * u1, G * h1, 0],
                      [0, 0, 0, 1],
                      [r * G * h2, 0, G * h2 - u2 ** 2, 2 * u2]])
        eps = (1 - r) * h1 * h2 / (h1 + h2) ** 2
        for p in range(4):
            s = out["s"][p]
            al = out["Z"][p, 3] / out["Z"][p, 0]
            v = np.array([1.0, s, al, al * s])
            res = A @ v - s * v
            nv = np.abs(v).max() * max(abs(s), 1.0) * 10
            assert np.abs(res[:3]).max() <= 1e-7 * nv
            assert abs(res[3]) <= 5 * eps * G * (h1 + h2) * np.abs(v).max()


def test_speeds_at_rest_and_quartic_roots():
    """At u = 0 the speeds are sqrt(g(h1+h2)) and sqrt(g(1-r)h1h2/(h1+h2)); these
    approximate the roots of l^4 - g(h1+h2) l^2 + g^2 (1-r) h1 h2 = 0 to O(eps)."""
    for (h1, h2, r) in [(200.0, 3800.0, 0.95), (100.0, 100.0, 0.97), (500.0, 1500.0, 0.9)]:
        q = np.array([h1, 0, 0, h2, 0, 0, -(h1 + h2)])
        q2 = q.copy(); q2[0] += 1e-9; q2[6] -= 1e-9  # tiny jump, same surfaces
        out = oracle.riemann(q, q2, r=r)
        hb1 = h1 + 0.5e-9
        H = hb1 + h2
        ce = np.sqrt(G * H)
        ci = np.sqrt(G * (1 - r) * hb1 * h2 / H)
        s = out["s"]
        assert abs(s[3] - ce) <= 2 * np.spacing(ce) and abs(s[0] + ce) <= 2 * np.spacing(ce)
        assert abs(s[2] - ci) <= 4 * np.spacing(ci) and abs(s[1] + ci) <= 4 * np.spacing(ci)
        disc = np.sqrt(H * H - 4 * (1 - r) * hb1 * h2)
        lam_e = np.sqrt(G * (H + disc) / 2)
        lam_i = np.sqrt(G * (H - disc) / 2)
        eps = (1 - r) * hb1 * h2 / H ** 2
        assert abs(s[3] - lam_e) / lam_e <= 2 * eps
        assert abs(s[2] - lam_i) / lam_i <= 2 * eps
    # worked numbers: h1 = 200, h2 = 3800, r = 0.95 give an external speed of 197.855 m/s
    H = 4000.0
    disc = np.sqrt(H * H - 4 * 0.05 * 200 * 3800)
    assert abs(np.sqrt(G * (H + disc) / 2) - 197.855) < 1e-3
    assert abs(np.sqrt(G * (H - disc) / 2) - 9.6653) < 1e-3


def test_lake_at_rest_all_wet_dry_patterns():
    """Flat surfaces (eta1 = 0, eta2 = -100 where the lower layer exists) over
    varying bathymetry give no fluctuations, for every wet-order-valid pattern
    on both sides: both layers wet, top layer only, dry land."""
    def cell(kind):
        if kind == "wet2":
            B = -1500.0
            return np.array([100.0, 0, 0, -100.0 - B, 0, 0, B])
        if kind == "top":
            B = -60.0
            return np.array([0.0 - B, 0, 0, 0, 0, 0, B])
        B = 25.0
        return np.array([0.0, 0, 0, 0, 0, 0, B])
    for a in ["wet2", "top", "land"]:
        for b in ["wet2", "top", "land"]:
            out = oracle.riemann(cell(a), cell(b))
            assert np.all(out["amdq"] == 0.0) and np.all(out["apdq"] == 0.0), (a, b, out)


def test_wall_gives_zero_mass_flux():
    """Top layer moving towards land higher than its surface: reflecting edge, so
    the edge mass flux m_L + A-dQ[0] vanishes (to rounding of the wave strengths)
    and nothing enters the dry cell."""
    qL = np.array([50.0, 50.0 * 0.7, 50.0 * 0.2, 0, 0, 0, -50.0])
    qR = np.array([0.0, 0, 0, 0, 0, 0, 10.0])
    out = oracle.riemann(qL, qR)
    assert abs(qL[1] + out["amdq"][0]) <= 4 * np.spacing(qL[1])
    assert np.all(out["apdq"] == 0.0)
    # the lower layer against a bottom step above its surface: also a wall
    qL = np.array([100.0, 10.0, 0, 400.0, 400.0 * 0.5, 0, -500.0])
    qR = np.array([140.0, 0, 0, 0.0, 0, 0, -40.0])
    out = oracle.riemann(qL, qR)
    assert abs(qL[4] + out["amdq"][3]) <= 4 * np.spacing(qL[4])
    assert out["apdq"][3] == 0.0 and out["apdq"][4] == 0.0


def test_overtopping_moves_water_onto_land():
    """Surface above the dry neighbour's ground: water at rest flows onto it
    (positive edge mass flux) and the f-wave sum still equals the jump."""
    qL = np.array([60.0, 0, 0, 0, 0, 0, -50.0])   # eta1 = 10
    qR = np.array([0.0, 0, 0, 0, 0, 0, 5.0])      # ground at 5 < 10
    out = oracle.riemann(qL, qR)
    F = qL[1] + out["amdq"][0]
    assert F > 0.0
    d = jump(qL, np.array([0.0, 0, 0, 0, 0, 0, 5.0]), 0.95)
    # with a dry right side the source term uses the surface jump of the wet layer
    s = out["Z"].sum(axis=0)
    assert abs(s[0] - d[0]) <= 1e-12 * 60


def test_mirror_symmetry():
    """Solving (L, R) equals the mirror image of solving (R*, L*) with the normal
    momenta negated: A-dQ <-> A+dQ with the normal-momentum components negated."""
    rng = np.random.default_rng(5)
    flip = np.array([1, -1, 1, 1, -1, 1.0])
    for _ in range(100):
        qL, qR = wet_state(rng), wet_state(rng)
        mL = qR * np.array([1, -1, 1, 1, -1, 1, 1.0])
        mR = qL * np.array([1, -1, 1, 1, -1, 1, 1.0])
        a = oracle.riemann(qL, qR)
        b = oracle.riemann(mL, mR)
        sc = np.abs(a["amdq"]).max() + np.abs(a["apdq"]).max()
        assert np.abs(a["amdq"] - flip * b["apdq"]).max() <= 1e-10 * sc
        assert np.abs(a["apdq"] - flip * b["amdq"]).max() <= 1e-10 * sc
        assert np.allclose(np.sort(np.abs(a["s"][:4])), np.sort(np.abs(b["s"][:4])), rtol=1e-12)


def test_single_layer_branch_is_einfeldt_fwave():
    """Lower layer dry on both sides: the top layer alone is single-layer shallow
    water over B; its two waves use the Einfeldt speeds and sum to the jump."""
    rng = np.random.default_rng(6)
    for _ in range(100):
        BL, BR = rng.uniform(-300, -60, 2)
        hL, hR = 10.0 - BL + rng.uniform(-1, 1), 10.0 - BR + rng.uniform(-1, 1)
        uL, uR = rng.uniform(-2, 2, 2)
        qL = np.array([hL, hL * uL, 0, 0, 0, 0, BL])
        qR = np.array([hR, hR * uR, 0, 0, 0, 0, BR])
        out = oracle.riemann(qL, qR)
        d = jump(qL, qR, 0.95)
        s = out["Z"].sum(axis=0)
        assert np.abs(s[:2] - d[:2]).max() <= 1e-10 * np.abs(d[:2]).max()
        cL, cR = np.sqrt(G * hL), np.sqrt(G * hR)
        uh = (np.sqrt(hL) * uL + np.sqrt(hR) * uR) / (np.sqrt(hL) + np.sqrt(hR))
        ch = np.sqrt(G * 0.5 * (hL + hR))
        assert np.isclose(out["s"][0], min(uL - cL, uh - ch), rtol=1e-13)
        assert np.isclose(out["s"][3], max(uR + cR, uh + ch), rtol=1e-13)
        assert np.all(out["Z"][[1, 2, 5]] == 0.0)
