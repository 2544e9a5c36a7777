"""Planted slips: each plausible mistake below, written into a copy of the
oracle's sources and compiled, must fail at least one of the oracle's pins
(the 50-digit brute force of the step, the MC table, the ghost cells'
time interpolation, the substep fractions, a lake at rest, mass with walls).

The slips are the ones a reader could make when restating the method:

* the downwind instead of the upwind neighbour edge in the limiter ratio;
* the minmod limiter in place of MC;
* the ghost-cell fraction (k + 1) / r_t instead of k / r_t for the k-th fine
  substep (Sec. 2);
* the old and new coarse states swapped in the time interpolation;
* the internal-wave speed without the hyperbolicity factor;
* the density ratio left out of the lower layer's pressure jump;
* the correction flux with the wrong sign;
* the lower layer's transverse momentum carried with the upper layer's
  transverse velocity;
* a dry neighbour taken as a wall when the wet surface lies above its bottom
  (and as open when below).
"""
import os
import shutil

import numpy as np
import pytest

import oracle
import test_oracle_bruteforce as BF
import test_oracle_limiter_ghost as LG

SLIPS = {
    "limiter_downwind_edge": ("ora_core.hpp", "const Waves<T>& U = (sv > 0.0) ? Wm : Wp;",
                              "const Waves<T>& U = (sv > 0.0) ? Wp : Wm;"),
    "minmod_for_mc": ("ora_core.hpp", "  T m = minv(minv(a, T(2.0)), b);\n",
                      "  T m = minv(T(1.0), th);\n"),
    "ghost_fraction_k_plus_1": ("ora_amr.cpp", "rc = adv(H, l + 1, dtf, double(k) / double(r));",
                                "rc = adv(H, l + 1, dtf, double(k + 1) / double(r));"),
    "old_new_swapped": ("ora_amr.cpp", "CoarseSrc S{&Lc, Lc.q[1 - Lc.cur].data(), Lc.q[Lc.cur].data(), th};",
                        "CoarseSrc S{&Lc, Lc.q[Lc.cur].data(), Lc.q[1 - Lc.cur].data(), th};"),
    "no_hyperbolicity_factor": ("ora_core.hpp", "T ci = sqrt_((((T(P.gp) * hb1) * hb2) * iH) * kap);",
                                "T ci = sqrt_((((T(P.gp) * hb1) * hb2) * iH));"),
    "no_density_ratio_in_lower_jump": ("ora_core.hpp", "T J2 = fma_(T(P.r), R.h1 - L.h1, R.eta2 - L.eta2);",
                                       "T J2 = R.eta2 - L.eta2;"),
    "correction_sign": ("ora_core.hpp", "T sg = T(sv > 0.0 ? 0.5 : -0.5);", "T sg = T(sv > 0.0 ? -0.5 : 0.5);"),
    "lower_transverse_with_upper_velocity": ("ora_core.hpp", "      W.Z[p][5] = ba * wb2;", "      W.Z[p][5] = ba * wb1;"),
    "wall_test_inverted": ("ora_core.hpp", "bool wall = wallIfDryR || val(etaL) <= val(botR);",
                           "bool wall = wallIfDryR || val(etaL) > val(botR);"),
}


def lake_at_rest_motion():
    """Largest momentum after 20 steps of a lake at rest over rough bathymetry."""
    rng = np.random.default_rng(5)
    n = 16
    B = -1500.0 + 200.0 * rng.uniform(-1, 1, (n, n))
    q = np.zeros((6, n, n))
    q[3] = -300.0 - B
    q[0] = 300.0
    qo, _, _ = oracle.fixed_steps(B, q, 1000.0, 1000.0, [3.0] * 20, r=0.95)
    return max(np.abs(qo[f]).max() for f in (1, 2, 4, 5))


def failed_pins():
    """Names of the pins that fail with the oracle currently loaded."""
    out = []
    for kind, nx, ny, seed in BF.CASES:
        err, serr, _, _ = BF.compare(kind, nx, ny, seed)
        if not (np.all(err <= BF.TOL) and serr <= BF.TOL):
            out.append("bruteforce_" + kind)
    if LG.mc_table_mismatch():
        out.append("mc_table")
    worst, _ = LG.ghost_fill_mismatch(thetas=(0.25, 0.5))
    if worst != 0.0:
        out.append("ghost_fill")
    if LG.subcycle_mismatch((2, 4)) != 0.0:
        out.append("subcycle_fractions")
    if lake_at_rest_motion() > 1e-9:
        out.append("lake_at_rest")
    return out


def test_unmodified_oracle_passes_every_pin():
    assert failed_pins() == []


@pytest.mark.parametrize("name", sorted(SLIPS))
def test_planted_slip_fails_a_pin(name, tmp_path):
    fname, old, new = SLIPS[name]
    for src in oracle.sources():
        shutil.copy(src, tmp_path)
    path = os.path.join(tmp_path, fname)
    text = open(path).read()
    assert text.count(old) == 1, "slip anchor not found once: " + old
    with open(path, "w") as f:
        f.write(text.replace(old, new))
    lib = oracle.compile_to(str(tmp_path), os.path.join(tmp_path, "liboracle_slip.so"))
    with oracle.variant(lib):
        failed = failed_pins()
    assert failed, name + " passed every pin"
