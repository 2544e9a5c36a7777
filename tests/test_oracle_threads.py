"""The oracle's multi-threaded timing mode (rows cut into strips, each stepped
as a box on its own thread) against its plain one-box stepping: the same
arithmetic on the same stencils, so the states agree bit for bit."""
import numpy as np

import oracle
from paper_1803_01450_amd import inputs


def test_threaded_steps_equal_one_box_steps():
    c = inputs.roofline_grid(n=96, L=409.6e3 * 96 / 4096)
    B = c["B"][:80, :]
    q = np.ascontiguousarray(c["q"][:, :80, :])
    dt = 0.9 * c["dx"] / np.sqrt(9.81 * 4000.0)
    H = oracle.Hierarchy(96, 80, c["dx"], c["dx"], r=c["r"])
    H.set_bathymetry(B)
    H.set_state(0, q)
    for _ in range(3):
        H.step_level(0, dt)
    ref = H.state(0)
    for threads in (1, 3, 7):
        _, sec, got = oracle.time_fixed_mt(B, q, c["dx"], c["dx"], 3, dt, threads, r=c["r"], want_state=True)
        assert sec > 0.0
        assert np.array_equal(got, ref), threads
