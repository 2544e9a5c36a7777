"""The allocation-free flag entry point (mlswe_flag_noalloc) against mlswe_flag.

Flags are bytes, so the bar is bit-exact.  The calls run back to back on one
GPU with shrinking levels (1024^2, 256^2, 128^2, then a 64^2 grid of a second
context), so each call reads a scratch array an earlier, larger call wrote.
"""
import ctypes
import sys

import numpy as np
import pytest

from paper_1803_01450_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def flags_both(S, p, level, tau, nbuf=2):
    import torch
    nx, ny = S.shapes[p][level][:2]
    ref = S.flag(p, level, tau, nbuf)
    out = torch.full((ny, nx), 7, dtype=torch.uint8, device="cuda")
    S.flag_noalloc(p, level, tau, out, nbuf)
    S.synchronize()
    return ref, out.cpu().numpy()


def test_flag_noalloc_matches_flag():
    import torch
    from paper_1803_01450_amd.binding import Solver
    torch.cuda.init()
    c = inputs.amr_shoreline(n0=128, L=200e3, ratios=(2, 4))
    S = Solver()
    p = S.define(128, 128, c["dx0"], c["dx0"], c["r"], (2, 4))
    S.set_bathymetry(p, c["Bf"])
    S.set_state(p, 0, c["q0"])
    tau = [[4e-6, 8e-6]]
    say("case: 3-level shoreline 128^2, regrid then 4 coarse steps")
    S.advance(4, 4, tau)
    assert len(S.patches(p, 2)) > 0
    calls = 0
    for level, t in ((2, 8e-6), (1, 4e-6), (0, 4e-6), (0, 1e-3)):
        ref, got = flags_both(S, p, level, t)
        say("level", level, "tau", t, "flagged", int(ref.sum()), int(got.sum()))
        assert np.array_equal(ref, got)
        calls += 1
    assert calls == 4
    # a second context on the same GPU, smaller input: the scratch holds the
    # last call's bytes, which must not leak into these flags
    q = inputs.fixed_small()
    T = Solver()
    pq = T.define(64, 64, q["dx"], q["dx"], q["r"])
    T.set_bathymetry(pq, q["B"])
    T.set_state(pq, 0, q["q"])
    T.advance(5)
    for t in (1e-6, 2e-5):
        ref, got = flags_both(T, pq, 0, t, nbuf=1)
        say("64^2 tau", t, "flagged", int(ref.sum()), int(got.sum()))
        assert np.array_equal(ref, got)
    T.close()
    S.close()


def test_flag_noalloc_rejects_bad_calls():
    import torch
    from paper_1803_01450_amd import binding
    from paper_1803_01450_amd.binding import Solver, MlsweError
    torch.cuda.init()
    S = Solver()
    p = S.define(64, 64, 1000.0, 1000.0, 0.95)
    L = binding.lib()
    assert L.mlswe_flag_noalloc(S.h, p, 0, 1e-5, 2, None) == binding.EINVAL
    out = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    assert L.mlswe_flag_noalloc(S.h, p, 1, 1e-5, 2, ctypes.c_void_p(out.data_ptr())) == binding.EINVAL
    assert L.mlswe_flag_noalloc(S.h, p, 0, 1e-5, -1, ctypes.c_void_p(out.data_ptr())) == binding.EINVAL
    with pytest.raises(MlsweError):
        S.flag_noalloc(p, 0, 1e-5, torch.zeros((64, 63), dtype=torch.uint8, device="cuda"))
    S.close()
    # a level above the scratch size (4160^2 cells > 16 MiB) is refused
    say("case: 520^2 level 0 with a ratio-8 level of 4160^2")
    B = Solver()
    pb = B.define(520, 520, 1000.0, 1000.0, 0.95, (8,))
    big = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    rc = L.mlswe_flag_noalloc(B.h, pb, 1, 1e-5, 2, ctypes.c_void_p(big.data_ptr()))
    assert rc == binding.EINVAL
    assert b"scratch" in L.mlswe_last_error(B.h)
    B.close()
