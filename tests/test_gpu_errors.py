"""Failure detection on the device: a non-finite value in the state (here one
cell set to NaN on the host before the run) must end a run with MLSWE_ENAN in
every launch mode, in a batch as well (the other problems' flags stay clear),
and in a fixed-dt substep that asks for the wave speeds.  The wave-speed
maximum alone can miss a NaN (a comparison with NaN is false), so the x-sweep
checks the depths of the cells it updates."""
import sys

import numpy as np
import pytest

from paper_1803_01450_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def poisoned(c, field=1, i=20, j=30):
    q = np.array(c["q"], copy=True)
    q[field, j, i] = np.nan
    return q


@pytest.mark.parametrize("mode,field", [(0, 1), (1, 2), (2, 3)])
def test_nan_state_ends_run(mode, field):
    """A NaN depth or normal momentum is seen by the first x-sweep; a NaN
    transverse momentum reaches the depths in the y-sweep and is seen by the
    next step's x-sweep."""
    from paper_1803_01450_amd import binding
    say("case: NaN in field %d of one cell, 64x64 with a fine patch, advance, mode %d" % (field, mode))
    c = inputs.fixed_small()
    S = binding.Solver()
    p = S.define(64, 64, c["dx"], c["dx"], c["r"], (2,))
    S.set_bathymetry(p, c["Bf"])
    S.set_state(p, 0, poisoned(c, field=field))
    S.refine(p, 1, [(16, 16, 32, 32)])
    with pytest.raises(binding.MlsweError) as e:
        S.advance(3, 0, None, mode=mode)
    say("error", e.value)
    assert e.value.code == binding.ENAN
    S.close()


def test_nan_in_one_problem_of_a_batch():
    from paper_1803_01450_amd import binding
    say("case: three problems, NaN in the second, batched")
    c = inputs.fixed_small()
    S = binding.Solver()
    for k in range(3):
        p = S.define(64, 64, c["dx"], c["dx"], c["r"])
        S.set_bathymetry(p, c["B"])
        S.set_state(p, 0, poisoned(c, field=0) if k == 1 else c["q"])
    with pytest.raises(binding.MlsweError) as e:
        S.advance(2, mode=binding.BATCHED)
    say("error", e.value)
    assert e.value.code == binding.ENAN
    assert "problem 1" in str(e.value) or "non-finite" in str(e.value)
    S.close()


def test_nan_fixed_substep():
    from paper_1803_01450_amd import binding
    say("case: NaN in one cell, fixed substep with wave speeds")
    c = inputs.fixed_small()
    S = binding.Solver()
    p = S.define(64, 64, c["dx"], c["dx"], c["r"])
    S.set_bathymetry(p, c["B"])
    S.set_state(p, 0, poisoned(c, field=4))
    with pytest.raises(binding.MlsweError) as e:
        S.step_level(0, [7.0])
    assert e.value.code == binding.ENAN
    S.close()


def test_finite_state_keeps_flag_clear():
    from paper_1803_01450_amd import binding
    say("case: finite state, fixed substeps, wave speeds returned")
    c = inputs.fixed_small()
    S = binding.Solver()
    p = S.define(64, 64, c["dx"], c["dx"], c["r"])
    S.set_bathymetry(p, c["B"])
    S.set_state(p, 0, c["q"])
    for _ in range(3):
        sm = S.step_level(0, [7.0])
        assert np.all(np.isfinite(sm))
    S.close()
