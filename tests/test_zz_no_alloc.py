"""lbf_diagnostics_noalloc (the static-scratch variant) against
lbf_diagnostics, through the C ABI, on two calls in a row: a 3D four-phase
case that uses every row of the scratch array, then a smaller 2D case that
uses 16 rows and leaves the first call's rows behind.  The two entry points
run the same kernels with the same block count, so the values must be
identical bit for bit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _pair(case, steps):
    from paper_2603_22902_amd import Solver
    s = Solver(case["params"])
    s.init_case(case)
    s.lbf_step(steps)
    ref = s.lbf_diagnostics()
    got = s.lbf_diagnostics(noalloc=True)
    for k in ref:
        assert np.array_equal(np.asarray(got[k]), np.asarray(ref[k])), (k, got[k], ref[k])
    return got


def test_noalloc_diagnostics_match_twice_second_smaller():
    big = synth.stress(synth.small(dim=3, shape=(96, 96, 96), nphase=4, precision="fp32"), phi_noise=1e-6)
    small = synth.stress(synth.small(dim=2, shape=(64, 64), nphase=2, precision="fp64"))
    a = _pair(big, 5)
    b = _pair(small, 5)
    assert len(a["mass"]) == 4 and len(b["mass"]) == 2
    assert not a["nonfinite"] and not b["nonfinite"]
