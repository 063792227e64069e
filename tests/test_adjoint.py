"""CPU checks of the hand-written reverse step (host emulator of the HIP
passes, lbf_adjoint.h): gradients of the frozen fraction and of the front
position against central finite differences of the same forward step and of
the FP64 oracle."""
import numpy as np
import pytest

import emulator
from adjoint_util import CASES, CASES_N14, central, checks, make_case, oracle_front, oracle_J

pytestmark = pytest.mark.skipif(not emulator.available(), reason="emulator not built")


@pytest.mark.parametrize("spec", CASES, ids=lambda s: f"N{s[0]}_{s[1][1]}_{s[2][1]}")
@pytest.mark.parametrize("nsteps", [6, 30])
def test_emulated_adjoint_matches_central_differences(spec, nsteps):
    """float64: the reverse sweep is the exact derivative of the forward
    step, so it meets central differences (O(h^2) + rounding / h) at 1e-6."""
    case = make_case(*spec)
    prm = case["params"]
    J, g = emulator.adjoint(prm, case["phi"], case["T"], nsteps)
    assert 0.0 < J < 1.0
    fj = lambda q: emulator.adjoint(q, case["phi"], case["T"], nsteps)[0]
    scale = max(abs(g[k]) for k in range(22))
    for key, idx, h, pick in checks(prm):
        fd = central(fj, prm, key, idx, h)
        assert abs(pick(g) - fd) <= 1e-6 * abs(fd) + 1e-9 * scale, (key, idx, pick(g), fd)


def test_emulated_adjoint_matches_oracle_gradient():
    """The gradient of the FP64 oracle by central differences (the oracle
    shares no code with the reverse step) within 1e-4."""
    case = make_case(*CASES[1])
    prm = case["params"]
    n = 20
    J, g = emulator.adjoint(prm, case["phi"], case["T"], n)
    assert abs(J - oracle_J(case, prm, n)) <= 1e-12
    fj = lambda q: oracle_J(case, q, n)
    for key, idx, h, pick in checks(prm):
        fd = central(fj, prm, key, idx, h)
        assert abs(pick(g) - fd) <= 1e-4 * abs(fd) + 1e-10, (key, idx, pick(g), fd)


def test_zero_steps_gradient_is_the_final_state_term():
    """n = 0: only the dependence of the start on L remains (no step, so no
    wall or wetting terms), and it matches central differences."""
    case = make_case(*CASES[0])
    prm = case["params"]
    J, g = emulator.adjoint(prm, case["phi"], case["T"], 0)
    assert g[0] == 0.0 and g[1] == 0.0 and not np.any(g[6:])
    fj = lambda q: emulator.adjoint(q, case["phi"], case["T"], 0)[0]
    fd = central(fj, prm, "latent", 0, 1e-5)
    assert abs(g[2] - fd) <= 1e-6 * abs(fd) + 1e-12


@pytest.mark.parametrize("spec", CASES, ids=lambda s: f"N{s[0]}_{s[1][1]}_{s[2][1]}")
def test_emulated_front_gradient_matches_central_differences(spec):
    """The front-position objective: its own seed (no normalisation by the
    freezing volume), checked like the frozen fraction."""
    case = make_case(*spec)
    prm = case["params"]
    n = 12
    J, g = emulator.adjoint(prm, case["phi"], case["T"], n, objective="front")
    Jf, gf = emulator.adjoint(prm, case["phi"], case["T"], n)
    assert J > 0.0 and abs(J - Jf) > 1e-3 * J  # a different objective
    fj = lambda q: emulator.adjoint(q, case["phi"], case["T"], n, objective="front")[0]
    scale = max(abs(g[k]) for k in range(22))
    for key, idx, h, pick in checks(prm):
        fd = central(fj, prm, key, idx, h)
        assert abs(pick(g) - fd) <= 1e-6 * abs(fd) + 1e-9 * scale, (key, idx, pick(g), fd)


def test_emulated_front_gradient_matches_oracle():
    """The front position and its gradient against the FP64 oracle's own
    diagnostic front, by central differences, within 1e-4."""
    case = make_case(*CASES[0])
    prm = case["params"]
    n = 20
    J, g = emulator.adjoint(prm, case["phi"], case["T"], n, objective="front")
    assert abs(J - oracle_front(case, prm, n)) <= 1e-12 * max(1.0, J)
    fj = lambda q: oracle_front(case, q, n)
    for key, idx, h, pick in checks(prm):
        fd = central(fj, prm, key, idx, h)
        assert abs(pick(g) - fd) <= 1e-4 * abs(fd) + 1e-10, (key, idx, pick(g), fd)


@pytest.mark.parametrize("spec", CASES_N14, ids=lambda s: f"N{s[0]}_{s[1][1]}_{s[2][1]}")
@pytest.mark.parametrize("nsteps", [6, 30])
def test_emulated_adjoint_one_and_four_phases(spec, nsteps):
    """N = 1 and N = 4: the reverse sweep against central differences of the
    same forward step (steps ten times those of checks(), see CASES_N14),
    at the 1e-6 relative bar."""
    case = make_case(*spec)
    prm = case["params"]
    J, g = emulator.adjoint(prm, case["phi"], case["T"], nsteps)
    assert 0.0 < J < 1.0
    fj = lambda q: emulator.adjoint(q, case["phi"], case["T"], nsteps)[0]
    scale = max(abs(g[k]) for k in range(22))
    for key, idx, h, pick in checks(prm):
        fd = central(fj, prm, key, idx, 10.0 * h)
        assert abs(pick(g) - fd) <= 1e-6 * abs(fd) + 1e-9 * scale, (key, idx, pick(g), fd)


@pytest.mark.parametrize("spec", CASES_N14, ids=lambda s: f"N{s[0]}_{s[1][1]}_{s[2][1]}")
def test_emulated_adjoint_one_and_four_phases_match_oracle(spec):
    """N = 1 and N = 4: J of both objectives equals the FP64 oracle's, and the
    frozen fraction's gradient meets the oracle's central differences within
    1e-4."""
    case = make_case(*spec)
    prm = case["params"]
    n = 20
    J, g = emulator.adjoint(prm, case["phi"], case["T"], n)
    assert abs(J - oracle_J(case, prm, n)) <= 1e-12
    Jf, _ = emulator.adjoint(prm, case["phi"], case["T"], n, objective="front")
    assert abs(Jf - oracle_front(case, prm, n)) <= 1e-12 * max(1.0, Jf)
    fj = lambda q: oracle_J(case, q, n)
    for key, idx, h, pick in checks(prm):
        fd = central(fj, prm, key, idx, h)
        assert abs(pick(g) - fd) <= 1e-4 * abs(fd) + 1e-10, (key, idx, pick(g), fd)
