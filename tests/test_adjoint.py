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


@pytest.mark.parametrize("N", [3, 4])
def test_emulated_adjoint_matches_oracle_gradient_across_tiles(N):
    """On a 261 x 12 grid (two full 128-cell row tiles and a 5-cell ragged
    one, periodic wrap across the last), so that the tiled collide reverse
    and the tiled gather run across tile boundaries: the emulated reverse
    sweep against central differences of the FP64 oracle within 1e-4, over
    10 steps."""
    spec = (N, ("wall", "open"), ("dirichlet", "dirichlet"), 70.0)
    case = make_case(*spec, shape=(261, 12))
    prm = case["params"]
    n = 10
    J, g = emulator.adjoint(prm, case["phi"], case["T"], n)
    assert 0.0 < J < 1.0
    assert abs(J - oracle_J(case, prm, n)) <= 1e-12
    fj = lambda q: oracle_J(case, q, n)
    scale = max(abs(g[k]) for k in range(22))
    for key, idx, h, pick in checks(prm):
        fd = central(fj, prm, key, idx, 10 * h)
        assert abs(pick(g) - fd) <= 1e-4 * abs(fd) + 1e-8 * scale, (key, idx, pick(g), fd)


def test_float32_overflow_of_the_reverse_sweep_is_reported():
    """A bulk two-phase mixture (phi_2 = phi_3 = 1/2 across the far field)
    drives the pairwise normal's Jacobian, A/|v| with |v| at rounding level,
    to about 1e8 per step; float32 cannot hold that over a few steps.  The
    sweep must then return LBF_ENAN (as lbf_adjoint_gradient does), not a
    non-finite gradient with a success status; float64 stays finite."""
    from paper_2603_22902_amd.lbfreeze import LBF_ENAN
    case = make_case(3, ("wall", "open"), ("dirichlet", "dirichlet"), 70.0, precision="fp32",
                     shape=(150, 21))
    phi = case["phi"].copy()
    gas = phi[1].copy()
    phi[1] = 0.5 * gas
    phi[2] = phi[2] + 0.5 * gas
    prm = case["params"]
    with pytest.raises(emulator.EmulatorError) as e:
        emulator.adjoint(prm, phi, case["T"], 7)
    assert e.value.rc == LBF_ENAN
    assert not np.all(np.isfinite(e.value.grad)) or not np.isfinite(e.value.J)
    p64 = dict(prm, precision="fp64")
    J, g = emulator.adjoint(p64, phi, case["T"], 7)
    assert np.isfinite(J) and np.all(np.isfinite(g))
