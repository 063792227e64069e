"""GPU reverse step (lbf_adjoint_* through the C ABI): gradients of the
frozen fraction and of the front position against the host emulator of the
same passes, against central differences of the FP64 oracle, across
checkpoint windows, in float32, and through torch autograd."""
import math

import numpy as np
import pytest

import emulator
import synth
from adjoint_util import CASES, CASES_N14, central, checks, make_case, oracle_front, oracle_J

pytestmark = pytest.mark.gpu


def _grad(case, nsteps, window, objective="frozen_fraction"):
    from paper_2603_22902_amd.adjoint import frozen_fraction_and_gradient
    return frozen_fraction_and_gradient(case, nsteps, window, objective=objective)


@pytest.mark.parametrize("spec", CASES + CASES_N14, ids=lambda s: f"N{s[0]}_{s[1][1]}_{s[2][1]}")
def test_gpu_adjoint_matches_emulator_fp64(spec):
    case = make_case(*spec)
    print("adjoint case", spec, flush=True)
    J, g = _grad(case, 30, 30)
    Je, ge = emulator.adjoint(case["params"], case["phi"], case["T"], 30)
    assert abs(J - Je) <= 1e-13
    scale = np.abs(ge).max()
    assert np.abs(g["raw"] - ge).max() <= 1e-10 * scale, (g["raw"], ge)


def test_gpu_adjoint_matches_oracle_gradient():
    case = make_case(*CASES[1])
    prm = case["params"]
    n = 20
    J, g = _grad(case, n, 7)
    fj = lambda q: oracle_J(case, q, n)
    for key, idx, h, pick in checks(prm):
        fd = central(fj, prm, key, idx, h)
        assert abs(pick(g["raw"]) - fd) <= 1e-4 * abs(fd) + 1e-10, (key, idx, pick(g["raw"]), fd)


@pytest.mark.parametrize("N", [2, 3])
def test_gpu_adjoint_matches_oracle_gradient_multi_tile(N):
    """300 x 40 (two full 128-cell row tiles and a ragged third, several
    wall-normal chunks of the tiled passes), float64, 12 steps: the GPU
    reverse sweep against central differences of the FP64 oracle within
    1e-4."""
    spec = (N, ("wall", "open"), ("dirichlet", "dirichlet"), 70.0)
    case = make_case(*spec, shape=(300, 40))
    prm = case["params"]
    n = 12
    print("multi-tile adjoint", spec, flush=True)
    J, g = _grad(case, n, 5)
    assert abs(J - oracle_J(case, prm, n)) <= 1e-12
    fj = lambda q: oracle_J(case, q, n)
    scale = np.abs(g["raw"]).max()
    for key, idx, h, pick in checks(prm):
        fd = central(fj, prm, key, idx, 10 * h)
        assert abs(pick(g["raw"]) - fd) <= 1e-4 * abs(fd) + 1e-8 * scale, (key, idx, pick(g["raw"]), fd)


@pytest.mark.parametrize("N", [3, 4])
def test_gpu_adjoint_matches_emulator_across_tiles(N):
    """261 x 12 (the tiled collide reverse and gather across two tile
    boundaries and the periodic wrap): the GPU sweep against the host
    emulator of the same passes, float64, within 1e-10 of the gradient's
    scale."""
    spec = (N, ("wall", "open"), ("dirichlet", "dirichlet"), 70.0)
    case = make_case(*spec, shape=(261, 12))
    J, g = _grad(case, 10, 10)
    Je, ge = emulator.adjoint(case["params"], case["phi"], case["T"], 10)
    assert abs(J - Je) <= 1e-13
    assert np.abs(g["raw"] - ge).max() <= 1e-10 * np.abs(ge).max(), (g["raw"], ge)


def test_gpu_two_phase_tiled_reverse_matches_emulator():
    """130 x 1024: 2 x 512 = 1 024 tiles of the step geometry, past the
    count from which two phases take the tiled collide reverse (below it,
    one thread per cell).  The GPU sweep against the host emulator of the
    same passes, float64, within 1e-10 of the gradient's scale."""
    spec = (2, ("wall", "open"), ("dirichlet", "dirichlet"), 70.0)
    case = make_case(*spec, shape=(130, 1024))
    print("two-phase tiled reverse", spec, flush=True)
    J, g = _grad(case, 6, 6)
    Je, ge = emulator.adjoint(case["params"], case["phi"], case["T"], 6)
    assert abs(J - Je) <= 1e-13
    assert np.abs(g["raw"] - ge).max() <= 1e-10 * np.abs(ge).max(), (g["raw"], ge)


def test_gpu_front_gradient_matches_emulator_and_oracle():
    """The front-position objective (sum f_s psi per wall-layer cell): the
    float64 sweep against the emulator, and against central differences of
    the FP64 oracle's diagnostic front."""
    case = make_case(*CASES[1])
    prm = case["params"]
    n = 20
    print("front objective", CASES[1], flush=True)
    J, g = _grad(case, n, 7, objective="front")
    Je, ge = emulator.adjoint(prm, case["phi"], case["T"], n, objective="front")
    assert abs(J - Je) <= 1e-13 * max(1.0, Je)
    assert abs(J - oracle_front(case, prm, n)) <= 1e-12 * max(1.0, J)
    scale = np.abs(ge).max()
    assert np.abs(g["raw"] - ge).max() <= 1e-10 * scale, (g["raw"], ge)
    fj = lambda q: oracle_front(case, q, n)
    for key, idx, h, pick in checks(prm):
        fd = central(fj, prm, key, idx, h)
        assert abs(pick(g["raw"]) - fd) <= 1e-4 * abs(fd) + 1e-10, (key, idx, pick(g["raw"]), fd)


def test_checkpoint_window_does_not_change_the_gradient():
    """Recomputation from checkpoints reproduces the states bitwise, so
    every window gives the same gradient bitwise."""
    case = make_case(*CASES[0])
    ref = None
    for window in (1, 7, 40):
        J, g = _grad(case, 40, window)
        if ref is None:
            ref = (J, g["raw"])
        assert J == ref[0] and np.array_equal(g["raw"], ref[1]), window


@pytest.mark.parametrize("objective", ["frozen_fraction", "front"])
def test_full_tape_equals_checkpointed_gradient(objective):
    """window = 0 writes every state of the forward run into a device tape
    and recomputes nothing: the same states, so the same gradient bitwise."""
    case = make_case(*CASES[1], precision="fp32")
    J0, g0 = _grad(case, 25, 7, objective=objective)
    J1, g1 = _grad(case, 25, 0, objective=objective)
    assert J0 == J1 and np.array_equal(g0["raw"], g1["raw"])


def test_automatic_window_chooses_the_full_tape_when_it_fits():
    """window = None keeps a small run's whole trajectory on the device and
    gives the checkpointed gradient bitwise."""
    from paper_2603_22902_amd import Solver
    from paper_2603_22902_amd.adjoint import choose_window
    case = make_case(*CASES[0], precision="fp32")
    s = Solver(case["params"])
    assert choose_window(s, 25) == 0 and choose_window(s, 25, 7) == 7
    s.close()
    J0, g0 = _grad(case, 25, 7)
    J1, g1 = _grad(case, 25, None)
    assert J0 == J1 and np.array_equal(g0["raw"], g1["raw"])


def test_float32_adjoint_close_to_float64():
    """float32 storage and arithmetic: the gradient of the same case within
    1e-3 relative of the float64 one (measured ~1e-5)."""
    c64 = make_case(*CASES[0])
    c32 = make_case(*CASES[0], precision="fp32")
    _, g64 = _grad(c64, 30, 10)
    _, g32 = _grad(c32, 30, 10)
    scale = np.abs(g64["raw"]).max()
    err = np.abs(g32["raw"] - g64["raw"]).max() / scale
    print("fp32 vs fp64 gradient", err)
    assert err <= 1e-3


@pytest.mark.parametrize("spec", CASES_N14, ids=lambda s: f"N{s[0]}_{s[1][1]}_{s[2][1]}")
def test_float32_adjoint_close_to_float64_one_and_four_phases(spec):
    """The same bar for N = 1 (per-cell collide reverse) and N = 4 (tiled),
    both objectives."""
    for objective in ("frozen_fraction", "front"):
        print("fp32 adjoint", spec, objective, flush=True)
        _, g64 = _grad(make_case(*spec), 30, 10, objective)
        _, g32 = _grad(make_case(*spec, precision="fp32"), 30, 10, objective)
        scale = np.abs(g64["raw"]).max()
        err = np.abs(g32["raw"] - g64["raw"]).max() / scale
        print("fp32 vs fp64 gradient", err)
        assert err <= 1e-3


@pytest.mark.parametrize("objective", ["frozen_fraction", "front"])
def test_autograd_stefan_number_and_contact_angle(objective):
    """torch autograd through the reverse step: J(T_w, Ste, theta) with
    L = C_s (T_melt - T_w) / Ste for the freezing phase and
    cos_theta = [[0, cos t], [-cos t, 0]]; the gradient against central
    differences of GPU forward runs, within 1e-4."""
    import torch

    from paper_2603_22902_amd.adjoint import frozen_fraction, front_position

    base = make_case(*CASES[0])
    prm = base["params"]
    Cs = prm["cp_s"][0]
    n = 25

    def J_of(Tw, Ste, th):
        L = torch.stack([Cs * (synth.T_MELT - Tw) / Ste, torch.zeros((), dtype=torch.float64)])
        c, s0 = torch.cos(th), torch.zeros((), dtype=torch.float64)
        ct = torch.stack([torch.stack([s0, c]), torch.stack([-c, s0])])
        fn = front_position if objective == "front" else frozen_fraction
        return fn(Tw, L, ct, base, n, 10)

    x = [torch.tensor(v, dtype=torch.float64, requires_grad=True)
         for v in (prm["T_face"][0], 0.1, math.radians(70.0))]
    J = J_of(*x)
    J.backward()
    for k, h in enumerate((1e-6, 1e-6, 1e-6)):
        xp = [v.detach().clone() for v in x]
        xm = [v.detach().clone() for v in x]
        xp[k] += h
        xm[k] -= h
        with torch.no_grad():
            fd = (J_of(*xp).item() - J_of(*xm).item()) / (2 * h)
        ga = x[k].grad.item()
        print("autograd", k, ga, fd)
        assert abs(ga - fd) <= 1e-4 * abs(fd) + 1e-10, (k, ga, fd)
