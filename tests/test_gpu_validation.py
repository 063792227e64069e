"""Validation of the HIP path against values the paper prints and closed
forms.

Table 1 (Sec. 4.1): a liquid film frozen through on a cold wall keeps its
mass, so its final height over the initial one is rho_l/rho_s; the paper
reports agreement within 5 % over rho_s/rho_l = 0.7..1 and Ste 0.1..0.2.
All 21 films run together as one batch (the batched path of the library).

Table 2 (Sec. 4.3): equilibrium wetting lengths of a Janus droplet on a
wall for four contact angles; and the Neumann closed form for three equal
surface tensions (120 deg junctions: a floating lens's thickness over width
is tan 30 deg).  Equal densities and viscosities in both: the static
equilibrium depends only on the surface tensions and the wall angles, and
equal properties relax fastest.
"""
import math
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_table1_full_freeze_sweep():
    from paper_2603_22902_amd import Solver
    from paper_2603_22902_amd.batch import Batch

    rows = np.loadtxt(os.path.join(GOLDEN, "table1_film_full_freeze.txt"))
    h0, ny, nx = 32.0, 128, 4
    runs = []
    for r in rows:
        for ste in (0.1, 0.15, 0.2):
            c = synth.film(ny=ny, nx=nx, h0=h0, ratio=float(r[0]), ste=ste, precision="fp64")
            s = Solver(c["params"])
            s.init_case(c)
            d0 = s.lbf_diagnostics()
            runs.append((float(r[0]), ste, float(r[1]), s, d0["vol"][0], d0["mass"][0]))
    b = Batch([run[3] for run in runs])
    b.capture()
    frozen = [False] * len(runs)
    for chunk in range(80):
        b.replay(2500)
        b.synchronize()
        for k, run in enumerate(runs):
            d = run[3].lbf_diagnostics()
            frozen[k] = d["vol_solid"][0] >= 0.999 * d["vol"][0]
        if all(frozen):
            break
    print(f"full freeze after {runs[0][3].step_count()} steps")
    worst = 0.0
    for (ratio, ste, analytic, s, v0, m0), fz in zip(runs, frozen):
        d = s.lbf_diagnostics()
        hf = d["vol"][0] / v0
        err = abs(hf - analytic) / analytic
        worst = max(worst, err)
        print(f"rho_s/rho_l {ratio:.2f} Ste {ste:.2f}: h_f/h_0 {hf:.4f} analytic {analytic:.4f} "
              f"error {err:.2e} mass drift {d['mass'][0] / m0 - 1:.2e} frozen {fz}")
        assert fz, (ratio, ste)
        # measured worst 1.6e-3; the paper's own numbers deviate by up to 2.4e-2
        assert err < 5e-3, (ratio, ste, hf, analytic)
        # the lagged divergence (reading R2) conserves sum phi exactly only
        # at u = 0; over ~1e5 steps of expansion flow the phase mass drifts
        # by O(1e-3) (measured 1.6e-3 at rho_s/rho_l = 0.7)
        assert abs(d["mass"][0] / m0 - 1.0) < 5e-3, (ratio, ste)
    print("worst relative error", worst)


def _three_fluids(shape, phi, cth, eps=5.0, sigma=0.01):
    """Inert fluids of equal density and viscosity, uniform T above melting,
    adiabatic walls top and bottom, periodic x."""
    phases = [synth.inert_phase(1.0, lam=0.1) for _ in range(3)]
    prm = synth.make_params(2, shape, phases, sigma=sigma, precision="fp64",
                            therm_bc=("adiabatic", "adiabatic"), T_face=(1.0, 1.0),
                            cos_theta=cth, eps=eps)
    return {"params": prm, "phi": phi, "T": np.ones(phi.shape[1:])}


def _relax(batch, solvers, measure, chunk=2500, max_chunks=60, tol=2e-4):
    """Replay until the measured lengths change by less than tol per chunk."""
    last = None
    for _ in range(max_chunks):
        batch.replay(chunk // 2)
        batch.synchronize()
        cur = [measure(s) for s in solvers]
        if last is not None and max(abs(a - b) for x, y in zip(cur, last) for a, b in zip(x, y)) < tol:
            break
        last = cur
    return cur


def test_table2_janus_wetting_lengths():
    from paper_2603_22902_amd import Solver
    from paper_2603_22902_amd.batch import Batch

    rows = np.loadtxt(os.path.join(GOLDEN, "table2_janus_wetting_lengths.txt"))
    nx, ny, R, eps = 300, 150, 60.0, 5.0
    x = np.arange(nx) + 0.5 - nx / 2
    y = np.arange(ny) + 0.5
    X, Y = np.meshgrid(x, y)
    drop = synth.tanh_in(R - np.sqrt(X ** 2 + Y ** 2), eps)
    left = 0.5 - 0.5 * np.tanh(2.0 * X / eps)
    phi = np.stack([drop * left, drop * (1.0 - left), 1.0 - drop])[:, None]
    solvers = []
    c13 = math.cos(math.radians(75.0))
    for th23 in rows[:, 0]:
        c23 = math.cos(math.radians(th23))
        cth = [[0.0, c13 - c23, c13], [c23 - c13, 0.0, c23], [-c13, -c23, 0.0]]
        case = _three_fluids((nx, ny), phi, cth, eps)
        s = Solver(case["params"])
        s.init_case(case)
        solvers.append(s)
    b = Batch(solvers)
    b.capture()

    def lengths(s):
        wall = s.lbf_get_moments()["phi"][:, 0, 0, :]  # first layer, [phase][x]
        return float(wall[0].sum() / R), float(wall[1].sum() / R)

    got = _relax(b, solvers, lengths)
    for (th23, L1, L2), (g1, g2) in zip(rows, got):
        e1, e2 = abs(g1 - L1) / L1, abs(g2 - L2) / L2
        print(f"theta_23 {th23:.0f}: L1 {g1:.4f} (analytic {L1:.4f}, {e1:.2e})  "
              f"L2 {g2:.4f} (analytic {L2:.4f}, {e2:.2e})")
        # measured worst 1.3e-2 (L_2 at 30 deg); the paper's own errors reach 3e-2
        assert e1 < 3e-2 and e2 < 3e-2, (th23, g1, g2)


def test_equal_tension_lens_has_120_degree_junctions():
    from paper_2603_22902_amd import Solver
    from paper_2603_22902_amd.batch import Batch

    nx, ny, R0, eps = 200, 120, 24.0, 4.0
    x = np.arange(nx) + 0.5 - nx / 2
    y = np.arange(ny) + 0.5 - ny / 2
    X, Y = np.meshgrid(x, y)
    lens = synth.tanh_in(R0 - np.sqrt(X ** 2 + Y ** 2), eps)
    below = synth.tanh_in(-Y, eps)
    phi = np.stack([lens, (1 - lens) * below, (1 - lens) * (1 - below)])[:, None]
    case = _three_fluids((nx, ny), phi, np.zeros((3, 3)).tolist(), eps)
    s = Solver(case["params"])
    s.init_case(case)
    b = Batch([s])
    b.capture()

    def shape(s):
        p = s.lbf_get_moments()["phi"][:, 0]
        lens_ = p[0]
        cols = lens_.sum(axis=0)
        xc = int(np.argmax(cols))
        # flat interface far from the lens: where phi_2 = phi_3 in the edge column
        edge = p[1][:, 0] - p[2][:, 0]
        k = int(np.argmax(edge < 0))
        yi = k - 1 + edge[k - 1] / (edge[k - 1] - edge[k])
        row = lens_[int(round(yi))]
        width = float((row > 0.5).sum())
        thick = float((lens_[:, xc] > 0.5).sum())
        return thick / width, width

    ratio, width = _relax(b, [s], shape, tol=5e-4)[0]
    print(f"lens thickness/width {ratio:.4f} (tan 30 = {math.tan(math.radians(30)):.4f}), width {width:.1f}")
    # measured 0.5758 against 0.5774 (0.3 %)
    assert abs(ratio - math.tan(math.radians(30.0))) < 0.02 * math.tan(math.radians(30.0))


def test_impurities_workload_full_length_is_stable():
    """The 192^3 D3Q19 N = 4 impurities workload for its full 10 000 steps in
    float32, from the Young-Laplace pressure of its round interfaces: no
    non-finite value, sum_p phi_p within 1e-2 of 1, the front
    (volume-equivalent solid thickness) rising monotonically, and every
    phase's mass near its start at every 1000 steps: the base liquid, the
    gas and the impurity droplet within 2e-3, the small gas bubble within
    BUBBLE_BAR (it follows the compression of the weakly compressible flow,
    whose bulk modulus scales with the density)."""
    from paper_2603_22902_amd import Solver
    c = synth.impurities()
    s = Solver(c["params"])
    s.init_case(c)
    m0 = s.lbf_diagnostics()["mass"]
    front = 0.0
    bars = np.array([2e-3, 2e-3, 2e-3, BUBBLE_BAR])
    for k in range(10):
        s.lbf_step(1000)
        d = s.lbf_diagnostics()
        drift = (d["mass"] - m0) / m0
        print("step", 1000 * (k + 1), "front", d["front"], "drift", drift,
              "sum_phi_err", d["max_sum_phi_err"], flush=True)
        assert not d["nonfinite"]
        assert d["max_sum_phi_err"] < 1e-2
        assert d["front"] > front
        front = d["front"]
        assert np.all(np.abs(drift) < bars), drift
    assert front > 2.0


# measured: the bubble breathes between -0.3 % and +4.4 % of its start over the run
BUBBLE_BAR = 6e-2


@pytest.mark.parametrize("workload,nsteps,drift_bar,sumphi_bar", [
    ("droplet", 20000, 5e-3, 1e-2),    # 256^2 D2Q9 N = 2
    ("compound", 500, 3e-3, 5e-2),     # 512^2 D2Q9 N = 3 (the adjoint's run)
])
def test_2d_workloads_full_length_are_stable(workload, nsteps, drift_bar, sumphi_bar):
    """The 2D workloads for their full runs in float32: finite, the front
    rising monotonically, sum_p phi_p near 1 and every phase mass within the
    bar of its start, checked ten times along the run."""
    from paper_2603_22902_amd import Solver
    c = synth.WORKLOADS[workload]()
    s = Solver(c["params"])
    s.init_case(c)
    m0 = s.lbf_diagnostics()["mass"]
    front = 0.0
    for k in range(10):
        s.lbf_step(nsteps // 10)
        d = s.lbf_diagnostics()
        drift = (d["mass"] - m0) / m0
        print(workload, "step", nsteps // 10 * (k + 1), "front", d["front"], "drift", drift, flush=True)
        assert not d["nonfinite"] and d["max_sum_phi_err"] < sumphi_bar
        assert d["front"] > front
        front = d["front"]
        assert np.all(np.abs(drift) < drift_bar), drift
