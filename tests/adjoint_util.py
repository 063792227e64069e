"""Cases and finite-difference helpers of the reverse-step tests.

J is the frozen fraction of the freezing material after n steps from an
equilibrium start, sum f_s psi / sum psi, or the front position, the
volume-equivalent solid thickness sum f_s psi / (cells per wall layer);
the parameters are T_face[0]
(the cold wall), the latent heats of the freezing phases and the wetting
cosines (perturbed antisymmetrically, as the wetting rule requires)."""
import copy

import numpy as np

import oracle
import synth

CASES = [
    # (N, flow_bc, therm_bc, theta_deg)
    (2, ("wall", "wall"), ("dirichlet", "adiabatic"), 70.0),
    (3, ("wall", "open"), ("dirichlet", "dirichlet"), 70.0),
]

# One phase (no interface terms) and four phases (the largest per-cell
# reverse state, tiled collide reverse).  Central differences of these take
# steps ten times those of checks(): the fourth phase's wetting entries are
# ~1e-3 of the largest, and over 30 steps the rounding of J / h with the
# smaller steps reaches 1e-10 (measured: h = 1e-6 misses the 1e-6 relative
# bar on them; h = 1e-5 meets it on every entry).
CASES_N14 = [
    (1, ("wall", "wall"), ("dirichlet", "adiabatic"), 70.0),
    (4, ("wall", "open"), ("dirichlet", "dirichlet"), 70.0),
]


def make_case(N, fbc, tbc, theta, precision="fp64", shape=(20, 12)):
    c = synth.small(dim=2, shape=shape, nphase=N, precision=precision, flow_bc=fbc, therm_bc=tbc,
                    theta_deg=theta)
    return synth.near_melting(c)


def perturbed(params, key, idx, h):
    q = copy.deepcopy(params)
    if key == "T_face":
        q["T_face"][idx] += h
    elif key == "latent":
        q["latent"][idx] += h
    else:
        p, r = idx
        q["cos_theta"][p][r] += h
        q["cos_theta"][r][p] -= h
    return q


def checks(params):
    """(key, index, step h, function mapping grad[22] to the derivative)."""
    N = params["nphase"]
    out = [("T_face", 0, 1e-6, lambda g: g[0])]
    for p in range(N):
        if params["freezes"][p]:
            out.append(("latent", p, 1e-5, lambda g, p=p: g[2 + p]))
    for p in range(N):
        for r in range(p + 1, N):
            out.append(("cos_theta", (p, r), 1e-6, lambda g, p=p, r=r: g[6 + 4 * p + r] - g[6 + 4 * r + p]))
    return out


def oracle_J(case, params, nsteps):
    """J of the FP64 oracle run with the given parameters."""
    o = oracle.Oracle(params)
    o.init_case({"phi": case["phi"], "T": case["T"]})
    o.step(nsteps)
    m = o.moments()
    N = params["nphase"]
    psi = sum(m["phi"][p] for p in range(N) if params["freezes"][p])
    return float(((1.0 - m["fl"]) * psi).sum() / psi.sum())


def oracle_front(case, params, nsteps):
    """Front position of the FP64 oracle run with the given parameters,
    from the oracle's own conservation diagnostics."""
    o = oracle.Oracle(params)
    o.init_case({"phi": case["phi"], "T": case["T"]})
    o.step(nsteps)
    return float(o.diagnostics()["front"])


def central(fn, params, key, idx, h):
    return (fn(perturbed(params, key, idx, +h)) - fn(perturbed(params, key, idx, -h))) / (2.0 * h)
