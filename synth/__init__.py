"""Seeded synthetic workloads for the coupled LB freezing solver.

This module is shared by the tests, the benchmark and the smoke check.  It
holds only parameter choices and initial-field geometry (tanh interface
profiles of films, droplets and spheres); none of the method's arithmetic.

Every case is a plain dict::

    {"name": str, "params": dict, "phi": (N, nz, ny, nx) float64,
     "T": (nz, ny, nx) float64, "u": (dim, nz, ny, nx) float64 or None,
     "p": (nz, ny, nx) float64 or None, "steps": int}

Cells sit at (i + 1/2, j + 1/2, k + 1/2); the wall-normal axis is y in 2D
and z in 3D, with the cold wall at coordinate 0.  Lateral axes are periodic.
Seeds: ``numpy.random.Generator(PCG64(260322902 + k))`` for workload k.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 260322902

# ---------------------------------------------------------------------------
# Materials (lattice units).  Densities are relative to the freezing liquid.
# Heat capacities make rho*C = 1 for every phase so that the total-enthalpy
# rest population stays non-negative with the reference E_ref = 1.
# ---------------------------------------------------------------------------
NU = 0.1        # kinematic viscosity of every phase: tau_f = 0.8
EPS = 4.0       # interface width parameter epsilon
TAU_G = 0.8     # phase-field relaxation: M = (tau_g - 1/2)/3 = 0.1
T_MELT = 0.0
T_HOT = 1.0     # initial temperature T_0
T_COLD = -1.0   # substrate temperature T_w


def freezing_phase(rho_l=1.0, ratio=0.9, lam=0.15, cp=1.0, ste=0.1):
    """A phase that freezes; ratio = rho_s/rho_l, latent heat from the Stefan
    number Ste = C_p,s (T_m - T_w) / L."""
    rho_s = rho_l * ratio
    return dict(rho_l=rho_l, rho_s=rho_s, mu_l=rho_l * NU, mu_s=rho_s * NU,
                lam_l=lam, lam_s=lam, cp_l=cp, cp_s=cp,
                latent=cp * (T_MELT - T_COLD) / ste, freezes=1)


def inert_phase(rho=0.001, lam=0.15):
    """A phase that never freezes (gas, bubbles); rho*C = 1."""
    cp = 1.0 / rho
    return dict(rho_l=rho, rho_s=rho, mu_l=rho * NU, mu_s=rho * NU,
                lam_l=lam, lam_s=lam, cp_l=cp, cp_s=cp, latent=0.0, freezes=0)


def make_params(dim, shape, phases, sigma, precision="fp32",
                flow_bc=("wall", "wall"), therm_bc=("dirichlet", "adiabatic"),
                T_face=(T_COLD, T_HOT), cos_theta=None, eps=EPS, tau_g=TAU_G,
                T_melt=T_MELT, E_ref=None, gravity=(0.0, 0.0, 0.0)):
    """Assemble a parameter dict.  shape = (nx, ny) in 2D, (nx, ny, nz) in 3D.

    E_ref = rho_ref C_p,ref with rho_ref = rho_1^l and
    C_p,ref = 2 C_s C_l / (C_s + C_l) of phase 1 (the paper's reference heat
    capacity) unless given."""
    N = len(phases)
    sig = np.zeros((4, 4))
    s = np.asarray(sigma, dtype=float)
    if s.ndim == 0:
        s = np.full((N, N), float(s))
    sig[:N, :N] = s
    np.fill_diagonal(sig, 0.0)
    ct = np.zeros((4, 4))
    if cos_theta is not None:
        ct[:N, :N] = np.asarray(cos_theta, dtype=float)
    if E_ref is None:
        p0 = phases[0]
        cref = 2.0 * p0["cp_s"] * p0["cp_l"] / (p0["cp_s"] + p0["cp_l"])
        E_ref = p0["rho_l"] * cref
    nx, ny = shape[0], shape[1]
    nz = shape[2] if dim == 3 else 1
    out = dict(dim=dim, nx=nx, ny=ny, nz=nz, nphase=N, precision=precision,
               flow_bc=list(flow_bc), therm_bc=list(therm_bc),
               T_face=[float(t) for t in T_face], sigma=sig.tolist(),
               cos_theta=ct.tolist(), eps=eps, tau_g=tau_g, T_melt=T_melt,
               E_ref=float(E_ref), gravity=list(gravity))
    for key in ("rho_l", "rho_s", "mu_l", "mu_s", "lam_l", "lam_s", "cp_l",
                "cp_s", "latent", "freezes"):
        out[key] = [ph[key] for ph in phases] + [0] * (4 - N)
    return out


# ---------------------------------------------------------------------------
# Geometry helpers
# ---------------------------------------------------------------------------
def grid(params):
    """Cell-centre coordinates X, Y, Z with shape (nz, ny, nx)."""
    nx, ny, nz = params["nx"], params["ny"], params["nz"]
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5,
                          np.arange(nx) + 0.5, indexing="ij")
    return x, y, z


def tanh_in(dist_inside, eps=EPS):
    """1/2 + 1/2 tanh(d / (eps/2)): 1 inside (d > 0), 0 outside."""
    return 0.5 + 0.5 * np.tanh(dist_inside / (eps / 2.0))


def laplace_pressure(bodies, dim):
    """Initial pressure of fluids at rest with curved interfaces: the
    Young-Laplace jump sigma * (dim - 1) / R across the outer interface of
    each round body, summed over nested bodies and smoothed by the bodies'
    tanh indicators.  bodies = [(indicator, sigma, R), ...]."""
    p = 0.0
    for ind, sig, R in bodies:
        p = p + sig * (dim - 1) / R * ind
    return np.ascontiguousarray(p, dtype=np.float64)


def _case(name, params, phi, T, steps, u=None, p=None):
    return dict(name=name, params=params, phi=np.ascontiguousarray(phi, dtype=np.float64),
                T=np.ascontiguousarray(T, dtype=np.float64), u=u, p=p, steps=steps)


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------
def film(ny=256, nx=8, h0=128.0, ratio=0.9, ste=0.1, steps=2000, precision="fp64"):
    """Film freezing with volume change: liquid below h0, gas above, cold wall
    at y = 0 (Dirichlet T_w, no slip), open top at T_0, periodic x."""
    phases = [freezing_phase(ratio=ratio, lam=0.15, ste=ste), inert_phase(0.01, lam=0.15)]
    prm = make_params(2, (nx, ny), phases, sigma=1e-3, precision=precision,
                      flow_bc=("wall", "open"), therm_bc=("dirichlet", "dirichlet"),
                      T_face=(T_COLD, T_HOT))
    x, y, z = grid(prm)
    p1 = tanh_in(h0 - y)
    phi = np.stack([p1, 1.0 - p1])
    T = np.full(p1.shape, T_HOT)
    return _case("film", prm, phi, T, steps)


def droplet(seed_k=2, n=256, radius=60.0, steps=20000, precision="fp32",
            theta_deg=90.0, ste=None):
    """Sessile droplet on a cold wall (centre on the wall), gas around,
    density ratio liquid:solid:gas 1:0.9:0.001."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_k))
    if ste is None:
        ste = float(rng.uniform(0.05, 0.2))
    phases = [freezing_phase(ratio=0.9, lam=0.1, ste=ste), inert_phase(0.001, lam=0.15)]
    ct = math.cos(math.radians(theta_deg))
    prm = make_params(2, (n, n), phases, sigma=1e-3, precision=precision,
                      cos_theta=[[0.0, ct], [-ct, 0.0]])
    x, y, z = grid(prm)
    r = np.sqrt((x - n / 2) ** 2 + y ** 2)
    p1 = tanh_in(radius - r)
    phi = np.stack([p1, 1.0 - p1])
    T = np.full(p1.shape, T_HOT)
    c = _case("droplet", prm, phi, T, steps, p=laplace_pressure([(p1, 1e-3, radius)], 2))
    c["ste"] = ste
    return c


def compound(seed_k=3, n=512, r_core=60.0, r_shell=120.0, steps=500, precision="fp32"):
    """Encapsulated compound droplet: core phase 1 (rho_s/rho_l = 1.1) inside
    shell phase 2 (0.9), gas phase 3; alpha_2/alpha_1 = 3, alpha_3/alpha_1 =
    1.5, Ste = 0.2, 90-degree wetting, pairwise sigma drawn from the seed."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_k))
    s12, s13, s23 = (float(v) for v in rng.uniform(0.5e-3, 1.5e-3, size=3))
    sig = [[0, s12, s13], [s12, 0, s23], [s13, s23, 0]]
    phases = [freezing_phase(ratio=1.1, lam=0.05, ste=0.2),
              freezing_phase(ratio=0.9, lam=0.15, ste=0.2),
              inert_phase(0.001, lam=0.075)]
    prm = make_params(2, (n, n), phases, sigma=sig, precision=precision)
    x, y, z = grid(prm)
    r = np.sqrt((x - n / 2) ** 2 + y ** 2)
    p1 = tanh_in(r_core - r)
    p2 = (1.0 - p1) * tanh_in(r_shell - r)
    phi = np.stack([p1, p2, 1.0 - p1 - p2])
    T = np.full(p1.shape, T_HOT)
    p = laplace_pressure([(p1 + p2, s23, r_shell), (p1, s12, r_core)], 2)
    return _case("compound", prm, phi, T, steps, p=p)


def impurities(seed_k=4, n=192, radius=64.0, steps=10000, precision="fp32"):
    """3D droplet with two insoluble impurities on a cold wall, D3Q19, N = 4:
    phase 1 base liquid (rho_s/rho_l = 0.95), phase 2 gas, phase 3 freezing
    impurity droplet (1.05, alpha 3x the base), phase 4 non-freezing bubble
    with gas properties.  Impurity radii r_A, r_B ~ U[8, 16], centres uniform
    in the droplet, at least r + eps inside its surface and above the wall,
    and at least eps apart."""
    if radius < 2.0 * (16.0 + EPS) + 2.0:
        raise ValueError("droplet radius too small to hold the impurities")
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_k))
    rA, rB = (float(v) for v in rng.uniform(8.0, 16.0, size=2))
    c0 = np.array([n / 2, n / 2, 0.0])

    def draw(r, others):
        for _ in range(100000):
            cand = np.array([rng.uniform(c0[0] - radius, c0[0] + radius),
                             rng.uniform(c0[1] - radius, c0[1] + radius),
                             rng.uniform(0.0, radius)])
            if np.linalg.norm(cand - c0) > radius - r - EPS:
                continue
            if cand[2] < r + EPS:
                continue
            if any(np.linalg.norm(cand - oc) < r + orr + EPS for oc, orr in others):
                continue
            return cand
        raise ValueError("could not place the impurities")

    cA = draw(rA, [])
    cB = draw(rB, [(cA, rA)])
    phases = [freezing_phase(ratio=0.95, lam=0.05, ste=0.1),
              inert_phase(0.001, lam=0.075),
              freezing_phase(ratio=1.05, lam=0.15, ste=0.1),
              inert_phase(0.001, lam=0.075)]
    prm = make_params(3, (n, n, n), phases, sigma=1e-3, precision=precision)
    x, y, z = grid(prm)
    d = tanh_in(radius - np.sqrt((x - c0[0]) ** 2 + (y - c0[1]) ** 2 + z ** 2))
    a = tanh_in(rA - np.sqrt((x - cA[0]) ** 2 + (y - cA[1]) ** 2 + (z - cA[2]) ** 2))
    b = tanh_in(rB - np.sqrt((x - cB[0]) ** 2 + (y - cB[1]) ** 2 + (z - cB[2]) ** 2))
    rest = 1.0 - a - b
    phi = np.stack([rest * d, rest * (1.0 - d), a, b])
    T = np.full(d.shape, T_HOT)
    p = laplace_pressure([(d, 1e-3, radius), (a, 1e-3, rA), (b, 1e-3, rB)], 3)
    c = _case("impurities", prm, phi, T, steps, p=p)
    c["impurity"] = dict(rA=rA, rB=rB, cA=cA.tolist(), cB=cB.tolist())
    return c


def bubble(n=96, radius=10.0, rho_g=0.001, sigma=1e-3, inverted=False, laplace=True,
           steps=500, precision="fp64"):
    """A round gas bubble (or, inverted, a liquid drop in gas) at the centre
    of a closed n x n box, no phase change (T above melting everywhere,
    adiabatic walls).  The bubble is phase 2 (non-freezing, gas
    properties), the liquid phase 1.  laplace=True starts from the
    Young-Laplace pressure of the round interface."""
    phases = [freezing_phase(ratio=0.9, lam=0.15, ste=0.1), inert_phase(rho_g, lam=0.15)]
    prm = make_params(2, (n, n), phases, sigma=sigma, precision=precision,
                      flow_bc=("wall", "wall"), therm_bc=("adiabatic", "adiabatic"),
                      T_face=(T_HOT, T_HOT))
    x, y, z = grid(prm)
    b = tanh_in(radius - np.sqrt((x - n / 2) ** 2 + (y - n / 2) ** 2))
    phi = np.stack([b, 1.0 - b]) if inverted else np.stack([1.0 - b, b])
    T = np.full(b.shape, T_HOT)
    p = laplace_pressure([(b, sigma, radius)], 2) if laplace else None
    return _case("drop" if inverted else "bubble", prm, phi, T, steps, p=p)


def small(dim=2, shape=(70, 37), nphase=2, precision="fp64", seed_k=11,
          flow_bc=("wall", "wall"), therm_bc=("dirichlet", "adiabatic"),
          theta_deg=90.0, steps=30, gravity=(0.0, 0.0, 0.0)):
    """A small droplet case with ragged sizes for element-wise parity: a
    (compound, for N >= 3) droplet on the wall, gas around, N = 2..4."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_k))
    phases = [freezing_phase(ratio=0.9, lam=0.1, ste=0.1),
              inert_phase(0.01, lam=0.15),
              freezing_phase(ratio=1.1, lam=0.05, ste=0.2),
              inert_phase(0.02, lam=0.1)][:nphase]
    sig = rng.uniform(0.5e-3, 1.5e-3, size=(4, 4))
    sig = 0.5 * (sig + sig.T)
    ct = np.zeros((4, 4))
    c = math.cos(math.radians(theta_deg))
    ct[0, 1], ct[1, 0] = c, -c
    prm = make_params(dim, shape, phases, sigma=sig[:nphase, :nphase],
                      precision=precision, flow_bc=flow_bc, therm_bc=therm_bc,
                      cos_theta=ct[:nphase, :nphase], gravity=gravity)
    x, y, z = grid(prm)
    L = shape[0]
    R = 0.3 * min(shape)
    if dim == 2:
        r = np.sqrt((x - L / 2) ** 2 + y ** 2)
    else:
        r = np.sqrt((x - L / 2) ** 2 + (y - shape[1] / 2) ** 2 + z ** 2)
    drop = tanh_in(R - r)
    if nphase == 1:
        phi = np.ones((1,) + drop.shape)
    elif nphase == 2:
        phi = np.stack([drop, 1.0 - drop])
    else:
        core = tanh_in(0.5 * R - r)
        parts = [drop * (1.0 - core), 1.0 - drop, drop * core]
        if nphase == 4:
            if dim == 2:
                rb = np.sqrt((x - 0.2 * L) ** 2 + (y - 0.7 * shape[1]) ** 2)
            else:
                rb = np.sqrt((x - 0.2 * L) ** 2 + (y - 0.3 * shape[1]) ** 2 +
                             (z - 0.7 * shape[2]) ** 2)
            bub = tanh_in(0.15 * min(shape) - rb)
            parts = [q * (1.0 - bub) for q in parts] + [bub]
        phi = np.stack(parts)
    T = np.full(drop.shape, T_HOT)
    return _case("small", prm, phi, T, steps)


def batch(n_cases=64, seed_k=5, precision="fp32", sizes=(64, 128, 256, 512)):
    """Independent 2D droplet-freezing cases for a batched run.  For each
    case, in this order: the side L from sizes, the contact angle
    theta ~ U[60, 120] deg, the Stefan number Ste ~ U[0.05, 0.2] and N from
    {2, 3}.  A droplet of radius L/4 sits on the cold wall (with an
    encapsulated core of radius L/8 for N = 3), gas elsewhere."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_k))
    out = []
    for _ in range(n_cases):
        L = int(rng.choice(sizes))
        theta = float(rng.uniform(60.0, 120.0))
        ste = float(rng.uniform(0.05, 0.2))
        N = int(rng.choice([2, 3]))
        c = math.cos(math.radians(theta))
        if N == 2:
            phases = [freezing_phase(ratio=0.9, lam=0.15, ste=ste), inert_phase(0.01, lam=0.225)]
            ct = [[0.0, c], [-c, 0.0]]
        else:
            phases = [freezing_phase(ratio=1.1, lam=0.05, ste=ste),
                      freezing_phase(ratio=0.9, lam=0.15, ste=ste), inert_phase(0.01, lam=0.075)]
            ct = [[0.0, 0.0, 0.0], [0.0, 0.0, c], [0.0, -c, 0.0]]
        prm = make_params(2, (L, L), phases, sigma=1e-3, precision=precision, cos_theta=ct)
        x, y, z = grid(prm)
        r = np.sqrt((x - L / 2) ** 2 + y ** 2)
        drop = tanh_in(L / 4 - r)
        if N == 2:
            phi = np.stack([drop, 1.0 - drop])
            p = laplace_pressure([(drop, 1e-3, L / 4)], 2)
        else:
            core = tanh_in(L / 8 - r)
            phi = np.stack([drop * core, drop * (1.0 - core), 1.0 - drop])
            p = laplace_pressure([(drop, 1e-3, L / 4), (core, 1e-3, L / 8)], 2)
        T = np.full(drop.shape, T_HOT)
        case = _case("batch", prm, phi, T, 200, p=p)
        case.update(theta_deg=theta, ste=ste)
        out.append(case)
    return out


def near_melting(case, T_wall=0.005, T_top=0.025):
    """The case with a liquid start just above the melting point, T rising
    linearly from T_wall at the cold wall to T_top at the far face, and no
    initial flow: freezing starts within the first steps (for short
    gradient checks of the reverse step)."""
    c = dict(case)
    prm = c["params"]
    x, y, z = grid(prm)
    wn = y if prm["dim"] == 2 else z
    nwn = prm["ny"] if prm["dim"] == 2 else prm["nz"]
    c["T"] = T_MELT + T_wall + (T_top - T_wall) * wn / nwn
    c.pop("u", None)
    c.pop("p", None)
    return c


def stress(case, seed_k=99, phi_noise=1e-3, T_band=0.05, u_amp=1e-3, p_amp=1e-4):
    """Perturbed copy of a case that exercises every branch in the first
    steps: U[-phi_noise, phi_noise] on phi (clipped at 0, renormalised so
    that sum_p phi_p = 1), T = T_melt + U[-T_band, T_band] wherever some
    freezing phase is present (so solid, mushy and liquid cells all occur
    within a few steps), and random velocity and pressure."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + seed_k))
    prm = case["params"]
    phi = case["phi"] + rng.uniform(-phi_noise, phi_noise, size=case["phi"].shape)
    phi = np.clip(phi, 0.0, None)
    phi = phi / phi.sum(axis=0, keepdims=True)
    N = prm["nphase"]
    psi = sum(phi[q] for q in range(N) if prm["freezes"][q])
    dT = rng.uniform(-T_band, T_band, size=case["T"].shape)
    T = np.where(psi > 1e-3, prm["T_melt"] + dT, case["T"])
    d = prm["dim"]
    u = rng.uniform(-u_amp, u_amp, size=(d,) + case["T"].shape)
    p = rng.uniform(-p_amp, p_amp, size=case["T"].shape)
    out = dict(case)
    out.update(name=case["name"] + "+stress", phi=np.ascontiguousarray(phi),
               T=np.ascontiguousarray(T), u=np.ascontiguousarray(u),
               p=np.ascontiguousarray(p))
    return out


WORKLOADS = {
    "film": film,
    "droplet": droplet,
    "compound": compound,
    "impurities": impurities,
}
