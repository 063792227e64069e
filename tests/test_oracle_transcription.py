"""The C oracle against an independent NumPy transcription of the step.

tests/transcription.py re-reads Sec. 2-3 as whole-array operations; the
oracle runs cell loops.  From a random valid state (three phases with
random fractions, temperatures across the melting point so that every
branch of eq. (H) runs, random velocity and pressure, perturbed
populations and random lagged fields, random wetting cosines), both
advance 1 and 5 steps on a 6 x 6 D2Q9 and a 5 x 5 x 5 D3Q19 grid, for
wall/open faces and Dirichlet/adiabatic thermal faces in three
combinations.  Populations and every lagged field must agree within
1e-14 of their largest magnitude (measured: 1e-18 after one step, 2e-15
after five).
"""
import numpy as np
import pytest

import oracle
import synth
from transcription import Step

FACES = [(("wall", "wall"), ("dirichlet", "adiabatic")),
         (("wall", "open"), ("dirichlet", "dirichlet")),
         (("open", "wall"), ("adiabatic", "dirichlet"))]


def _random_state(dim, shape, flow_bc, therm_bc, seed):
    rng = np.random.default_rng(seed)
    c = synth.small(dim=dim, shape=shape, nphase=3, flow_bc=flow_bc, therm_bc=therm_bc)
    prm = c["params"]
    ct = np.zeros((4, 4))
    a = rng.uniform(-0.5, 0.5, size=(3, 3))
    ct[:3, :3] = a - a.T
    prm["cos_theta"] = ct.tolist()
    sh = c["T"].shape
    phi = rng.uniform(0.05, 1.0, size=(3,) + sh)
    phi /= phi.sum(0)
    T = prm["T_melt"] + rng.uniform(-0.05, 0.05, size=sh)
    u = rng.uniform(-1e-3, 1e-3, size=(dim,) + sh)
    p = rng.uniform(-1e-4, 1e-4, size=sh)
    o = oracle.Oracle(prm)
    o.init(phi, T, u, p)
    pop = o.populations() * (1 + rng.uniform(-1e-3, 1e-3, size=(o.nlat * o.Q,) + sh))
    aux = o.aux()
    aux[:3] += rng.uniform(-1e-3, 1e-3, size=(3,) + sh)
    aux[3] = rng.uniform(0, 1, size=sh)
    aux[4:] = rng.uniform(-1e-3, 1e-3, size=aux[4:].shape)
    o.set_state(pop, aux)
    return prm, o, pop, aux


@pytest.mark.parametrize("dim,shape", [(2, (6, 6)), (3, (5, 5, 5))])
@pytest.mark.parametrize("faces", range(len(FACES)))
def test_oracle_matches_independent_transcription(dim, shape, faces):
    flow_bc, therm_bc = FACES[faces]
    prm, o, pop, aux = _random_state(dim, shape, flow_bc, therm_bc, seed=100 + 10 * dim + faces)
    step = Step(prm)
    moved = False
    for n in (1, 4):
        for _ in range(n):
            pop2, aux2 = step(pop, aux)
            moved |= np.abs(pop2 - pop).max() > 1e-3
            pop, aux = pop2, aux2
        o.step(n)
        po, ao = o.populations(), o.aux()
        for k in range(po.shape[0]):
            scale = np.abs(po[k]).max()
            assert np.abs(po[k] - pop[k]).max() <= 1e-14 * scale, ("population", k)
        for k in range(ao.shape[0]):
            scale = max(np.abs(ao[k]).max(), 1e-300)
            assert np.abs(ao[k] - aux[k]).max() <= 1e-14 * scale, ("lagged field", k)
    assert moved
