"""GPU batched cases (lbf_batch_* through the C ABI): a batch of uneven 2D
cases gives bitwise the states of stepping each solver alone, eagerly and
from every replay of the captured graph; the autotuner leaves the states
unchanged."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _cases():
    # a few uneven cases of both phase counts (the 64-case sweep's recipe)
    cs = synth.batch(n_cases=6, seed_k=7, sizes=(64, 128))
    return [synth.stress(c, phi_noise=1e-6) for c in cs]


def _solvers(cases):
    from paper_2603_22902_amd import Solver
    out = []
    for c in cases:
        s = Solver(c["params"])
        s.init_case(c)
        out.append(s)
    return out


def test_batch_equals_single_steps():
    from paper_2603_22902_amd.batch import Batch
    cases = _cases()
    assert len({c["params"]["nphase"] for c in cases}) == 2
    ref = _solvers(cases)
    for s in ref:
        s.lbf_step(5)
    got = _solvers(cases)
    b = Batch(got)
    b.set_tiles({2: 64, 3: 256})
    b.step(5)
    b.synchronize()
    for s, r in zip(got, ref):
        assert s.step_count() == 5
        assert np.array_equal(s.lbf_get_populations(), r.lbf_get_populations())
        assert np.array_equal(s.lbf_get_aux(), r.lbf_get_aux())


def test_graph_replays_equal_eager_steps():
    from paper_2603_22902_amd.batch import Batch
    cases = _cases()
    ref = _solvers(cases)
    got = _solvers(cases)
    b = Batch(got)
    b.capture()
    for k in range(1, 4):
        for s in ref:
            s.lbf_step(2)
        b.replay(1)
        b.synchronize()
        for s, r in zip(got, ref):
            assert s.step_count() == 2 * k
            assert np.array_equal(s.lbf_get_populations(), r.lbf_get_populations()), k


def test_autotune_keeps_the_states():
    from paper_2603_22902_amd.batch import Batch
    cases = _cases()
    got = _solvers(cases)
    before = [s.lbf_get_populations() for s in got]
    b = Batch(got)
    tiles = b.tune(2)
    b.synchronize()
    assert set(tiles) == {2, 3} and all(t in (64, 128, 256) for t in tiles.values())
    for s, p in zip(got, before):
        assert s.step_count() == 0
        assert np.array_equal(s.lbf_get_populations(), p)


def test_member_stepped_alone_is_refused():
    from paper_2603_22902_amd.batch import Batch
    from paper_2603_22902_amd.lbfreeze import LbfError, LBF_ESTATE
    got = _solvers(_cases()[:2])
    b = Batch(got)
    b.step(1)
    b.synchronize()
    got[0].lbf_step(1)
    with pytest.raises(LbfError) as e:
        b.step(1)
    assert e.value.status == LBF_ESTATE
