"""Host logic of the checkpointed sweeps: which windows are recomputed and
how many device states the forward run keeps (no GPU call)."""
import types

import pytest

from paper_2603_22902_amd.adjoint import last_window, reverse_sweep
from paper_2603_22902_amd.batch import batch_reverse_sweep


@pytest.mark.parametrize("nsteps,window,expect", [
    (500, 50, (10, 450, 50)),   # the compound run: ten windows, the last kept
    (200, 50, (4, 150, 50)),    # the batched sweep
    (7, 3, (3, 6, 1)),          # a ragged last window of one step
    (10, 20, (1, 0, 10)),       # one window: the whole run is kept, nothing recomputed
    (1, 1, (1, 0, 1)),
    (0, 5, (1, 0, 0)),          # no step: one checkpoint, nothing to reverse
])
def test_last_window(nsteps, window, expect):
    nck, start, n_last = last_window(nsteps, window)
    assert (nck, start, n_last) == expect
    # every step lies in exactly one window, and the last one ends the run
    assert start + n_last == nsteps
    assert nck == 1 or (nck - 1) * window == start
    # the rows the forward run keeps: the checkpoints, then x^{s+1} .. x^K
    rows = nck + n_last
    assert rows >= 1
    # steps recomputed by the reverse sweep: every window but the last
    recomputed = sum(min(window, nsteps - k * window) - 1 for k in range(nck - 1))
    assert recomputed == max(0, (nck - 1) * (window - 1))


@pytest.mark.parametrize("sweep", [reverse_sweep, batch_reverse_sweep])
def test_sweep_rejects_checkpoints_of_another_run(sweep):
    # checkpoints laid out for (100, 50) given with (100, 25): refused before
    # any device work (the solver or batch is never touched)
    ck = types.SimpleNamespace(shape=(2 + 50, 16))
    with pytest.raises(ValueError):
        sweep(None, ck, 100, 25)
