"""Batched cases (include/lbfreeze.h, lbf_batch_*): many independent 2D
solvers advance together, one moments and one collide launch per phase count
and time step, optionally replayed from a captured HIP graph; the row tile of
each phase count is picked by the library's autotuner.  Each case's result
is bitwise that of stepping its :class:`Solver` alone."""
from __future__ import annotations

import ctypes

from .lbfreeze import LBF_OK, LbfError, Solver, lib


class Batch:
    def __init__(self, solvers: list, stream=None):
        import torch

        if not solvers:
            raise ValueError("a batch needs at least one solver")
        self.solvers = list(solvers)
        dev = self.solvers[0].device
        torch.cuda.synchronize(dev)
        self.stream = stream if stream is not None else torch.cuda.Stream(dev)
        n = len(self.solvers)
        self._arr = (ctypes.c_void_p * n)(*[s._h.value for s in self.solvers])
        nb = ctypes.c_size_t(0)
        st = lib().lbf_batch_bytes(self._arr, n, ctypes.byref(nb))
        if st != LBF_OK:
            raise LbfError(st, "lbf_batch_bytes: " + lib().lbf_last_error(self.solvers[0]._h).decode())
        nbytes = max(int(nb.value), 256)
        self.buffer = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        aligned = (self.buffer.data_ptr() + 255) & ~255
        h = ctypes.c_void_p(0)
        self._check(lib().lbf_batch_create(self._arr, n, ctypes.c_void_p(aligned), nbytes,
                                           ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.ncell = sum(s.ncell for s in self.solvers)

    def _check(self, s):
        if s != LBF_OK:
            raise LbfError(s, lib().lbf_last_error(self.solvers[0]._h).decode())

    def set_tiles(self, tiles: dict) -> None:
        """tiles: {N: row tile in (64, 128, 256)}."""
        t = (ctypes.c_int * 4)(*[int(tiles.get(n, 0)) for n in range(1, 5)])
        self._check(lib().lbf_batch_set_tiles(self._h, t))

    def tune(self, trial_steps: int = 3) -> dict:
        """Autotune the row tile per phase count; returns {N: tile}."""
        t = (ctypes.c_int * 4)()
        self._check(lib().lbf_batch_tune(self._h, int(trial_steps), t))
        return {n: t[n - 1] for n in range(1, 5) if t[n - 1]}

    def step(self, n: int = 1) -> None:
        self._check(lib().lbf_batch_step(self._h, int(n)))

    def capture(self) -> None:
        """Capture two batched steps into a HIP graph."""
        self._check(lib().lbf_batch_capture(self._h))

    def replay(self, times: int = 1) -> None:
        """Launch the captured graph times times (2 * times steps)."""
        self._check(lib().lbf_batch_replay(self._h, int(times)))

    def synchronize(self) -> None:
        self.stream.synchronize()

    def close(self):
        if getattr(self, "_h", None):
            lib().lbf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
