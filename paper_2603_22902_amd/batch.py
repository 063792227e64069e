"""Batched cases (include/lbfreeze.h, lbf_batch_*): many independent 2D
solvers advance together, one moments and one collide launch per phase count
and time step, optionally replayed from a captured HIP graph; the row tile of
each phase count is picked by the library's autotuner.  Each case's result
is bitwise that of stepping its :class:`Solver` alone.

The batched reverse sweep (:func:`batch_forward_with_checkpoints`,
:func:`batch_reverse_sweep`) differentiates every case's objective at once:
packed batch states hold the checkpoints and the tape, each recomputed step
and each reverse step is one launch per pass and phase count over all
cases, and every case's gradient is bitwise that of its single-case sweep."""
from __future__ import annotations

import ctypes

import numpy as np

from .adjoint import NPAR, OBJECTIVES
from .lbfreeze import LBF_OK, LbfError, Solver, _ptr, lib


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

    def set_launch(self, persistent: bool = False, concurrent: bool = False, grid: int = 0) -> None:
        """persistent: each pass launched with grid blocks (0: as many as the
        GPU holds at once) striding over the work items; concurrent: the
        phase-count groups on streams of their own (parallel graph
        branches; the creation default when there are several groups).
        Drops a captured graph."""
        flags = (1 if persistent else 0) | (2 if concurrent else 0)
        self._check(lib().lbf_batch_set_launch(self._h, flags, int(grid)))

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

    # ----- packed batch states (checkpoints and tapes of a batched sweep)
    def state_bytes(self) -> int:
        n = ctypes.c_size_t(0)
        self._check(lib().lbf_batch_state_bytes(self._h, ctypes.byref(n)))
        return int(n.value)

    def states(self, k: int):
        """k packed batch states, one per row of a uint8 device tensor."""
        import torch

        t = torch.empty((k, self.state_bytes()), dtype=torch.uint8, device=self.solvers[0].device)
        if t.data_ptr() & 255:
            raise RuntimeError("packed batch states need a 256-byte aligned allocation")
        return t

    def state_to_device(self, dst) -> None:
        """Copy every member's current state into the packed state dst."""
        self._check(lib().lbf_batch_state_to_device(self._h, ctypes.c_void_p(dst.data_ptr())))

    def state_from_device(self, src, advance: int) -> None:
        """Every member's state from the packed state src, which is advance
        steps ahead of the members' current states (their step counts
        advance by that much)."""
        self._check(lib().lbf_batch_state_from_device(self._h, ctypes.c_void_p(src.data_ptr()), int(advance)))

    def step_states(self, src, dst) -> None:
        """One batched step from packed state src to dst (members untouched)."""
        self._check(lib().lbf_batch_step_states(self._h, ctypes.c_void_p(src.data_ptr()),
                                                ctypes.c_void_p(dst.data_ptr())))

    def close(self):
        if getattr(self, "_h", None):
            lib().lbf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchAdjoint:
    """Batched reverse step over a :class:`Batch` (its stream and cases)."""

    def __init__(self, batch: Batch):
        import torch

        self.batch = batch
        n = ctypes.c_size_t(0)
        st = lib().lbf_batch_adjoint_bytes(batch._h, ctypes.byref(n))
        if st != LBF_OK:
            raise LbfError(st, "lbf_batch_adjoint_bytes: the batched reverse step needs 2D float32 or float64 cases")
        nbytes = int(n.value)
        self.buffer = torch.empty(nbytes + 256, dtype=torch.uint8, device=batch.solvers[0].device)
        aligned = (self.buffer.data_ptr() + 255) & ~255
        h = ctypes.c_void_p(0)
        batch._check(lib().lbf_batch_adjoint_create(batch._h, ctypes.c_void_p(aligned), nbytes, ctypes.byref(h)))
        self._h = h

    def seed(self, state, objective: str = "frozen_fraction") -> np.ndarray:
        """Objective of every case of the packed state (caller order)."""
        if objective not in OBJECTIVES:
            raise ValueError(f"objective must be one of {sorted(OBJECTIVES)}")
        J = np.zeros(len(self.batch.solvers))
        self.batch._check(lib().lbf_batch_adjoint_seed(self._h, OBJECTIVES[objective],
                                                        ctypes.c_void_p(state.data_ptr()), _ptr(J)))
        return J

    def step(self, state, next_state) -> None:
        self.batch._check(lib().lbf_batch_adjoint_step(self._h, ctypes.c_void_p(state.data_ptr()),
                                                        ctypes.c_void_p(next_state.data_ptr())))

    def finish(self, state0) -> None:
        self.batch._check(lib().lbf_batch_adjoint_finish(self._h, ctypes.c_void_p(state0.data_ptr())))

    def gradient(self) -> np.ndarray:
        """(ncase, 22) rows as lbf_adjoint_gradient."""
        g = np.zeros((len(self.batch.solvers), NPAR))
        self.batch._check(lib().lbf_batch_adjoint_gradient(self._h, _ptr(g)))
        return g

    def close(self):
        if getattr(self, "_h", None):
            lib().lbf_batch_adjoint_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def relax_contact_angles(cases: list, max_steps: int = 20000, chunk: int = 1000, tol: float = 0.05,
                         device: int = 0) -> tuple:
    """Isothermal pre-relaxation of the droplets whose wall angle is not 90
    degrees (a semicircle on the wall, the shape they start as, is the
    equilibrium only at 90 degrees): those cases run together as one batch
    with their cold face held at the initial temperature (so nothing
    freezes) until the wetted length of each -- the freezing material on the
    wall layer, sum_x psi -- changes by less than tol cells over chunk
    steps, or until max_steps.  Returns (states, steps, lengths): one device
    state per case (None where theta = 90 degrees) to start the cooled run
    from with Solver.lbf_state_from_device, the steps taken and each case's
    last two wetted lengths."""
    import copy as _copy

    import torch

    idx = [k for k, c in enumerate(cases) if abs(c.get("theta_deg", 90.0) - 90.0) > 1e-9]
    states = [None] * len(cases)
    if not idx:
        return states, 0, {}
    solvers = []
    for k in idx:
        prm = _copy.deepcopy(cases[k]["params"])
        prm["T_face"] = [float(np.max(cases[k]["T"])), prm["T_face"][1]]
        s = Solver(prm, device=device)
        s.init_case(cases[k])
        solvers.append(s)
    b = Batch(solvers)

    def wetted(s):
        phi = s.lbf_get_moments(mask=1)["phi"]  # LBF_M_PHI
        frz = [p for p in range(s.N) if s.params["freezes"][p]]
        wall = phi[:, 0, 0, :] if s.dim == 2 else phi[:, 0]
        return float(sum(wall[p].sum() for p in frz))

    last = [wetted(s) for s in solvers]
    steps, lengths = 0, {}
    while steps < max_steps:
        b.step(chunk)
        b.synchronize()
        steps += chunk
        cur = [wetted(s) for s in solvers]
        lengths = {idx[j]: (last[j], cur[j]) for j in range(len(idx))}
        done = all(abs(c - l) < tol for c, l in zip(cur, last))
        last = cur
        if done:
            break
    b.close()
    for j, k in enumerate(idx):
        st = torch.empty(solvers[j].state_device_bytes(), dtype=torch.uint8, device=solvers[j].device)
        solvers[j].lbf_state_to_device(st)
        torch.cuda.synchronize(solvers[j].device)
        states[k] = st
        solvers[j].close()
    return states, steps, lengths


def batch_forward_with_checkpoints(batch: Batch, nsteps: int, window: int, graph: bool = False):
    """nsteps batched steps from the members' current states (taken as step
    0); returns the packed states at steps 0, window, 2 window, ... (one row
    each), followed by the packed states of the last window after its
    checkpoint (x^{s+1} .. x^nsteps, batched steps between packed states),
    which the reverse sweep then need not recompute.  The members end at
    x^nsteps.  graph: the other windows' even stretches replay the captured
    two-step graph (capture first)."""
    from .adjoint import last_window

    nck, start, n_last = last_window(nsteps, window)
    ck = batch.states(nck + n_last)
    for k in range(nck - 1):
        batch.state_to_device(ck[k])
        if graph:
            batch.replay(window // 2)
            batch.step(window % 2)
        else:
            batch.step(window)
    batch.state_to_device(ck[nck - 1])
    for j in range(n_last):
        batch.step_states(ck[nck - 1 + j], ck[nck + j])
    if n_last > 0:
        batch.state_from_device(ck[nck + n_last - 1], n_last)
    return ck


def batch_reverse_sweep(batch: Batch, ck, nsteps: int, window: int, objective: str = "frozen_fraction",
                        timing: dict = None) -> tuple:
    """(J[ncase], grad[ncase, 22]) by batched reverse steps over the
    checkpoints of :func:`batch_forward_with_checkpoints`: the last window's
    packed states come with them; every earlier window is re-run from its
    checkpoint into a packed tape with batched steps (reusing the last
    window's rows once those are done).  timing (a dict) receives the
    milliseconds of recomputation and of reverse steps (events on the
    batch's stream)."""
    import torch

    from .adjoint import last_window

    ev = []

    def mark():
        if timing is not None:
            e = torch.cuda.Event(enable_timing=True)
            e.record(batch.stream)
            ev.append(e)

    nck, s_last, n_last = last_window(nsteps, window)
    if ck.shape[0] != nck + n_last:
        raise ValueError("checkpoints do not match nsteps and window (use batch_forward_with_checkpoints)")
    adj = BatchAdjoint(batch)
    J = adj.seed(ck[nck + n_last - 1], objective)
    tape = None
    for k in range(nck - 1, -1, -1):
        start = k * window
        n = min(window, nsteps - start)
        if n <= 0:
            continue
        mark()
        if k == nck - 1:
            states = [ck[k + j] for j in range(n + 1)]
        else:
            if tape is None:
                tape = ck[nck:nck + window - 1] if n_last >= window - 1 else batch.states(window - 1)
            states = [ck[k]] + [tape[j] for j in range(n - 1)] + [ck[k + 1]]
            for j in range(1, n):
                batch.step_states(states[j - 1], states[j])
        mark()
        for j in range(n - 1, -1, -1):
            adj.step(states[j], states[j + 1])
        mark()
    adj.finish(ck[0])
    g = adj.gradient()
    adj.close()
    if timing is not None:
        batch.synchronize()
        timing["recompute_ms"] = sum(ev[i].elapsed_time(ev[i + 1]) for i in range(0, len(ev), 3))
        timing["reverse_ms"] = sum(ev[i + 1].elapsed_time(ev[i + 2]) for i in range(0, len(ev), 3))
    return J, g


def batch_forward_to_tape(batch: Batch, nsteps: int):
    """nsteps batched steps from the members' current states, every packed
    state written straight into a device tape (row j = x^j, nsteps + 1
    rows); the members' own states are not advanced."""
    tape = batch.states(nsteps + 1)
    batch.state_to_device(tape[0])
    for j in range(1, nsteps + 1):
        batch.step_states(tape[j - 1], tape[j])
    return tape


def batch_reverse_from_tape(batch: Batch, tape, nsteps: int, objective: str = "frozen_fraction",
                            timing: dict = None) -> tuple:
    """(J[ncase], grad[ncase, 22]) from the full tape of
    :func:`batch_forward_to_tape`, with no recomputation; timing (a dict)
    receives the milliseconds of the reverse steps."""
    import torch

    adj = BatchAdjoint(batch)
    J = adj.seed(tape[nsteps], objective)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(batch.stream)
    for j in range(nsteps - 1, -1, -1):
        adj.step(tape[j], tape[j + 1])
    e1.record(batch.stream)
    adj.finish(tape[0])
    g = adj.gradient()
    adj.close()
    if timing is not None:
        batch.synchronize()
        timing["reverse_ms"] = e0.elapsed_time(e1)
    return J, g


def batch_choose_window(batch: Batch, nsteps: int, window=None) -> int:
    """window as given, else 0 (every packed state of the run in a device
    tape, no recomputation) when that tape fits in three quarters of the
    free device memory, else checkpoints every 50 steps."""
    if window is not None:
        return int(window)
    import torch
    free, _ = torch.cuda.mem_get_info(batch.solvers[0].device)
    return 0 if (nsteps + 1) * batch.state_bytes() < 0.75 * free else 50


def batch_objective_and_gradient(batch: Batch, nsteps: int, window=None, objective: str = "frozen_fraction",
                                 graph: bool = False) -> tuple:
    """nsteps batched steps from the members' current states, then the
    batched reverse sweep: (J[ncase], grad[ncase, 22]) of the objective
    ("frozen_fraction" or "front").  window = 0 keeps every packed state in
    HBM; None chooses that when it fits (batch_choose_window).  graph: the
    checkpointed forward replays the captured two-step graph (capture
    first).  The members end at step nsteps either way."""
    window = batch_choose_window(batch, nsteps, window)
    if window == 0:
        tape = batch_forward_to_tape(batch, nsteps)
        batch.state_from_device(tape[nsteps], nsteps)
        return batch_reverse_from_tape(batch, tape, nsteps, objective=objective)
    ck = batch_forward_with_checkpoints(batch, nsteps, window, graph=graph)
    return batch_reverse_sweep(batch, ck, nsteps, window, objective=objective)
