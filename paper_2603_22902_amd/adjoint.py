"""Reverse mode of the coupled-LB step (include/lbfreeze.h, lbf_adjoint_*).

Gradient of an objective of the state at the end of a run -- the frozen
fraction of the freezing material, J = sum f_s psi / sum psi, or the front
position, J = sum f_s psi / (cells per wall layer) -- with respect to the
wall temperatures, the latent heats and the wetting cosines, by the
hand-written discrete adjoint of every step (2D, float32 or float64).  Long runs use checkpoint-and-
recompute: the forward run keeps the device state every ``window`` steps;
the reverse sweep re-runs each window forward from its checkpoint, keeping
its states on the device, and then steps the adjoint back through it.  When
the whole trajectory fits in device memory (``window = 0``), the forward run
writes every state straight into an HBM-resident tape instead and the
reverse sweep recomputes nothing.

:class:`FrozenFraction` exposes this as a ``torch.autograd.Function`` of
(T_w, latent[N], cos_theta[N, N]), for either objective; derived parameters such as the Stefan
number (L = C (T_melt - T_w) / Ste) or the contact angle (cos_theta) are
composed in torch around it.
"""
from __future__ import annotations

import copy
import ctypes

import numpy as np

from .lbfreeze import LBF_OK, LbfError, Solver, _ptr, lib, make_params

NPAR = 22
OBJECTIVES = {"frozen_fraction": 0, "front": 1}


class Adjoint:
    """Adjoint context bound to a :class:`Solver` (same device and stream)."""

    def __init__(self, solver: Solver):
        import torch

        self.solver = solver
        n = ctypes.c_size_t(0)
        s = lib().lbf_adjoint_bytes(ctypes.byref(solver._P), ctypes.byref(n))
        if s != LBF_OK:
            raise LbfError(s, "lbf_adjoint_bytes: the reverse step needs dim 2 and fp32 or fp64")
        nbytes = int(n.value)
        self.buffer = torch.empty(nbytes + 256, dtype=torch.uint8, device=solver.device)
        aligned = (self.buffer.data_ptr() + 255) & ~255
        h = ctypes.c_void_p(0)
        solver._check(lib().lbf_adjoint_create(solver._h, ctypes.c_void_p(aligned), nbytes, ctypes.byref(h)))
        self._h = h

    def _check(self, s):
        self.solver._check(s)

    def seed(self, objective: str = "frozen_fraction") -> float:
        """Objective of the current state ("frozen_fraction" or "front")."""
        if objective not in OBJECTIVES:
            raise ValueError(f"objective must be one of {sorted(OBJECTIVES)}")
        J = np.zeros(1)
        self._check(lib().lbf_adjoint_seed_objective(self._h, OBJECTIVES[objective], _ptr(J)))
        return float(J[0])

    def step(self, state, next_state=None) -> None:
        """Reverse step through x^n = state; next_state = x^{n+1} if at
        hand (saves recomputing the moments of x^n)."""
        nxt = ctypes.c_void_p(next_state.data_ptr()) if next_state is not None else None
        self._check(lib().lbf_adjoint_step(self._h, ctypes.c_void_p(state.data_ptr()), nxt))

    def finish(self, state0) -> None:
        self._check(lib().lbf_adjoint_finish(self._h, ctypes.c_void_p(state0.data_ptr())))

    def gradient(self) -> dict:
        g = np.zeros(NPAR)
        self._check(lib().lbf_adjoint_gradient(self._h, _ptr(g)))
        N = self.solver.N
        return dict(T_face=g[0:2].copy(), latent=g[2:2 + N].copy(),
                    cos_theta=g[6:22].reshape(4, 4)[:N, :N].copy(), raw=g)

    def state(self):
        s = self.solver
        pops = np.empty(((s.N + 2) * s.Q,) + s.shape)
        aux = np.empty((s.N + s.dim + 3,) + s.shape)
        self._check(lib().lbf_adjoint_state(self._h, _ptr(pops), _ptr(aux)))
        return pops, aux

    def close(self):
        if getattr(self, "_h", None):
            lib().lbf_adjoint_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _states(solver: Solver, k: int):
    import torch
    return torch.empty((k, solver.state_device_bytes()), dtype=torch.uint8, device=solver.device)


def last_window(nsteps: int, window: int) -> tuple:
    """(number of checkpoints, first step of the last window, its length)."""
    nck = (nsteps + window - 1) // window if nsteps > 0 else 1
    start = (nck - 1) * window
    return nck, start, nsteps - start


def forward_with_checkpoints(solver: Solver, case: dict, nsteps: int, window: int):
    """Equilibrium start from case, nsteps steps; returns the device states
    at steps 0, window, 2 window, ... (one row each), followed by the states
    of the last window after its checkpoint (x^{s+1} .. x^nsteps): the
    reverse sweep goes through that window first and need not recompute
    it.  The solver's own state ends at x^nsteps."""
    solver.init_case(case)
    nck, start, n_last = last_window(nsteps, window)
    ck = _states(solver, nck + n_last)
    for k in range(nck - 1):
        solver.lbf_state_to_device(ck[k])
        solver.lbf_step(window)
    solver.lbf_state_to_device(ck[nck - 1])
    for j in range(n_last):
        solver.lbf_step_states(ck[nck - 1 + j], ck[nck + j])
    if n_last > 0:
        solver.lbf_state_from_device(ck[nck + n_last - 1], nsteps)
    return ck


def reverse_sweep(solver: Solver, ck, nsteps: int, window: int, timing: dict = None,
                  objective: str = "frozen_fraction") -> tuple:
    """With the final state current: J and its gradient (dict) by the
    reverse steps.  The last window's states come with the checkpoints
    (forward_with_checkpoints); every earlier window is re-run forward from
    its checkpoint straight into a device tape (the solver's own state is
    not touched), which reuses the last window's rows once those are done.
    timing (a dict) receives the milliseconds spent in recomputation and in
    reverse steps, measured with events on the solver's stream."""
    import torch

    ev = []

    def mark():
        if timing is not None:
            e = torch.cuda.Event(enable_timing=True)
            e.record(solver.stream)
            ev.append(e)

    nck, s_last, n_last = last_window(nsteps, window)
    if ck.shape[0] != nck + n_last:
        raise ValueError("checkpoints do not match nsteps and window (use forward_with_checkpoints)")
    adj = Adjoint(solver)
    J = adj.seed(objective)
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
                tape = ck[nck:nck + window - 1] if n_last >= window - 1 else _states(solver, window - 1)
            states = [ck[k]] + [tape[j] for j in range(n - 1)] + [ck[k + 1]]
            for j in range(1, n):
                solver.lbf_step_states(states[j - 1], states[j])
        mark()
        for j in range(n - 1, -1, -1):
            adj.step(states[j], states[j + 1])
        mark()
    adj.finish(ck[0])
    g = adj.gradient()
    adj.close()
    if timing is not None:
        torch.cuda.synchronize(solver.device)
        rec = sum(ev[i].elapsed_time(ev[i + 1]) for i in range(0, len(ev), 3))
        rev = sum(ev[i + 1].elapsed_time(ev[i + 2]) for i in range(0, len(ev), 3))
        timing["recompute_ms"] = rec
        timing["reverse_ms"] = rev
    return J, g


def tape_bytes(solver: Solver, nsteps: int) -> int:
    """Device bytes of the full tape of an nsteps run (nsteps + 1 states)."""
    return (nsteps + 1) * solver.state_device_bytes()


def choose_window(solver: Solver, nsteps: int, window=None) -> int:
    """window as given, else 0 (the whole trajectory in a device tape, no
    recomputation) when that tape fits in half the free device memory, else
    checkpoints every 50 steps."""
    if window is not None:
        return int(window)
    import torch
    free, _ = torch.cuda.mem_get_info(solver.device)
    return 0 if tape_bytes(solver, nsteps) < 0.5 * free else 50


def forward_to_tape(solver: Solver, case: dict, nsteps: int):
    """Equilibrium start from case, then nsteps steps written straight into
    a device tape (row j = x^j, nsteps + 1 rows, no copies); the solver's
    own state ends at x^nsteps."""
    solver.init_case(case)
    tape = _states(solver, nsteps + 1)
    solver.lbf_state_to_device(tape[0])
    for j in range(1, nsteps + 1):
        solver.lbf_step_states(tape[j - 1], tape[j])
    solver.lbf_state_from_device(tape[nsteps], nsteps)
    return tape


def reverse_from_tape(solver: Solver, tape, nsteps: int, timing: dict = None,
                      objective: str = "frozen_fraction") -> tuple:
    """J and its gradient from the full tape of :func:`forward_to_tape`, with
    no recomputation; timing (a dict) receives the milliseconds of the
    reverse steps (events on the solver's stream)."""
    import torch

    adj = Adjoint(solver)
    J = adj.seed(objective)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(solver.stream)
    for j in range(nsteps - 1, -1, -1):
        adj.step(tape[j], tape[j + 1])
    e1.record(solver.stream)
    adj.finish(tape[0])
    g = adj.gradient()
    adj.close()
    if timing is not None:
        torch.cuda.synchronize(solver.device)
        timing["reverse_ms"] = e0.elapsed_time(e1)
    return J, g


def case_with(case: dict, T_w=None, latent=None, cos_theta=None) -> dict:
    """A copy of case whose parameters take T_face[0] = T_w, latent[:N] and
    cos_theta[:N, :N] (plain floats / arrays)."""
    c = dict(case)
    prm = copy.deepcopy(case["params"])
    N = prm["nphase"]
    if T_w is not None:
        prm["T_face"] = [float(T_w), float(prm["T_face"][1])]
    if latent is not None:
        lat = list(prm["latent"])
        for p in range(N):
            lat[p] = float(latent[p])
        prm["latent"] = lat
    if cos_theta is not None:
        ct = [list(r) for r in prm["cos_theta"]]
        for p in range(N):
            for q in range(N):
                ct[p][q] = float(cos_theta[p][q])
        prm["cos_theta"] = ct
    c["params"] = prm
    make_params(prm)  # validates the layout of the dict
    return c


def frozen_fraction_and_gradient(case: dict, nsteps: int, window=None, device: int = 0,
                                 objective: str = "frozen_fraction"):
    """Forward run with checkpoints, then the reverse sweep: (J, gradient)
    of the objective ("frozen_fraction" or "front").  window = 0 keeps the
    whole trajectory on the device (no recomputation); None chooses that
    when it fits (choose_window)."""
    s = Solver(case["params"], device=device)
    window = choose_window(s, nsteps, window)
    if window == 0:
        tape = forward_to_tape(s, case, nsteps)
        J, g = reverse_from_tape(s, tape, nsteps, objective=objective)
    else:
        ck = forward_with_checkpoints(s, case, nsteps, window)
        J, g = reverse_sweep(s, ck, nsteps, window, objective=objective)
    s.close()
    return J, g


def _torch_function():
    import torch

    class FrozenFraction(torch.autograd.Function):
        """J = the objective after nsteps (frozen fraction or front
        position), as a function of T_w (0-d), latent (N,) and cos_theta
        (N, N) float64 CPU tensors.  The forward keeps checkpoints on the
        GPU; backward runs the reverse sweep."""

        @staticmethod
        def forward(ctx, T_w, latent, cos_theta, case, nsteps, window, device=0, objective="frozen_fraction"):
            c = case_with(case, float(T_w), latent.detach().cpu().numpy(),
                          cos_theta.detach().cpu().numpy())
            s = Solver(c["params"], device=device)
            window = choose_window(s, nsteps, window)
            ck = forward_to_tape(s, c, nsteps) if window == 0 else forward_with_checkpoints(s, c, nsteps, window)
            d = s.lbf_diagnostics()
            N = s.N
            frz = [p for p in range(N) if c["params"]["freezes"][p]]
            area = s.shape[2] * (s.shape[1] if s.dim == 3 else 1)
            B = float(sum(d["vol"][p] for p in frz))
            J = d["front"] if objective == "front" else d["front"] * area / B
            ctx.solver, ctx.ck, ctx.nsteps, ctx.window = s, ck, nsteps, window
            ctx.objective = objective
            ctx.shapes = (latent.shape, cos_theta.shape)
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            if ctx.window == 0:
                _, g = reverse_from_tape(ctx.solver, ctx.ck, ctx.nsteps, objective=ctx.objective)
            else:
                _, g = reverse_sweep(ctx.solver, ctx.ck, ctx.nsteps, ctx.window, objective=ctx.objective)
            N = ctx.solver.N
            gT = torch.tensor(g["T_face"][0], dtype=torch.float64) * gJ
            gL = torch.tensor(g["latent"][:N], dtype=torch.float64) * gJ
            gC = torch.tensor(g["cos_theta"], dtype=torch.float64) * gJ
            ctx.solver.close()
            ctx.solver = ctx.ck = None
            return gT, gL, gC, None, None, None, None, None

    return FrozenFraction


_FF = None


def frozen_fraction(T_w, latent, cos_theta, case: dict, nsteps: int, window=None, device: int = 0):
    """torch entry point: the frozen fraction J(T_w, latent, cos_theta) with
    autograd support."""
    global _FF
    if _FF is None:
        _FF = _torch_function()
    return _FF.apply(T_w, latent, cos_theta, case, nsteps, window, device, "frozen_fraction")


def front_position(T_w, latent, cos_theta, case: dict, nsteps: int, window=None, device: int = 0):
    """torch entry point: the front position s(T_w, latent, cos_theta) =
    sum f_s psi / (cells per wall layer) with autograd support."""
    global _FF
    if _FF is None:
        _FF = _torch_function()
    return _FF.apply(T_w, latent, cos_theta, case, nsteps, window, device, "front")
