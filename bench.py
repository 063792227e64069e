"""Throughput of the coupled-LB time step on one MI355X.

One "step" is one time step of the whole coupled method (three LBs,
moments, enthalpy inversion, finite differences, interface physics,
collision and streaming) over the whole grid of one workload.  Default
workload: freezing with impurities, 192^3 D3Q19, N = 4, float32 storage
(the largest single-GPU configuration).  Inputs are generated in host
memory, uploaded, and resident in HBM before timing starts.

Prints one JSON line with MLUPS (million lattice updates per second, with
the conservation diagnostics inside the timed region: after every 100
steps and after the last step), the HBM roofline of the step (the state's
algorithmic bytes per step over the average durations of its two launches,
the moments and the collide pass, measured with HIP events on the
solver's stream around each launch), the same for each kernel, and the
FP64 CPU oracle timed on a bounded sample of the same workload.

  python bench.py [--steps K] [--warmup W] [--workload impurities|droplet|compound|film]
                  [--precision fp32|mixed|fp64] [--no-cpu-baseline]
  python bench.py --probe MIB   only the library's float4 copy and read
                                sweeps over MIB-MiB buffers (the known-size
                                kernels that calibrate the HBM counters)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "MLUPS of coupled LB step + % HBM roofline; adjoint/forward cost ratio"
KERNEL_SOURCES = ["lbf_step.h", "lbf_kernels.h", "lbf_lattice.h", "lbf_kernels_f32_ilp.hip"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_22902_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes_per_cell(dim: int, N: int, elt: int) -> dict:
    """Bytes per cell that each pass must move at least, and the step's
    state (every population and lagged field read once and written once).

    moments: reads g, h ((N+1) Q), D, q; writes phi_p, f_s (N+1).
    collide: reads f, g, h ((N+2) Q), phi_p and f_s at n and n-1 (2(N+1)),
             u^{n-1} (dim), q^{n-1}; writes f, g, h, u (dim), D, q.
    """
    Q = 9 if dim == 2 else 19
    return {"moments": elt * ((N + 1) * Q + 2 + (N + 1)),
            "collide": elt * (2 * (N + 2) * Q + 2 * (N + 1) + 2 * dim + 3),
            "step": 2 * elt * ((N + 2) * Q + (N + dim + 3))}


def algorithmic_bytes_reverse(dim: int, N: int, elt: int) -> dict:
    """Bytes per cell the two reverse-step passes must move at least (2D
    tiled passes; every value read once and written once).

    collide reverse: reads the populations of x^n and their adjoints
        (2 (N+2) Q), phi_p and f_s of x^n (N+1), the lagged fields it uses
        (N + dim + 2), the per-cell adjoint scalars (N+1) and the adjoints of
        u, D, q (dim + 2); writes the population adjoints ((N+2) Q) and its
        work planes (finite-difference, own-cell and lagged adjoints, rho H:
        2 N dim + 3 N + 2 dim + 5).
    gather: reads those work planes and the moments it reverses
        (2 N dim + 6 N + 2 dim + 8); writes the adjoint scalars and lagged
        fields (2 N + dim + 4).
    """
    Q = 9 if dim == 2 else 19
    col = elt * ((2 * (N + 2) * Q + 3 * N + 2 * dim + 6) + ((N + 2) * Q + 2 * N * dim + 3 * N + 2 * dim + 5))
    gat = elt * ((2 * N * dim + 6 * N + 2 * dim + 8) + (2 * N + dim + 4))
    return {"collide_reverse": col, "gather": gat, "reverse_step": col + gat}


def measured_traffic(workload: str, precision: str, kernel: str = "collide"):
    """HBM bytes per launch (kernel="collide") or per step (kernel="step",
    both launches) from the committed rocprofv3 counter summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch" if kernel == "collide" else "bytes_per_step")


def traffic_rate(workload: str, precision: str, ms: float) -> float:
    """Measured HBM bytes per second of the collide kernel at ms per launch."""
    return measured_traffic(workload, precision) / (ms * 1e-3)


def make_case(workload: str, precision: str):
    import synth
    fn = synth.WORKLOADS[workload]
    case = fn()
    case["params"]["precision"] = precision
    return case


def describe(case) -> dict:
    p = case["params"]
    shape = (p["nx"], p["ny"]) + ((p["nz"],) if p["dim"] == 3 else ())
    return {"workload": f"{case['name']} {'x'.join(map(str, shape))} D{p['dim']}Q{9 if p['dim'] == 2 else 19} "
                        f"N={p['nphase']}",
            "cells": int(p["nx"] * p["ny"] * (p["nz"] if p["dim"] == 3 else 1)),
            "nphase": p["nphase"], "lattice": f"D{p['dim']}Q{9 if p['dim'] == 2 else 19}",
            "storage": "f64" if p["precision"] == "fp64" else "f32",
            "diagnostics": "every 100 steps and after the last, inside the timed region"}


def cpu_baseline(case, budget_s: float = 20.0) -> dict:
    """The FP64 oracle on the same workload: initialisation, then whole
    steps until about budget_s seconds of stepping have passed (at least
    one step)."""
    import oracle
    o = oracle.Oracle(case["params"])
    o.init_case(case)
    ncell = case["T"].size
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el / steps * (steps + 1) > 1.5 * budget_s:
            break
    return {"value": ncell * steps / el / 1e6, "unit": "MLUPS", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{steps} full step(s) of the same {ncell}-cell workload in float64 "
                      f"({el:.1f} s, OpenMP over cells)",
            "host": host_info()}


def host_info() -> dict:
    """The host the oracle ran on: CPU model, logical CPUs, and a triad
    bandwidth (a = b + 3 c over 2^27 float64 per array, torch's CPU threads)
    for the oracle's own memory roofline."""
    import torch
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n = 1 << 27
    b = torch.ones(n, dtype=torch.float64)
    c = torch.ones(n, dtype=torch.float64)
    a = torch.empty(n, dtype=torch.float64)
    torch.add(b, c, alpha=3.0, out=a)
    best = float("inf")
    for _ in range(3):
        t0 = time.perf_counter()
        torch.add(b, c, alpha=3.0, out=a)
        best = min(best, time.perf_counter() - t0)
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "torch_threads": torch.get_num_threads(),
            "triad_GB_s": round(3 * n * 8 / best / 1e9, 1)}


def adjoint_leg(precision: str = "fp32", nsteps: int = 500, window: int = 50) -> dict:
    """Forward plus reverse sweep on the compound droplet (512^2 D2Q9, N=3)
    from a start just above melting, checkpoint every window steps:
    wall-clock of each part with events on the solver's stream, their
    ratio, and the gradient of the frozen fraction w.r.t. T_w and Ste
    (L_p = C_s (T_melt - T_w) / Ste for both freezing phases)."""
    import torch

    import synth
    from paper_2603_22902_amd import Solver
    import numpy as np

    from paper_2603_22902_amd.adjoint import (forward_to_tape, forward_with_checkpoints, reverse_from_tape,
                                               reverse_sweep, tape_bytes)

    case = synth.near_melting(synth.compound(precision=precision))
    prm = case["params"]
    s = Solver(prm)
    forward_with_checkpoints(s, case, window, window)  # warm-up
    reverse_sweep(s, forward_with_checkpoints(s, case, window, window), window, window)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(s.stream)
    ck = forward_with_checkpoints(s, case, nsteps, window)
    e1.record(s.stream)
    t = {}
    J, g = reverse_sweep(s, ck, nsteps, window, timing=t)
    e2.record(s.stream)
    torch.cuda.synchronize()
    fwd, bwd = e0.elapsed_time(e1), e1.elapsed_time(e2)
    # plain forward steps (no checkpoint copies) for the per-step ratio
    s.init_case(case)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.lbf_step(nsteps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / nsteps
    # the whole trajectory in an HBM-resident tape (no recomputation), when
    # it fits in half the free device memory
    full = None
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    need = tape_bytes(s, nsteps)
    if need < 0.5 * free:
        torch.cuda.synchronize()
        e0.record(s.stream)
        tape = forward_to_tape(s, case, nsteps)
        e1.record(s.stream)
        t2 = {}
        J2, g2 = reverse_from_tape(s, tape, nsteps, timing=t2)
        torch.cuda.synchronize()
        ftape = e0.elapsed_time(e1)
        full = {"tape_GB": round(need / 1e9, 2), "forward_to_tape_ms": round(ftape, 2),
                "reverse_ms": round(t2["reverse_ms"], 2),
                "ratio_vs_plain_forward": round(t2["reverse_ms"] / (step_ms * nsteps), 3),
                "ratio_vs_forward_to_tape": round(t2["reverse_ms"] / ftape, 3),
                "gradient_bitwise_equal_checkpointed": bool(J2 == J and np.array_equal(g2["raw"], g["raw"]))}
        del tape
        torch.cuda.empty_cache()
    N = prm["nphase"]
    Tw, Tm = prm["T_face"][0], synth.T_MELT
    frz = [p for p in range(N) if prm["freezes"][p]]
    dL = g["latent"]
    # L_p = C_s,p (T_m - T_w) / Ste (one Stefan number for the freezing phases)
    ste = prm["cp_s"][frz[0]] * (Tm - Tw) / prm["latent"][frz[0]]
    dJ_dSte = sum(dL[p] * (-prm["latent"][p] / ste) for p in frz)
    dJ_dTw = g["T_face"][0] + sum(dL[p] * (-prm["cp_s"][p] / ste) for p in frz)
    rb = algorithmic_bytes_reverse(2, N, 8 if precision == "fp64" else 4)
    rev_step_s = t["reverse_ms"] / nsteps * 1e-3
    ncell = prm["nx"] * prm["ny"]
    return {"workload": f"compound {prm['nx']}x{prm['ny']} D2Q9 N={N}, start just above melting",
            # both reverse passes against their algorithmic bytes (HBM bound)
            "reverse_roofline": {"bound": "hbm", "bytes_per_cell": rb["reverse_step"],
                                 "achieved": round(rb["reverse_step"] * ncell / rev_step_s / 1e9, 1),
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(rb["reverse_step"] * ncell / rev_step_s / 1e9 / HBM_PEAK_GBS, 4)},
            "steps": nsteps, "window": window, "precision": precision,
            "forward_ms": round(fwd, 2), "reverse_ms": round(bwd, 2),
            "ratio": round(bwd / fwd, 3),
            "reverse_step_ms": round(t["reverse_ms"] / nsteps, 4),
            "forward_step_ms": round(step_ms, 4),
            "ratio_no_recompute": round(t["reverse_ms"] / nsteps / step_ms, 3),
            # what the library's default (window=None) takes at this size:
            # the full tape when it fits in half the free memory
            "default_window": "full tape" if full else window,
            "ratio_default_window": full["ratio_vs_plain_forward"] if full else round(bwd / fwd, 3),
            "full_tape": full,
            "J": J, "dJ_dTw": float(dJ_dTw), "dJ_dSte": float(dJ_dSte)}


def batch_leg(nsteps: int = 200, precision: str = "fp32", adjoint: bool = True,
              relax_steps: int = 20000) -> dict:
    """The 64-case 2D sweep (sides 64..512, N 2 or 3): total-cells MLUPS of
    (a) the batch replayed from its captured graph after autotuning, (b) the
    same batch launched step by step, (c) the cases looped one by one with
    their own launches; each from the same start, timed with events.  The
    cases whose wall angle is not 90 degrees first relax isothermally (not
    timed) for at most relax_steps steps."""
    import torch

    import synth
    from paper_2603_22902_amd import Solver
    from paper_2603_22902_amd.batch import Batch, relax_contact_angles

    cases = synth.batch(n_cases=64, precision=precision)
    relaxed, rsteps, lengths = relax_contact_angles(cases, max_steps=relax_steps, chunk=1000) \
        if relax_steps > 0 else ([None] * len(cases), 0, {})
    solvers = []
    for c, st in zip(cases, relaxed):
        s = Solver(c["params"])
        s.init_case(c)
        if st is not None:
            s.lbf_state_from_device(st, 0)
        solvers.append(s)
    del relaxed
    relax = {"cases": len(lengths), "steps": rsteps,
             "max_wetted_change_last_1000": round(max((abs(b - a) for a, b in lengths.values()), default=0.0), 3)}
    print(f"[bench] contact-angle pre-relaxation {relax}", file=sys.stderr, flush=True)
    ncell = sum(s.ncell for s in solvers)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, stream):
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    # (c) looped single-case solves on the solvers' own stream
    for s in solvers:
        s.lbf_step(2)
    t_loop = timed(lambda: [s.lbf_step(nsteps) for s in solvers], solvers[0].stream)
    b = Batch(solvers)
    tiles = b.tune(10)
    b.step(2)
    t_eager = timed(lambda: b.step(nsteps), b.stream)
    b.capture()
    b.replay(1)
    t_graph = timed(lambda: b.replay(nsteps // 2), b.stream)
    mlups = lambda ms: round(ncell * nsteps / (ms * 1e-3) / 1e6, 1)
    # the same graph in each launch mode: one block per work item or
    # persistent blocks (resident count, striding over the items), the
    # phase-count groups on one stream or on parallel branches (the default)
    modes = {}
    for name, pers, conc in (("one_stream", False, False), ("persistent", True, False),
                             ("concurrent_groups", False, True), ("persistent_concurrent", True, True)):
        b.set_launch(persistent=pers, concurrent=conc)
        b.capture()
        b.replay(1)
        modes[name] = mlups(timed(lambda: b.replay(nsteps // 2), b.stream))
    out = {"workload": f"{len(cases)} 2D cases, sides 64..512, N 2 or 3, {ncell} cells",
           "steps": nsteps, "precision": precision, "tiles": {str(k): v for k, v in tiles.items()},
           "mlups_graph": mlups(t_graph), "mlups_batch_eager": mlups(t_eager), "graph_launch_modes": modes,
           "mlups_looped_single": mlups(t_loop),
           "speedup_graph_vs_looped": round(t_loop / t_graph, 3), "prerelaxation": relax}
    b.close()
    if adjoint:
        print(f"[bench] batch forward {out}; batched adjoint sweep next", file=sys.stderr, flush=True)
        out["adjoint"] = batch_adjoint_leg(cases, solvers, tiles, nsteps, window=50)
    return out


def batch_adjoint_leg(cases, solvers, tiles, nsteps: int, window: int) -> dict:
    """Forward plus reverse sweep of every case (frozen fraction, start just
    above melting): the batched sweep (forward from the captured graph with
    packed checkpoints, batched recomputation and reverse steps) against the
    same sweeps looped case by case; wall-clock seconds around each, after
    a device synchronisation.  Both give bitwise the same gradients."""
    import time

    import numpy as np
    import torch

    import synth
    from paper_2603_22902_amd.adjoint import forward_with_checkpoints, reverse_sweep
    from paper_2603_22902_amd.batch import (Batch, batch_forward_to_tape, batch_forward_with_checkpoints,
                                            batch_reverse_from_tape, batch_reverse_sweep)

    adj_cases = [synth.near_melting(c) for c in cases]
    for s, c in zip(solvers, adj_cases):
        s.init_case(c)
    ncell = sum(s.ncell for s in solvers)
    b = Batch(solvers)
    b.set_tiles(tiles)
    b.capture()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ck = batch_forward_with_checkpoints(b, nsteps, window, graph=True)
    b.synchronize()
    t1 = time.perf_counter()
    tm = {}
    J, g = batch_reverse_sweep(b, ck, nsteps, window, timing=tm)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    b.close()
    del ck
    # the same sweep from a full packed tape (no recomputation), if it fits
    full = None
    torch.cuda.empty_cache()
    for s, c in zip(solvers, adj_cases):
        s.init_case(c)
    b = Batch(solvers)
    b.set_tiles(tiles)
    need = (nsteps + 1) * b.state_bytes()
    free, _ = torch.cuda.mem_get_info()
    if need < 0.75 * free:
        try:
            torch.cuda.synchronize()
            t5 = time.perf_counter()
            tape = batch_forward_to_tape(b, nsteps)
            b.synchronize()
            t6 = time.perf_counter()
            t7 = {}
            J2, g2 = batch_reverse_from_tape(b, tape, nsteps, timing=t7)
            torch.cuda.synchronize()
            t8 = time.perf_counter()
            full = {"tape_GB": round(need / 1e9, 1), "forward_to_tape_s": round(t6 - t5, 4),
                    "reverse_s": round(t8 - t6, 4), "reverse_steps_ms": round(t7["reverse_ms"], 2),
                    "ratio_vs_graph_forward": round((t8 - t6) / (t1 - t0), 3),
                    "gradients_bitwise_equal_checkpointed": bool(np.array_equal(J2, J) and np.array_equal(g2, g))}
            del tape
        except torch.cuda.OutOfMemoryError:
            full = {"skipped": f"out of device memory for a {need / 1e9:.0f} GB tape"}
    else:
        full = {"skipped": f"a {need / 1e9:.0f} GB tape needs more than 3/4 of the free device memory"}
    b.close()
    torch.cuda.empty_cache()
    # the same sweeps, one case at a time
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    gl = []
    for s, c in zip(solvers, adj_cases):
        ckk = forward_with_checkpoints(s, c, nsteps, window)
        gl.append(reverse_sweep(s, ckk, nsteps, window)[1]["raw"])
        del ckk
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    fwd, rev, loop = t1 - t0, t2 - t1, t4 - t3
    return {"steps": nsteps, "window": window, "objective": "frozen_fraction",
            "forward_s": round(fwd, 4), "reverse_sweep_s": round(rev, 4),
            "recompute_ms": round(tm["recompute_ms"], 2), "reverse_steps_ms": round(tm["reverse_ms"], 2),
            "ratio_adjoint_forward": round(rev / fwd, 3),
            "mlups_forward_plus_adjoint": round(ncell * nsteps / (fwd + rev) / 1e6, 1),
            "looped_single_s": round(loop, 4),
            "speedup_vs_looped": round(loop / (fwd + rev), 3),
            "gradients_bitwise_equal_looped": bool(all(np.array_equal(g[k], gl[k]) for k in range(len(gl)))),
            "full_tape": full,
            # what adjoint.choose_window's policy takes for this batch: the
            # whole trajectory in HBM when it fits, else the checkpoints
            "default_window": "full tape" if full and "ratio_vs_graph_forward" in full else window,
            "ratio_default_window": (full["ratio_vs_graph_forward"] if full and "ratio_vs_graph_forward" in full
                                     else round(rev / fwd, 3)),
            "J_range": [float(J.min()), float(J.max())]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="impurities", choices=["impurities", "droplet", "compound", "film"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "mixed", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--probe", type=int, default=0, metavar="MIB")
    ap.add_argument("--relax-steps", type=int, default=20000,
                    help="isothermal pre-relaxation of the batch cases with a wall angle other than 90 deg")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solver's time step runs on one device; "
              "a multi-GPU slab decomposition is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_22902_amd import Solver

    if args.probe:
        from paper_2603_22902_amd.lbfreeze import bandwidth_probe
        bw = bandwidth_probe(0, mib=args.probe, reps=3)
        print(json.dumps({"probe_mib": args.probe, "reps": 3,
                          "bytes_per_copy_launch": 2 * (args.probe << 20),
                          "bytes_per_read_launch": args.probe << 20,
                          "copy_GB_s": round(bw["copy"] / 1e9, 1), "read_GB_s": round(bw["read"] / 1e9, 1)}))
        return

    case = make_case(args.workload, args.precision)
    prm = case["params"]
    print(f"[bench] workload {case['name']} precision {args.precision} steps {args.steps} "
          f"warmup {args.warmup}", file=sys.stderr, flush=True)
    s = Solver(prm)
    s.init_case(case)
    stream = s.stream
    ncell = s.ncell
    d0 = s.lbf_diagnostics(check_nan=False)
    s.lbf_step(args.warmup)
    torch.cuda.synchronize()
    # per-phase mass and front position every 100 steps of the timed run
    # (the diagnostics are part of the timed work)
    dlog = {"interval": "every 100 steps and after the last", "step": [], "front": [], "mass_drift_max_rel": []}

    # Timed region 1 (the metric): K steps with diagnostics every 100 steps.
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    done = 0
    while done < args.steps:
        n = min(100, args.steps - done)
        s.lbf_step(n)
        done += n
        d = s.lbf_diagnostics(check_nan=False)
        dlog["step"].append(args.warmup + done)
        dlog["front"].append(d["front"])
        dlog["mass_drift_max_rel"].append(d["mass"])
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms_total = start.elapsed_time(stop)
    print(f"[bench] timed {args.steps} steps: {ms_total:.2f} ms (host wall {wall * 1e3:.2f} ms)",
          file=sys.stderr, flush=True)

    # Timed region 2 (roofline): HIP events around each launch of K steps.
    k_steps = max(20, args.steps // 2)
    ms_mom, ms_col = s.lbf_step_timed(k_steps)
    diag = s.lbf_diagnostics(check_nan=False)
    print(f"[bench] moments {ms_mom * 1e3:.1f} us, collide {ms_col * 1e3:.1f} us per launch; "
          f"front {diag['front']:.4f} nonfinite {diag['nonfinite']}", file=sys.stderr, flush=True)

    # The same K steps as a whole job through the host boundary (context,
    # never the metric): float64 phi, T from host memory into the equilibrium
    # start, the steps, and every moment back to float64 host memory.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.init_case(case)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.lbf_step(args.steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.lbf_get_moments()
    t3 = time.perf_counter()
    host_io = {"init_fields_ms": round((t1 - t0) * 1e3, 2), "steps_ms": round((t2 - t1) * 1e3, 2),
               "get_moments_ms": round((t3 - t2) * 1e3, 2),
               # float64 fields up (phi, T, u and p if given) and down (every moment)
               "host_bytes": int(8 * ncell * (prm["nphase"] + 1 + (prm["dim"] if case.get("u") is not None else 0)
                                              + (1 if case.get("p") is not None else 0)
                                              + prm["nphase"] + prm["dim"] + 6)),
               "mlups_with_host_io": round(ncell * args.steps / (t3 - t0) / 1e6, 1)}
    print(f"[bench] with host I/O {host_io}", file=sys.stderr, flush=True)

    # same-box HBM rates of a plain float4 copy and read sweep, for context
    from paper_2603_22902_amd.lbfreeze import bandwidth_probe
    bw = bandwidth_probe(s.device)
    probe = {"copy_GB_s": round(bw["copy"] / 1e9, 1), "read_GB_s": round(bw["read"] / 1e9, 1),
             "collide_raw_vs_copy": round(traffic_rate(args.workload, args.precision, ms_col) / bw["copy"], 3)
             if measured_traffic(args.workload, args.precision) else None}
    elt = 8 if args.precision == "fp64" else 4
    bpc = algorithmic_bytes_per_cell(prm["dim"], prm["nphase"], elt)
    achieved = bpc["collide"] * ncell / (ms_col * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, args.precision)
    step_ms = ms_mom + ms_col
    step_achieved = bpc["step"] * ncell / (step_ms * 1e-3) / 1e9
    # the step's state bytes per second against the same box's copy rate
    probe["step_state_vs_copy"] = round(step_achieved * 1e9 / bw["copy"], 3)
    step_traffic = measured_traffic(args.workload, args.precision, kernel="step")
    ms_per_step = ms_total / args.steps
    mlups = ncell * args.steps / (ms_total * 1e-3) / 1e6
    dtype = {"fp32": "f32", "mixed": "f32 storage / f64 arithmetic", "fp64": "f64"}[args.precision]
    m0 = d0["mass"]
    masses = dlog.pop("mass_drift_max_rel")
    dlog["mass_drift_rel_per_phase"] = [[round(float((m[p] - m0[p]) / m0[p]), 7) if m0[p] != 0.0 else 0.0
                                         for p in range(len(m0))] for m in masses]
    dlog["front_initial"] = float(d0["front"])
    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic", "config": describe(case),
        # The step (its two launches together) against the state's bytes:
        # every population and lagged field read once and written once.
        "roofline": {"bound": "hbm", "achieved": round(step_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(step_achieved / HBM_PEAK_GBS, 4), "traffic": step_traffic,
                     "kernel": "step = moment_kernel + collide_kernel", "kernel_us": round(step_ms * 1e3, 2),
                     "bytes_per_cell": bpc["step"],
                     "dominant_kernel": {"kernel": "collide_kernel", "achieved": round(achieved, 1),
                                         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                                         "kernel_us": round(ms_col * 1e3, 2), "bytes_per_cell": bpc["collide"]}},
        "bandwidth_probe": probe,
        "host_io": host_io,
        "diagnostics": dlog,
        "kernels": {
            "moment_kernel": {"us": round(ms_mom * 1e3, 2), "bytes_per_cell": bpc["moments"],
                              "GB/s": round(bpc["moments"] * ncell / (ms_mom * 1e-3) / 1e9, 1)},
            "collide_kernel": {"us": round(ms_col * 1e3, 2), "bytes_per_cell": bpc["collide"],
                               "GB/s": round(achieved, 1)},
            "step": {"us": round((ms_mom + ms_col) * 1e3, 2), "state_bytes_per_cell": bpc["step"],
                     "GB/s": round(bpc["step"] * ncell / ((ms_mom + ms_col) * 1e-3) / 1e9, 1),
                     "mlups_kernels_only": round(ncell / ((ms_mom + ms_col) * 1e-3) / 1e6, 2)}},
    }
    del s
    torch.cuda.synchronize()
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg()
        print(f"[bench] adjoint leg {out['adjoint']}", file=sys.stderr, flush=True)
    if not args.no_batch:
        out["batch"] = batch_leg(relax_steps=args.relax_steps)
        print(f"[bench] batch leg {out['batch']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
