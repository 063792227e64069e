"""Forward run with checkpoints and the reverse sweep on a 2D workload,
printing J (the frozen fraction, or the front position) and its gradient.

  python paper_2603_22902_amd/adjoint_run.py [--workload compound|droplet]
        [--steps 100] [--window 50] [--precision fp32|fp64]
        [--objective frozen_fraction|front] [--batch NCASES]

With --batch, the batched sweep over NCASES uneven droplet cases (sides 64
to 512, N 2 or 3, contact angle and Stefan number drawn per case): packed
checkpoints from the captured forward graph, batched recomputation and
batched reverse steps.  The start is the fields with the temperature just
above melting (freezing begins at once), so that J and its gradient are
non-zero."""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="compound", choices=["compound", "droplet"])
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--window", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--objective", default="frozen_fraction", choices=["frozen_fraction", "front"])
    ap.add_argument("--batch", type=int, default=0)
    a = ap.parse_args()
    import torch

    import synth
    from paper_2603_22902_amd import Solver
    from paper_2603_22902_amd.adjoint import forward_with_checkpoints, reverse_sweep

    if a.batch > 0:
        from paper_2603_22902_amd.batch import Batch, batch_forward_with_checkpoints, batch_reverse_sweep
        cases = [synth.near_melting(c) for c in synth.batch(n_cases=a.batch, precision=a.precision)]
        solvers = []
        for c in cases:
            s = Solver(c["params"])
            s.init_case(c)
            solvers.append(s)
        b = Batch(solvers)
        print(f"cases {len(cases)}, cells {sum(s.ncell for s in solvers)}, tiles {b.tune(2)}", flush=True)
        b.capture()
        ck = batch_forward_with_checkpoints(b, a.steps, a.window, graph=True)
        t = {}
        J, g = batch_reverse_sweep(b, ck, a.steps, a.window, objective=a.objective, timing=t)
        torch.cuda.synchronize()
        print(f"J min {J.min():.6g} max {J.max():.6g}")
        print(f"dJ/dT_face[0] per case {g[:, 0].tolist()}")
        print(f"recompute {t['recompute_ms']:.2f} ms, reverse steps {t['reverse_ms']:.2f} ms")
        return

    case = synth.near_melting(synth.WORKLOADS[a.workload](precision=a.precision))
    s = Solver(case["params"])
    ck = forward_with_checkpoints(s, case, a.steps, a.window)
    t = {}
    J, g = reverse_sweep(s, ck, a.steps, a.window, timing=t, objective=a.objective)
    torch.cuda.synchronize()
    print(f"J {J:.10g}")
    print(f"dJ/dT_face {g['T_face']}")
    print(f"dJ/dlatent {g['latent']}")
    print(f"dJ/dcos_theta {g['cos_theta'].tolist()}")
    print(f"recompute {t['recompute_ms']:.2f} ms, reverse steps {t['reverse_ms']:.2f} ms")


if __name__ == "__main__":
    main()
