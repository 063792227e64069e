"""Forward run with checkpoints and the reverse sweep on a 2D workload,
printing J (the frozen fraction) and its gradient.

  python paper_2603_22902_amd/adjoint_run.py [--workload compound|droplet]
        [--steps 100] [--window 50] [--precision fp32|fp64]

The start is the workload's fields with the temperature just above melting
(freezing begins at once), so that J and its gradient are non-zero."""
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
    a = ap.parse_args()
    import torch

    import synth
    from paper_2603_22902_amd import Solver
    from paper_2603_22902_amd.adjoint import forward_with_checkpoints, reverse_sweep

    case = synth.near_melting(synth.WORKLOADS[a.workload](precision=a.precision))
    s = Solver(case["params"])
    ck = forward_with_checkpoints(s, case, a.steps, a.window)
    t = {}
    J, g = reverse_sweep(s, ck, a.steps, a.window, timing=t)
    torch.cuda.synchronize()
    print(f"J {J:.10g}")
    print(f"dJ/dT_face {g['T_face']}")
    print(f"dJ/dlatent {g['latent']}")
    print(f"dJ/dcos_theta {g['cos_theta'].tolist()}")
    print(f"recompute {t['recompute_ms']:.2f} ms, reverse steps {t['reverse_ms']:.2f} ms")


if __name__ == "__main__":
    main()
