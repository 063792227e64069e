"""Plain device-to-device copy of a known size, run under rocprofv3 counter
collection to calibrate FETCH_SIZE / WRITE_SIZE against known HBM traffic.

  python -m paper_2603_22902_amd.copy_probe [--mib 1024] [--reps 5]

Each repetition copies --mib MiB from one buffer to another (one read and
one write of every byte).
"""
import argparse
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    import torch

    n = a.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}", file=sys.stderr)


if __name__ == "__main__":
    main()
