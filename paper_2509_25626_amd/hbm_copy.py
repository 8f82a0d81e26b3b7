"""Plain device-to-device copy of a known size, for calibrating HBM traffic
counters (rocprofv3 FETCH_SIZE / WRITE_SIZE): the copy moves exactly
`--gib` GiB in and out per repetition.

    python -m paper_2509_25626_amd.hbm_copy [--gib 1] [--reps 3]
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gib", type=int, default=1)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    n = (a.gib << 30) // 4
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(a.reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {a.reps} x {a.gib} GiB", flush=True)


if __name__ == "__main__":
    main()
