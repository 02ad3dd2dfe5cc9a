"""Calibration workload for the HBM traffic counters.

Copies a buffer of known size a few times on the GPU (one plain device copy
per repetition), so that what FETCH_SIZE and WRITE_SIZE report for that copy
can be compared with the bytes it must move:

    python3 -m paper_2204_04678_amd.pmc_copy [MiB] [repetitions]
"""
import sys

import torch


def main(mib: int = 1024, reps: int = 4) -> None:
    n = mib * (1 << 20) // 8
    x = torch.arange(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps}: {n * 8} bytes read and written per copy", flush=True)


if __name__ == "__main__":
    args = [int(a) for a in sys.argv[1:3]]
    main(*args)
