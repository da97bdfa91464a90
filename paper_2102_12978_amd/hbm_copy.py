"""Plain device-to-device copy of a known size, used to calibrate the HBM
byte counters (FETCH_SIZE, WRITE_SIZE) read by rocprofv3 --pmc.

    python -m paper_2102_12978_amd.hbm_copy [--mib 1024] [--reps 5]
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}: {a.mib * (1 << 20)} bytes read and written per copy")


if __name__ == "__main__":
    main()
