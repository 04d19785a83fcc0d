"""Plain device-to-device copy of a known size, for calibrating HBM counters.

Run under `rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE): each copy kernel
reads and writes exactly --mib MiB, so counter / (mib * 1024) KiB gives the
scale between the counter and true bytes moved.
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=2048)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    n = a.mib * (1 << 20)
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}", flush=True)


if __name__ == "__main__":
    main()
