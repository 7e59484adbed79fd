"""Plain device-to-device copy of a known size (HBM traffic calibration).

    python -m paper_2509_17340_amd.hbm_copy [--mib 512] [--reps 5]

Hardware counters such as FETCH_SIZE / WRITE_SIZE are read for this copy (its
true traffic is exactly `mib` MiB read and written per repetition) to scale the
same counters of the planning kernels into bytes.
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}", flush=True)


if __name__ == "__main__":
    main()
