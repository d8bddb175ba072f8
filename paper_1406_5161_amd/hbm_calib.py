"""Calibration run for HBM byte counters: device-to-device copies of a known size.

    python -m paper_1406_5161_amd.hbm_calib [--mib 1024] [--reps 4]

Each repetition copies `mib` MiB from one device buffer to another (torch's
copy kernel reads and writes exactly that many bytes).  Profiled with
rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE), the counter value per copy
dispatch against the known size gives the factor that turns the counters of
other kernels into bytes.
"""
import argparse


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=4)
    a = ap.parse_args()
    import torch
    n = a.mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied %d x %d MiB" % (a.reps, a.mib), flush=True)


if __name__ == "__main__":
    main()
