"""Small fixed workloads for profiling runs.

  python -m paper_2607_06045_amd.probes copy --mib 512
      a plain device-to-device copy of known size (calibrates rocprofv3's
      FETCH_SIZE / WRITE_SIZE counters against known bytes)
"""
import argparse
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["copy"])
    ap.add_argument("--mib", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    import torch
    n = a.mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(a.reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
