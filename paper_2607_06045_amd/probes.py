"""Small fixed workloads for profiling runs.

  python -m paper_2607_06045_amd.probes copy --mib 512
      a plain device-to-device copy of known size (calibrates rocprofv3's
      FETCH_SIZE / WRITE_SIZE counters against known bytes)

  python -m paper_2607_06045_amd.probes throughput --workload shear59k --precision fp64
      SSP-RK3 steps of one of the synthetic workloads (vortex304, blast22k,
      shear59k: N = 3; quadrants247k: N = 4) and the stage-kernel time;
      prints one JSON line
"""
import argparse
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["copy", "throughput"])
    ap.add_argument("--mib", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--workload", default="shear59k")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--steps", type=int, default=50)
    a = ap.parse_args(argv)
    if a.mode == "throughput":
        return throughput(a)
    import torch
    n = a.mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(a.reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}", flush=True)


def throughput(a):
    import json
    import os
    import time
    import torch
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_2607_06045_amd as P
    from workloads import states
    from workloads.meshes import workload_mesh, workload_order
    N = workload_order(a.workload)
    spec = workload_mesh(a.workload)
    s = P.Solver(N, precision=P.MIXED if a.precision == "mixed" else P.FP64)
    s.set_mesh(*spec.args())
    x, y = s.node_coords()
    s.upload(states.workload_state(a.workload, x, y))
    for _ in range(3):
        s.step(0.5, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s.step(0.5, stats=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = s.step(0.5)
    km = s.time_kernels(reps=20)
    dofs = s.E * (N + 1) ** 2
    alg = (64.0 + 96.0 + 96.0) / 3.0 * dofs
    print(json.dumps({"workload": a.workload, "N": N, "precision": a.precision, "elements": s.E,
                      "mortars": s.M, "dof_updates_per_s": dofs * 3 * a.steps / el,
                      "ms_per_step": el / a.steps * 1e3, "stage_ms": km["stage"],
                      "stage_hbm_frac": alg / (km["stage"] * 1e-3) / 8e12,
                      "mortar_ms": km["mortar"], "dt_ms": km["dt"],
                      "violations": st["violations"]}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
