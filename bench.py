"""Throughput of the IDP-limited LGL-DGSEM hot path on one MI355X.

One step = one SSP-RK3 step of the whole path: the IDP time step, then three
stages of (high-order and low-order fluxes, volume limiter, mortar limiter, SSP
combination).  Workload: the Sedov-type blast "blast22k" (2D
Euler, gamma = 1.4, [-1,1]^2 periodic, 64^2 base mesh refined by three levels
inside r <= 0.3 and 2:1 balanced: 22,156 leaves, 552 mortars, N = 3,
rho = 1, v = 0, p = 1e-5 plus a Gaussian energy bump of width 0.06, positivity
limiting, CFL 0.5 on the IDP time step).  Inputs are synthetic and generated
on the host from the library's node coordinates, then resident in HBM.

Prints one JSON line.  value = DOF-updates/s = (elements (N+1)^2) x 3 stages x
steps / seconds.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s (RHS+IDP limiter+RK stage), FP64 vs mixed; % HBM roofline"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes of the element stage kernel per node and launch: the
# first stage reads u and writes u^(1) (64 B); the other two also read u^n
# (96 B); averaged over the three launches of a step
STAGE_BYTES_PER_NODE = (64.0 + 96.0 + 96.0) / 3.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_2607_06045_amd", "csrc", "dgidp_kernels.hip")


def kernel_hash():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(name):
    """HBM bytes per launch of the stage kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def copy_bandwidth(mib=1024, reps=10):
    """Measured device-to-device copy bandwidth (read + write bytes per second,
    GB/s) of a plain torch copy in this process: the practical HBM ceiling that
    the stage kernel's algorithmic bandwidth is also compared with."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        y.copy_(x)
    ev1.record()
    torch.cuda.synchronize()
    sec = ev0.elapsed_time(ev1) * 1e-3 / reps
    del x, y
    return 2.0 * mib * (1 << 20) / sec / 1e9


def cpu_baseline(spec, N, seconds=12.0):
    """The oracle as it stands, timed on this host's cores on a bounded sample
    of the same workload (whole SSP-RK3 steps of the same mesh and state)."""
    import numpy as np
    import oracle as O
    from workloads import states
    cores = len(os.sched_getaffinity(0))
    threads = O.set_threads(cores)
    M = O.Mesh(N, *spec.args())
    x, y, m = M.geometry()
    u = states.workload_state("blast22k", x, y)
    t0 = time.perf_counter()
    steps = 0
    while True:
        u, st = M.ssprk3(u, 0.5)
        steps += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    dofs = M.E * (N + 1) ** 2
    return {"value": dofs * 3 * steps / dt, "unit": "DOF-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} SSP-RK3 steps of the same 22,156-leaf blast workload, "
                      f"{dt:.1f} s, OpenMP over elements"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2607_06045_amd as P
    from workloads import states
    from workloads.meshes import workload_mesh

    N = 3
    spec = workload_mesh("blast22k")

    def run(precision, limiter=P.LIMIT_POSITIVITY, dt_mode=P.DT_IDP, cfl=0.5):
        s = P.Solver(N, gamma=1.4, beta=0.1, precision=precision, dt_mode=dt_mode,
                     limiter=limiter)
        s.set_mesh(*spec.args())
        x, y = s.node_coords()
        s.upload(states.workload_state("blast22k", x, y))
        for _ in range(args.warmup):
            s.step(cfl, stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s.step(cfl, stats=False)
        torch.cuda.synchronize()
        return s, time.perf_counter() - t0

    s, elapsed = run(P.FP64)
    dofs = s.E * (N + 1) ** 2
    value = dofs * 3 * args.steps / elapsed

    # one more step with statistics: bounds and limiter activity of the run
    st = s.step(0.5, stats=True)
    km = s.time_kernels(reps=50)
    stage_bytes = STAGE_BYTES_PER_NODE * dofs
    achieved = stage_bytes / (km["stage"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic("traffic_k_stage_blast22k.json"),
            "kernel": "k_stage<3>", "kernel_ms": km["stage"], "bytes_per_launch": stage_bytes,
            "other_kernels_ms": {"k_mortar": km["mortar"], "k_dt": km["dt"]}}
    copy_gbs = copy_bandwidth()
    roof["copy_gbs_measured"] = copy_gbs
    roof["frac_of_measured_copy"] = achieved / copy_gbs
    out = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "sedov-gaussian blast, 22156 leaves (64^2 base +3 levels, r<=0.3), "
                               "552 mortars, N=3, positivity limiting, IDP dt CFL 0.5",
                   "elements": s.E, "mortars": s.M, "dofs": dofs, "N": N},
        "roofline": roof,
        "run_stats": {"violations": st["violations"], "theta_vol_min": st["theta_vol_min"],
                      "theta_mort_min": st["theta_mort_min"], "dt": st["dt"]},
    }
    # the same workload in the mixed mode (FP32 volume flux differencing and
    # mortar interpolation / projection; FP64 state, bounds, limiter, update)
    sm, el_m = run(P.MIXED)
    stm = sm.step(0.5, stats=True)
    kmm = sm.time_kernels(reps=50)
    out["mixed"] = {"value": dofs * 3 * args.steps / el_m, "unit": "DOF-updates/s",
                    "ms_per_step": el_m / args.steps * 1e3, "kernel_ms": kmm["stage"],
                    "dtype": "f64 state and limiter, f32 volume fluxes and mortar projection",
                    "violations": stm["violations"]}
    # the same workload with local limiting (eq. Bounds_Barstates: bar-state
    # density and specific-entropy bounds on top of the positivity bounds), FP64
    sl, el_l = run(P.FP64, P.LIMIT_LOCAL)
    stl = sl.step(0.5, stats=True)
    kml = sl.time_kernels(reps=50)
    out["local"] = {"value": dofs * 3 * args.steps / el_l, "unit": "DOF-updates/s",
                    "ms_per_step": el_l / args.steps * 1e3, "kernel_ms": kml["stage"],
                    "dtype": "f64", "violations": stl["violations"],
                    "alpha_vol_mean": stl["alpha_vol_mean"]}
    # combined limiting (eq. combination_posLim_local): local factors where the
    # pressure shock indicator fires, positivity factors elsewhere, FP64
    sc, el_c = run(P.FP64, P.LIMIT_COMBINED)
    stc = sc.step(0.5, stats=True)
    kmc = sc.time_kernels(reps=50)
    out["combined"] = {"value": dofs * 3 * args.steps / el_c, "unit": "DOF-updates/s",
                       "ms_per_step": el_c / args.steps * 1e3, "kernel_ms": kmc["stage"],
                       "dtype": "f64", "violations": stc["violations"],
                       "alpha_vol_mean": stc["alpha_vol_mean"]}
    # local bounds from the low-order solution (eq. Bounds_LowOrder) with the
    # low-order time step at CFL 0.4, FP64: per step one more residual launch
    # and the bounds kernel; each step advances a larger dt
    so, el_o = run(P.FP64, P.LIMIT_LOCAL_LOWORDER, P.DT_LOWORDER, 0.4)
    sto = so.step(0.4, stats=True)
    out["local_lowsol"] = {"value": dofs * 3 * args.steps / el_o, "unit": "DOF-updates/s",
                           "ms_per_step": el_o / args.steps * 1e3, "dtype": "f64",
                           "violations": sto["violations"], "dt": sto["dt"], "dt_idp_cfl_0.5": st["dt"],
                           "alpha_vol_mean": sto["alpha_vol_mean"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, N)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
