"""Throughput of the IDP-limited LGL-DGSEM hot path on one MI355X.

One step = one SSP-RK3 step of the whole path: the IDP time step, then three
stages of (high-order and low-order fluxes, volume limiter, mortar limiter, SSP
combination).

Headline workload "quadrants247k": 2D Euler (gamma = 1.4) on [0,1]^2,
periodic, 256^2 base mesh refined by two levels within 0.022 of the four
periodic discontinuity lines x, y in {0, 0.5} and 2:1 balanced: 246,736
leaves, 5,536 mortars, N = 4 (6,168,400 DOF, one FP64 state 197 MB); four
constant quadrant states drawn from seed 5 (rho in [0.1, 1.5], p in
[0.03, 1.5], v in [-1, 1]^2); positivity limiting; IDP time step at CFL 0.5.
Its three state buffers (3 x 197 MB) do not fit the 256 MB last-level cache,
so the stage kernel streams from HBM.  Inputs are synthetic, generated on the
host from the library's node coordinates, and resident in HBM before the
timed region starts.

Further legs (same JSON line): the mixed-precision mode on the same workload
with its error against the FP64 run of the same steps; the 22,156-leaf blast
and the 59,392-leaf shear layer (N = 3) in FP64 and mixed; the other limiter
modes on the blast; the CPU oracle on a bounded sample of the headline
workload, single-threaded and on all host cores.

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
# MI355X: 256 compute units of 4 SIMDs; a wave64 VALU instruction occupies its
# SIMD for 4 cycles; peak engine clock 2.4 GHz
SIMDS = 1024
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector peak
CLOCK_HZ = 2.4e9
# algorithmic HBM bytes of the element stage kernel per node and launch: the
# first stage reads u and writes u^(1) (64 B); the other two also read u^n
# (96 B); averaged over the three launches of a step
STAGE_BYTES_PER_NODE = (64.0 + 96.0 + 96.0) / 3.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_2607_06045_amd", "csrc", "dgidp_kernels.hip")
HEADLINE = "quadrants247k"
DESCRIBE = {
    "quadrants247k": "four-quadrant Riemann states (seed 5) on [0,1]^2 periodic, 256^2 base "
                     "+2 levels within 0.022 of x,y in {0,0.5}: 246736 leaves, 5536 mortars, "
                     "N=4 (6168400 DOF), positivity limiting, IDP dt CFL 0.5",
    "blast22k": "sedov-gaussian blast, 22156 leaves (64^2 base +3 levels, r<=0.3), 552 mortars, "
                "N=3, positivity limiting, IDP dt CFL 0.5",
    "shear59k": "shear layer, 59392 leaves (128^2 base +3 levels in a band), 3584 mortars, N=3, "
                "positivity limiting, IDP dt CFL 0.5",
}


def kernel_hash():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def committed_counters(workload):
    """rocprofv3 counter summary of the stage kernel on this workload, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"counters_k_stage_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return d


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


def cpu_baseline(spec, N, name, all_core_seconds=6.0):
    """The oracle as it stands, timed on this host's cores on a bounded sample
    of the same workload: whole SSP-RK3 steps of the same mesh and state, one
    step single-threaded, then steps on all cores for about all_core_seconds."""
    import oracle as O
    from workloads import states
    cores = len(os.sched_getaffinity(0))
    M = O.Mesh(N, *spec.args())
    x, y, m = M.geometry()
    u0 = states.workload_state(name, x, y)
    dofs = M.E * (N + 1) ** 2

    def timed(threads, min_seconds):
        used = O.set_threads(threads)
        u = u0
        t0 = time.perf_counter()
        steps = 0
        while True:
            u, _ = M.ssprk3(u, 0.5)
            steps += 1
            if time.perf_counter() - t0 > min_seconds:
                break
        return used, steps, time.perf_counter() - t0

    t1, s1, d1 = timed(1, 0.0)
    tn, sn, dn = timed(cores, all_core_seconds)
    return {"value": dofs * 3 * sn / dn, "unit": "DOF-updates/s", "cores": tn, "kind": "oracle",
            "sample": f"{sn} SSP-RK3 steps of the {name} workload ({M.E} leaves, N={N}), {dn:.1f} s, "
                      f"OpenMP over elements on {tn} threads",
            "single_thread": {"value": dofs * 3 * s1 / d1, "unit": "DOF-updates/s", "cores": t1,
                              "sample": f"{s1} SSP-RK3 step of the same workload, {d1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--legs", choices=["all", "none"], default="all",
                    help="none: the headline workload in FP64 only (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2607_06045_amd as P
    from workloads import states
    from workloads.meshes import workload_mesh, workload_order

    specs = {}

    def spec_of(name):
        if name not in specs:
            specs[name] = workload_mesh(name)
        return specs[name]

    def run(name, precision, limiter=P.LIMIT_POSITIVITY, dt_mode=P.DT_IDP, cfl=0.5):
        N = workload_order(name)
        s = P.Solver(N, gamma=1.4, beta=0.1, precision=precision, dt_mode=dt_mode, limiter=limiter)
        s.set_mesh(*spec_of(name).args())
        x, y = s.node_coords()
        s.upload(states.workload_state(name, x, y))
        for _ in range(args.warmup):
            s.step(cfl, stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s.step(cfl, stats=False)
        torch.cuda.synchronize()
        return s, time.perf_counter() - t0

    def dofs_of(s):
        return s.E * (s.N + 1) ** 2

    def hbm_frac(s, km):
        return STAGE_BYTES_PER_NODE * dofs_of(s) / (km["stage"] * 1e-3) / (HBM_PEAK_GBS * 1e9)

    def rel_err(a, b):
        """relative L1 per variable and the largest relative deviation per
        variable (against the variable's largest magnitude) of a against b"""
        a = a.reshape(a.shape[0], 4, -1)
        b = b.reshape(b.shape[0], 4, -1)
        l1 = [float(np.abs(a[:, v] - b[:, v]).sum() / max(np.abs(b[:, v]).sum(), 1e-300)) for v in range(4)]
        mx = [float(np.abs(a[:, v] - b[:, v]).max() / max(np.abs(b[:, v]).max(), 1e-300)) for v in range(4)]
        return {"rel_l1": l1, "rel_max": mx}

    # ---- headline: quadrants247k, FP64 ----
    name = HEADLINE
    s, elapsed = run(name, P.FP64)
    N, dofs = s.N, dofs_of(s)
    value = dofs * 3 * args.steps / elapsed
    u64 = s.download()
    # one more step with statistics: bounds and limiter activity of the run
    st = s.step(0.5, stats=True)
    km = s.time_kernels(reps=50)
    stage_bytes = STAGE_BYTES_PER_NODE * dofs
    achieved = stage_bytes / (km["stage"] * 1e-3) / 1e9
    # one stage: the launch over the element batches with a mortar element and
    # the launch over the others (the second template flag)
    kname = f"k_stage<{N}, 0, false, 0, true> + k_stage<{N}, 0, false, 0, false>"
    cnt = committed_counters(name)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": cnt["hbm_bytes_per_launch"] if cnt else None,
            "kernel": kname, "kernel_ms": km["stage"], "bytes_per_launch": stage_bytes,
            "other_kernels_ms": {"k_mortar": km["mortar"], "k_dt": km["dt"]}}
    if cnt and cnt.get("valu_wave_insts_per_launch"):
        vw = cnt["valu_wave_insts_per_launch"]
        roof["valu"] = {
            "bound": "valu", "wave_insts_per_launch": vw,
            "lane_insts_per_node_stage": vw * 64.0 / dofs,
            "f64_share": cnt.get("valu_f64_share"),
            # issue-limited time of the counted instructions against the live
            # kernel duration: 4 cycles per wave instruction on 1,024 SIMDs
            "issue_floor_ms": vw * 4.0 / (SIMDS * CLOCK_HZ) * 1e3,
            "frac": vw * 4.0 / (SIMDS * CLOCK_HZ) / (km["stage"] * 1e-3),
            "source": f"profiles/counters_k_stage_{name}.json"}
        sq = cnt.get("sq_per_launch", {})
        if all(k in sq for k in ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64")):
            # FP64 arithmetic of the counted instructions (64 lanes each, an FMA
            # counting two) against the live duration and the FP64 vector peak
            flop = 64.0 * (sq["SQ_INSTS_VALU_ADD_F64"] + sq["SQ_INSTS_VALU_MUL_F64"] +
                           2.0 * sq["SQ_INSTS_VALU_FMA_F64"])
            tf = flop / (km["stage"] * 1e-3) / 1e12
            roof["valu"].update({"f64_tflops": tf, "f64_peak_tflops": FP64_PEAK_TFLOPS,
                                 "f64_frac": tf / FP64_PEAK_TFLOPS})
    copy_gbs = copy_bandwidth()
    roof["copy_gbs_measured"] = copy_gbs
    roof["frac_of_measured_copy"] = achieved / copy_gbs
    out = {
        "metric": METRIC, "value": value, "unit": "DOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{name}: {DESCRIBE[name]}", "elements": s.E, "mortars": s.M,
                   "dofs": dofs, "N": N},
        "roofline": roof,
        "run_stats": {"violations": st["violations"], "fv_inadmissible": st["fv_inadmissible"],
                      "theta_vol_min": st["theta_vol_min"], "theta_mort_min": st["theta_mort_min"],
                      "dt": st["dt"]},
    }
    del s
    if args.legs == "all":
        # the same workload and steps in the mixed mode (FP32 volume flux
        # differencing and mortar interpolation / projection; FP64 state,
        # bounds, limiter, update), with its error against the FP64 run
        sm, el_m = run(name, P.MIXED)
        err = rel_err(sm.download(), u64)
        stm = sm.step(0.5, stats=True)
        kmm = sm.time_kernels(reps=50)
        out["mixed"] = {"value": dofs * 3 * args.steps / el_m, "unit": "DOF-updates/s",
                        "speedup_vs_fp64": elapsed / el_m,
                        "ms_per_step": el_m / args.steps * 1e3, "kernel_ms": kmm["stage"],
                        "hbm_frac": hbm_frac(sm, kmm),
                        "dtype": "f64 state and limiter, f32 volume fluxes and mortar projection",
                        "error_vs_fp64": dict(err, steps=args.warmup + args.steps),
                        "violations": stm["violations"]}
        del sm
        legs = {}
        for wname in ("blast22k", "shear59k"):
            leg = {"workload": DESCRIBE[wname]}
            for prec, key in ((P.FP64, "fp64"), (P.MIXED, "mixed")):
                sw, el = run(wname, prec)
                kmw = sw.time_kernels(reps=50)
                stw = sw.step(0.5, stats=True)
                leg[key] = {"value": dofs_of(sw) * 3 * args.steps / el,
                            "ms_per_step": el / args.steps * 1e3, "kernel_ms": kmw["stage"],
                            "hbm_frac": hbm_frac(sw, kmw), "violations": stw["violations"]}
                del sw
            legs[wname] = leg
        out["legs"] = legs
        # the other limiter modes on the blast, FP64
        modes = {"local": (P.LIMIT_LOCAL, P.DT_IDP, 0.5),            # eq. Bounds_Barstates
                 "combined": (P.LIMIT_COMBINED, P.DT_IDP, 0.5),      # eq. combination_posLim_local
                 "local_lowsol": (P.LIMIT_LOCAL_LOWORDER, P.DT_LOWORDER, 0.4)}  # eq. Bounds_LowOrder
        for key, (lim, dtm, cfl) in modes.items():
            sl, el = run("blast22k", P.FP64, lim, dtm, cfl)
            stl = sl.step(cfl, stats=True)
            leg = {"workload": "blast22k", "value": dofs_of(sl) * 3 * args.steps / el,
                   "ms_per_step": el / args.steps * 1e3, "dtype": "f64",
                   "violations": stl["violations"], "dt": stl["dt"],
                   "alpha_vol_mean": stl["alpha_vol_mean"]}
            if lim != P.LIMIT_LOCAL_LOWORDER:
                leg["kernel_ms"] = sl.time_kernels(reps=50)["stage"]
            out[key] = leg
            del sl
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec_of(name), N, name)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
