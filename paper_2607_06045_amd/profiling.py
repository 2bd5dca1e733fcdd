"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_2607_06045_amd.profiling stats --csv RUN_kernel_stats.csv \\
      --out profiles/kernels_blast22k.txt --command "..."
      per-kernel call count and mean / min / max duration of a --kernel-trace
      --stats run, as a short text table

  python -m paper_2607_06045_amd.profiling counters --fetch DIR --write DIR \\
      --copy-fetch DIR --copy-write DIR --copy-mib 512 --sq DIR [DIR ...] \\
      --kernel k_stage --dofs D --algorithmic-bytes-per-node B \\
      --out profiles/counters_....json
      per launch of one kernel: HBM bytes from a FETCH_SIZE pass and a
      WRITE_SIZE pass (KiB per dispatch), each scaled by the ratio of known
      bytes to what the same counter reads for a plain device copy of
      --copy-mib MiB; and the instruction counters (SQ_INSTS_*) of the --sq
      passes, as wave instructions per launch and lane instructions per node

  python -m paper_2607_06045_amd.profiling copy --mib 512
      a plain device-to-device copy of known size, the calibration workload of
      the FETCH_SIZE / WRITE_SIZE counters
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCE = os.path.join(ROOT, "paper_2607_06045_amd", "csrc", "dgidp_kernels.hip")


def kernel_source_hash():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _counter_rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _mean_counter_opt(rows, name_part, counter):
    """Counter per launch of the kernels whose names contain name_part: the
    mean over the dispatches of each matching kernel, summed over the matching
    kernels (one stage of the element kernel is a launch of each of its
    variants that the mesh needs), and the number of dispatches per kernel."""
    per = {}
    for r in rows:
        if name_part in r["Kernel_Name"] and r["Counter_Name"] == counter:
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    if not per:
        return None, 0
    return sum(sum(v) / len(v) for v in per.values()), {k.split("(")[0]: len(v) for k, v in per.items()}


def _mean_counter(rows, name_part, counter):
    v, k = _mean_counter_opt(rows, name_part, counter)
    if v is None:
        raise SystemExit(f"no {counter} rows for kernels matching {name_part!r}")
    return v, k


def counters(a):
    f_kib, nf = _mean_counter(_counter_rows(a.fetch), a.kernel, "FETCH_SIZE")
    w_kib, nw = _mean_counter(_counter_rows(a.write), a.kernel, "WRITE_SIZE")
    cf_kib, _ = _mean_counter(_counter_rows(a.copy_fetch), a.copy_kernel, "FETCH_SIZE")
    cw_kib, _ = _mean_counter(_counter_rows(a.copy_write), a.copy_kernel, "WRITE_SIZE")
    known_kib = a.copy_mib * 1024.0
    ff, wf = known_kib / cf_kib, known_kib / cw_kib
    fetch_b = f_kib * 1024.0 * ff
    write_b = w_kib * 1024.0 * wf
    alg = a.algorithmic_bytes_per_node * a.dofs if a.dofs else None
    out = {
        "kernel": a.kernel, "workload": a.workload,
        "fetch_kib_per_dispatch_raw": f_kib, "write_kib_per_dispatch_raw": w_kib,
        "dispatches": [nf, nw],
        "copy_calibration": {"mib": a.copy_mib, "fetch_kib_raw": cf_kib, "write_kib_raw": cw_kib,
                             "fetch_factor": ff, "write_factor": wf},
        "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
        "hbm_bytes_per_launch": fetch_b + write_b,
        "algorithmic_bytes_per_launch": alg,
    }
    # instruction counters: wave instructions per dispatch of the kernel
    sq = {}
    for d in a.sq or []:
        rows = _counter_rows(d)
        for c in sorted({r["Counter_Name"] for r in rows}):
            v, k = _mean_counter_opt(rows, a.kernel, c)
            if v is not None:
                sq[c] = v
    if sq:
        out["sq_per_launch"] = sq
        vw = sq.get("SQ_INSTS_VALU")
        if vw:
            out["valu_wave_insts_per_launch"] = vw
            if a.dofs:
                out["valu_lane_insts_per_node"] = vw * 64.0 / a.dofs
            f64 = sum(sq.get(k, 0.0) for k in ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
                                               "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64"))
            if f64:
                out["valu_f64_share"] = f64 / vw
    out["kernel_source_sha256_16"] = kernel_source_hash()
    out["command"] = a.command
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def copy(a):
    import torch
    n = a.mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(a.reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}", flush=True)


def timed_region(a):
    """Mean duration of the last --tail dispatches of --kernel in the kernel trace
    (bench.py's kernel-timing region) beside the HIP-event figure that the same
    profiled bench.py run printed for that kernel."""
    with open(a.trace_csv) as fh:
        rows = [r for r in csv.DictReader(fh) if r["Kernel_Name"].startswith("void dgidp::" + a.kernel)]
    if not rows:
        raise SystemExit(f"no dispatches of {a.kernel!r} in {a.trace_csv}")
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    # per kernel whose name starts so (the variants of one stage, launched
    # side by side on two streams): the mean over its last --tail dispatches;
    # one stage spans from the first start to the last end of its i-th
    # dispatches
    per = {}
    for r in rows:
        per.setdefault(r["Kernel_Name"].split("(")[0], []).append(
            (int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    out = []
    for k, d in per.items():
        d = d[-a.tail:]
        m = sum((e - b) / 1e3 for b, e in d) / len(d)
        out.append(f"# {k}: mean over its last {len(d)} dispatches (bench.py's kernel-timing region): "
                   f"{m:.2f} us")
    runs = [d[-a.tail:] for d in per.values()]
    ns = min(len(d) for d in runs)
    spans = [(max(d[i][1] for d in runs) - min(d[i][0] for d in runs)) / 1e3 for i in range(ns)]
    mean = sum(spans) / ns
    if len(per) > 1:
        out.append(f"# one stage (first start to last end of {' and '.join(per)}): {mean:.2f} us "
                   f"over {ns} stages")
    if a.bench_log:
        with open(a.bench_log) as fh:
            js = [json.loads(l) for l in fh if l.startswith('{"metric"')]
        if js:
            live = js[-1]["roofline"]["kernel_ms"] * 1e3
            out.append(f"# same run, bench.py's HIP-event figure for that kernel: {live:.2f} us "
                       f"(trace / events = {mean / live:.3f})")
    return out


def stats(a):
    with open(a.csv) as fh:
        rows = list(csv.DictReader(fh))
    lines = [f"# {a.title}", f"# command: {a.command}", "",
             f"{'kernel':60s} {'calls':>6s} {'mean_us':>9s} {'min_us':>8s} {'max_us':>8s} {'pct':>6s}"]
    for r in rows:
        name = r["Name"].split("(")[0][:60]
        lines.append(f"{name:60s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} "
                     f"{float(r['MinNs']) / 1e3:8.2f} {float(r['MaxNs']) / 1e3:8.2f} "
                     f"{float(r['Percentage']):6.2f}")
    if a.trace_csv and a.kernel and a.tail > 0:
        lines += [""] + timed_region(a)
    text = "\n".join(lines) + "\n"
    with open(a.out, "w") as fh:
        fh.write(text)
    print(text)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("counters")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--sq", nargs="*", default=[])
    t.add_argument("--copy-mib", type=float, default=512)
    t.add_argument("--copy-kernel", default="copyBuffer")
    t.add_argument("--kernel", default="k_stage")
    t.add_argument("--workload", default="")
    t.add_argument("--dofs", type=int, default=0)
    t.add_argument("--algorithmic-bytes-per-node", type=float, default=0.0)
    t.add_argument("--command", default="")
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--title", default="rocprofv3 kernel statistics")
    s.add_argument("--command", default="")
    s.add_argument("--trace-csv", default="")
    s.add_argument("--kernel", default="")
    s.add_argument("--tail", type=int, default=0)
    s.add_argument("--bench-log", default="")
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=512)
    c.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    {"counters": counters, "stats": stats, "copy": copy}[a.mode](a)


if __name__ == "__main__":
    sys.exit(main())
