#!/bin/bash
# rocprofv3 profiles of the benchmark workload (Sedov-type blast, 22,156 leaves,
# N = 3, FP64): kernel-trace statistics of bench.py, then a FETCH_SIZE pass and
# a WRITE_SIZE pass of the same benchmark and of a plain 512 MiB device copy
# (counter calibration).  Run from the repository root on a machine with the
# GPU; raw output and the two summaries go to $PROFILE_OUT (default prof_out,
# not tracked): kernels_k_stage_blast22k.txt, traffic_k_stage_blast22k.json
# under summary/.
set -o pipefail
ROOT=$(pwd)
OUT=$ROOT/${PROFILE_OUT:-prof_out}
mkdir -p "$OUT/summary"
cd /tmp && export TMPDIR=/tmp && cd "$ROOT" || exit 1
CMD="bash paper_2607_06045_amd/profile_bench.sh"
BT="python3 bench.py --steps 20 --warmup 2 --no-cpu-baseline"
BC="python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline"
CP="python3 -m paper_2607_06045_amd.probes copy --mib 512"

echo "== kernel trace: $BT"
timeout -k 10 300 rocprofv3 --kernel-trace --stats -d "$OUT/trace" -o trace --output-format csv -- $BT \
    > "$OUT/trace.log" 2>&1 || { echo "kernel trace failed"; tail -20 "$OUT/trace.log"; exit 1; }
tail -1 "$OUT/trace.log" | cut -c1-160
pmc() {
    local name=$1 counter=$2; shift 2
    echo "== $counter: $*"
    timeout -s KILL 120 rocprofv3 --pmc "$counter" -d "$OUT/$name" -o "$name" --output-format csv -- "$@" \
        > "$OUT/$name.log" 2>&1 || { echo "$name pass failed"; tail -20 "$OUT/$name.log"; exit 1; }
}
pmc fetch FETCH_SIZE $BC || exit 1
pmc write WRITE_SIZE $BC || exit 1
pmc copyfetch FETCH_SIZE $CP || exit 1
pmc copywrite WRITE_SIZE $CP || exit 1

STATS=$(find "$OUT/trace" -name '*kernel_stats.csv' | head -1)
python3 -m paper_2607_06045_amd.profiling stats --csv "$STATS" \
    --out "$OUT/summary/kernels_k_stage_blast22k.txt" \
    --title "kernel durations, bench.py workload (Sedov blast, 22,156 leaves, N=3; 20 steps + kernel timing, FP64 then mixed; k_stage<3, 0, false, 0> is the FP64 stage kernel, <3, 0, true, 0> the mixed one)" \
    --command "$CMD" --trace-csv "$(find "$OUT/trace" -name '*kernel_trace.csv' | head -1)" \
    --kernel "k_stage<3, 0, false, 0>" --tail 150 --bench-log "$OUT/trace.log" || exit 1
python3 -m paper_2607_06045_amd.profiling traffic --fetch "$OUT/fetch" --write "$OUT/write" \
    --copy-fetch "$OUT/copyfetch" --copy-write "$OUT/copywrite" --copy-mib 512 --kernel "k_stage<3, 0, false, 0>" \
    --workload "Sedov blast, 22,156 leaves, N=3, FP64; mean over the three stage configurations" \
    --dofs 354496 --algorithmic-bytes-per-node 85.33333333333333 \
    --out "$OUT/summary/traffic_k_stage_blast22k.json" --command "$CMD" || exit 1
echo "profiles done"
