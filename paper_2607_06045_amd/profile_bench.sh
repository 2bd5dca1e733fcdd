#!/bin/bash
# rocprofv3 profiles of the headline benchmark workload (four-quadrant states,
# 246,736 leaves, N = 4, FP64): kernel-trace statistics of bench.py, then
# counter passes of the same benchmark (FETCH_SIZE, WRITE_SIZE, two passes of
# instruction counters) and of a plain 512 MiB device copy (calibration of the
# byte counters).  Run from the repository root on a machine with the GPU; raw
# output and the two summaries go to $PROFILE_OUT (default prof_out, not
# tracked): kernels_k_stage_quadrants247k.txt and
# counters_k_stage_quadrants247k.json under summary/.
set -o pipefail
ROOT=$(pwd)
OUT=$ROOT/${PROFILE_OUT:-prof_out}
mkdir -p "$OUT/summary"
cd /tmp && export TMPDIR=/tmp && cd "$ROOT" || exit 1
CMD="bash paper_2607_06045_amd/profile_bench.sh"
BT="python3 bench.py --steps 20 --warmup 2 --no-cpu-baseline --legs none"
BC="python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline --legs none"
CP="python3 -m paper_2607_06045_amd.profiling copy --mib 512"
# one stage is two launches of the element kernel: k_stage<4, 0, false, 0, true>
# over the element batches with a mortar element, k_stage<4, 0, false, 0, false>
# over the others; the summaries add the two per stage
KERNEL="k_stage<4, 0, false, 0,"

echo "== kernel trace: $BT"
timeout -k 10 300 rocprofv3 --kernel-trace --stats -d "$OUT/trace" -o trace --output-format csv -- $BT \
    > "$OUT/trace.log" 2>&1 || { echo "kernel trace failed"; tail -20 "$OUT/trace.log"; exit 1; }
tail -1 "$OUT/trace.log" | cut -c1-160
pmc() {
    local name=$1 counters=$2; shift 2
    echo "== $counters: $*"
    timeout -s KILL 150 rocprofv3 --pmc $counters -d "$OUT/$name" -o "$name" --output-format csv -- "$@" \
        > "$OUT/$name.log" 2>&1 || { echo "$name pass failed"; tail -20 "$OUT/$name.log"; return 1; }
}
pmc fetch FETCH_SIZE $BC || exit 1
pmc write WRITE_SIZE $BC || exit 1
pmc copyfetch FETCH_SIZE $CP || exit 1
pmc copywrite WRITE_SIZE $CP || exit 1
pmc sqa "SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_VALU_INT32 SQ_BUSY_CYCLES" $BC || exit 1
pmc sqb "SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64" $BC || exit 1
# issue and stall counters (optional: the summary goes without them if this pass fails)
SQC=""
pmc sqc "SQ_WAVE_CYCLES SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_ANY SQ_INSTS_LDS SQ_WAIT_ANY" $BC \
    && SQC="$OUT/sqc"

STATS=$(find "$OUT/trace" -name '*kernel_stats.csv' | head -1)
python3 -m paper_2607_06045_amd.profiling stats --csv "$STATS" \
    --out "$OUT/summary/kernels_k_stage_quadrants247k.txt" \
    --title "kernel durations, bench.py headline workload (four-quadrant states, 246,736 leaves, N=4, FP64; 20 steps + kernel timing; one stage = the two k_stage<4, 0, false, 0, *> launches)" \
    --command "$CMD" --trace-csv "$(find "$OUT/trace" -name '*kernel_trace.csv' | head -1)" \
    --kernel "$KERNEL" --tail 150 --bench-log "$OUT/trace.log" || exit 1
python3 -m paper_2607_06045_amd.profiling counters --fetch "$OUT/fetch" --write "$OUT/write" \
    --copy-fetch "$OUT/copyfetch" --copy-write "$OUT/copywrite" --copy-mib 512 \
    --sq "$OUT/sqa" "$OUT/sqb" $SQC --kernel "$KERNEL" \
    --workload "four-quadrant states, 246,736 leaves, N=4, FP64; mean over the three stage configurations" \
    --dofs 6168400 --algorithmic-bytes-per-node 85.33333333333333 \
    --out "$OUT/summary/counters_k_stage_quadrants247k.json" --command "$CMD" || exit 1
echo "profiles done"
