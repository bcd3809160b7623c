#!/bin/bash
# Writes the profiles/ summaries from the rocprofv3 output of the profiling
# commands they record (run on the GPU machine from the repository root,
# output under gpurun_out/pa/).
set -e
P="python -m paper_2409_03771_amd.profsum"
RP='cd /tmp && export TMPDIR=/tmp && timeout -s KILL 150 rocprofv3'
B='python3 bench.py'
SEG='--steps 2 --warmup 1 --no-cpu-baseline --no-serve --no-batch'
O=gpurun_out/pa
$P stats $O/kt_seg/run_kernel_trace.csv --title "MS segmentation, gauss1024 (1024^3 float32, 512 Gaussians, seed 1), 32x16x16 tiles; 5 timed + 2 warm-up + 3 bench warm-up + 5 traced steps" --cmd "$RP --kernel-trace --stats --output-format csv -d $O/kt_seg -o run -- $B --steps 5 --warmup 2 --no-cpu-baseline --no-serve --no-batch" --out profiles/segment_gauss1024_kernel_stats.md
$P traffic --fetch $O/fetch_seg/run_counter_collection.csv --write $O/write_seg/run_counter_collection.csv --copy-fetch $O/fetch_copy/run_counter_collection.csv --copy-write $O/write_copy/run_counter_collection.csv --copy-bytes 1073741824 --title "MS segmentation, gauss1024" --cmd "$RP --pmc FETCH_SIZE --output-format csv -d $O/fetch_seg -o run -- $B $SEG
$RP --pmc WRITE_SIZE --output-format csv -d $O/write_seg -o run -- $B $SEG
$RP --pmc FETCH_SIZE --output-format csv -d $O/fetch_copy -o run -- $B --calibrate-copy 1
$RP --pmc WRITE_SIZE --output-format csv -d $O/write_copy -o run -- $B --calibrate-copy 1" --out profiles/segment_gauss1024_traffic.md --json profiles/traffic_gauss1024.json
$P counters $O/sqa_seg/run_counter_collection.csv --title "MS segmentation, gauss1024: instruction counts" --cmd "$RP --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_WAIT_INST_LDS SQ_LDS_BANK_CONFLICT --output-format csv -d $O/sqa_seg -o run -- $B $SEG" --out profiles/segment_gauss1024_sq_instructions.md
$P counters $O/sqb_seg/run_counter_collection.csv --title "MS segmentation, gauss1024: cycles" --cmd "$RP --pmc SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_VMEM --output-format csv -d $O/sqb_seg -o run -- $B $SEG" --out profiles/segment_gauss1024_sq_cycles.md
$P stats $O/kt_cc/run_kernel_trace.csv --title "grid connected components, cc1024 (gauss1024 field above its 70th percentile, int64 labels); 5 timed + 2 warm-up steps" --cmd "$RP --kernel-trace --stats --output-format csv -d $O/kt_cc -o run -- $B --workload cc1024 --steps 5 --warmup 2" --out profiles/cc_grid_cc1024_kernel_stats.md
$P traffic --fetch $O/fetch_cc/run_counter_collection.csv --write $O/write_cc/run_counter_collection.csv --copy-fetch $O/fetch_copy/run_counter_collection.csv --copy-write $O/write_copy/run_counter_collection.csv --copy-bytes 1073741824 --title "grid CC, cc1024" --cmd "$RP --pmc FETCH_SIZE --output-format csv -d $O/fetch_cc -o run -- $B --workload cc1024 --steps 2 --warmup 1
$RP --pmc WRITE_SIZE --output-format csv -d $O/write_cc -o run -- $B --workload cc1024 --steps 2 --warmup 1
(copy calibration as in segment_gauss1024_traffic.md)" --out profiles/cc_grid_cc1024_traffic.md --json profiles/traffic_cc1024.json
$P stats $O/kt_b256/run_kernel_trace.csv --top 14 --title "batch256: 256 uneven float32 fields (axes log-uniform [32,256], 8-128 bumps, seed 3): autotune over the 5 tile shapes, then per step one batched call and 256 plain calls; 5 timed + 2 warm-up steps of each. Rows with the full batched grid (e.g. [grid 23689728] for 32x16x16) are the batched call's kernels; the plain calls' kernels have per-field grids" --cmd "$RP --kernel-trace --stats --output-format csv -d $O/kt_b256 -o run -- $B --workload batch256 --steps 5 --warmup 2" --out profiles/segment_batch256_kernel_stats.md
