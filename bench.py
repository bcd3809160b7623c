"""Benchmark: Morse-Smale segmentation throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload gauss1024]

A step is one msc_segment call (steepest pointers, pointer jumping, pairing
into Morse-Smale cells) over a 1024^3 float32 field already resident in HBM.
Prints one JSON line with Gvertices/s, the roofline of the dominant kernel
(timed with HIP events on the call's stream by the library's own trace) and
the CPU oracle timed on a bounded slab of the same field.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Gvertices/s MS segmentation @1024^3 f32 (vs plain); "
          "served p50/p99 latency")
HBM_PEAK_GBS = 8000.0
BATCH_TEXT = ("batch256: 256 float32 fields, each axis round(exp(U[ln32, "
              "ln256])), Gaussian sums with U{8..128} bumps, seed 3")
WORKLOAD_TEXT = {
    "gauss1024": "gauss1024: 1024^3 float32, sum of 512 Gaussians "
                 "(sigma U[0.02,0.1]*1024) + U[-1e-4,1e-4] noise, seed 1",
    "gauss64": "gauss64: 64^3 float32, sum of 8 Gaussians + noise, seed 0",
    "perlin512": "perlin512: 512^3 float32, one layer of Perlin gradient "
                 "noise, frequency 0.1, amplitude 1, seed 5",
    "perlin1024": "perlin1024: 1024^3 float32, one layer of Perlin gradient "
                  "noise, frequency 0.1, amplitude 1, seed 5",
    "perlin2048s": "perlin2048s: 2048x2048x256 float32, z-planes [0, 256) of "
                   "the 2048^3 one-layer Perlin field (frequency 0.1, "
                   "amplitude 1, seed 5): one GPU's share of an 8-way z-slab "
                   "split",
}

# The paper's one-node times (seconds; 12 cores of an Intel Xeon Gold 6126)
# on the same synthetic workloads: segmentation at 512^3 and 1024^3 (table
# "overview") and implicit connected components of the 1024^3 field under
# the three feature thresholds (table "different_thresholds"; its rows are
# labelled top 10 / 50 / 90 %), and implicit connected components of the
# 512^3 and 1024^3 fields with the top 10 % of vertices masked (table
# "overview", the CC scaling figure).  Another machine's numbers: context
# only.
PAPER_1N_SECONDS = {
    "perlin512": 11.291, "perlin1024": 86.044,
    "ccperlin_t90": 47.285, "ccperlin_t50": 163.410, "ccperlin_t10": 226.593,
    "ccperlin512_top10": 5.973, "ccperlin1024_top10": 44.7504,
}


def paper_reference(workload, n, value_gvs):
    """(vs_baseline, reference record) against the paper's one-node time."""
    sec = PAPER_1N_SECONDS.get(workload)
    if sec is None:
        return None, None
    ref = n / sec / 1e9
    return round(value_gvs / ref, 1), {
        "seconds": sec, "gvertices_per_s": round(ref, 5),
        "hardware": "1 CPU node, 12 cores (Intel Xeon Gold 6126)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(field_dev, depth: int):
    """The oracle, single-threaded, on the first `depth` z-planes of the
    field taken as a grid of their own."""
    from oracle import oracle as O
    slab = field_dev[:depth].cpu().numpy()
    n = slab.size
    t0 = time.perf_counter()
    O.segment(slab, memo=True)
    dt = time.perf_counter() - t0
    return {"value": n / dt / 1e9, "unit": "Gvertices/s", "cores": 1,
            "kind": "oracle", "nproc": os.cpu_count(),
            "cpu_model": cpu_model(), "build": "gcc -O3",
            "sample": f"first {depth} z-planes ({slab.shape[2]}x{slab.shape[1]}"
                      f"x{depth} = {n} vertices) of the same field, "
                      f"{dt:.1f} s, serial C oracle (successors, memoised "
                      "walks, sort-based cells) on one core"}


def timed_steps(torch, stream, run, steps):
    """Time `steps` calls: synchronise, then per call a HIP event pair on the
    call's stream, synchronise.  Returns (median ms, mean wall ms)."""
    import statistics
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in zip(starts, ends):
        a.record(stream)
        run()
        b.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    per = [a.elapsed_time(b) for a, b in zip(starts, ends)]
    return statistics.median(per), wall


def traced_steps(msc, torch, run, steps):
    """The library's per-kernel event trace over `steps` calls (a pass of
    its own: the trace adds two event records per launch)."""
    torch.cuda.synchronize()
    msc.profile(True)
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    msc.profile(False)
    return msc.profile_read()


def traffic_of(workload, kernel, folder=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    record of this workload, or None when there is none or the kernel
    sources changed since it was taken."""
    path = os.path.join(folder or os.path.join(ROOT, "profiles"),
                        f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    from paper_2409_03771_amd.profsum import source_hash
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != source_hash():
        return None
    k = rec["kernels"].get(kernel)
    return None if k is None else int(round(k["hbm_bytes"]))


def path_traffic(workload, folder=None):
    """HBM bytes of one call summed over all kernels of the committed
    counter record, or None when absent or taken on other kernel sources."""
    path = os.path.join(folder or os.path.join(ROOT, "profiles"),
                        f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    from paper_2409_03771_amd.profsum import source_hash
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != source_hash():
        return None
    return int(round(sum(k["hbm_bytes"] for k in rec["kernels"].values())))


def roofline_of(prof, workload=None, tile=None):
    """Roofline object of the kernel with the most device time in `prof`
    (the library's own event trace: per-kernel launches, milliseconds and
    algorithmic bytes)."""
    name, dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    bpl = dom["bytes"] / dom["launches"]
    achieved = bpl / (avg_ms * 1e-3) / 1e9
    templated = name in ("tile_local", "tile_pairs", "tile_write", "exit_link")
    kname = "k_" + name + ("<%d,%d,%d>" % tile if tile and templated else "")
    out = {"bound": "hbm", "achieved": round(achieved, 1),
           "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": traffic_of(workload, kname) if workload else None,
           "kernel": kname, "avg_ms": round(avg_ms, 4),
           "bytes_per_launch": bpl}
    if name == "tile_local":
        # The steepest pass's algorithmic bytes counted as the field and
        # two int32 pointers (f 4 + 8 = 12 B/vertex); the kernel itself
        # writes one packed 32-bit code per vertex (f 4 + code 4 = 8 B).
        n = bpl / 12.0
        out["bytes_per_vertex"] = 12
        out["frac_own_bytes_8"] = round(8 * n / (avg_ms * 1e-3) / 1e9 /
                                        HBM_PEAK_GBS, 4)
    return out


def log_prof(prof):
    for k, p in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"]):
        avg = p["total_ms"] / max(1, p["launches"])
        gbs = p["bytes"] / max(1, p["launches"]) / (avg * 1e-3) / 1e9 if avg else 0
        log(f"[bench]   {k:16s} launches {p['launches']:5d} "
            f"avg {avg:8.3f} ms  {gbs:8.1f} GB/s (algorithmic)")


CC_TEXT = {
    "cc1024": "cc1024: mask = gauss1024 field (1024^3 float32, 512 Gaussians, "
              "seed 1) above its 70th percentile (k = floor(0.7 N)-th smallest "
              "value), Freudenthal connectivity, int64 labels",
    "ccperlin_t90": "ccperlin_t90: perlin1024 field normalised to [0,1] by "
                    "its min and max, mask = value above 0.9, Freudenthal "
                    "connectivity, int64 labels",
    "ccperlin_t50": "ccperlin_t50: perlin1024 field normalised to [0,1], "
                    "mask = value above 0.5, int64 labels",
    "ccperlin_t10": "ccperlin_t10: perlin1024 field normalised to [0,1], "
                    "mask = value above 0.1, int64 labels",
    "ccperlin512_top10": "ccperlin512_top10: perlin512 field (512^3 float32, "
                         "one layer of Perlin noise, frequency 0.1, seed 5), "
                         "mask = the top 10 % of vertices (above the "
                         "floor(0.9 N)-th smallest value), Freudenthal "
                         "connectivity, int64 labels",
    "ccperlin1024_top10": "ccperlin1024_top10: perlin1024 field, mask = the "
                          "top 10 % of vertices (above the floor(0.9 N)-th "
                          "smallest value), Freudenthal connectivity, int64 "
                          "labels",
    "csr50m": "csr50m: 368^3 = 49.8M-vertex jittered Kuhn tetrahedralisation "
              "as symmetric CSR (int64 row_ptr, int32 col_idx), vertex ids "
              "randomly permuted, seed 2; mask = Gaussian sum (24 bumps) at "
              "the jittered positions above its 70th percentile; int64 labels",
}


def bench_cc(args, msc, synth, torch, dev):
    """Connected components: the grid mask at 1024^3 or the 50M-vertex CSR
    mesh, one labelling call per step, inputs resident on the device."""
    stream = torch.cuda.current_stream(dev)

    def cc_grid(mask, labels):
        if args.ranks > 1:
            msc.cc_label_grid_ranks_into(mask, args.ranks, labels,
                                         stream=stream)
        else:
            msc.cc_label_grid_into(mask, labels, stream=stream)

    if args.workload == "cc1024":
        log("[bench] generating gauss1024 and its 70th-percentile mask")
        f = synth.config_field("gauss1024", device=dev)
        n = f.numel()
        k = int(0.7 * n)
        tau = torch.sort(f.reshape(-1)).values[k]
        mask = (f > tau).to(torch.uint8)
        del f
        torch.cuda.empty_cache()
        labels = torch.empty(n, dtype=torch.int64, device=dev)
        run = lambda: cc_grid(mask, labels)
        fg = int(mask.sum().item())
    elif args.workload.endswith("_top10"):
        name = args.workload[2:-len("_top10")]
        log(f"[bench] generating {name} and its top-10 % mask")
        f = synth.config_field(name, device=dev)
        n = f.numel()
        mask = synth.threshold_mask(f, 0.9)
        del f
        torch.cuda.empty_cache()
        labels = torch.empty(n, dtype=torch.int64, device=dev)
        run = lambda: cc_grid(mask, labels)
        fg = int(mask.sum().item())
    elif args.workload.startswith("ccperlin_t"):
        level = int(args.workload[-2:]) / 100.0
        log(f"[bench] generating perlin1024 and its mask above {level}")
        f = synth.config_field("perlin1024", device=dev)
        n = f.numel()
        mask = synth.normalized_mask(f, level)
        del f
        torch.cuda.empty_cache()
        labels = torch.empty(n, dtype=torch.int64, device=dev)
        run = lambda: cc_grid(mask, labels)
        fg = int(mask.sum().item())
    else:
        log("[bench] generating the 368^3 Kuhn CSR mesh on the host")
        t0 = time.perf_counter()
        d = synth.kuhn_csr(368, seed=2)
        log(f"[bench] mesh ready in {time.perf_counter() - t0:.1f} s")
        rp = torch.from_numpy(d["row_ptr"]).to(dev)
        ci = torch.from_numpy(d["col_idx"]).to(dev)
        mask = torch.from_numpy(d["mask"]).to(dev)
        del d
        n = rp.numel() - 1
        labels = torch.empty(n, dtype=torch.int64, device=dev)
        run = lambda: msc.cc_label_csr_into(rp, ci, labels, mask, stream=stream)
        fg = int(mask.sum().item())
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    msc.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    msc.profile(False)
    prof = msc.profile_read()
    log(f"[bench] {args.steps} steps: {dt * 1e3:.2f} ms/step")
    log_prof(prof)
    ncomp = int((labels == torch.arange(n, device=dev)).sum().item())
    vs, ref = paper_reference(args.workload, n, n / dt / 1e9)
    out = {
        "metric": "Gvertices/s connected components (" + args.workload + ")",
        "value": round(n / dt / 1e9, 3), "unit": "Gvertices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": vs, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": CC_TEXT[args.workload], "vertices": n,
                   "foreground": fg, "components": ncomp,
                   "virtual_ranks": args.ranks},
        "roofline": roofline_of(prof, args.workload),
    }
    if ref:
        out["paper_one_node"] = ref
    print(json.dumps(out), flush=True)


SEGCSR_TEXT = {
    "segcsr50m": "segcsr50m: MS segmentation of the csr50m mesh (368^3 = "
                 "49.8M vertices of a jittered Kuhn tetrahedralisation, "
                 "symmetric CSR, randomly permuted ids, seed 2) with the "
                 "Gaussian-sum field at its jittered positions; int32 asc, "
                 "desc, ms",
}


def bench_segcsr(args, msc, synth, torch, dev):
    """Segmentation over CSR adjacency: the 50M-vertex mesh, one call per
    step, inputs resident on the device."""
    stream = torch.cuda.current_stream(dev)
    log("[bench] generating the 368^3 Kuhn CSR mesh on the host")
    t0 = time.perf_counter()
    d = synth.kuhn_csr(368, seed=2)
    log(f"[bench] mesh ready in {time.perf_counter() - t0:.1f} s")
    import numpy as np
    f = np.empty_like(d["field"])
    f[d["perm"]] = d["field"]
    rp = torch.from_numpy(d["row_ptr"]).to(dev)
    ci = torch.from_numpy(d["col_idx"]).to(dev)
    fd = torch.from_numpy(f).to(dev)
    nnz = int(d["row_ptr"][-1])
    del d, f
    n = rp.numel() - 1
    asc = torch.empty(n, dtype=torch.int32, device=dev)
    desc = torch.empty_like(asc)
    ms = torch.empty_like(asc)
    run = lambda: msc.segment_csr_into(rp, ci, fd, asc, desc, ms,
                                       stream=stream)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    stats = msc.last_stats()
    msc.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    msc.profile(False)
    prof = msc.profile_read()
    log(f"[bench] {args.steps} steps: {dt * 1e3:.2f} ms/step")
    log_prof(prof)
    out = {
        "metric": "Gvertices/s MS segmentation over CSR adjacency "
                  "(" + args.workload + ")",
        "value": round(n / dt / 1e9, 3), "unit": "Gvertices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": SEGCSR_TEXT[args.workload], "vertices": n,
                   "edges": nnz, "maxima": stats["n_maxima"],
                   "minima": stats["n_minima"], "cells": stats["n_cells"]},
        "roofline": roofline_of(prof, args.workload),
    }
    print(json.dumps(out), flush=True)


def bench_tets(args, msc, synth, torch, dev):
    """CSR adjacency of the 368^3 Kuhn mesh from its 296M tetrahedra (ids
    randomly permuted, seed 2), one build per step into resident buffers."""
    stream = torch.cuda.current_stream(dev)
    import numpy as np
    na = 368
    perm = np.random.default_rng(2).permutation(na ** 3).astype(np.int64)
    log("[bench] generating the tetrahedra")
    tets = torch.from_numpy(synth.kuhn_tets(na, perm=perm)).to(dev)
    del perm
    n = na ** 3
    rp = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nnz = msc.csr_from_tets_into(n, tets, rp, None, stream=stream)
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    run = lambda: msc.csr_from_tets_into(n, tets, rp, col, stream=stream)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    msc.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    msc.profile(False)
    prof = msc.profile_read()
    log(f"[bench] {args.steps} steps: {dt * 1e3:.2f} ms/step")
    log_prof(prof)
    ntets = tets.numel() // 4
    out = {
        "metric": "Gtetrahedra/s CSR adjacency from a tetrahedra list",
        "value": round(ntets / dt / 1e9, 3), "unit": "Gtetrahedra/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": TETS_TEXT[args.workload], "vertices": n,
                   "tetrahedra": ntets, "entries": nnz},
        "roofline": roofline_of(prof, args.workload),
    }
    print(json.dumps(out), flush=True)


CRIT_TEXT = {
    "crit_gauss1024": "crit_gauss1024: link components of every vertex and "
                      "the extremum graph of the gauss1024 field",
    "crit_perlin1024": "crit_perlin1024: link components of every vertex and "
                       "the extremum graph of the perlin1024 field",
}


def bench_crit(args, msc, synth, torch, dev):
    """Critical points by link components, then the extremum graph from the
    field's segmentation (computed once, outside the timed region); one of
    each per step."""
    stream = torch.cuda.current_stream(dev)
    name = args.workload.split("_", 1)[1]
    log(f"[bench] generating {name}")
    f = synth.config_field(name, device=dev)
    n = f.numel()
    code = torch.empty(n, dtype=torch.uint8, device=dev)
    a, d, _ = msc.segment(f, want=("asc", "desc"))
    m = msc.extremum_graph(f, a, d).shape[0]
    edges = torch.empty((m, 3), dtype=torch.int32, device=dev)
    def run():
        msc.critical_points_into(f, code, stream=stream)
        msc.extremum_graph_into(f, a, d, edges, stream=stream)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    msc.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    msc.profile(False)
    prof = msc.profile_read()
    log(f"[bench] {args.steps} steps: {dt * 1e3:.2f} ms/step")
    log_prof(prof)
    saddles = int(((code & 15) >= 2).sum() + ((code >> 4) >= 2).sum())
    out = {
        "metric": "Gvertices/s critical points + extremum graph "
                  "(" + args.workload + ")",
        "value": round(n / dt / 1e9, 3), "unit": "Gvertices/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": CRIT_TEXT[args.workload], "vertices": n,
                   "saddle_sides": saddles, "edges": m},
        "roofline": roofline_of(prof, args.workload),
    }
    print(json.dumps(out), flush=True)


TETS_TEXT = {
    "tets368": "tets368: the 6*367^3 = 296M Kuhn tetrahedra of a 368^3 grid "
               "with randomly permuted vertex ids (seed 2) to symmetric CSR "
               "(int64 row_ptr, int32 col_idx)",
}


def batch_leg(args, msc, synth, torch, dev):
    """batch256: one batched call vs. 256 plain calls on one stream (both
    asynchronous, no host synchronisation inside the timed loop)."""
    specs = synth.batch_specs(256, seed=3)
    log("[bench] generating batch256")
    fields = [synth.gaussian_field(d, nb, sd, device=dev) for d, nb, sd in specs]
    torch.cuda.synchronize()
    n = sum(f.numel() for f in fields)
    outs = [tuple(torch.empty(f.numel(), dtype=torch.int32, device=dev)
                  for _ in range(3)) for f in fields]
    stream = torch.cuda.current_stream(dev)
    tune = msc.autotune(fields, outs, stream=stream)
    log(f"[bench] autotune {tune}")

    def batched():
        msc.segment_batched_into(fields, outs, stream=stream, check=False)

    def plain():
        for f, (a, d, m) in zip(fields, outs):
            msc.segment_into(f, a, d, m, stream=stream, check=False)

    for _ in range(max(1, args.warmup)):
        batched()
        plain()
    torch.cuda.synchronize()
    if msc.last_status() != msc.MSC_OK:
        raise msc.MscError(msc.last_status(), "batch256")
    steps = max(3, args.steps)
    b_ms, b_wall = timed_steps(torch, stream, batched, steps)
    p_ms, p_wall = timed_steps(torch, stream, plain, steps)
    prof = traced_steps(msc, torch, batched, 2)
    # The same batch captured into a HIP graph and replayed.
    graph = msc.Graph(fields, outs, stream=stream)
    for _ in range(max(1, args.warmup)):
        graph.launch(stream=stream)
    torch.cuda.synchronize()
    g_ms, _ = timed_steps(torch, stream, lambda: graph.launch(stream=stream),
                          steps)
    graph.close()
    msc.set_tile(*msc.tile_shapes()[0])
    log(f"[bench] batch256: batched {b_ms:.2f} ms (graph replay {g_ms:.2f} "
        f"ms) vs plain {p_ms:.2f} ms for {n} vertices")
    return {"workload": BATCH_TEXT, "vertices": n, "tile": list(tune["tile"]),
            "batched_ms": round(b_ms, 3), "plain_ms": round(p_ms, 3),
            "graph_replay_ms": round(g_ms, 3),
            "batched_wall_ms": round(b_wall, 3),
            "plain_wall_ms": round(p_wall, 3),
            "batched_gvps": round(n / (b_ms * 1e-3) / 1e9, 3),
            "plain_gvps": round(n / (p_ms * 1e-3) / 1e9, 3),
            "speedup_vs_plain": round(p_ms / b_ms, 2),
            "steps": steps,
            "roofline": roofline_of(prof, tile=tuple(tune["tile"]))}


def bench_batch(args, msc, synth, torch, dev):
    """256 uneven fields: one batched call per step vs. 256 plain calls."""
    leg = batch_leg(args, msc, synth, torch, dev)
    out = {
        "metric": "Gvertices/s batched MS segmentation (256 uneven fields)",
        "value": leg["batched_gvps"], "unit": "Gvertices/s",
        "n_gpus": 1, "steps": leg["steps"], "warmup": args.warmup,
        "ms_per_step": leg["batched_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": BATCH_TEXT, "vertices": leg["vertices"],
                   "tile": leg["tile"], "plain_ms_per_step": leg["plain_ms"],
                   "speedup_vs_plain": leg["speedup_vs_plain"]},
        "roofline": leg["roofline"],
    }
    print(json.dumps(out), flush=True)


SERVE_TEXT = ("served: open-loop Poisson arrivals (seed 4), 70% MS segmentation"
              " / 30% mask CC (mask above the 70th percentile), each axis "
              "round(exp(U[ln64, ln512])), Gaussian sums with U{{8..128}} bumps; "
              "inputs from a pool of {pool} pre-generated page-locked host "
              "fields (request i uses entry i mod {pool}); H2D copy counted in "
              "latency (arrival -> results resident on the device); "
              "{budget} GiB HBM budget, at most {max_batch} fields per launch")


_POOLS = {}


def serve_pool(synth, torch, dev, size):
    """Page-locked host inputs: a float32 field and its mask per entry
    (generated once per size)."""
    if size in _POOLS:
        return _POOLS[size]
    pool = []
    for spec in synth.poisson_trace(1.0, size, seed=4):
        f = synth.gaussian_field(spec["dims"], spec["nbumps"], spec["seed"],
                                 device=dev).cpu().numpy()
        fh = torch.from_numpy(f).pin_memory()
        mh = torch.from_numpy(synth.threshold_mask(f, 0.7)).pin_memory()
        pool.append((fh, mh))
    _POOLS[size] = pool
    return pool


def _percentiles(lat_ms):
    import numpy as np
    a = np.asarray(lat_ms)
    return round(float(np.percentile(a, 50)), 3), round(float(np.percentile(a, 99)), 3)


def run_served(msc, pool, trace, warm, budget, max_batch):
    """Open loop through the request queue: a submitter thread at the trace's
    arrival times, this thread collecting and releasing results in order."""
    import queue
    import threading
    srv = msc.Server(hbm_budget=budget, max_batch=max_batch)
    handoff = queue.Queue()
    t0 = time.monotonic_ns() + 20_000_000

    def submitter():
        for i, req in enumerate(trace):
            at = t0 + int(req["t"] * 1e9)
            dt = (at - time.monotonic_ns()) / 1e9
            if dt > 0:
                time.sleep(dt)
            fh, mh = pool[i % len(pool)]
            kind = msc.REQ_SEGMENT if req["kind"] == "ms" else msc.REQ_CC_GRID
            t = srv.submit(kind, fh if kind == msc.REQ_SEGMENT else mh)
            handoff.put((t, at, fh.numel()))
        handoff.put(None)

    th = threading.Thread(target=submitter)
    th.start()
    lat, verts, first, last, batches, k = [], 0, None, 0, [], 0
    while True:
        item = handoff.get()
        if item is None:
            break
        t, at, n = item
        rc = srv.wait(t)
        if rc != msc.MSC_OK:
            raise msc.MscError(rc, f"served request {k}")
        r = srv.result(t)
        srv.release(t)
        if k >= warm:
            lat.append((r["t_done_ns"] - at) / 1e6)
            verts += n
            first = at if first is None else first
            last = max(last, r["t_done_ns"])
            batches.append(r["batch_size"])
        k += 1
    th.join()
    srv.close()
    p50, p99 = _percentiles(lat)
    return {"p50_ms": p50, "p99_ms": p99,
            "gvps": round(verts / ((last - first) / 1e9) / 1e9, 3),
            "mean_batch": round(sum(batches) / len(batches), 2)}


def run_plain(msc, torch, dev, pool, trace, warm):
    """The same trace served one request at a time in arrival order: copy the
    input to the device, one plain call, wait for it."""
    stream = torch.cuda.current_stream(dev)
    t0 = time.monotonic_ns() + 20_000_000
    lat, verts, first, last = [], 0, None, 0
    for i, req in enumerate(trace):
        at = t0 + int(req["t"] * 1e9)
        dt = (at - time.monotonic_ns()) / 1e9
        if dt > 0:
            time.sleep(dt)
        fh, mh = pool[i % len(pool)]
        if req["kind"] == "ms":
            f = fh.to(dev, non_blocking=True)
            a = torch.empty(f.numel(), dtype=torch.int32, device=dev)
            d, m = torch.empty_like(a), torch.empty_like(a)
            msc.segment_into(f, a, d, m, stream=stream, check=False)
        else:
            msc.cc_label_grid(mh.to(dev, non_blocking=True), stream=stream)
        torch.cuda.synchronize()
        done = time.monotonic_ns()
        if i >= warm:
            lat.append((done - at) / 1e6)
            verts += fh.numel()
            first = at if first is None else first
            last = done
    p50, p99 = _percentiles(lat)
    return {"p50_ms": p50, "p99_ms": p99,
            "gvps": round(verts / ((last - first) / 1e9) / 1e9, 3)}


def run_saturated(msc, torch, dev, pool, kinds, budget, max_batch):
    """Closed-loop saturation: every request submitted at once (inputs
    already in device memory), then the same sequence as plain sequential
    calls (one call, wait, next).  Throughput over all requests; latency
    from the common start."""
    srv = msc.Server(hbm_budget=budget, max_batch=max_batch)
    t0 = time.monotonic_ns()
    tickets = []
    for i, kind in enumerate(kinds):
        fd, md = pool[i % len(pool)]
        k = msc.REQ_SEGMENT if kind == "ms" else msc.REQ_CC_GRID
        tickets.append((srv.submit(k, fd if k == msc.REQ_SEGMENT else md),
                        fd.numel()))
    lat, verts, last, batches = [], 0, 0, []
    for t, n in tickets:
        rc = srv.wait(t)
        if rc != msc.MSC_OK:
            raise msc.MscError(rc, "saturated request")
        r = srv.result(t)
        srv.release(t)
        lat.append((r["t_done_ns"] - t0) / 1e6)
        verts += n
        last = max(last, r["t_done_ns"])
        batches.append(r["batch_size"])
    info = srv.info()
    srv.close()
    served_s = (last - t0) / 1e9
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    p0 = time.monotonic_ns()
    plain_lat = []
    for i, kind in enumerate(kinds):
        fd, md = pool[i % len(pool)]
        if kind == "ms":
            a = torch.empty(fd.numel(), dtype=torch.int32, device=dev)
            d, m = torch.empty_like(a), torch.empty_like(a)
            msc.segment_into(fd, a, d, m, stream=stream, check=False)
        else:
            msc.cc_label_grid(md, stream=stream)
        torch.cuda.synchronize()
        plain_lat.append((time.monotonic_ns() - p0) / 1e6)
    plain_s = (time.monotonic_ns() - p0) / 1e9
    if msc.last_status() != msc.MSC_OK:
        raise msc.MscError(msc.last_status(), "plain request")
    sp50, sp99 = _percentiles(lat)
    pp50, pp99 = _percentiles(plain_lat)
    return {"requests": len(kinds), "gvps": round(verts / served_s / 1e9, 3),
            "p50_ms": sp50, "p99_ms": sp99,
            "mean_batch": round(sum(batches) / len(batches), 2),
            "launches": info["launches"],
            "host_waits": info["host_waits"],
            "workspace_grows": info["workspace_grows"],
            "plain_gvps": round(verts / plain_s / 1e9, 3),
            "plain_p50_ms": pp50, "plain_p99_ms": pp99,
            "speedup_vs_plain": round(plain_s / served_s, 2)}


def saturated_leg(msc, synth, torch, dev, count, pool_size, budget_gib=64,
                  max_batch=64):
    log(f"[bench] saturated device-resident load: {count} requests")
    pool = [(fh.to(dev), mh.to(dev))
            for fh, mh in serve_pool(synth, torch, dev, pool_size)]
    torch.cuda.synchronize()
    kinds = [r["kind"] for r in synth.poisson_trace(1.0, count, seed=4)]
    # One untimed pass warms the queue's contexts and the plain path.
    run_saturated(msc, torch, dev, pool, kinds[:32], budget_gib << 30,
                  max_batch)
    res = run_saturated(msc, torch, dev, pool, kinds, budget_gib << 30,
                        max_batch)
    log(f"[bench] saturated {res}")
    res["workload"] = ("closed loop: all requests submitted at once from a "
                       f"pool of {pool_size} device-resident inputs of the "
                       "served mix (70% MS / 30% mask CC, axes "
                       "log-uniform [64, 512]); plain = the same sequence "
                       "as one call at a time, each waited for; latency "
                       "from the common start")
    return res


def served_sweep(msc, synth, torch, dev, rates, warm, count, pool_size,
                 budget_gib=64, max_batch=64, resident_rates=()):
    """Per rate: the queue and plain sequential calls on the same trace with
    host inputs (the H2D copy is part of each request); per resident rate,
    the same with the inputs already in device memory."""
    log(f"[bench] serve pool of {pool_size} fields")
    pool = serve_pool(synth, torch, dev, pool_size)
    out, out_res = {}, {}
    for rates_, pool_, dst, tag in ((rates, pool, out, "host"),
                                    (resident_rates, None, out_res,
                                     "resident")):
        if tag == "resident" and resident_rates:
            pool_ = [(fh.to(dev), mh.to(dev)) for fh, mh in pool]
        for rate in rates_:
            trace = synth.poisson_trace(float(rate), warm + count, seed=4)
            srv = run_served(msc, pool_, trace, warm, budget_gib << 30,
                             max_batch)
            plain = run_plain(msc, torch, dev, pool_, trace, warm)
            log(f"[bench] {rate:5d} req/s {tag} served {srv} plain {plain}")
            dst[str(rate)] = {**srv, "plain_p50_ms": plain["p50_ms"],
                              "plain_p99_ms": plain["p99_ms"],
                              "plain_gvps": plain["gvps"],
                              "speedup_vs_plain": round(
                                  srv["gvps"] / plain["gvps"], 2)}
    text = SERVE_TEXT.format(pool=pool_size, budget=budget_gib,
                             max_batch=max_batch)
    return text, out, out_res


def bench_serve(args, msc, synth, torch, dev):
    rates = [int(r) for r in args.rates.split(",")]
    text, res, res_dev = served_sweep(
        msc, synth, torch, dev, rates, args.serve_warmup, args.serve_requests,
        args.serve_pool, resident_rates=rates)
    sat = saturated_leg(msc, synth, torch, dev, args.serve_requests,
                        args.serve_pool)
    top = res[str(rates[-1])]
    out = {
        "metric": "Gvertices/s served MS segmentation + mask CC; "
                  "p50/p99 latency",
        "value": top["gvps"], "unit": "Gvertices/s", "n_gpus": 1,
        "steps": args.serve_requests, "warmup": args.serve_warmup,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": text, "requests_per_rate": args.serve_requests,
                   "rates": res, "rates_device_resident_inputs": res_dev,
                   "saturated_device_resident": sat,
                   "speedup_vs_plain": round(top["gvps"] / top["plain_gvps"], 2)},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="gauss1024",
                    choices=sorted(WORKLOAD_TEXT) + ["batch256", "serve"]
                    + sorted(CC_TEXT) + sorted(SEGCSR_TEXT)
                    + sorted(TETS_TEXT) + sorted(CRIT_TEXT))
    ap.add_argument("--cpu-depth", type=int, default=100,
                    help="z-planes of the field the CPU oracle is timed on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rates", default="50,100,200,500,1000,2000",
                    help="served mode: arrival rates (req/s)")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--serve-pool", type=int, default=48)
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the short served leg of the default run")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch256 leg of the default run")
    ap.add_argument("--ranks", type=int, default=1,
                    help="virtual z-slab ranks on the one device (the "
                         "paper's distributed scheme; 1 = single domain)")
    ap.add_argument("--tile", default=None,
                    help="tile shape of the fused pass, e.g. 32x16x16")
    ap.add_argument("--calibrate-copy", type=float, default=None,
                    metavar="GIB",
                    help="only run torch's device copy of a GIB-sized float32 "
                         "buffer 3 times (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        n = int(args.calibrate_copy * (1 << 30)) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 4 * n, "launches": 3}))
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): "
              "the segmentation path is single-device; there is no multi-GPU "
              "mode to measure.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2409_03771_amd import msc, synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.tile:
        msc.set_tile(*(int(t) for t in args.tile.split("x")))

    if args.workload == "batch256":
        return bench_batch(args, msc, synth, torch, dev)
    if args.workload == "serve":
        return bench_serve(args, msc, synth, torch, dev)
    if args.workload in CC_TEXT:
        return bench_cc(args, msc, synth, torch, dev)
    if args.workload in SEGCSR_TEXT:
        return bench_segcsr(args, msc, synth, torch, dev)
    if args.workload in TETS_TEXT:
        return bench_tets(args, msc, synth, torch, dev)
    if args.workload in CRIT_TEXT:
        return bench_crit(args, msc, synth, torch, dev)

    log(f"[bench] generating {args.workload} on {dev}")
    t0 = time.perf_counter()
    field = synth.config_field(args.workload, device=dev)
    torch.cuda.synchronize()
    log(f"[bench] field ready in {time.perf_counter() - t0:.1f} s, "
        f"shape {tuple(field.shape)}")
    n = field.numel()
    asc = torch.empty(n, dtype=torch.int32, device=dev)
    desc = torch.empty_like(asc)
    ms = torch.empty_like(asc)
    stream = torch.cuda.current_stream(dev)

    def segment(field, asc, desc, ms):
        if args.ranks > 1:
            msc.segment_ranks_into(field, args.ranks, asc, desc, ms,
                                   stream=stream)
        else:
            msc.segment_into(field, asc, desc, ms, stream=stream, check=False)

    for i in range(args.warmup):
        segment(field, asc, desc, ms)
        log(f"[bench] warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    stats = msc.last_stats()
    log(f"[bench] stats {stats}")
    if stats["status"] != msc.MSC_OK:
        raise msc.MscError(stats["status"], "segmentation")

    run = lambda: segment(field, asc, desc, ms)
    ms_per_step, wall_ms = timed_steps(torch, stream, run, args.steps)
    value = n / (ms_per_step * 1e-3) / 1e9
    log(f"[bench] {args.steps} steps: median {ms_per_step:.3f} ms/step "
        f"(HIP events), wall {wall_ms:.3f} ms/step")
    prof = traced_steps(msc, torch, run, args.steps)
    log_prof(prof)
    tile = (stats["tile_x"], stats["tile_y"], stats["tile_z"])
    roofline = roofline_of(prof, args.workload, tile)

    vs, ref = paper_reference(args.workload, n, value)
    # The headline metric names the 1024^3 shape; other shapes name theirs.
    dims = tuple(field.shape[::-1])
    metric = METRIC if dims == (1024, 1024, 1024) else (
        "Gvertices/s MS segmentation @%dx%dx%d f32 (vs plain); served "
        "p50/p99 latency" % dims)
    out = {
        "metric": metric, "value": round(value, 3), "unit": "Gvertices/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": vs, "dtype": "f32",
        "data": "synthetic",
        "timing": "median of per-step HIP events on the call's stream, "
                  "trace off; wall_ms_per_step is the synchronised wall "
                  "clock over the same steps",
        "wall_ms_per_step": round(wall_ms, 3),
        "config": {"workload": WORKLOAD_TEXT[args.workload],
                   "vertices": n, "outputs": "int32 asc, desc, ms",
                   "maxima": stats["n_maxima"], "minima": stats["n_minima"],
                   "cells": stats["n_cells"], "exits": stats["n_exits"],
                   "virtual_ranks": args.ranks},
        "roofline": roofline,
        # Whole call: the compulsory 16 B per vertex (read f, write asc, desc,
        # ms) and the rocprofv3-measured HBM bytes of all kernels, per step.
        "path_roofline": {
            "compulsory_bytes": 16 * n,
            "compulsory_frac": round(16 * n / (ms_per_step * 1e-3) /
                                     (HBM_PEAK_GBS * 1e9), 4),
            "measured_bytes": path_traffic(args.workload),
            "measured_frac": None},
    }
    if ref:
        out["paper_one_node"] = ref
    pr = out["path_roofline"]
    if pr["measured_bytes"]:
        pr["measured_frac"] = round(pr["measured_bytes"] / (ms_per_step * 1e-3)
                                    / (HBM_PEAK_GBS * 1e9), 4)
    if not args.no_cpu_baseline:
        depth = min(args.cpu_depth, field.shape[0])
        log(f"[bench] timing the CPU oracle on {depth} z-planes")
        out["cpu_baseline"] = cpu_baseline(field, depth)
    if not args.no_batch:
        del field, asc, desc, ms
        torch.cuda.empty_cache()
        out["batched"] = batch_leg(args, msc, synth, torch, dev)
    if not args.no_serve:
        # Short served leg: a light, a busy and a saturating arrival rate.
        torch.cuda.empty_cache()
        text, res, res_dev = served_sweep(msc, synth, torch, dev,
                                          [200, 1000, 2000], 50, 300, 24,
                                          resident_rates=[2000])
        out["served"] = {"workload": text, "requests_per_rate": 300,
                         "rates": res,
                         "rates_device_resident_inputs": res_dev}
        out["served"]["saturated_device_resident"] = saturated_leg(
            msc, synth, torch, dev, 400, 24)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
