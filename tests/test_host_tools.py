"""Host-side tooling, on the CPU: the rocprofv3 summariser, the benchmark's
use of committed counter records, and its single-GPU contract."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2409_03771_amd import profsum  # noqa: E402


def test_short_names():
    assert profsum.short_name(
        "void msc::(anonymous namespace)::k_tile_local<msc::(anonymous "
        "namespace)::Cfg<32, 16, 16> >(msc::(anonymous namespace)::FieldDev "
        "const*, unsigned int const*)") == "k_tile_local<32,16,16>"
    assert profsum.short_name(
        "msc::(anonymous namespace)::k_cc_cross(msc::(anonymous namespace)::"
        "CGeo, unsigned short const*, long*)") == "k_cc_cross"
    assert not profsum.short_name("__amd_rocclr_copyBuffer").startswith("k_")


def _counter_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size",
                                           "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow({"Grid_Size": 4096, **r})


def test_stats_one_row_per_kernel_and_grid(tmp_path):
    """A kernel launched with two grid sizes (a pass and its rerun) gets a
    row per grid size; the shares add up to the whole."""
    k = ("void msc::(anonymous namespace)::k_tile_pairs<msc::(anonymous "
         "namespace)::Cfg<32, 16, 16> >(int)")
    rows = [(k, 1024, 0, 3000), (k, 1024, 5000, 9000), (k, 64, 9000, 9010),
            ("void msc::(anonymous namespace)::k_key_hist(int)", 256,
             10000, 10990)]
    path = tmp_path / "trace.csv"
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size_X",
                                           "Start_Timestamp",
                                           "End_Timestamp"])
        w.writeheader()
        for name, grid, a, b in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size_X": grid,
                        "Start_Timestamp": a, "End_Timestamp": b})
    out = tmp_path / "s.md"
    subprocess.run([sys.executable, "-m", "paper_2409_03771_amd.profsum",
                    "stats", str(path), "--cmd", "demo", "--out", str(out)],
                   check=True, cwd=ROOT)
    text = out.read_text()
    assert "| k_tile_pairs<32,16,16> [grid 1024] | 2 | 0.004 |" in text
    assert "| k_tile_pairs<32,16,16> [grid 64] | 1 | 0.000 |" in text
    assert "| k_key_hist | 1 | 0.001 |" in text
    assert "8.000 ms" not in text and "0.008 ms." in text


def test_traffic_scaling_and_source_guard(tmp_path):
    k = "void msc::(anonymous namespace)::k_cc_final(long*)"
    copy = "__amd_rocclr_copyBuffer"
    _counter_csv(tmp_path / "f.csv", [
        {"Kernel_Name": k, "Counter_Name": "FETCH_SIZE", "Counter_Value": 100},
        {"Kernel_Name": k, "Counter_Name": "FETCH_SIZE", "Counter_Value": 300}])
    _counter_csv(tmp_path / "w.csv", [
        {"Kernel_Name": k, "Counter_Name": "WRITE_SIZE", "Counter_Value": 50}])
    _counter_csv(tmp_path / "cf.csv", [
        {"Kernel_Name": copy, "Counter_Name": "FETCH_SIZE", "Counter_Value": 512}])
    _counter_csv(tmp_path / "cw.csv", [
        {"Kernel_Name": copy, "Counter_Name": "WRITE_SIZE", "Counter_Value": 1024}])
    out_json = tmp_path / "traffic_demo.json"
    subprocess.run([sys.executable, "-m", "paper_2409_03771_amd.profsum",
                    "traffic", "--fetch", str(tmp_path / "f.csv"),
                    "--write", str(tmp_path / "w.csv"),
                    "--copy-fetch", str(tmp_path / "cf.csv"),
                    "--copy-write", str(tmp_path / "cw.csv"),
                    "--copy-bytes", str(1024 * 1024), "--cmd", "demo",
                    "--out", str(tmp_path / "t.md"), "--json", str(out_json)],
                   check=True, cwd=ROOT)
    rec = json.loads(out_json.read_text())
    # the copy of 1 MiB reads 512 KiB of FETCH_SIZE: factor 2; writes: 1
    assert rec["fetch_factor"] == pytest.approx(2.0)
    assert rec["write_factor"] == pytest.approx(1.0)
    # mean FETCH 200 KiB * 2 + WRITE 50 KiB = 450 KiB per launch
    assert rec["kernels"]["k_cc_final"]["hbm_bytes"] == pytest.approx(450 * 1024)
    sys.argv = ["bench.py"]
    import bench
    assert bench.traffic_of("demo", "k_cc_final", str(tmp_path)) == 450 * 1024
    assert bench.path_traffic("demo", str(tmp_path)) == 450 * 1024
    assert bench.traffic_of("demo", "k_other", str(tmp_path)) is None
    rec["source_sha256"] = "0" * 64      # taken on other kernel sources
    out_json.write_text(json.dumps(rec))
    assert bench.traffic_of("demo", "k_cc_final", str(tmp_path)) is None
    assert bench.path_traffic("demo", str(tmp_path)) is None
    assert bench.traffic_of("absent", "k_cc_final", str(tmp_path)) is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_perlin_generator_properties():
    """Perlin noise vanishes at lattice points, stays within the bound of
    the twelve-gradient noise (|n| <= 1), does not depend on the z chunking
    or on the grid's extent, and its normalised masks nest (0.9 within 0.5
    within 0.1)."""
    import numpy as np
    from paper_2409_03771_amd import synth
    f = synth.perlin_field((33, 25, 17), seed=5, frequency=0.125)
    assert np.all(f[::8, ::8, ::8] == 0.0)
    g = synth.perlin_field((40, 30, 20), seed=5)
    assert np.abs(g).max() <= 1.0 and g.std() > 0.1
    h = synth.perlin_field((40, 30, 20), seed=5, z_chunk=3)
    assert np.array_equal(g, h)
    assert not np.array_equal(g, synth.perlin_field((40, 30, 20), seed=6))
    # The value at a point does not depend on the grid's extent, so a field
    # generated at a slab's dims is that slab of the larger field.
    assert np.array_equal(synth.perlin_field((23, 17, 9), seed=5),
                          g[:9, :17, :23])
    m9, m5, m1 = (synth.normalized_mask(g, t) for t in (0.9, 0.5, 0.1))
    assert np.all(m9 <= m5) and np.all(m5 <= m1)
    assert 0 < m9.sum() < m5.sum() < m1.sum() < g.size
    assert synth.normalized_mask(g, 0.0).sum() == g.size - (g == g.min()).sum()
