"""Segmentation on a complex given as CSR adjacency (msc_segment_csr)
through the C ABI, bit-exact against the oracle: permuted Kuhn meshes, the
Freudenthal grid's own adjacency (equal to the grid path), random graphs
with ties and one-sided rows, edge cases and errors, and the pair table's
regrowth."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2409_03771_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def msc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_03771_amd import msc as m
    return m


def gpu_csr(msc, rp, ci, f, **kw):
    out = msc.segment_csr(torch.from_numpy(rp).cuda(),
                          torch.from_numpy(ci).cuda(),
                          torch.from_numpy(np.ascontiguousarray(f)).cuda(),
                          **kw)
    torch.cuda.synchronize()
    return [None if x is None else x.cpu().numpy() for x in out]


def check(msc, rp, ci, f, tag):
    want = O.segment_csr(rp, ci, f)
    got = gpu_csr(msc, rp, ci, f)
    for name, g, w in zip(("asc", "desc", "ms"), got, want):
        np.testing.assert_array_equal(g, w, err_msg=f"{tag} {name}")
    st = msc.last_stats()
    assert st["n_maxima"] == len(np.unique(want[0]))
    assert st["n_minima"] == len(np.unique(want[1]))
    assert st["n_cells"] == len(np.unique(want[2]))


@pytest.mark.parametrize("n_axis,seed", [(40, 9), (23, 3)])
def test_permuted_kuhn_mesh(msc, n_axis, seed):
    print(f"[csr segment] kuhn {n_axis} seed {seed}", flush=True)
    d = synth.kuhn_csr(n_axis, seed=seed, nbumps=20)
    f = np.empty_like(d["field"])
    f[d["perm"]] = d["field"]
    check(msc, d["row_ptr"], d["col_idx"], f, f"kuhn {n_axis}")


@pytest.mark.parametrize("levels", [None, 4])
def test_grid_adjacency_equals_grid_path(msc, levels):
    n = 33
    d = synth.kuhn_csr(n, seed=5, nbumps=12, permute=False)
    f = d["field"] if levels is None else \
        synth.random_field((n, n, n), seed=6, levels=levels).reshape(-1)
    got = gpu_csr(msc, d["row_ptr"], d["col_idx"], f)
    grid = msc.segment(torch.from_numpy(f.reshape(n, n, n)).cuda())
    torch.cuda.synchronize()
    for g, w in zip(got, grid):
        np.testing.assert_array_equal(g, w.cpu().numpy())


def random_graph(n, p, seed, symmetric):
    rng = np.random.default_rng(seed)
    deg = rng.binomial(max(n - 1, 0), p, size=n) if n else np.zeros(0, int)
    rows = [rng.choice(n, size=int(k), replace=True) for k in deg]
    if symmetric:
        sets = [set() for _ in range(n)]
        for v, r in enumerate(rows):
            for u in r:
                sets[v].add(int(u))
                sets[int(u)].add(v)
        rows = [sorted(s) for s in sets]
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = (np.concatenate([np.asarray(r, np.int32) for r in rows])
          if n and rp[-1] else np.zeros(0, np.int32))
    return rp, ci.astype(np.int32)


@pytest.mark.parametrize("n,p,symmetric", [
    (1, 0.0, True), (2, 1.0, True), (17, 0.3, True), (1000, 0.01, True),
    (5000, 0.002, False), (3000, 0.0, True)])
@pytest.mark.parametrize("levels", [None, 3])
def test_random_graphs(msc, n, p, symmetric, levels):
    rp, ci = random_graph(n, p, seed=n + int(100 * p), symmetric=symmetric)
    rng = np.random.default_rng(n)
    f = (rng.standard_normal(n) if levels is None
         else rng.integers(0, levels, n)).astype(np.float32)
    check(msc, rp, ci, f, f"n={n} p={p} sym={symmetric} levels={levels}")


def test_edgeless_and_empty(msc):
    rp = np.zeros(6, np.int64)
    ci = np.zeros(0, np.int32)
    a, d, m = gpu_csr(msc, rp, ci, np.arange(5, dtype=np.float32))
    assert (a == np.arange(5)).all() and (d == a).all() and (m == a).all()
    a, d, m = gpu_csr(msc, np.zeros(1, np.int64), ci,
                      np.zeros(0, np.float32))
    assert a.size == d.size == m.size == 0


def test_partial_outputs(msc):
    d = synth.kuhn_csr(20, seed=4, nbumps=8)
    f = np.empty_like(d["field"])
    f[d["perm"]] = d["field"]
    want = O.segment_csr(d["row_ptr"], d["col_idx"], f)
    for keep in (("ms",), ("asc",), ("desc", "ms")):
        got = gpu_csr(msc, d["row_ptr"], d["col_idx"], f, want=keep)
        for name, g, w in zip(("asc", "desc", "ms"), got, want):
            if name in keep:
                np.testing.assert_array_equal(g, w, err_msg=f"{keep} {name}")
            else:
                assert g is None


def test_errors(msc):
    rp = np.array([0, 2, 3, 4], np.int64)
    f = np.zeros(3, np.float32)
    for bad in (np.array([1, 3, 0, 1], np.int32),
                np.array([1, -1, 0, 1], np.int32)):
        with pytest.raises(Exception):
            gpu_csr(msc, rp, bad, f)
    with pytest.raises(Exception):   # a row pointer past the last entry
        gpu_csr(msc, np.array([0, 2, 9, 4], np.int64),
                np.array([1, 2, 0, 1], np.int32), f)
    nan = np.array([0, np.nan, 1], np.float32)
    with pytest.raises(Exception):
        gpu_csr(msc, rp, np.array([1, 2, 0, 1], np.int32), nan)
    # the context still works
    check(msc, rp, np.array([1, 2, 0, 1], np.int32),
          np.array([3, 1, 2], np.float32), "after errors")


def test_pair_table_regrows(msc):
    d = synth.kuhn_csr(30, seed=7, nbumps=4)
    rng = np.random.default_rng(1)
    f = rng.standard_normal(d["row_ptr"].size - 1).astype(np.float32)
    try:
        msc.set_table_capacity(1024)
        check(msc, d["row_ptr"], d["col_idx"], f, "small table")
        assert msc.last_stats()["n_cells"] > 4096
    finally:
        msc.set_table_capacity(0)
