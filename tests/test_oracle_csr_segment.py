"""Pins of the oracle's segmentation on a complex given as CSR adjacency:
on the Freudenthal grid's own adjacency (built in the input module from its
edge vectors, not from the oracle's tetrahedra) it must equal the grid
oracle label for label, ties included; relabelling the vertices must map
the results through the permutation; and on tiny random graphs it must
equal a brute-force restatement that compares every pair of candidates."""
import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from paper_2409_03771_amd import synth


@pytest.mark.parametrize("levels", [None, 3])
def test_csr_on_grid_adjacency_equals_grid_oracle(levels):
    n = 9
    d = synth.kuhn_csr(n, seed=1, nbumps=6, permute=False)
    f = d["field"] if levels is None else \
        synth.random_field((n, n, n), seed=4, levels=levels).reshape(-1)
    got = O.segment_csr(d["row_ptr"], d["col_idx"], f)
    want = O.segment(f.reshape(n, n, n))
    for g, w in zip(got, want):
        np.testing.assert_array_equal(g, w)


def test_csr_relabelling_maps_through_permutation():
    n = 10
    d0 = synth.kuhn_csr(n, seed=2, nbumps=6, permute=False)
    d1 = synth.kuhn_csr(n, seed=2, nbumps=6)
    f = d0["field"]
    assert len(np.unique(f)) == f.size  # distinct values: ids never decide
    perm = d1["perm"]
    fp = np.empty_like(f)
    fp[perm] = f
    a0, dd0, m0 = O.segment_csr(d0["row_ptr"], d0["col_idx"], f)
    a1, dd1, m1 = O.segment_csr(d1["row_ptr"], d1["col_idx"], fp)
    np.testing.assert_array_equal(a1[perm], perm[a0])
    np.testing.assert_array_equal(dd1[perm], perm[dd0])
    # the cell of perm[g] is the image of g's cell; its id is its smallest
    # permuted id
    cls = {}
    for g in range(f.size):
        cls.setdefault(m0[g], []).append(perm[g])
    want = np.empty(f.size, np.int64)
    for g in range(f.size):
        want[perm[g]] = min(cls[m0[g]])
    np.testing.assert_array_equal(m1, want)


@pytest.mark.parametrize("seed", range(6))
def test_csr_random_graphs_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 11))
    rows = [[] for _ in range(n)]
    for u in range(n):
        for v in range(n):
            if u != v and rng.random() < 0.3:
                rows[u].append(v)          # one-sided entries on purpose
    if n > 1:
        rows[0].append(0)                  # a self entry is harmless
    row_ptr = np.zeros(n + 1, np.int64)
    row_ptr[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([u for r in rows for u in r], np.int32)
    F = rng.integers(0, 3, size=(12, n)).astype(np.float32)
    A, D, M = brute.segment_graph(rows, F)
    for b in range(F.shape[0]):
        got = O.segment_csr(row_ptr, col, F[b])
        for g, w in zip(got, (A[b], D[b], M[b])):
            np.testing.assert_array_equal(g, w, err_msg=f"seed {seed} b {b}")
