"""Pins of the oracle's CSR construction from a tetrahedra list: on the Kuhn
subdivision of a grid it gives the Freudenthal adjacency that the input
module builds from edge vectors (grid ids and permuted ids), and on random
tetrahedra (repeated vertices included) it equals a set-based restatement."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2409_03771_amd import synth


@pytest.mark.parametrize("n", [2, 3, 7])
def test_kuhn_tets_give_freudenthal_adjacency(n):
    rp, ci = O.csr_from_tets(n ** 3, synth.kuhn_tets(n))
    d = synth.kuhn_csr(n, seed=1, permute=False)
    np.testing.assert_array_equal(rp, d["row_ptr"])
    np.testing.assert_array_equal(ci, d["col_idx"])


def test_kuhn_tets_permuted():
    n = 6
    d = synth.kuhn_csr(n, seed=3)
    rp, ci = O.csr_from_tets(n ** 3, synth.kuhn_tets(n, perm=d["perm"]))
    np.testing.assert_array_equal(rp, d["row_ptr"])
    np.testing.assert_array_equal(ci, d["col_idx"])


@pytest.mark.parametrize("seed", range(5))
def test_random_tets_against_sets(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 30))
    tets = rng.integers(0, n, size=(int(rng.integers(0, 40)), 4))
    rows = [set() for _ in range(n)]
    for t in tets:
        for a in t:
            for b in t:
                if a != b:
                    rows[a].add(int(b))
    rp, ci = O.csr_from_tets(n, tets)
    assert rp[0] == 0 and rp[-1] == ci.size
    for v in range(n):
        assert list(ci[rp[v]:rp[v + 1]]) == sorted(rows[v])
