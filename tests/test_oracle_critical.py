"""Pins of the oracle's critical point classification and extremum graph:
Banchoff's critical point theorem (the sum over vertices of 1 - chi(lower
link) is the Euler characteristic of the domain, 1 for a grid box of any
dimension); the link's extrema are exactly the segmentation's roots; the
component counts equal those of the lattice-rule link; and the extremum
graph's edges end at extrema, one per link component, the steepest path's
extremum among them."""
import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from paper_2409_03771_amd import synth

DIMS = [(6, 5, 4), (7, 6, 1), (1, 9, 8), (12, 1, 1), (1, 1, 1), (2, 2, 2),
        (5, 1, 6), (17, 13, 9)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("levels", [None, 2])
def test_banchoff_and_extrema(dims, levels):
    X, Y, Z = dims
    f = synth.random_field(dims, seed=X + 3 * Y + 7 * Z, levels=levels)
    lc, uc, chi = O.critical(f)
    assert int((1 - chi.astype(np.int64)).sum()) == 1
    asc, desc, _ = O.segment(f)
    ids = np.arange(X * Y * Z)
    np.testing.assert_array_equal(uc == 0, asc == ids)
    np.testing.assert_array_equal(lc == 0, desc == ids)


def test_gaussian_field_banchoff():
    f = synth.gaussian_field((40, 33, 27), 12, seed=2)
    lc, uc, chi = O.critical(f)
    assert int((1 - chi.astype(np.int64)).sum()) == 1
    assert (lc > 1).sum() > 0 and (uc > 1).sum() > 0


@pytest.mark.parametrize("dims", [(4, 4, 3), (5, 4, 1), (1, 6, 5), (3, 3, 3)])
@pytest.mark.parametrize("levels", [None, 2])
def test_components_equal_lattice_rule_link(dims, levels):
    f = synth.random_field(dims, seed=sum(dims), levels=levels)
    lc, uc, _ = O.critical(f)
    blc, buc = brute.link_components(f, *dims)
    np.testing.assert_array_equal(lc, blc)
    np.testing.assert_array_equal(uc, buc)


@pytest.mark.parametrize("dims", [(9, 8, 7), (11, 10, 1)])
def test_extremum_graph_invariants(dims):
    f = synth.random_field(dims, seed=5)
    asc, desc, _ = O.segment(f)
    lc, uc, _ = O.critical(f)
    E = O.extremum_edges(f, asc, desc)
    n = f.size
    ids = np.arange(n)
    for tag, cnt, lab in ((1, uc, asc), (-1, lc, desc)):
        rows = E[E[:, 2] == tag]
        saddles = ids[cnt >= 2]
        np.testing.assert_array_equal(np.unique(rows[:, 0]), saddles)
        per = np.bincount(rows[:, 0], minlength=n)
        np.testing.assert_array_equal(per[saddles], cnt[saddles])
        assert np.all(lab[rows[:, 1]] == rows[:, 1])   # ends at an extremum
        for s in saddles[:200]:                        # the steepest path's
            assert lab[s] in rows[rows[:, 0] == s, 1]  # extremum is one end
    assert np.all(np.diff(E[:, 0]) >= 0)
