"""Pins of the CPU oracle against things other than itself: an independent
brute force on exhaustive tiny grids, closed forms, invariants and the
paper's worked example.  CPU only."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from paper_2409_03771_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
with open(os.path.join(GOLDEN, "gauss64_counts.json")) as _fh:
    GAUSS64 = json.load(_fh)


# ---------------------------------------------------------------------------
# Triangulation
# ---------------------------------------------------------------------------

def test_stencil_from_kuhn_matches_lattice_rule():
    """Edges derived from the six Kuhn tetrahedra equal the lattice rule
    (non-zero difference with entries all in {0,1} or all in {0,-1})."""
    st = {tuple(int(t) for t in r) for r in O.stencil()}
    rule = {d for d in itertools.product((-1, 0, 1), repeat=3)
            if any(d) and (all(t >= 0 for t in d) or all(t <= 0 for t in d))}
    assert len(st) == 14
    assert st == rule
    assert all(tuple(-t for t in d) in st for d in st)


def test_stencil_2d_restriction_is_freudenthal_2d():
    """On a Z=1 grid the edges left are +-(1,0), +-(0,1), +-(1,1)."""
    E = brute.edges(3, 3, 1)
    diffs = set()
    cs = brute.coords(3, 3, 1)
    for u, v in E:
        diffs.add(tuple(cs[v][i] - cs[u][i] for i in range(2)))
    assert diffs == {(1, 0), (0, 1), (1, 1)}


# ---------------------------------------------------------------------------
# Exhaustive tiny fields: C oracle == brute force
# ---------------------------------------------------------------------------

def _oracle_batch(F, dims):
    X, Y, Z = dims
    A, D, M = [], [], []
    for f in F:
        a, d, m = O.segment(f.reshape(Z, Y, X))
        A.append(a), D.append(d), M.append(m)
    return np.array(A), np.array(D), np.array(M)


def _compare_exhaustive(F, dims):
    F = np.asarray(F, np.float32)
    a0, d0, m0 = brute.segment_batch(F, *dims)
    a1, d1, m1 = _oracle_batch(F, dims)
    np.testing.assert_array_equal(a1, a0)
    np.testing.assert_array_equal(d1, d0)
    np.testing.assert_array_equal(m1, m0)


def test_exhaustive_permutations_2x2x2():
    """All 8! orderings of distinct values on a 2x2x2 grid."""
    F = np.array(list(itertools.permutations(range(8))), np.float32)
    _compare_exhaustive(F, (2, 2, 2))


def test_exhaustive_three_levels_2x2x2():
    """All 3^8 fields over {0,1,2}: heavy ties, so the id tie-break decides."""
    F = np.array(list(itertools.product((0, 1, 2), repeat=8)), np.float32)
    _compare_exhaustive(F, (2, 2, 2))


def test_exhaustive_binary_3x3x2():
    """All 2^18 fields over {0,1} on a 3x3x2 grid."""
    F = np.array(list(itertools.product((0, 1), repeat=18)), np.float32)
    _compare_exhaustive(F, (3, 3, 2))


@pytest.mark.parametrize("dims", [(5, 1, 1), (4, 3, 1), (1, 4, 3), (3, 1, 4),
                                  (3, 3, 3), (1, 1, 1)])
def test_random_small_grids_vs_brute(dims):
    rng = np.random.default_rng(sum(dims))
    n = int(np.prod(dims))
    F = np.concatenate([rng.standard_normal((40, n)),
                        rng.integers(0, 3, (40, n))]).astype(np.float32)
    _compare_exhaustive(F, dims)


def test_signed_zero_is_a_tie():
    """-0.0 and +0.0 compare equal, so the id decides."""
    f = np.array([[[0.0, -0.0]]], np.float32)
    a, d, _ = O.segment(f)
    assert list(a) == [1, 1] and list(d) == [0, 0]
    f = np.array([[[-0.0, 0.0]]], np.float32)
    a, d, _ = O.segment(f)
    assert list(a) == [1, 1] and list(d) == [0, 0]


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

DIMS = [(7, 5, 4), (16, 1, 1), (6, 9, 1), (1, 1, 1), (1, 6, 5)]


@pytest.mark.parametrize("dims", DIMS)
def test_constant_field_is_pure_tie_break(dims):
    X, Y, Z = dims
    n = X * Y * Z
    a, d, m = O.segment(np.zeros((Z, Y, X), np.float32))
    assert (a == n - 1).all() and (d == 0).all() and (m == 0).all()


@pytest.mark.parametrize("dims", DIMS)
def test_identity_and_negated_identity(dims):
    X, Y, Z = dims
    n = X * Y * Z
    ids = np.arange(n, dtype=np.float32).reshape(Z, Y, X)
    a, d, m = O.segment(ids)
    assert (a == n - 1).all() and (d == 0).all() and (m == 0).all()
    a, d, m = O.segment(-ids)
    assert (a == 0).all() and (d == n - 1).all() and (m == 0).all()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_ramp_one_max_one_min(axis):
    X, Y, Z = 9, 7, 6
    zz, yy, xx = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X),
                             indexing="ij")
    f = [xx, yy, zz][axis].astype(np.float32)
    a, d, _ = O.segment(f)
    assert (a == X * Y * Z - 1).all()
    assert (d == 0).all()


@pytest.mark.parametrize("n,centre", [(32, (11, 20, 5)), (20, (0, 19, 7))])
def test_single_gaussian_bump_one_ascending_manifold(n, centre):
    sigma = n / 3.0
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                             indexing="ij")
    cx, cy, cz = centre
    r2 = (xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2
    f = np.exp(-r2 / (2 * sigma ** 2)).astype(np.float32)
    a, d, _ = O.segment(f)
    cid = cx + n * cy + n * n * cz
    assert (a == cid).all()
    sp, _ = O.successors(f)
    assert int((sp == np.arange(n ** 3)).sum()) == 1


# ---------------------------------------------------------------------------
# Invariants at the 64^3 workload
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1():
    f = synth.config_field("c1")
    asc, desc, ms = O.segment(f)
    return f, asc, desc, ms


def _key_gt(f, a, b):
    fa, fb = f[a], f[b]
    return (fa > fb) | ((fa == fb) & (a > b))


def test_c1_labels_are_extrema_and_counts(c1):
    f, asc, desc, ms = c1
    ff = f.reshape(-1)
    n = ff.size
    sp, sm = O.successors(f)
    ids = np.arange(n)
    maxima = ids[sp == ids]
    minima = ids[sm == ids]
    assert (sp[asc] == asc).all() and (sm[desc] == desc).all()
    assert set(np.unique(asc)) == set(maxima)
    assert set(np.unique(desc)) == set(minima)
    # regression values the oracle wrote (tests/golden/make_gauss64_counts.py)
    assert len(maxima) == GAUSS64["n_maxima"]
    assert len(minima) == GAUSS64["n_minima"]
    # monotone: the ascent root is never below v, the descent root never above
    assert (_key_gt(ff, asc, ids) | (asc == ids)).all()
    assert (_key_gt(ff, ids, desc) | (desc == ids)).all()


def test_c1_ms_cells(c1):
    f, asc, desc, ms = c1
    n = asc.size
    ids = np.arange(n)
    key = asc.astype(np.int64) * n + desc
    assert (ms <= ids).all()
    assert (ms[ms] == ms).all()
    assert (key[ms] == key).all()
    # brute definition via grouping: the class minimum of every key
    uk, inv = np.unique(key, return_inverse=True)
    mins = np.full(uk.size, n, np.int64)
    np.minimum.at(mins, inv, ids)
    np.testing.assert_array_equal(ms, mins[inv])
    assert len(np.unique(ms)) == uk.size == GAUSS64["n_cells"]


def test_memo_walk_equals_plain_walk(c1):
    f = c1[0]
    sp, sm = O.successors(f)
    for s in (sp, sm):
        np.testing.assert_array_equal(O.walk(s, memo=True),
                                      O.walk(s, memo=False))


def test_walk_from_matches_full_walk(c1):
    f, asc, desc, _ = c1
    rng = np.random.default_rng(1)
    for v in rng.integers(0, asc.size, 200):
        assert O.walk_from(f, v, +1) == asc[v]
        assert O.walk_from(f, v, -1) == desc[v]


def test_local_checker_accepts_truth_and_flags_a_planted_mistake(c1):
    f, asc, desc, _ = c1
    assert O.check_roots(f, asc, +1) == (0, -1)
    assert O.check_roots(f, desc, -1) == (0, -1)
    bad = asc.copy()
    v = int(np.flatnonzero(asc != np.arange(asc.size))[1234])
    bad[v] = asc[v - 1] if asc[v - 1] != asc[v] else v
    nbad, first = O.check_roots(f, bad, +1)
    assert nbad >= 1 and first <= v


# ---------------------------------------------------------------------------
# Worked example (Fig. 2): spiral polyline A..P
# ---------------------------------------------------------------------------

def _fig2_table():
    rows = {}
    with open(os.path.join(GOLDEN, "fig2_pointer_table.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            rows[parts[0]] = parts[1:]
    return rows


def test_fig2_synchronous_doubling_reproduces_columns():
    rows = _fig2_table()
    letter = {c: i for i, c in enumerate("ABCDEFGHIJKLMNOP")}
    d = np.arange(16, dtype=np.int64)
    for c in "ABCDEFGHIJKLMNOP":
        if c in rows:
            d[letter[c]] = letter[rows[c][0]]
        elif c != "P":
            d[letter[c]] = letter[c] + 1      # G, J, M: never a target
    for r in (1, 2, 3):
        got = O.sync_doubling(d, r)
        for c, cols in rows.items():
            want = cols[r]
            want = "P" if want == "-" else want
            assert got[letter[c]] == letter[want], (c, r)
    assert (O.sync_doubling(d, 3)[[letter[c] for c in rows]] == 15).all()


def test_fig2_polyline_labels():
    """f = id along the 16-vertex polyline: every vertex ascends to P and
    descends to A; as one masked component its min-id label is A."""
    f = np.arange(16, dtype=np.float32)
    a, d, m = O.segment(f)
    assert (a == 15).all() and (d == 0).all() and (m == 0).all()
    lab, k = O.cc_grid(np.ones(16, np.uint8))
    assert k == 1 and (lab == 0).all()
    cols, row_ptr = [], [0]
    for v in range(16):
        cols += [u for u in (v - 1, v + 1) if 0 <= u < 16]
        row_ptr.append(len(cols))
    row_ptr = np.array(row_ptr, np.int64)
    lab, k = O.cc_csr(row_ptr, np.array(cols, np.int32))
    assert k == 1 and (lab == 0).all()


def test_oracle_is_reentrant():
    """Concurrent oracle calls (thread pool; the C calls release the GIL)
    give the serial results: the cell sort keeps no global state."""
    from concurrent.futures import ThreadPoolExecutor
    specs = synth.batch_specs(8, seed=5, lo=12, hi=40)
    fields = [synth.gaussian_field(d, nb, sd) for d, nb, sd in specs]
    with ThreadPoolExecutor(8) as pool:
        par = list(pool.map(O.segment, fields))
    for f, p in zip(fields, par):
        for x, y in zip(p, O.segment(f)):
            np.testing.assert_array_equal(x, y)
