"""Pins of the oracle's connected components: union-find against BFS, an
independent label-propagation brute force on every mask of tiny grids, and
scipy's labelling routines (ndimage.label with the Freudenthal structuring
element, csgraph.connected_components).  CPU only."""
import itertools

import numpy as np
import pytest
import scipy.ndimage as ndi
from scipy.sparse import csr_matrix, diags
from scipy.sparse.csgraph import connected_components

from oracle import brute
from oracle import oracle as O
from paper_2409_03771_amd import synth


def _freudenthal_structure():
    s = np.zeros((3, 3, 3), bool)
    s[1, 1, 1] = True
    for dx, dy, dz in O.stencil():
        s[1 + dz, 1 + dy, 1 + dx] = True
    return s


def _min_id_labels(lab_scipy, mask):
    """Turn scipy's component numbering into smallest-id labels."""
    flat = lab_scipy.reshape(-1)
    m = mask.reshape(-1).astype(bool)
    out = np.full(flat.size, -1, np.int64)
    ids = np.arange(flat.size)
    k = flat.max()
    first = np.full(k + 1, flat.size, np.int64)
    np.minimum.at(first, flat[m], ids[m])
    out[m] = first[flat[m]]
    return out


def _stacked(masks, dims):
    """Stack tiny masks along z with an all-zero separator plane between
    them, so one oracle call labels every mask independently."""
    X, Y, Z = dims
    B = masks.shape[0]
    big = np.zeros((B, Z + 1, Y, X), np.uint8)
    big[:, :Z] = masks.reshape(B, Z, Y, X)
    return big.reshape(B * (Z + 1), Y, X)


def _unstack(label, B, dims):
    X, Y, Z = dims
    per = (Z + 1) * Y * X
    lab = label.reshape(B, per)[:, : X * Y * Z]
    off = (np.arange(B) * per)[:, None]
    return np.where(lab >= 0, lab - off, -1)


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 3, 2)])
def test_every_mask_matches_brute_force(dims):
    X, Y, Z = dims
    n = X * Y * Z
    M = np.array(list(itertools.product((0, 1), repeat=n)), np.uint8)
    want = brute.cc_batch(M, X, Y, Z)
    big = _stacked(M, dims)
    for method in ("uf", "bfs"):
        lab, _ = O.cc_grid(big, method)
        np.testing.assert_array_equal(_unstack(lab, M.shape[0], dims), want)


@pytest.mark.parametrize("density", [0.1, 0.3, 0.5, 0.7, 0.95])
@pytest.mark.parametrize("dims", [(40, 30, 20), (64, 48, 1), (200, 1, 1)])
def test_grid_cc_vs_scipy_label(density, dims):
    X, Y, Z = dims
    rng = np.random.default_rng(int(density * 100) + X)
    mask = (rng.uniform(size=(Z, Y, X)) < density).astype(np.uint8)
    lab_uf, k_uf = O.cc_grid(mask, "uf")
    lab_bfs, k_bfs = O.cc_grid(mask, "bfs")
    sl, ks = ndi.label(mask, structure=_freudenthal_structure())
    want = _min_id_labels(sl, mask)
    np.testing.assert_array_equal(lab_uf, want)
    np.testing.assert_array_equal(lab_bfs, want)
    assert k_uf == k_bfs == ks


def test_threshold_mask_c1_properties():
    f = synth.config_field("c1")
    mask = synth.threshold_mask(f, 0.7)
    n = f.size
    assert abs(int(mask.sum()) - (n - int(0.7 * n) - 1)) <= 0
    lab, k = O.cc_grid(mask)
    ids = np.arange(n)
    m = mask.reshape(-1).astype(bool)
    assert (lab[~m] == -1).all()
    assert (lab[m] <= ids[m]).all()
    assert (lab[lab[m]] == lab[m]).all()
    sl, ks = ndi.label(mask, structure=_freudenthal_structure())
    np.testing.assert_array_equal(lab, _min_id_labels(sl, mask))


def _csr_from_edges(n, E):
    rows = [[] for _ in range(n)]
    for u, v in E:
        rows[u].append(v)
        rows[v].append(u)
    row_ptr = np.zeros(n + 1, np.int64)
    cols = []
    for v in range(n):
        cols += sorted(rows[v])
        row_ptr[v + 1] = len(cols)
    return row_ptr, np.array(cols, np.int32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_csr_cc_vs_scipy_csgraph(seed):
    rng = np.random.default_rng(seed)
    n = 3000
    E = rng.integers(0, n, size=(2600, 2))
    row_ptr, col = _csr_from_edges(n, [tuple(e) for e in E])
    lab, k = O.cc_csr(row_ptr, col)
    lab2, k2 = O.cc_csr(row_ptr, col, method="bfs")
    A = csr_matrix((np.ones(col.size), col, row_ptr), shape=(n, n))
    ks, comp = connected_components(A, directed=False)
    first = np.full(ks, n, np.int64)
    np.minimum.at(first, comp, np.arange(n))
    np.testing.assert_array_equal(lab, first[comp])
    np.testing.assert_array_equal(lab2, first[comp])
    assert k == k2 == ks
    # with a mask: vertices outside it drop out, with their edges
    mask = (rng.uniform(size=n) < 0.6).astype(np.uint8)
    lab, k = O.cc_csr(row_ptr, col, mask)
    keep = mask.astype(bool)
    D = diags(keep.astype(np.float64))
    sub = (D @ A @ D).tocsr()
    sub.eliminate_zeros()
    _, comp = connected_components(sub, directed=False)
    first = np.full(comp.max() + 1, n, np.int64)
    np.minimum.at(first, comp[keep], np.arange(n)[keep])
    np.testing.assert_array_equal(lab[keep], first[comp[keep]])
    assert (lab[~keep] == -1).all()


def test_csr_of_kuhn_grid_equals_grid_partition():
    """The permuted Kuhn CSR of a grid and the grid itself give the same
    foreground partition (mask given both ways, and as explicit geometry)."""
    g = synth.kuhn_csr(12, seed=2, nbumps=6)
    perm, mask = g["perm"], g["mask"]
    n = perm.size
    gmask = mask[perm].reshape(12, 12, 12)
    lab_grid, kg = O.cc_grid(gmask)
    lab_csr, kc = O.cc_csr(g["row_ptr"], g["col_idx"], mask)
    lab_fg, _ = O.cc_csr(g["fg_row_ptr"], g["fg_col_idx"])
    assert kg == kc
    m = gmask.reshape(-1).astype(bool)
    # same partition: pairs of grid vertices share a label in both
    a = lab_grid[m]
    b = lab_csr[perm[np.flatnonzero(m)]]
    _, ia = np.unique(a, return_inverse=True)
    _, ib = np.unique(b, return_inverse=True)
    pairs = set(zip(ia.tolist(), ib.tolist()))
    assert len(pairs) == len(set(ia.tolist())) == len(set(ib.tolist()))
    # explicit geometry: foreground labels equal the masked CSR labels
    fg = mask.astype(bool)
    np.testing.assert_array_equal(lab_fg[fg], lab_csr[fg])
    assert (lab_fg[~fg] == np.arange(n)[~fg]).all()   # isolated vertices
    # full CSR without mask is one component labelled 0
    lab_all, k_all = O.cc_csr(g["row_ptr"], g["col_idx"])
    assert k_all == 1 and (lab_all == 0).all()
