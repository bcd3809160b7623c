"""Parity of the HIP connected components (grid mask and CSR) and of the
pointer-jumping entry point with the CPU oracle, bit-exact."""
import itertools
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2409_03771_amd import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def msc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_03771_amd import msc as m
    return m


def gpu_cc_grid(msc, mask):
    lab = msc.cc_label_grid(torch.from_numpy(np.ascontiguousarray(mask)).cuda())
    torch.cuda.synchronize()
    return lab.cpu().numpy()


def gpu_cc_csr(msc, row_ptr, col, mask=None):
    mt = None if mask is None else torch.from_numpy(mask).cuda()
    lab = msc.cc_label_csr(torch.from_numpy(row_ptr).cuda(),
                           torch.from_numpy(col).cuda(), mt)
    torch.cuda.synchronize()
    return lab.cpu().numpy()


def test_gauss64_threshold_mask(msc):
    f = synth.config_field("gauss64")
    mask = synth.threshold_mask(f, 0.7)
    want, _ = O.cc_grid(mask)
    np.testing.assert_array_equal(gpu_cc_grid(msc, mask), want)


@pytest.mark.parametrize("density", [0.05, 0.3, 0.55, 0.9, 1.0, 0.0])
@pytest.mark.parametrize("dims", [(61, 47, 33), (1, 1, 1), (500, 1, 1),
                                  (1, 70, 60), (80, 90, 1), (129, 3, 2)])
def test_random_masks(msc, dims, density):
    X, Y, Z = dims
    rng = np.random.default_rng(X * 7 + int(density * 100))
    mask = (rng.uniform(size=(Z, Y, X)) < density).astype(np.uint8)
    want, _ = O.cc_grid(mask)
    np.testing.assert_array_equal(gpu_cc_grid(msc, mask), want)


def test_every_mask_3x3x2_in_one_call(msc):
    """All 2^18 masks of a 3x3x2 grid stacked along z with an empty plane
    between them: one call labels every mask independently."""
    M = np.array(list(itertools.product((0, 1), repeat=18)), np.uint8)
    big = np.zeros((M.shape[0], 3, 3, 3), np.uint8)
    big[:, :2] = M.reshape(-1, 2, 3, 3)
    big = big.reshape(-1, 3, 3)
    want, _ = O.cc_grid(big)
    np.testing.assert_array_equal(gpu_cc_grid(msc, big), want)


def test_gaussian_mask_ragged(msc):
    f = synth.gaussian_field((190, 171, 93), 60, seed=5)
    for q in (0.1, 0.5, 0.7, 0.9):
        mask = synth.threshold_mask(f, q)
        want, _ = O.cc_grid(mask)
        np.testing.assert_array_equal(gpu_cc_grid(msc, mask), want, str(q))


@pytest.fixture(scope="module")
def kuhn():
    return synth.kuhn_csr(28, seed=2, nbumps=10)


def test_csr_masked_explicit_and_full(msc, kuhn):
    g = kuhn
    want, _ = O.cc_csr(g["row_ptr"], g["col_idx"], g["mask"])
    np.testing.assert_array_equal(
        gpu_cc_csr(msc, g["row_ptr"], g["col_idx"], g["mask"]), want)
    want, _ = O.cc_csr(g["fg_row_ptr"], g["fg_col_idx"])
    np.testing.assert_array_equal(
        gpu_cc_csr(msc, g["fg_row_ptr"], g["fg_col_idx"]), want)
    got = gpu_cc_csr(msc, g["row_ptr"], g["col_idx"])
    assert (got == 0).all()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_csr_random_graph_one_sided(msc, seed):
    """Random sparse graph listed one-sided (each edge in one row only)."""
    rng = np.random.default_rng(seed)
    n = 20000
    E = rng.integers(0, n, size=(int(n * (0.3 + 0.3 * seed)), 2))
    E = np.sort(E, axis=1)
    order = np.lexsort((E[:, 1], E[:, 0]))
    E = E[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, E[:, 0] + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    col = E[:, 1].astype(np.int32)
    want, _ = O.cc_csr(row_ptr, col)
    np.testing.assert_array_equal(gpu_cc_csr(msc, row_ptr, col), want)
    mask = (rng.uniform(size=n) < 0.7).astype(np.uint8)
    want, _ = O.cc_csr(row_ptr, col, mask)
    np.testing.assert_array_equal(gpu_cc_csr(msc, row_ptr, col, mask), want)


def test_csr_edge_cases(msc):
    # no edges at all
    n = 1000
    rp = np.zeros(n + 1, np.int64)
    col = np.zeros(0, np.int32)
    lab = msc.cc_label_csr(torch.from_numpy(rp).cuda(),
                           torch.empty(0, dtype=torch.int32, device="cuda"))
    assert (lab.cpu().numpy() == np.arange(n)).all()
    # a long path listed in decreasing order: worst case for hooking by id
    n = 5000
    perm = np.random.default_rng(3).permutation(n)
    rows = [[] for _ in range(n)]
    for i in range(n - 1):
        a, b = perm[i], perm[i + 1]
        rows[a].append(b)
        rows[b].append(a)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([u for r in rows for u in sorted(r)], np.int32)
    assert (gpu_cc_csr(msc, rp, col) == 0).all()
    # out-of-range column index is rejected
    bad = col.copy()
    bad[17] = n + 5
    with pytest.raises(msc.MscError) as e:
        gpu_cc_csr(msc, rp, bad)
    assert e.value.code == msc.MSC_EINVAL


def _fig2_rows():
    rows = {}
    with open(os.path.join(GOLDEN, "fig2_pointer_table.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            p = line.split()
            rows[p[0]] = p[1:]
    return rows


def test_pointer_jump_reproduces_fig2(msc):
    rows = _fig2_rows()
    L = {c: i for i, c in enumerate("ABCDEFGHIJKLMNOP")}
    d0 = np.arange(16, dtype=np.int64)
    for c in "ABCDEFGHIJKLMNO":
        d0[L[c]] = L[rows[c][0]] if c in rows else L[c] + 1
    for r in (1, 2, 3):
        d = torch.from_numpy(d0).cuda()
        msc.pointer_jump(d, rounds=r, synchronous=True)
        got = d.cpu().numpy()
        for c, cols in rows.items():
            want = "P" if cols[r] == "-" else cols[r]
            assert got[L[c]] == L[want], (c, r)
    d = torch.from_numpy(d0).cuda()
    msc.pointer_jump(d)             # in place, to convergence
    assert (d.cpu().numpy() == 15).all()


def test_pointer_jump_random_forest(msc):
    rng = np.random.default_rng(9)
    n = 1 << 20
    parent = np.arange(n, dtype=np.int64)
    # random forest: each vertex points to a smaller id or itself
    nonroot = rng.uniform(size=n) < 0.999
    parent[nonroot] = (rng.uniform(size=nonroot.sum()) *
                       np.arange(n)[nonroot]).astype(np.int64)
    want = O.sync_doubling(parent, 25)
    for sync in (True, False):
        d = torch.from_numpy(parent).cuda()
        msc.pointer_jump(d, synchronous=sync)
        np.testing.assert_array_equal(d.cpu().numpy(), want)


def test_batched_masks_equal_oracle(msc):
    """70 masks of uneven shapes (more than one launch's worth, with edge
    shapes and empty and full masks) in one batched call: every mask's
    labels equal the oracle's, ids local to the mask."""
    rng = np.random.default_rng(31)
    masks = []
    shapes = [(1, 1, 1), (33, 17, 17), (64, 1, 1), (1, 40, 3), (32, 16, 16)]
    for k in range(70):
        dims = shapes[k] if k < len(shapes) else tuple(
            int(x) for x in rng.integers(1, 70, size=3))
        X, Y, Z = dims
        if k == 5:
            m = np.zeros((Z, Y, X), np.uint8)
        elif k == 6:
            m = np.ones((Z, Y, X), np.uint8)
        elif k % 3 == 0:
            f = synth.gaussian_field(dims, 6, 300 + k)
            m = synth.threshold_mask(f, 0.6)
        else:
            m = (rng.uniform(size=(Z, Y, X)) < rng.uniform(0.1, 0.9)).astype(
                np.uint8)
        masks.append(m)
    dev = [torch.from_numpy(m).cuda() for m in masks]
    labels = [torch.full((m.size,), -7, dtype=torch.int64, device="cuda")
              for m in masks]
    msc.cc_label_grid_batched_into(dev, labels)
    torch.cuda.synchronize()
    for k, (m, lab) in enumerate(zip(masks, labels)):
        want, _ = O.cc_grid(m)
        np.testing.assert_array_equal(lab.cpu().numpy(), want,
                                      err_msg=f"mask {k} {m.shape}")


def test_batched_masks_edge_cases(msc):
    assert msc.cc_label_grid_batched([]) == []
    m = torch.ones((5, 4, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(TypeError):
        msc.cc_label_grid_batched_into([m], [torch.empty(60, dtype=torch.int32,
                                                         device="cuda")])
    with pytest.raises(ValueError):
        msc.cc_label_grid_batched_into([m], [torch.empty(59, dtype=torch.int64,
                                                         device="cuda")])
    (lab,) = msc.cc_label_grid_batched([m])
    torch.cuda.synchronize()
    assert (lab == 0).all()
