"""CSR adjacency from a tetrahedra list on the device (msc_csr_from_tets),
row for row against the oracle: Kuhn subdivisions with grid and permuted
ids, random tetrahedra with repeated vertices, empty inputs; the explicit
pipeline (tetrahedra whose vertices are all in the mask -> adjacency ->
components) and segmentation over the built adjacency; bad vertex ids."""
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


def build(msc, n, tets):
    t = torch.from_numpy(np.ascontiguousarray(tets, np.int32).reshape(-1, 4))
    rp, ci = msc.csr_from_tets(n, t.cuda())
    torch.cuda.synchronize()
    return rp.cpu().numpy(), ci.cpu().numpy()


def check(msc, n, tets, tag):
    rp, ci = build(msc, n, tets)
    wrp, wci = O.csr_from_tets(n, tets)
    np.testing.assert_array_equal(rp, wrp, err_msg=f"{tag} row_ptr")
    np.testing.assert_array_equal(ci, wci, err_msg=f"{tag} col_idx")
    return rp, ci


@pytest.mark.parametrize("n_axis,permute", [(20, False), (24, True),
                                            (2, False)])
def test_kuhn_subdivisions(msc, n_axis, permute):
    d = synth.kuhn_csr(n_axis, seed=4, permute=permute)
    tets = synth.kuhn_tets(n_axis, perm=d["perm"] if permute else None)
    rp, ci = check(msc, n_axis ** 3, tets, f"kuhn {n_axis}")
    np.testing.assert_array_equal(rp, d["row_ptr"])
    np.testing.assert_array_equal(ci, d["col_idx"])


@pytest.mark.parametrize("n,ntets", [(1, 0), (1, 3), (5, 40), (100, 700),
                                     (2000, 9000), (64, 0)])
def test_random_tetrahedra(msc, n, ntets):
    rng = np.random.default_rng(n + ntets)
    tets = rng.integers(0, n, size=(ntets, 4)).astype(np.int32)
    if ntets:
        tets[0] = tets[0, 0]           # a fully degenerate tetrahedron
    check(msc, n, tets, f"random n={n} T={ntets}")


def test_zero_vertices(msc):
    rp, ci = build(msc, 0, np.zeros((0, 4), np.int32))
    assert rp.tolist() == [0] and ci.size == 0


def test_explicit_pipeline(msc):
    """Extracted geometry: the tetrahedra whose four vertices are all in
    the mask, their adjacency built on the device, then components; and the
    segmentation over the full mesh's built adjacency."""
    n_axis = 40
    d = synth.kuhn_csr(n_axis, seed=8, nbumps=16, quantile=0.9)
    n = n_axis ** 3
    tets = synth.kuhn_tets(n_axis, perm=d["perm"])
    keep = d["mask"][tets].all(axis=1)
    kept = np.ascontiguousarray(tets[keep])
    in_geom = np.zeros(n, np.uint8)
    in_geom[kept.reshape(-1)] = 1
    rp, ci = check(msc, n, kept, "extracted")
    lab = msc.cc_label_csr(torch.from_numpy(rp).cuda(),
                           torch.from_numpy(ci).cuda(),
                           torch.from_numpy(in_geom).cuda())
    torch.cuda.synchronize()
    want, k = O.cc_csr(rp, ci, in_geom)
    np.testing.assert_array_equal(lab.cpu().numpy(), want)
    print(f"[explicit] {int(in_geom.sum())} vertices in the geometry, "
          f"{k} components", flush=True)
    assert k >= 1
    rp, ci = check(msc, n, tets, "full")
    f = np.empty_like(d["field"])
    f[d["perm"]] = d["field"]
    got = msc.segment_csr(torch.from_numpy(rp).cuda(),
                          torch.from_numpy(ci).cuda(),
                          torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    for g, w in zip(got, O.segment_csr(d["row_ptr"], d["col_idx"], f)):
        np.testing.assert_array_equal(g.cpu().numpy(), w)


def test_bad_vertex_ids(msc):
    for bad in ([0, 1, 2, 5], [0, -1, 2, 3]):
        with pytest.raises(Exception):
            build(msc, 5, np.array([[0, 1, 2, 3], bad], np.int32))
    check(msc, 5, np.array([[0, 1, 2, 3], [1, 2, 3, 4]], np.int32), "after")
