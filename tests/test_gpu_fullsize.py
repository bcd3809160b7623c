"""Parity at the full 1024^3 workload, in the launch configuration the
benchmark times.  The oracle cannot segment 2^30 vertices in seconds, so:

  * asc and desc are checked on every vertex by the oracle's local
    characterisation (root[v] == v iff v is a fixed point of the steepest
    step, else root[v] == root[S(v)]), which determines the root maps
    uniquely;
  * sampled vertices are walked by the oracle from scratch;
  * ms is checked on every vertex by properties that pin it to the
    smallest-id definition: ms[v] <= v, pair(ms[v]) == pair(v),
    ms[ms[v]] == ms[v], and the fixed points carry distinct pairs.

Connected components are compared label by label with the oracle's
union-find at full size: the 1024^3 grid mask and the 368^3 CSR mesh.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2409_03771_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    from paper_2409_03771_amd import msc
    assert torch.cuda.is_available()
    print("[fullsize] generating gauss1024 on the device", flush=True)
    f = synth.config_field("gauss1024", device="cuda")
    asc, desc, ms = msc.segment(f)
    torch.cuda.synchronize()
    stats = msc.last_stats()
    print(f"[fullsize] stats {stats}", flush=True)
    out = (f.cpu().numpy(), asc.cpu().numpy(), desc.cpu().numpy(),
           ms.cpu().numpy(), stats)
    del f, asc, desc, ms
    torch.cuda.empty_cache()
    return out


def test_fullsize_roots_local_characterisation(full):
    f, asc, desc, _, _ = full
    bad, first = O.check_roots(f, asc, +1, threads=16)
    assert bad == 0, f"asc: {bad} violations, first at {first}"
    bad, first = O.check_roots(f, desc, -1, threads=16)
    assert bad == 0, f"desc: {bad} violations, first at {first}"


def test_fullsize_sampled_walks(full):
    f, asc, desc, _, _ = full
    rng = np.random.default_rng(7)
    for v in rng.integers(0, asc.size, 300):
        assert O.walk_from(f, v, +1) == asc[v], v
        assert O.walk_from(f, v, -1) == desc[v], v


def test_fullsize_ms_properties(full):
    _, asc, desc, ms, stats = full
    n = asc.size
    chunk = 1 << 26
    reps = []
    for v0 in range(0, n, chunk):
        v1 = min(n, v0 + chunk)
        ids = np.arange(v0, v1, dtype=np.int64)
        m = ms[v0:v1].astype(np.int64)
        assert (m >= 0).all() and (m <= ids).all()
        assert (asc[m] == asc[v0:v1]).all() and (desc[m] == desc[v0:v1]).all()
        assert (ms[m] == m).all()
        fixed = ids[m == ids]
        reps.append(asc[fixed].astype(np.int64) * n + desc[fixed])
    reps = np.concatenate(reps)
    assert np.unique(reps).size == reps.size
    assert reps.size == stats["n_cells"]


def test_fullsize_extrema_counts(full):
    _, asc, desc, _, stats = full
    for roots, key in ((asc, "n_maxima"), (desc, "n_minima")):
        seen = np.zeros(roots.size, bool)
        seen[roots] = True
        assert int(seen.sum()) == stats[key]


def test_fullsize_cc_grid(full):
    """Mask at the 70th percentile of the 1024^3 field, every label."""
    from paper_2409_03771_amd import msc
    mask = synth.threshold_mask(full[0], 0.7)
    print("[fullsize] cc grid on the device", flush=True)
    lab = msc.cc_label_grid(torch.from_numpy(mask).cuda())
    torch.cuda.synchronize()
    got = lab.cpu().numpy()
    del lab
    torch.cuda.empty_cache()
    print("[fullsize] cc grid oracle", flush=True)
    want, ncomp = O.cc_grid(mask)
    print(f"[fullsize] {ncomp} components", flush=True)
    np.testing.assert_array_equal(got, want)


@pytest.fixture(scope="module")
def kuhn50m():
    print("[fullsize] generating the 368^3 Kuhn CSR mesh", flush=True)
    return synth.kuhn_csr(368, seed=2)


def test_fullsize_cc_csr(kuhn50m):
    """The 49.8M-vertex permuted Kuhn mesh: masked CSR, the explicit
    foreground graph, and the full mesh with no mask (one component over
    every vertex: the longest union chains), every label."""
    from paper_2409_03771_amd import msc
    d = kuhn50m
    cases = [("masked", d["row_ptr"], d["col_idx"], d["mask"]),
             ("explicit", d["fg_row_ptr"], d["fg_col_idx"], None),
             ("full", d["row_ptr"], d["col_idx"], None)]
    for name, rp, ci, mask in cases:
        print(f"[fullsize] csr {name} on the device", flush=True)
        lab = msc.cc_label_csr(
            torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
            None if mask is None else torch.from_numpy(mask).cuda())
        torch.cuda.synchronize()
        got = lab.cpu().numpy()
        del lab
        want, _ = O.cc_csr(rp, ci, mask)
        np.testing.assert_array_equal(got, want, err_msg=name)
        if name == "full":  # a connected mesh: every label is vertex 0
            assert (want == 0).all()


def test_fullsize_segment_csr(kuhn50m):
    """Segmentation of the mesh's field (values at the jittered positions,
    in permuted ids) over its CSR adjacency: asc, desc and ms of every vertex
    equal the oracle's."""
    from paper_2409_03771_amd import msc
    d = kuhn50m
    f = np.empty_like(d["field"])
    f[d["perm"]] = d["field"]
    print("[fullsize] csr segmentation on the device", flush=True)
    got = msc.segment_csr(torch.from_numpy(d["row_ptr"]).cuda(),
                          torch.from_numpy(d["col_idx"]).cuda(),
                          torch.from_numpy(f).cuda())
    torch.cuda.synchronize()
    got = [x.cpu().numpy() for x in got]
    st = msc.last_stats()
    print("[fullsize] csr segmentation on the oracle", flush=True)
    want = O.segment_csr(d["row_ptr"], d["col_idx"], f)
    for name, g, w in zip(("asc", "desc", "ms"), got, want):
        np.testing.assert_array_equal(g, w, err_msg=name)
    assert st["n_maxima"] == len(np.unique(want[0]))
    assert st["n_cells"] == len(np.unique(want[2]))


def test_fullsize_csr_from_tets(kuhn50m):
    """The 368^3 mesh's 296M Kuhn tetrahedra (permuted ids) give, on the
    device, exactly the adjacency the input module builds from edge
    vectors."""
    from paper_2409_03771_amd import msc
    d = kuhn50m
    print("[fullsize] generating the 296M tetrahedra", flush=True)
    tets = synth.kuhn_tets(368, perm=d["perm"])
    t = torch.from_numpy(tets).cuda()
    del tets
    print("[fullsize] building the adjacency on the device", flush=True)
    rp, ci = msc.csr_from_tets(368 ** 3, t)
    torch.cuda.synchronize()
    del t
    np.testing.assert_array_equal(rp.cpu().numpy(), d["row_ptr"])
    np.testing.assert_array_equal(ci.cpu().numpy(), d["col_idx"])
