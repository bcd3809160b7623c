"""The paper's distributed scheme with virtual ranks (z-slabs, ghost planes
as extrema, ghost-graph exchange and relabelling) gives exactly the
single-domain labels and the oracle's, for any number of ranks."""
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


def _check(msc, f, ranks_list, oracle=True):
    t = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    want = O.segment(f) if oracle else None
    base = [x.cpu().numpy() for x in msc.segment(t)]
    if want is not None:
        for b, w in zip(base, want):
            np.testing.assert_array_equal(b, w)
    for r in ranks_list:
        got = msc.segment_ranks(t, r)
        torch.cuda.synchronize()
        st = msc.last_stats()
        for name, g, b in zip(("asc", "desc", "ms"), got, base):
            np.testing.assert_array_equal(g.cpu().numpy(), b,
                                          err_msg=f"{f.shape} ranks={r} {name}")
        assert st["n_maxima"] == len(np.unique(base[0]))
        assert st["n_minima"] == len(np.unique(base[1]))
        assert st["n_cells"] == len(np.unique(base[2]))


@pytest.mark.parametrize("dims,levels", [
    ((37, 29, 23), None), ((37, 29, 23), 3), ((64, 64, 17), None),
    ((20, 30, 9), 2), ((33, 1, 31), None), ((1, 1, 40), 3)])
def test_ranks_random_fields(msc, dims, levels):
    f = synth.random_field(dims, seed=sum(dims) + (levels or 0), levels=levels)
    Z = dims[2]
    _check(msc, f, sorted({1, 2, 3, min(5, Z), Z}))


def test_ranks_gaussian(msc):
    f = synth.gaussian_field((131, 77, 90), 30, seed=3)
    _check(msc, f, [1, 2, 4, 7, 16, 90])


def test_ranks_gauss64_and_partial_outputs(msc):
    f = synth.config_field("gauss64")
    _check(msc, f, [2, 8, 64])
    t = torch.from_numpy(f).cuda()
    a, d, m = msc.segment_ranks(t, 4, want=("ms",))
    torch.cuda.synchronize()
    assert a is None and d is None
    np.testing.assert_array_equal(m.cpu().numpy(), O.segment(f)[2])


def test_ranks_errors(msc):
    f = torch.zeros((5, 4, 3), dtype=torch.float32, device="cuda")
    for r in (0, -1, 6):
        with pytest.raises(msc.MscError) as e:
            msc.segment_ranks(f, r)
        assert e.value.code == msc.MSC_EINVAL
    g = torch.from_numpy(synth.random_field((9, 8, 7), seed=1)).cuda()
    g.view(-1)[100] = float("nan")
    with pytest.raises(msc.MscError) as e:
        msc.segment_ranks(g, 3)
    assert e.value.code == msc.MSC_ENAN


def _check_cc(msc, mask, ranks_list):
    t = torch.from_numpy(np.ascontiguousarray(mask)).cuda()
    want, _ = O.cc_grid(mask)
    base = msc.cc_label_grid(t)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(base.cpu().numpy(), want)
    for r in ranks_list:
        got = msc.cc_label_grid_ranks(t, r)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), want,
                                      err_msg=f"{mask.shape} ranks={r}")


@pytest.mark.parametrize("dims,density", [
    ((37, 29, 23), 0.3), ((37, 29, 23), 0.6), ((64, 64, 17), 0.45),
    ((33, 1, 31), 0.5), ((1, 1, 40), 0.7), ((50, 40, 8), 1.0),
    ((40, 30, 12), 0.0)])
def test_cc_ranks_random_masks(msc, dims, density):
    """Random masks near the percolation threshold of the Freudenthal grid
    make components that cross many slab boundaries."""
    X, Y, Z = dims
    rng = np.random.default_rng(sum(dims))
    mask = (rng.random((Z, Y, X)) < density).astype(np.uint8)
    print(f"[cc ranks] dims={dims} density={density}", flush=True)
    _check_cc(msc, mask, sorted({1, 2, 3, min(5, Z), Z}))


@pytest.mark.parametrize("level", [0.9, 0.5, 0.1])
def test_cc_ranks_perlin_thresholds(msc, level):
    f = synth.perlin_field((90, 70, 60), seed=8)
    _check_cc(msc, synth.normalized_mask(f, level), [2, 4, 7, 60])


def test_cc_ranks_gaussian_mask(msc):
    f = synth.gaussian_field((120, 90, 77), 25, seed=4)
    _check_cc(msc, synth.threshold_mask(f, 0.7), [2, 3, 8, 77])


def test_cc_ranks_errors(msc):
    t = torch.ones((5, 4, 3), dtype=torch.uint8, device="cuda")
    for bad in (0, 6, -1):
        with pytest.raises(Exception):
            msc.cc_label_grid_ranks(t, bad)
