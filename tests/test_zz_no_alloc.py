"""The grid connected-components entry point that allocates nothing
(cc_label_grid_noalloc) against cc_label_grid, through the C-ABI: two calls
in a row, the second on a smaller input (the static scratch keeps the first
call's contents), bit-exact."""
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


def _pair(msc, mask_np):
    m = torch.from_numpy(np.ascontiguousarray(mask_np)).cuda()
    want = msc.cc_label_grid(m)
    got = torch.full_like(want, -7)
    msc.cc_label_grid_noalloc_into(m, got)
    torch.cuda.synchronize()
    return got.cpu().numpy(), want.cpu().numpy()


def test_noalloc_equals_cc_label_grid_two_calls(msc):
    big = synth.threshold_mask(synth.gaussian_field((200, 180, 150), 40, 21),
                               0.6)
    small = synth.threshold_mask(synth.gaussian_field((67, 45, 33), 10, 22),
                                 0.5)
    got, want = _pair(msc, big)
    np.testing.assert_array_equal(got, want, err_msg="first (larger) call")
    got, want = _pair(msc, small)
    np.testing.assert_array_equal(got, want, err_msg="second (smaller) call")
    np.testing.assert_array_equal(got, O.cc_grid(small)[0])


@pytest.mark.parametrize("dims", [(1, 1, 1), (37, 1, 1), (40, 30, 1),
                                  (33, 17, 18)])
def test_noalloc_degenerate_and_ragged(msc, dims):
    rng = np.random.default_rng(sum(dims))
    mask = (rng.random(dims[::-1]) < 0.55).astype(np.uint8)
    got, want = _pair(msc, mask)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(got, O.cc_grid(mask)[0])


def test_noalloc_rejects_more_than_its_scratch(msc):
    m = torch.zeros(8, dtype=torch.uint8, device="cuda")
    lab = torch.zeros(8, dtype=torch.int64, device="cuda")
    with pytest.raises(msc.MscError) as e:
        msc.cc_label_grid_noalloc_into(m, lab, dims=(1024, 1024, 129))
    assert e.value.code == msc.MSC_ERANGE
