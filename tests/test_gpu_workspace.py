"""Caller-owned workspace and the depth of the asynchronous call queue.

A context given a workspace carves every call's scratch from it: results
equal the oracle, a call that does not fit fails with MSC_ENOMEM without
allocating, and the context returns to its own memory afterwards.  More
asynchronous segmentation calls than the context keeps records for run back
to back, and the stats calls report the most recent one."""
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


def test_caller_workspace(msc):
    f = synth.gaussian_field((70, 45, 38), 10, 41)
    m = synth.threshold_mask(f, 0.6)
    seg_ws = msc.workspace_size(msc.REQ_SEGMENT, [(70, 45, 38)])
    cc_ws = msc.workspace_size(msc.REQ_CC_GRID, [(70, 45, 38)])
    # Needs grow with the field and with the number of fields.
    assert msc.workspace_size(msc.REQ_SEGMENT, [(140, 45, 38)]) > seg_ws
    assert msc.workspace_size(msc.REQ_SEGMENT,
                              [(70, 45, 38)] * 3) >= 2 * seg_ws
    assert cc_ws >= 70 * 45 * 38 * 2
    buf = torch.empty(max(seg_ws, cc_ws) + 512, dtype=torch.uint8,
                      device="cuda")
    assert buf.data_ptr() % 256 == 0
    try:
        with pytest.raises(msc.MscError) as e:
            msc.set_workspace(buf[1:])  # misaligned
        assert e.value.code == msc.MSC_EINVAL
        msc.set_workspace(buf)
        tf = torch.from_numpy(f).cuda()
        got = msc.segment(tf)
        lab = msc.cc_label_grid(torch.from_numpy(m).cuda())
        torch.cuda.synchronize()
        for name, g, w in zip(("asc", "desc", "ms"), got, O.segment(f)):
            np.testing.assert_array_equal(g.cpu().numpy(), w, err_msg=name)
        np.testing.assert_array_equal(lab.cpu().numpy(), O.cc_grid(m)[0])
        big = torch.from_numpy(synth.gaussian_field((140, 90, 38), 10, 42))
        with pytest.raises(msc.MscError) as e:
            msc.segment(big.cuda())
        assert e.value.code == msc.MSC_ENOMEM
    finally:
        msc.set_workspace(None)
    got = msc.segment(big.cuda())  # the context's own memory again
    torch.cuda.synchronize()
    for name, g, w in zip(("asc", "desc", "ms"), got,
                          O.segment(big.numpy())):
        np.testing.assert_array_equal(g.cpu().numpy(), w, err_msg=name)


def test_more_calls_than_records(msc):
    """Ten asynchronous calls on one stream (more than the four records a
    context keeps): each equals the oracle; the stats are the last call's,
    a NaN in an earlier call does not leak into them, and a NaN in the last
    call is reported."""
    fields = [synth.gaussian_field((40 + 3 * i, 33, 29 - i), 6, 60 + i)
              for i in range(10)]
    bad = fields[2].copy()
    bad.reshape(-1)[5] = np.nan
    s = torch.cuda.Stream()
    dev = [torch.from_numpy(x).cuda() for x in fields[:2] + [bad] + fields[3:]]
    outs = [tuple(torch.empty(t.numel(), dtype=torch.int32, device="cuda")
                  for _ in range(3)) for t in dev]
    torch.cuda.synchronize()
    for t, o in zip(dev, outs):
        msc.segment_into(t, *o, stream=s, check=False)
    assert msc.last_status() == msc.MSC_OK
    st = msc.last_stats()
    assert st["n_vertices"] == fields[-1].size
    for i, (f, o) in enumerate(zip(fields, outs)):
        if i == 2:
            continue
        want = O.segment(f)
        for name, g, w in zip(("asc", "desc", "ms"), o, want):
            np.testing.assert_array_equal(g.cpu().numpy(), w,
                                          err_msg=f"call {i} {name}")
        if i == len(fields) - 1:
            assert st["n_maxima"] == np.unique(want[0]).size
            assert st["n_cells"] == np.unique(want[2]).size
    t = torch.from_numpy(bad).cuda()
    msc.segment_into(t, *outs[2], stream=s, check=False)
    assert msc.last_status() == msc.MSC_ENAN
