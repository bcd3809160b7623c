"""Failure handling forced from the host (msc_debug_inject): an allocation
or a HIP runtime call is made to report failure, every kernel still runs
and exits normally.  The failing call reports MSC_ENOMEM / MSC_EHIP, the
requests it touched fail alone, and the context and the queue go on to give
exact results."""
import ctypes

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
    yield m
    m.debug_inject(m.INJECT_ENOMEM, -1)
    m.debug_inject(m.INJECT_EHIP, -1)


def _segment_raw(msc, ctx, t):
    outs = tuple(torch.empty(t.numel(), dtype=torch.int32, device="cuda")
                 for _ in range(3))
    dims = (ctypes.c_int64 * 3)(*msc.grid_dims(t.shape))
    rc = msc._lib.msc_segment(ctx, ctypes.c_void_p(t.data_ptr()), dims,
                              *(ctypes.c_void_p(o.data_ptr()) for o in outs),
                              None)
    return rc, outs


def test_allocation_failures(msc):
    f = synth.gaussian_field((45, 38, 30), 8, 81)
    t = torch.from_numpy(f).cuda()
    # Context creation.
    ctx = ctypes.c_void_p()
    msc.debug_inject(msc.INJECT_ENOMEM, 0)
    assert msc._lib.msc_create(ctypes.byref(ctx), 0) == msc.MSC_ENOMEM
    assert not ctx.value
    assert msc._lib.msc_create(ctypes.byref(ctx), 0) == msc.MSC_OK
    try:
        # The first call of a fresh context allocates its records and its
        # workspace: each failing allocation fails the call cleanly.
        for after in (0, 1, 2):
            msc.debug_inject(msc.INJECT_ENOMEM, after)
            rc, _ = _segment_raw(msc, ctx, t)
            msc.debug_inject(msc.INJECT_ENOMEM, -1)
            assert rc in (msc.MSC_OK, msc.MSC_ENOMEM), rc
        rc, outs = _segment_raw(msc, ctx, t)
        assert rc == msc.MSC_OK
        torch.cuda.synchronize()
        for name, g, w in zip(("asc", "desc", "ms"), outs, O.segment(f)):
            np.testing.assert_array_equal(g.cpu().numpy(), w, err_msg=name)
    finally:
        msc._lib.msc_destroy(ctx)
    # Queue creation.
    msc.debug_inject(msc.INJECT_ENOMEM, 0)
    with pytest.raises(msc.MscError) as e:
        msc.Server(hbm_budget=64 << 20, max_batch=4)
    assert e.value.code == msc.MSC_ENOMEM
    msc.debug_inject(msc.INJECT_ENOMEM, -1)


def test_runtime_failure_in_a_plain_call(msc):
    f = synth.gaussian_field((50, 41, 33), 8, 82)
    t = torch.from_numpy(f).cuda()
    msc.debug_inject(msc.INJECT_EHIP, 0)
    with pytest.raises(msc.MscError) as e:
        msc.segment(t)
    assert e.value.code == msc.MSC_EHIP
    msc.debug_inject(msc.INJECT_EHIP, -1)
    got = msc.segment(t)
    torch.cuda.synchronize()
    for name, g, w in zip(("asc", "desc", "ms"), got, O.segment(f)):
        np.testing.assert_array_equal(g.cpu().numpy(), w, err_msg=name)


@pytest.mark.parametrize("after", [1, 3, 9, 20])
def test_runtime_failure_in_the_queue(msc, after):
    """A runtime failure somewhere in the queue's threads (a copy, a launch)
    fails the requests it touched with MSC_EHIP; every other request is
    exact, and the queue serves new requests afterwards."""
    fields = [synth.gaussian_field((30 + i, 26, 21), 5, 90 + i)
              for i in range(8)]
    reqs = [(1, f) if i % 3 else (2, synth.threshold_mask(f, 0.6))
            for i, f in enumerate(fields)]
    with msc.Server(hbm_budget=256 << 20, max_batch=4) as srv:
        msc.debug_inject(msc.INJECT_EHIP, after)
        tickets = [srv.submit(k, a) for k, a in reqs]
        codes = [srv.wait(t) for t in tickets]
        # Disarmed before any result is copied back (the copy is a checked
        # call of this thread).
        msc.debug_inject(msc.INJECT_EHIP, -1)
        for t, (k, a), rc in zip(tickets, reqs, codes):
            assert rc in (msc.MSC_OK, msc.MSC_EHIP), rc
            if rc == msc.MSC_OK:
                got = srv.fetch(t)
                if k == 1:
                    for g, w in zip(got, O.segment(a)):
                        np.testing.assert_array_equal(g, w)
                else:
                    np.testing.assert_array_equal(got, O.cc_grid(a)[0])
            srv.release(t)
        assert msc.MSC_EHIP in codes
        for k, a in reqs[:3]:
            t = srv.submit(k, a)
            assert srv.wait(t) == msc.MSC_OK
            got = srv.fetch(t)
            if k == 1:
                for g, w in zip(got, O.segment(a)):
                    np.testing.assert_array_equal(g, w)
            else:
                np.testing.assert_array_equal(got, O.cc_grid(a)[0])
            srv.release(t)
        assert srv.info()["arena_used"] == 0
