"""Request queue with continuous batching: every result is bit-identical to
the CPU oracle and to the plain call, alone and in a mix of kinds and sizes;
admission respects the HBM budget; cancellation, errors and NaN requests
stay local to their request."""
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


def _requests(count, seed, lo=8, hi=64):
    """Mixed trace: 70 % segmentation (some tie-heavy), 30 % mask CC."""
    rng = np.random.default_rng(seed)
    specs = synth.batch_specs(count, seed=seed, lo=lo, hi=hi)
    out = []
    for k, (dims, nb, fseed) in enumerate(specs):
        if rng.random() < 0.7:
            f = (synth.random_field(dims, seed=fseed, levels=4) if k % 4 == 1
                 else synth.gaussian_field(dims, nb, fseed))
            out.append((1, f))
        else:
            f = synth.gaussian_field(dims, nb, fseed)
            out.append((2, synth.threshold_mask(f, 0.7)))
    return out


def _check(kind, arr, got, tag):
    if kind == 1:
        want = O.segment(arr)
        for name, g, w in zip(("asc", "desc", "ms"), got, want):
            np.testing.assert_array_equal(g, w, err_msg=f"{tag} {name}")
    else:
        np.testing.assert_array_equal(got, O.cc_grid(arr)[0], err_msg=tag)


def test_mix_matches_oracle_alone_and_plain(msc):
    reqs = _requests(40, seed=11)
    with msc.Server(hbm_budget=1 << 30, max_batch=16) as srv:
        tickets = [srv.submit(k, a) for k, a in reqs]
        batches = []
        for t, (k, a) in zip(tickets, reqs):
            assert srv.wait(t) == msc.MSC_OK
            r = srv.result(t)
            assert r["t_submit_ns"] <= r["t_start_ns"] <= r["t_done_ns"]
            batches.append(r["batch_size"])
            _check(k, a, srv.fetch(t), f"ticket {t} {a.shape}")
            srv.release(t)
        info = srv.info()
        assert info["arena_used"] == 0
        assert info["pending"] == info["running"] == info["finished"] == 0
        # The workspaces were fixed at creation and never reallocated.
        assert info["workspace_grows"] == 0
        assert info["arena_size"] + info["workspace_reserved"] == 1 << 30
        assert 1 <= info["launches"] < len(reqs)
    # Requests submitted together were packed into shared launches.
    assert max(batches) > 1
    # The same requests alone, each in a fresh queue, and as plain calls.
    with msc.Server(hbm_budget=1 << 30, max_batch=16) as srv:
        for k, a in reqs[:6]:
            t = srv.submit(k, a)
            assert srv.wait(t) == msc.MSC_OK
            assert srv.result(t)["batch_size"] == 1
            got = srv.fetch(t)
            if k == 1:
                plain = msc.segment(torch.from_numpy(a).cuda())
                torch.cuda.synchronize()
                for g, p in zip(got, plain):
                    np.testing.assert_array_equal(g, p.cpu().numpy())
            else:
                lab = msc.cc_label_grid(torch.from_numpy(a).cuda())
                torch.cuda.synchronize()
                np.testing.assert_array_equal(got, lab.cpu().numpy())
            srv.release(t)


def _resident(kind, n):
    """Arena bytes a request holds: input, outputs, alignment."""
    b = (4 * n if kind == 1 else n) + (12 * n if kind == 1 else 8 * n) + 256
    return (b + 255) // 256 * 256


def test_budget_backpressure(msc):
    """A budget whose arena holds a handful of requests: later ones wait for
    releases, arrival order is kept and every result is still exact."""
    dims = (40, 36, 32)
    n = dims[0] * dims[1] * dims[2]
    # The segmentation workspace (a quarter of the budget) holds one launch
    # of one request; the arena then holds about seven results.
    budget = 4 * msc.workspace_size(msc.REQ_SEGMENT, [dims]) + (64 << 10)
    fields = [synth.gaussian_field(dims, 6, 100 + i) for i in range(20)]
    with msc.Server(hbm_budget=budget, max_batch=8) as srv:
        arena = srv.info()["arena_size"]
        assert 3 * _resident(1, n) < arena < len(fields) * _resident(1, n)
        tickets = [srv.submit(1, f) for f in fields]
        starts = []
        for t, f in zip(tickets, fields):
            assert srv.info()["arena_used"] <= arena
            assert srv.wait(t) == msc.MSC_OK
            starts.append(srv.result(t)["t_start_ns"])
            _check(1, f, srv.fetch(t), f"ticket {t}")
            srv.release(t)
        assert starts == sorted(starts)
        info = srv.info()
        assert info["arena_used"] == 0 and info["workspace_grows"] == 0


def test_rejects_and_cancel(msc):
    fa = synth.gaussian_field((60, 50, 40), 6, 5)       # 120000 vertices
    fb = synth.gaussian_field((50, 40, 30), 4, 6)       # 60000 vertices
    budget = 8 * msc.workspace_size(msc.REQ_SEGMENT, [(60, 50, 40)])
    with msc.Server(hbm_budget=budget, max_batch=4) as srv:
        arena = srv.info()["arena_size"]
        big = np.zeros(arena // 16 + 1, np.float32)
        with pytest.raises(msc.MscError) as e:
            srv.submit(1, big)                      # alone exceeds the arena
        assert e.value.code == msc.MSC_EBUDGET
        with pytest.raises(TypeError):
            srv.submit(1, fa.astype(np.float64))
        with pytest.raises(msc.MscError):
            srv.poll(987654)                        # unknown ticket
        ta = srv.submit(1, fa)
        assert srv.wait(ta) == msc.MSC_OK
        # Fill the arena with held results until fb no longer fits.
        held = []
        while arena - srv.info()["arena_used"] >= _resident(1, fb.size):
            held.append(srv.submit(1, fb))
            assert srv.wait(held[-1]) == msc.MSC_OK
        tb = srv.submit(1, fb)                      # waits for a release
        assert srv.poll(tb) == msc.MSC_EBUSY
        assert srv.info()["pending"] == 1
        srv.cancel(tb)
        assert srv.poll(tb) == msc.MSC_ECANCELED
        assert srv.wait(tb) == msc.MSC_ECANCELED
        with pytest.raises(msc.MscError):
            srv.fetch(tb)
        srv.release(tb)
        with pytest.raises(msc.MscError):           # labels of a segmentation
            srv.copy_output(ta, 3)
        tc = srv.submit(1, fb)
        assert srv.poll(tc) == msc.MSC_EBUSY
        _check(1, fa, srv.fetch(ta), "held")
        srv.release(ta)                             # lets fb in
        assert srv.wait(tc) == msc.MSC_OK
        _check(1, fb, srv.fetch(tc), "after release")
        with pytest.raises(msc.MscError):
            srv.cancel(tc)                          # already finished
        srv.release(tc)
        _check(1, fb, srv.fetch(held[0]), "held filler")
        for t in held:
            srv.release(t)
        t = srv.submit(2, synth.threshold_mask(fb, 0.5))
        assert srv.wait(t) == msc.MSC_OK
        with pytest.raises(msc.MscError):           # outputs of a CC
            srv.copy_output(t, 0)
        srv.release(t)
        assert srv.info()["arena_used"] == 0


def test_nan_request_fails_alone(msc):
    reqs = [(1, synth.gaussian_field((30, 22, 18), 5, 200 + i)) for i in range(8)]
    bad = reqs[3][1].copy()
    bad.reshape(-1)[17] = np.nan
    reqs[3] = (1, bad)
    reqs.insert(5, (2, synth.threshold_mask(reqs[0][1], 0.6)))
    with msc.Server(hbm_budget=256 << 20, max_batch=16) as srv:
        tickets = [srv.submit(k, a) for k, a in reqs]
        for i, (t, (k, a)) in enumerate(zip(tickets, reqs)):
            rc = srv.wait(t)
            if i == 3:
                assert rc == msc.MSC_ENAN
                with pytest.raises(msc.MscError):
                    srv.fetch(t)
            else:
                assert rc == msc.MSC_OK
                _check(k, a, srv.fetch(t), f"request {i}")
            srv.release(t)


def test_device_inputs_match_host_inputs(msc):
    """Inputs already in device memory are copied within the device and give
    the same results as host inputs."""
    reqs = _requests(12, seed=21)
    with msc.Server(hbm_budget=512 << 20, max_batch=8) as srv:
        host = [srv.submit(k, a) for k, a in reqs]
        dev = [srv.submit(k, torch.from_numpy(a).cuda()) for k, a in reqs]
        for th, td, (k, a) in zip(host, dev, reqs):
            assert srv.wait(th) == msc.MSC_OK and srv.wait(td) == msc.MSC_OK
            gh, gd = srv.fetch(th), srv.fetch(td)
            if k == 1:
                for x, y in zip(gh, gd):
                    np.testing.assert_array_equal(x, y)
            else:
                np.testing.assert_array_equal(gh, gd)
            _check(k, a, gd, f"device input {a.shape}")
            srv.release(th)
            srv.release(td)
