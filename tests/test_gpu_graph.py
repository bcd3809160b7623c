"""Graph-captured batched segmentation (msc_graph_*): the captured call is
replayed several times with the program's own eager work between replays
(new field contents written into the same buffers, outputs cleared,
synchronisations), and every replay equals the oracle on the contents it
read; a NaN written into one field between replays fails that field alone.
"""
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


SHAPES = [(70, 45, 38), (33, 17, 90), (64, 64, 1), (5, 3, 2)]


def _fields(seed):
    return [synth.gaussian_field(d, 8, seed + i) if i % 2 == 0
            else synth.random_field(d, seed + i, levels=5)
            for i, d in enumerate(SHAPES)]


def _check(outs, host, tag):
    for i, (o, f) in enumerate(zip(outs, host)):
        want = O.segment(f)
        for name, g, w in zip(("asc", "desc", "ms"), o, want):
            np.testing.assert_array_equal(g.cpu().numpy(), w,
                                          err_msg=f"{tag} field {i} {name}")


def test_replays_follow_new_contents(msc):
    host = _fields(500)
    dev = [torch.from_numpy(f).cuda() for f in host]
    outs = [tuple(torch.empty(f.size, dtype=torch.int32, device="cuda")
                  for _ in range(3)) for f in host]
    g = msc.Graph(dev, outs)
    try:
        _check(outs, host, "first call")
        s = torch.cuda.Stream()
        for r, seed in enumerate((600, 700, 800)):
            new = _fields(seed)
            for t, f in zip(dev, new):
                t.copy_(torch.from_numpy(f))  # eager work between replays
            for o in outs:
                for x in o:
                    x.fill_(-7)
            torch.cuda.synchronize()
            g.launch(stream=s if r % 2 else None)
            torch.cuda.synchronize()
            _check(outs, new, f"replay {r}")
            for i, f in enumerate(new):
                st = g.field_stats(i)
                assert st["status"] == msc.MSC_OK
                assert st["n_vertices"] == f.size
                assert st["n_maxima"] == np.unique(O.segment(f)[0]).size
    finally:
        g.close()


def test_nan_in_one_field_between_replays(msc):
    host = _fields(900)
    dev = [torch.from_numpy(f).cuda() for f in host]
    outs = [tuple(torch.empty(f.size, dtype=torch.int32, device="cuda")
                  for _ in range(3)) for f in host]
    g = msc.Graph(dev, outs)
    try:
        bad = host[1].copy()
        bad.reshape(-1)[11] = np.nan
        dev[1].copy_(torch.from_numpy(bad))
        torch.cuda.synchronize()
        g.launch()
        assert g.field_stats(1)["status"] == msc.MSC_ENAN
        for i in (0, 2, 3):
            assert g.field_stats(i)["status"] == msc.MSC_OK
        torch.cuda.synchronize()
        _check([outs[i] for i in (0, 2, 3)], [host[i] for i in (0, 2, 3)],
               "beside a NaN field")
        dev[1].copy_(torch.from_numpy(host[1]))
        torch.cuda.synchronize()
        g.launch()
        assert g.field_stats(1)["status"] == msc.MSC_OK
        torch.cuda.synchronize()
        _check(outs, host, "after the NaN")
    finally:
        g.close()


def test_graph_arguments(msc):
    with pytest.raises(ValueError):
        msc.Graph([], [])
    t = torch.zeros(10, dtype=torch.float32, device="cuda")
    g = msc.Graph([t], [(None, None, torch.empty(10, dtype=torch.int32,
                                                  device="cuda"))])
    try:
        with pytest.raises(msc.MscError):
            g.field_stats(5)   # no such field
    finally:
        g.close()
