"""Parity of the virtual-rank path at full size, in the configuration
`bench.py --ranks R` times: the paper's distributed scheme (Alg. 1 with its
ghost rule, the exchange and relabelling of Alg. 2, Alg. 3's shared
communication phase for components) on R z-slabs of the 1024^3 headline
field must give the single-domain labels on every vertex.  The single-domain
outputs themselves are pinned to the oracle at this size by
test_gpu_fullsize.py; here the two device results are compared on the
device, label for label.
"""
import pytest
import torch

from paper_2409_03771_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def field():
    assert torch.cuda.is_available()
    print("[fullsize ranks] generating gauss1024 on the device", flush=True)
    f = synth.config_field("gauss1024", device="cuda")
    yield f
    del f
    torch.cuda.empty_cache()


@pytest.mark.parametrize("ranks", [8, 32])
def test_segment_ranks_equal_single_domain(field, ranks):
    from paper_2409_03771_amd import msc
    print(f"[fullsize ranks] segment R={ranks}", flush=True)
    want = msc.segment(field)
    st = msc.last_stats()
    got = msc.segment_ranks(field, ranks)
    sr = msc.last_stats()
    torch.cuda.synchronize()
    for name, a, b in zip(("asc", "desc", "ms"), got, want):
        diff = int((a != b).sum())
        assert diff == 0, f"R={ranks} {name}: {diff} vertices differ"
    for key in ("n_maxima", "n_minima", "n_cells"):
        assert sr[key] == st[key], key
    del want, got
    torch.cuda.empty_cache()


@pytest.mark.parametrize("ranks", [8, 32])
def test_cc_ranks_equal_single_domain(field, ranks):
    from paper_2409_03771_amd import msc
    print(f"[fullsize ranks] cc R={ranks}", flush=True)
    # The threshold study's middle mask: one large component and many small.
    mask = synth.normalized_mask(field, 0.5)
    want = msc.cc_label_grid(mask)
    got = msc.cc_label_grid_ranks(mask, ranks)
    torch.cuda.synchronize()
    diff = int((got != want).sum())
    assert diff == 0, f"R={ranks}: {diff} labels differ"
    del mask, want, got
    torch.cuda.empty_cache()
