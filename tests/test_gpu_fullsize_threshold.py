"""The threshold study at full size, in the configuration the benchmark times
(ccperlin_t90 / t50 / t10): the perlin1024 field normalised by its minimum
and maximum, masked above 0.9, 0.5 and 0.1, labelled on the device and
compared label by label with the oracle's union-find on the same masks.
The scaling study's masks (ccperlin512_top10 / ccperlin1024_top10): the
top 10 % of the vertices of perlin512 and perlin1024, the same way.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2409_03771_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def perlin():
    assert torch.cuda.is_available()
    print("[threshold] generating perlin1024 on the device", flush=True)
    f = synth.config_field("perlin1024", device="cuda")
    yield f
    del f
    torch.cuda.empty_cache()


@pytest.mark.parametrize("level", [0.9, 0.5, 0.1])
def test_threshold_mask_cc_full(perlin, level):
    from paper_2409_03771_amd import msc
    print(f"[threshold] level {level} on the device", flush=True)
    mask = synth.normalized_mask(perlin, level)
    lab = msc.cc_label_grid(mask)
    torch.cuda.synchronize()
    got = lab.cpu().numpy()
    mask_h = mask.cpu().numpy()
    del lab, mask
    torch.cuda.empty_cache()
    print(f"[threshold] level {level} oracle", flush=True)
    want, ncomp = O.cc_grid(mask_h)
    print(f"[threshold] level {level}: {int(mask_h.sum())} foreground, "
          f"{ncomp} components", flush=True)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("name", ["perlin512", "perlin1024"])
def test_top10_mask_cc_full(name):
    from paper_2409_03771_amd import msc
    print(f"[top10] {name} on the device", flush=True)
    f = synth.config_field(name, device="cuda")
    mask = synth.threshold_mask(f, 0.9)
    del f
    torch.cuda.empty_cache()
    lab = msc.cc_label_grid(mask)
    torch.cuda.synchronize()
    got = lab.cpu().numpy()
    mask_h = mask.cpu().numpy()
    del lab, mask
    torch.cuda.empty_cache()
    frac = mask_h.mean()
    assert 0.099 < frac < 0.101, frac
    print(f"[top10] {name} oracle", flush=True)
    want, ncomp = O.cc_grid(mask_h)
    print(f"[top10] {name}: {int(mask_h.sum())} foreground, {ncomp} "
          "components", flush=True)
    np.testing.assert_array_equal(got, want)
