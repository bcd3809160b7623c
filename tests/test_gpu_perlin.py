"""The paper's synthetic workload, one layer of Perlin noise (frequency 0.1,
amplitude 1), through the HIP path: MS segmentation and the normalised
threshold masks of the threshold study, bit-exact against the CPU oracle;
and the pair table's regrowth when its first capacity is far too small."""
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


def segment(msc, f):
    a, d, m = msc.segment(torch.from_numpy(np.ascontiguousarray(f)).cuda())
    torch.cuda.synchronize()
    return a.cpu().numpy(), d.cpu().numpy(), m.cpu().numpy()


def check_segment(msc, f, tag):
    want = O.segment(f)
    got = segment(msc, f)
    for name, g, w in zip(("asc", "desc", "ms"), got, want):
        np.testing.assert_array_equal(g, w, err_msg=f"{tag} {name}")
    return msc.last_stats()


@pytest.mark.parametrize("dims", [(64, 64, 64), (97, 75, 66)])
def test_perlin_segment_parity(msc, dims):
    print(f"[perlin segment] dims={dims}", flush=True)
    f = synth.perlin_field(dims, seed=5)
    st = check_segment(msc, f, f"perlin {dims}")
    assert st["n_cells"] > st["n_maxima"]


@pytest.mark.parametrize("level", [0.9, 0.5, 0.1])
def test_perlin_threshold_cc_parity(msc, level):
    print(f"[perlin cc] level={level}", flush=True)
    f = synth.perlin_field((80, 72, 64), seed=6)
    mask = synth.normalized_mask(f, level)
    lab = msc.cc_label_grid(torch.from_numpy(mask).cuda())
    torch.cuda.synchronize()
    want, ncomp = O.cc_grid(mask)
    np.testing.assert_array_equal(lab.cpu().numpy(), want)
    assert ncomp >= 1


def test_perlin_gpu_generator_matches_cpu(msc):
    """The device evaluation of the noise equals the host one to float32
    rounding of the same float64 expression (the benchmark generates its
    1024^3 fields on the device)."""
    dims = (70, 50, 40)
    a = synth.perlin_field(dims, seed=5)
    b = synth.perlin_field(dims, seed=5, device="cuda").cpu().numpy()
    assert np.abs(a.astype(np.float64) - b).max() <= 1e-7


@pytest.mark.parametrize("case", ["noise", "perlin"])
def test_pair_table_regrows(msc, case):
    """A first table capacity far below the cell count overflows the pair
    pass, which runs again on larger tables until the cells fit: results
    equal the oracle's and the next call, back on automatic sizing, too."""
    print(f"[table regrow] {case}", flush=True)
    if case == "noise":
        f = synth.random_field((60, 50, 40), seed=3)
    else:
        f = synth.perlin_field((96, 96, 96), seed=7, frequency=0.3)
    try:
        msc.set_table_capacity(1024)
        st = check_segment(msc, f, f"{case} small table")
        assert st["n_cells"] > 4 * 1024
    finally:
        msc.set_table_capacity(0)
    check_segment(msc, f, f"{case} automatic table")
    with pytest.raises(Exception):
        msc.set_table_capacity(1 << 33)
