"""Parity of the HIP segmentation (through the C-ABI) with the CPU oracle,
bit-exact, on seeded inputs; degenerate grids, ties and error paths."""
import itertools
import json
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2409_03771_amd import synth

pytestmark = pytest.mark.gpu


def load_golden(name):
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def msc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_03771_amd import msc as m
    return m


def gpu_segment(msc, f_np, **kw):
    t = torch.from_numpy(np.ascontiguousarray(f_np)).cuda()
    a, d, m = msc.segment(t, **kw)
    torch.cuda.synchronize()
    cpu = lambda x: None if x is None else x.cpu().numpy()
    return cpu(a), cpu(d), cpu(m)


def assert_parity(msc, f_np, tag=""):
    want = O.segment(f_np)
    got = gpu_segment(msc, f_np)
    for name, g, w in zip(("asc", "desc", "ms"), got, want):
        np.testing.assert_array_equal(g, w, err_msg=f"{tag} {name}")


def test_gauss64_parity(msc):
    f = synth.config_field("gauss64")
    assert_parity(msc, f, "gauss64")
    st = msc.last_stats()
    # counts the oracle wrote (tests/golden/make_gauss64_counts.py)
    want = load_golden("gauss64_counts.json")
    assert st["n_maxima"] == want["n_maxima"]
    assert st["n_minima"] == want["n_minima"]
    assert st["n_cells"] == want["n_cells"]


@pytest.mark.parametrize("dims", [
    (37, 29, 23), (128, 64, 17), (300, 7, 5), (1, 1, 1), (100, 1, 1),
    (1, 100, 1), (1, 1, 100), (40, 30, 1), (1, 30, 40), (33, 1, 31),
    (2, 2, 2), (257, 3, 2), (65, 65, 65)])
@pytest.mark.parametrize("levels", [None, 3])
def test_random_grids_parity(msc, dims, levels):
    f = synth.random_field(dims, seed=sum(dims) + (levels or 0), levels=levels)
    assert_parity(msc, f, f"{dims} levels={levels}")


def test_gaussian_ragged_parity(msc):
    f = synth.gaussian_field((203, 151, 77), 40, seed=11)
    assert_parity(msc, f, "gauss ragged")


def test_exhaustive_ties_2x2x2(msc):
    """Every field over {0,1,2} on 2x2x2 (3^8) and a seeded sample of the
    8! orderings of distinct values."""
    F = list(itertools.product((0, 1, 2), repeat=8))
    perms = list(itertools.permutations(range(8)))
    rng = np.random.default_rng(0)
    F += [perms[i] for i in rng.choice(len(perms), 3000, replace=False)]
    for vals in F:
        f = np.array(vals, np.float32).reshape(2, 2, 2)
        want = O.segment(f)
        got = gpu_segment(msc, f)
        for g, w in zip(got, want):
            assert np.array_equal(g, w), vals


@pytest.mark.parametrize("dims", [(50, 40, 30), (16, 1, 1), (9, 7, 1)])
def test_closed_forms(msc, dims):
    X, Y, Z = dims
    n = X * Y * Z
    a, d, m = gpu_segment(msc, np.zeros((Z, Y, X), np.float32))
    assert (a == n - 1).all() and (d == 0).all() and (m == 0).all()
    ids = np.arange(n, dtype=np.float32).reshape(Z, Y, X)
    a, d, m = gpu_segment(msc, ids)
    assert (a == n - 1).all() and (d == 0).all() and (m == 0).all()
    a, d, m = gpu_segment(msc, -ids)
    assert (a == 0).all() and (d == n - 1).all() and (m == 0).all()


def test_single_bump_one_ascending_manifold(msc):
    n, c = 48, (30, 7, 19)
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                             indexing="ij")
    r2 = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2
    f = np.exp(-r2 / (2 * (n / 3) ** 2)).astype(np.float32)
    a, _, _ = gpu_segment(msc, f)
    assert (a == c[0] + n * c[1] + n * n * c[2]).all()
    assert msc.last_stats()["n_maxima"] == 1


def test_signed_zero_tie(msc):
    f = np.array([[[0.0, -0.0, 0.0, -0.0]]], np.float32)
    a, d, _ = gpu_segment(msc, f)
    assert list(a) == [3] * 4 and list(d) == [0] * 4


def test_partial_outputs_agree(msc):
    f = synth.random_field((31, 17, 9), seed=5)
    full = gpu_segment(msc, f)
    for want in (("asc",), ("desc",), ("ms",), ("asc", "ms"), ("desc", "ms")):
        got = gpu_segment(msc, f, want=want)
        for k, g, w in zip(("asc", "desc", "ms"), got, full):
            if k in want:
                np.testing.assert_array_equal(g, w)
            else:
                assert g is None


def test_nan_is_rejected(msc):
    f = synth.random_field((20, 20, 20), seed=1)
    f[3, 4, 5] = np.nan
    with pytest.raises(msc.MscError) as e:
        gpu_segment(msc, f)
    assert e.value.code == msc.MSC_ENAN
    # the context stays usable
    assert_parity(msc, synth.random_field((20, 20, 20), seed=2))


def test_bad_dims_rejected(msc):
    t = torch.zeros(8, device="cuda")
    out = torch.empty(8, dtype=torch.int32, device="cuda")
    for dims in ((0, 1, 1), (2, -1, 4)):
        with pytest.raises(msc.MscError) as e:
            msc.segment_into(t, out, None, None, dims=dims)
        assert e.value.code == msc.MSC_EINVAL
    with pytest.raises(msc.MscError) as e:
        msc.segment_into(t, out, None, None, dims=(1 << 16, 1 << 16, 1))
    assert e.value.code == msc.MSC_ERANGE


def test_every_tile_shape_parity(msc):
    """Results do not depend on the tile shape of the fused pass."""
    cases = [synth.gaussian_field((131, 77, 45), 30, seed=3),
             synth.random_field((70, 33, 37), seed=4, levels=3),
             synth.random_field((200, 1, 1), seed=5),
             synth.random_field((1, 45, 70), seed=6),
             synth.random_field((65, 17, 1), seed=7, levels=2),
             # noise-dominated: thousands of cells per tile, more than the
             # per-tile pair table takes, so most vertices take the
             # per-vertex path of the pair and write passes
             synth.random_field((96, 80, 40), seed=8),
             synth.gaussian_field((150, 90, 50), 4, seed=9)]
    want = [O.segment(f) for f in cases]
    try:
        for shape in msc.tile_shapes():
            msc.set_tile(*shape)
            for f, w in zip(cases, want):
                got = gpu_segment(msc, f)
                for name, g, ww in zip(("asc", "desc", "ms"), got, w):
                    np.testing.assert_array_equal(
                        g, ww, err_msg=f"tile {shape} dims {f.shape} {name}")
                assert msc.last_stats()["n_cells"] == len(np.unique(w[2]))
            assert tuple(msc.last_stats()[k] for k in
                         ("tile_x", "tile_y", "tile_z")) == shape
    finally:
        msc.set_tile(*msc.tile_shapes()[0])


def test_side_stream_and_determinism(msc):
    f = torch.from_numpy(synth.gaussian_field((96, 80, 64), 20, 7)).cuda()
    a0, d0, m0 = msc.segment(f)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a1, d1, m1 = msc.segment(f, stream=s)
    s.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(a0, a1) and torch.equal(d0, d1) and torch.equal(m0, m1)


def test_calls_queue_without_host_sync(msc):
    """msc_segment returns with its work only enqueued: calls queued back to
    back on one stream, with no host synchronisation between them (and the
    stream still busy when the last one returns), reuse the context's
    workspace in stream order and each equal the oracle."""
    small = [synth.gaussian_field(d, 12, sd) for d, sd in
             (((96, 80, 64), 1), ((64, 70, 50), 2), ((33, 17, 90), 3))]
    big = synth.gaussian_field((512, 512, 256), 64, 4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dev = [torch.from_numpy(f).cuda() for f in small + [big] + small]
        outs = [tuple(torch.empty(t.numel(), dtype=torch.int32, device="cuda")
                      for _ in range(3)) for t in dev]
    s.synchronize()
    for t, (a, d, m) in zip(dev, outs):
        msc.segment_into(t, a, d, m, stream=s, check=False)
    busy = not s.query()
    s.synchronize()
    assert busy, "the calls waited for the device"
    assert msc.last_status() == msc.MSC_OK
    wants = {}
    for i, f in enumerate(small + [big] + small):
        key = id(f)
        if key not in wants:
            wants[key] = O.segment(f)
        for name, g, w in zip(("asc", "desc", "ms"), outs[i], wants[key]):
            np.testing.assert_array_equal(g.cpu().numpy(), w,
                                          err_msg=f"call {i} {name}")


def test_calls_on_two_streams_are_ordered(msc):
    """Consecutive calls on one context from two streams: the second waits
    for the first's work on the device (shared workspace)."""
    f1 = synth.gaussian_field((200, 150, 120), 30, 11)
    f2 = synth.gaussian_field((120, 200, 150), 30, 12)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    t1, t2 = torch.from_numpy(f1).cuda(), torch.from_numpy(f2).cuda()
    o1 = tuple(torch.empty(t1.numel(), dtype=torch.int32, device="cuda")
               for _ in range(3))
    o2 = tuple(torch.empty(t2.numel(), dtype=torch.int32, device="cuda")
               for _ in range(3))
    torch.cuda.synchronize()
    msc.segment_into(t1, *o1, stream=s1, check=False)
    msc.segment_into(t2, *o2, stream=s2, check=False)
    s2.synchronize()
    s1.synchronize()
    for f, o in ((f1, o1), (f2, o2)):
        for name, g, w in zip(("asc", "desc", "ms"), o, O.segment(f)):
            np.testing.assert_array_equal(g.cpu().numpy(), w, err_msg=name)


def _mixed_pair_field():
    """96 x 48 x 48 (3 x 3 x 3 tiles of 32 x 16 x 16): one smooth bump, with
    U[-0.05, 0.05] noise added in the far corner tile.  Its tiles hold one
    (asc, desc) pair, a few, and hundreds to thousands, so the output pass
    takes all three of its paths in one call (no bytes for a one-pair tile,
    the byte per vertex for up to 255 pairs, the per-vertex path beyond)."""
    X, Y, Z = 96, 48, 48
    z, y, x = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X),
                          indexing="ij")
    f = np.exp(-(((x - 40.5) / 25.0) ** 2 + ((y - 20.5) / 12.0) ** 2 +
                 ((z - 20.5) / 12.0) ** 2)).astype(np.float32)
    rng = np.random.default_rng(7)
    f[32:48, 32:48, 64:96] += rng.uniform(-0.05, 0.05,
                                          size=(16, 16, 32)).astype(np.float32)
    return f


def _pairs_per_tile(a, d, shape, tile=(16, 16, 32)):
    a = a.reshape(shape)
    d = d.reshape(shape)
    out = []
    for z0 in range(0, shape[0], tile[0]):
        for y0 in range(0, shape[1], tile[1]):
            for x0 in range(0, shape[2], tile[2]):
                sl = (slice(z0, z0 + tile[0]), slice(y0, y0 + tile[1]),
                      slice(x0, x0 + tile[2]))
                out.append(len(set(zip(a[sl].ravel().tolist(),
                                       d[sl].ravel().tolist()))))
    return out


def test_output_pass_paths_in_one_call(msc):
    f = _mixed_pair_field()
    want = O.segment(f)
    # The input covers every path: decided on the oracle's labels alone.
    counts = _pairs_per_tile(want[0], want[1], f.shape)
    assert min(counts) == 1 and max(counts) > 255
    assert any(1 < c <= 255 for c in counts)
    msc.set_tile(32, 16, 16)
    got = gpu_segment(msc, f)
    for name, g, w in zip(("asc", "desc", "ms"), got, want):
        np.testing.assert_array_equal(g, w, err_msg=name)
    # The same field inside a batch, beside a pure-noise field whose every
    # tile takes the per-vertex path.
    noise = np.random.default_rng(8).random((20, 40, 70)).astype(np.float32)
    dev = [torch.from_numpy(f).cuda(), torch.from_numpy(noise).cuda()]
    outs = msc.segment_batched(dev)
    torch.cuda.synchronize()
    for fld, out in zip((f, noise), outs):
        ref = O.segment(fld)
        for name, g, w in zip(("asc", "desc", "ms"), out, ref):
            np.testing.assert_array_equal(g.cpu().numpy(), w, err_msg=name)
