"""Parity at the full batched and served workloads, in the configurations
the benchmark times; every result is compared with the CPU oracle.

batch256: the 256 uneven fields segmented in one batched call with the
autotuned tile; every field's asc, desc and ms equal the oracle's label by
label (the oracle runs on a thread pool: its C calls release the GIL), and
the per-field counters equal the oracle's extremum and cell counts.

Served: requests drawn from the served size distribution (each axis
64..512) go through the queue all at once, first from device memory (the
inputs are staged far ahead of the worker, so requests queue up and get
batched) and then from page-locked host memory (the copies cross the host
link while earlier launches run); every result equals the oracle's for that
request's input.
"""
from concurrent.futures import ThreadPoolExecutor

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


def test_batch256_full(msc):
    specs = synth.batch_specs(256, seed=3)
    print("[batch256] generating", flush=True)
    fields = [synth.gaussian_field(d, nb, sd, device="cuda")
              for d, nb, sd in specs]
    outs = [tuple(torch.empty(f.numel(), dtype=torch.int32, device="cuda")
                  for _ in range(3)) for f in fields]
    try:
        tune = msc.autotune(fields, outs)
        print(f"[batch256] tile {tune['tile']}", flush=True)
        for o in outs:
            for x in o:
                x.fill_(-7)
        msc.segment_batched_into(fields, outs)
        torch.cuda.synchronize()
        stats = [msc.last_field_stats(i) for i in range(len(fields))]
        host = [f.cpu().numpy() for f in fields]
        print(f"[batch256] oracle on all {len(host)} fields", flush=True)
        with ThreadPoolExecutor(16) as pool:
            wants = list(pool.map(O.segment, host))
        for i, want in enumerate(wants):
            for name, g, w in zip(("asc", "desc", "ms"), outs[i], want):
                np.testing.assert_array_equal(
                    g.cpu().numpy(), w, err_msg=f"field {i} {specs[i][0]} {name}")
            assert stats[i]["n_maxima"] == np.unique(want[0]).size, i
            assert stats[i]["n_minima"] == np.unique(want[1]).size, i
            assert stats[i]["n_cells"] == np.unique(want[2]).size, i
    finally:
        msc.set_tile(*msc.tile_shapes()[0])


@pytest.fixture(scope="module")
def served_inputs():
    """48 requests over a pool of 16 fields of the served size mix, and the
    oracle's result for every pool entry (segmentation of its field, CC of
    its 70th-percentile mask)."""
    trace = synth.poisson_trace(1.0, 48, seed=4)
    pool_specs = synth.poisson_trace(1.0, 16, seed=4)
    pool = []
    for sp in pool_specs:
        f = synth.gaussian_field(sp["dims"], sp["nbumps"], sp["seed"])
        pool.append((f, synth.threshold_mask(f, 0.7)))
    print(f"[served] oracle on {len(pool)} fields and masks", flush=True)
    with ThreadPoolExecutor(16) as ex:
        segs = list(ex.map(O.segment, [f for f, _ in pool]))
        ccs = list(ex.map(lambda m: O.cc_grid(m)[0], [m for _, m in pool]))
    reqs = []
    for i, r in enumerate(trace):
        j = i % len(pool)
        if r["kind"] == "ms":
            reqs.append((1, pool[j][0], segs[j]))
        else:
            reqs.append((2, pool[j][1], ccs[j]))
    print(f"[served] {len(reqs)} requests, "
          f"{sum(a.size for _, a, _ in reqs) / 1e6:.0f}M vertices", flush=True)
    return reqs


def _serve_and_check(msc, reqs, inputs, tag):
    with msc.Server(hbm_budget=64 << 30, max_batch=64) as srv:
        tickets = [srv.submit(k, x) for (k, _, _), x in zip(reqs, inputs)]
        batches = []
        for i, (t, (k, _, want)) in enumerate(zip(tickets, reqs)):
            assert srv.wait(t) == msc.MSC_OK, (tag, i)
            batches.append(srv.result(t)["batch_size"])
            got = srv.fetch(t)
            if k == 1:
                for name, g, w in zip(("asc", "desc", "ms"), got, want):
                    np.testing.assert_array_equal(
                        g, w, err_msg=f"{tag} request {i} {name}")
            else:
                np.testing.assert_array_equal(
                    got, want, err_msg=f"{tag} request {i} cc")
            srv.release(t)
        info = srv.info()
    assert info["arena_used"] == 0 and info["workspace_grows"] == 0
    return batches


def test_served_full_sizes_device_inputs(msc, served_inputs):
    reqs = served_inputs
    dev_in = [torch.from_numpy(a).cuda() for _, a, _ in reqs]
    torch.cuda.synchronize()
    batches = _serve_and_check(msc, reqs, dev_in, "device")
    assert max(batches) > 1


def test_served_full_sizes_pinned_host_inputs(msc, served_inputs):
    reqs = served_inputs
    host_in = [torch.from_numpy(a).pin_memory() for _, a, _ in reqs]
    _serve_and_check(msc, reqs, host_in, "pinned host")


def test_plain_calls_full_sizes(msc, served_inputs):
    """The same requests as plain calls on one stream, queued back to back
    with no host synchronisation between them, equal the oracle."""
    reqs = served_inputs
    outs = []
    for k, a, _ in reqs:
        t = torch.from_numpy(a).cuda()
        outs.append(msc.segment(t) if k == 1 else msc.cc_label_grid(t))
    torch.cuda.synchronize()
    for i, ((k, _, want), got) in enumerate(zip(reqs, outs)):
        if k == 1:
            for name, g, w in zip(("asc", "desc", "ms"), got, want):
                np.testing.assert_array_equal(
                    g.cpu().numpy(), w, err_msg=f"plain request {i} {name}")
        else:
            np.testing.assert_array_equal(got.cpu().numpy(), want,
                                          err_msg=f"plain request {i} cc")
