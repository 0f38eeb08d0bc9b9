"""The library's default device memory source, the block cache: a repeated
CP-ALS step takes every buffer from idle blocks (no hipMalloc), a block
released on one stream serves another stream once that work is done, and
emptying the cache leaves every call working."""
import numpy as np
import pytest

import oracle
from paper_2509_00280_amd import synth
from _gpu_helpers import factors_dev, mttkrp_error, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_00280_amd import spt as _spt
    _spt.lib()
    _spt.use_torch_allocator(False)
    return _spt


def _tensor(seed=91, dims=(900, 700, 300, 12), nnz=120_000):
    t = synth.distinct_coo(seed, dims, nnz, [("zipf", 1.2)] * 3 + ["uniform"], "lognormal")
    F = synth.normal_factors(seed + 1, dims, 16)
    return t, F


def test_repeated_steps_allocate_nothing(spt):
    import torch
    t, F = _tensor()
    coords, vals = to_dev(t)
    iters = 4

    def step():
        Fw = factors_dev(F)
        h = spt.encode(t.dims, coords, vals)
        lam, fit, its = spt.cp_als(h, Fw, iters)
        h.free()
        torch.cuda.synchronize()
        return fit, Fw, lam

    fits = [step()[0]]
    before = spt.memory_stats()
    for _ in range(3):
        fit, Fw, lam = step()
        fits.append(fit)
    after = spt.memory_stats()
    print(f"cache before {before} after {after}", flush=True)
    assert after["device_allocs"] == before["device_allocs"]  # every buffer came from an idle block
    assert after["reuses"] > before["reuses"]
    assert after["bytes_live"] == before["bytes_live"]  # everything taken was given back
    ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
    for f in fits:
        assert abs(f - ref["fit"]) <= 1e-4 and abs(f - fits[0]) <= 1e-6


def test_block_released_on_one_stream_serves_another(spt):
    import torch
    t, F = _tensor(seed=93)
    coords, vals = to_dev(t)
    Fd = factors_dev(F)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for s in (sa, sb, sa):
        h = spt.encode(t.dims, coords, vals, stream=s)
        h.prepare(16, stream=s)
        o = torch.empty((t.dims[0], 16), device="cuda")
        with torch.cuda.stream(s):
            o.zero_()
        spt.mttkrp(h, Fd, 0, out=o, stream=s)
        h.free(stream=s)
        s.synchronize()
        outs.append(o)
        if len(outs) == 1:
            first = spt.memory_stats()
    last = spt.memory_stats()
    print(f"after the first stream {first}, after both {last}", flush=True)
    # the first stream's work had completed: its blocks served the second stream and back
    assert last["device_allocs"] == first["device_allocs"] and last["reuses"] > first["reuses"]
    for o in outs:
        err, bad = mttkrp_error(t, F, 0, o.cpu().numpy())
        assert bad == 0 and err <= 1e-4


def test_streams_in_flight_together(spt):
    """Two streams encode, plan and run MTTKRP at once, each releasing and
    re-taking blocks while the other's work may still be pending."""
    import torch
    ts = [_tensor(seed=95 + 2 * k, nnz=60_000 + 30_000 * k) for k in range(2)]
    dev = [(to_dev(t), factors_dev(F)) for t, F in ts]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    results = [[], []]
    for rep in range(3):
        for k, ((t, F), ((coords, vals), Fd), s) in enumerate(zip(ts, dev, streams)):
            h = spt.encode(t.dims, coords, vals, stream=s)
            h.prepare(16, stream=s)
            o = torch.empty((t.dims[1], 16), device="cuda")
            spt.mttkrp(h, Fd, 1, out=o, stream=s)
            h.free(stream=s)
            results[k].append(o)
    torch.cuda.synchronize()
    for k, (t, F) in enumerate(ts):
        for o in results[k]:
            err, bad = mttkrp_error(t, F, 1, o.cpu().numpy())
            assert bad == 0 and err <= 1e-4


def test_empty_cache_then_calls_work(spt):
    import torch
    t, F = _tensor(seed=99, nnz=50_000)
    coords, vals = to_dev(t)
    h = spt.encode(t.dims, coords, vals)
    h.free()
    torch.cuda.synchronize()
    spt.empty_cache()
    st = spt.memory_stats()
    assert st["bytes_idle"] == 0
    Fd = factors_dev(F)
    h = spt.encode(t.dims, coords, vals)
    o = spt.mttkrp(h, Fd, 2)
    torch.cuda.synchronize()
    assert spt.memory_stats()["device_allocs"] > st["device_allocs"]
    err, bad = mttkrp_error(t, F, 2, o.cpu().numpy())
    assert bad == 0 and err <= 1e-4
    h.free()
    torch.cuda.synchronize()
    assert spt.memory_stats()["bytes_live"] == st["bytes_live"]
