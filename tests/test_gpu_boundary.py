"""The C-ABI's memory and synchronisation contract, on the GPU.

* spt_set_allocator: every library-owned buffer comes from the hook and goes
  back to it (PyTorch's caching allocator behind counting hooks).
* spt_mttkrp and spt_mttkrp_batched on prepared tensors, spt_tensor_set_plan
  and spt_tensor_free never synchronise: a spin kernel queued first on the
  stream is still running when each call returns.
* spt_mttkrp on an unprepared tensor is rejected (it never plans itself).
* spt_cp_als / spt_cp_als_batched leave the caller's factors and lambda
  untouched when they fail (a NaN initial factor makes the normal equations
  fail every ridge retry).
"""
import ctypes

import numpy as np
import pytest

from paper_2509_00280_amd import synth
from _gpu_helpers import factors_dev, mttkrp_error, to_dev

pytestmark = pytest.mark.gpu
E_INVALID, E_NOT_SPD = -1, -6


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_00280_amd import spt as _spt
    _spt.lib()
    return _spt


@pytest.fixture(scope="module")
def cycles_per_ms():
    import torch
    torch.cuda._sleep(1000)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    torch.cuda._sleep(20_000_000)
    b.record()
    b.synchronize()
    return 20_000_000 / max(a.elapsed_time(b), 1e-3)


def _spin(cycles_per_ms, ms=300.0):
    """Queue a spin kernel of about `ms` on the current stream."""
    import torch
    torch.cuda._sleep(int(cycles_per_ms * ms))
    return torch.cuda.current_stream()


def test_mttkrp_and_batched_do_not_synchronise(spt, cycles_per_ms):
    import torch
    t, F, R, _ = synth.config("ratings", nnz=300_000)
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    h.prepare(R)
    h.prepare(R, batched=True)
    Fd = factors_dev(F)
    out = torch.empty((t.dims[1], R), device="cuda")
    torch.cuda.synchronize()
    s = _spin(cycles_per_ms)
    spt.mttkrp(h, Fd, 1, out=out)
    assert not s.query(), "spt_mttkrp waited for the stream"
    outs = [torch.empty((t.dims[2], R), device="cuda")]
    spt.mttkrp_batched([h], [Fd], 2, outs)
    assert not s.query(), "spt_mttkrp_batched waited for the stream"
    torch.cuda.synchronize()
    err, bad = mttkrp_error(t, F, 1, out.cpu().numpy())
    assert bad == 0 and err <= 1e-4
    err, bad = mttkrp_error(t, F, 2, outs[0].cpu().numpy())
    assert bad == 0 and err <= 1e-4


def test_set_plan_and_free_do_not_synchronise(spt, cycles_per_ms):
    import torch
    t, F, R, _ = synth.config("small")
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    Fd = factors_dev(F)
    out = spt.mttkrp(h, Fd, 0)
    torch.cuda.synchronize()
    s = _spin(cycles_per_ms)
    spt.mttkrp(h, Fd, 0, out=out)      # queued behind the spin, reads the old plan
    h.set_plan(tile=2048)               # releases the old plan in stream order
    assert not s.query(), "spt_tensor_set_plan waited for the stream"
    h.free()
    assert not s.query(), "spt_tensor_free waited for the stream"
    torch.cuda.synchronize()
    err, bad = mttkrp_error(t, F, 0, out.cpu().numpy())
    assert bad == 0 and err <= 1e-4


def test_unprepared_mttkrp_is_rejected(spt):
    t, F, R, _ = synth.config("small")
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    Fd = factors_dev(F)
    import torch
    out = torch.empty((t.dims[0], R), device="cuda")
    st = spt.lib().spt_mttkrp(h.handle, spt._ptr_array(Fd), R, 0, spt._ptr(out), spt._stream(None))
    assert st == E_INVALID and b"prepare" in spt.lib().spt_last_error()
    h.prepare(R)
    st = spt.lib().spt_mttkrp(h.handle, spt._ptr_array(Fd), R, 0, spt._ptr(out), spt._stream(None))
    assert st == 0


def test_allocator_hook_supplies_and_receives_every_buffer(spt):
    import torch
    counts = {"alloc": 0, "release": 0, "live": set()}

    def _alloc(nbytes, stream, ctx):
        p = torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0))
        counts["alloc"] += 1
        counts["live"].add(p)
        return p

    def _release(ptr, stream, ctx):
        counts["release"] += 1
        counts["live"].discard(int(ptr))
        torch.cuda.caching_allocator_delete(int(ptr))

    hooks = (spt.ALLOC_FN(_alloc), spt.RELEASE_FN(_release))
    assert spt.lib().spt_set_allocator(hooks[0], hooks[1], None) == 0
    try:
        t, F, R, iters = synth.config("small")
        c, v = to_dev(t)
        Fd = factors_dev(F)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        h = spt.encode(t.dims, c, v)
        h.prepare(R)
        held = torch.cuda.memory_allocated() - before
        assert held >= h.info()["encoded_bytes"]      # the encoding lives in torch's pool
        assert counts["alloc"] > 0 and counts["live"]
        lam = torch.empty(R, dtype=torch.float64, device="cuda")
        fit, its = spt.cp_als(h, Fd, 3, lam=lam)[1:]
        assert its == 3 and np.isfinite(fit)
        del lam  # the test's own tensor: only library buffers are counted below
        h.free()
        torch.cuda.synchronize()
        assert not counts["live"], f"{len(counts['live'])} buffers never released"
        assert counts["alloc"] == counts["release"]
        assert torch.cuda.memory_allocated() == before
        # exactly one hook NULL is rejected
        assert spt.lib().spt_set_allocator(hooks[0], spt.RELEASE_FN(), None) == E_INVALID
    finally:
        spt.use_torch_allocator(False)


def test_cp_als_failure_leaves_outputs_untouched(spt):
    import torch
    t, F, R, _ = synth.config("small")
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    bad = [f.copy() for f in F]
    bad[1][3, 2] = np.nan
    Fd = factors_dev(bad)
    before = [f.clone() for f in Fd]
    lam = torch.full((R,), 5.0, dtype=torch.float64, device="cuda")
    with pytest.raises(spt.SptError) as e:
        spt.cp_als(h, Fd, 3, lam=lam)
    assert e.value.status == E_NOT_SPD
    for a, b in zip(Fd, before):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))  # bit for bit, NaN included
    assert (lam == 5.0).all()
    # batched: one failing member leaves every member's factors untouched
    t2, F2, R2, _ = synth.config("small")
    h2 = spt.encode(t2.dims, *to_dev(t2))
    F2d = factors_dev(F2)
    keep = [f.clone() for f in F2d]
    with pytest.raises(spt.SptError) as e:
        spt.cp_als_batched([h2, h], [F2d, Fd], 3)
    assert e.value.status == E_NOT_SPD
    for a, b in zip(F2d, keep):
        assert torch.equal(a, b)
