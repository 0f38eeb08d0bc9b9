"""spt_mttkrp_noalloc (the entry point that allocates nothing) against
spt_mttkrp and the oracle: two calls in a row, the second on a smaller
tensor, every mode; a workspace above the fixed maximum is rejected."""
import numpy as np
import pytest

from paper_2509_00280_amd import synth
from _gpu_helpers import factors_dev, mttkrp_error, to_dev

pytestmark = pytest.mark.gpu
E_INVALID = -1


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_00280_amd import spt as _spt
    _spt.lib()
    return _spt


def _check_same(spt, h, t, F, R):
    import torch
    Fd = factors_dev(F)
    h.prepare(R)
    for n in range(t.nmodes):
        ref = spt.mttkrp(h, Fd, n)
        got = torch.full_like(ref, float("nan"))
        spt.mttkrp_noalloc(h, Fd, n, got)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        err, bad = mttkrp_error(t, F, n, g)
        print(f"dims {t.dims} nnz {t.nnz} R {R} mode {n}: noalloc err {err:.2e}", flush=True)
        assert bad == 0 and err <= 1e-4
        scale = np.abs(r).max(axis=1, keepdims=True) + 1e-30
        assert (np.abs(g - r) / scale).max() <= 1e-5


def test_noalloc_matches_mttkrp_twice_then_smaller(spt):
    big, Fb, Rb, _ = synth.config("skewed4d", nnz=600_000)
    hb = spt.encode(big.dims, *to_dev(big))
    _check_same(spt, hb, big, Fb, Rb)
    small, Fs, Rs, _ = synth.config("small")
    hs = spt.encode(small.dims, *to_dev(small))
    _check_same(spt, hs, small, Fs, Rs)


def test_noalloc_other_strategies_and_limits(spt):
    import torch
    t, F, R, _ = synth.config("small")
    h = spt.encode(t.dims, *to_dev(t))
    h.set_plan(strategy=1)  # REGROUP: no workspace
    _check_same(spt, h, t, F, R)
    h.set_plan(strategy=3)  # PRIV keeps partials: not served without allocation
    h.prepare(R)
    out = torch.empty((t.dims[0], R), device="cuda")
    with pytest.raises(spt.SptError) as e:
        spt.mttkrp_noalloc(h, factors_dev(F), 0, out)
    assert e.value.status == E_INVALID
    # a workspace above the maximum: 2M ratings nonzeros at rank 256
    t2, _, _, _ = synth.config("ratings", nnz=2_000_000)
    F2 = synth.normal_factors(3, t2.dims, 256)
    h2 = spt.encode(t2.dims, *to_dev(t2))
    h2.prepare(256)
    out2 = torch.empty((t2.dims[0], 256), device="cuda")
    with pytest.raises(spt.SptError) as e:
        spt.mttkrp_noalloc(h2, factors_dev(F2), 0, out2)
    assert e.value.status == E_INVALID and "maximum" in e.value.message
    # unprepared tensors are rejected, as by spt_mttkrp
    h3 = spt.encode(t.dims, *to_dev(t))
    with pytest.raises(spt.SptError):
        spt.mttkrp_noalloc(h3, factors_dev(F), 0, out)
