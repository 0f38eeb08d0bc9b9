"""FP64 MTTKRP (FP64 values, factors and accumulation: the paper's precision,
Section IV-A) against the FP64-valued oracle, at a stated FP64 tolerance:
max row error <= 1e-12 of the row's |X|,|C| scale (both sides sum in FP64,
in different orders)."""
import numpy as np
import pytest

import oracle
from paper_2509_00280_amd import synth
from _gpu_helpers import to_dev

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_00280_amd import spt as _spt
    _spt.lib()
    return _spt


def _f64_case(t, seed, rank):
    rng = np.random.default_rng(seed)
    vals64 = rng.random(t.nnz) / 3.0 + 1e-3  # not representable in FP32
    F = [rng.standard_normal((d, rank)) for d in t.dims]
    return vals64, F


def _check(spt, h, t, vals64, F):
    import torch
    Fd = [torch.from_numpy(f).cuda() for f in F]
    for n in range(t.nmodes):
        out = spt.mttkrp_f64(h, Fd, n).cpu().numpy()
        ref = oracle.mttkrp_f64vals(t.coords, vals64, t.dims, F, n)
        sc = oracle.mttkrp_f64vals(t.coords, np.abs(vals64), t.dims, [np.abs(f) for f in F], n)
        err, bad = oracle.row_error(out, ref, sc)
        print(f"f64 dims {t.dims} mode {n}: err {err:.2e}", flush=True)
        assert bad == 0 and err <= TOL64


@pytest.mark.parametrize("tile", [4096, 2048, 1024])
def test_f64_mttkrp_skewed(spt, tile):
    import torch
    t, _, _, _ = synth.config("skewed4d", nnz=300_001)
    vals64, F = _f64_case(t, 1, 16)
    h = spt.encode(t.dims, *to_dev(t))
    h.set_plan(tile=tile)
    spt.attach_f64(h, torch.from_numpy(vals64).cuda())
    _check(spt, h, t, vals64, F)


@pytest.mark.parametrize("rank", [5, 16, 64, 130])
def test_f64_mttkrp_small_ranks(spt, rank):
    import torch
    t, _, _, _ = synth.config("small")
    vals64, F = _f64_case(t, rank, rank)
    h = spt.encode(t.dims, *to_dev(t))
    spt.attach_f64(h, torch.from_numpy(vals64).cuda())
    _check(spt, h, t, vals64, F)


def test_f64_wide_keys_and_after_autotune(spt):
    import torch
    dims = (300_000, 200_000, 100_000, 5_000)  # 67-bit keys
    t = synth.distinct_coo(31, dims, 100_000, [("zipf", 1.2)] * 3 + ["uniform"], "u01")
    vals64, F = _f64_case(t, 2, 16)
    h = spt.encode(t.dims, *to_dev(t))
    spt.attach_f64(h, torch.from_numpy(vals64).cuda())
    _check(spt, h, t, vals64, F)
    F32 = [torch.from_numpy(f.astype(np.float32)).cuda() for f in F]
    spt.autotune(h, F32, budget_ms=1500.0, random_samples=2, seed=3)   # re-encodes: FP64 values follow
    _check(spt, h, t, vals64, F)


def test_f64_requires_values_and_segment(spt):
    import torch
    t, _, _, _ = synth.config("small")
    _, F = _f64_case(t, 3, 8)
    h = spt.encode(t.dims, *to_dev(t))
    Fd = [torch.from_numpy(f).cuda() for f in F]
    with pytest.raises(spt.SptError):
        spt.mttkrp_f64(h, Fd, 0)  # no FP64 values attached
    spt.attach_f64(h, torch.ones(t.nnz, dtype=torch.float64, device="cuda"))
    h.set_plan(strategy=1)
    with pytest.raises(spt.SptError):
        spt.mttkrp_f64(h, Fd, 0)  # REGROUP plan
