"""GPU parity of the row-cached SEGMENT kernel (tile dictionaries, 4096-nonzero tiles).

A nonzero reads its factor rows from the LDS cache or from memory; the
products and the order of the per-piece sums are the same either way, and
only the record reduction's atomic merges of rows that straddle reduction
chunks vary from run to run.  Both kernels must match the FP64 oracle within
1e-4 in every mode.
"""
import numpy as np
import pytest

from paper_2509_00280_amd import synth
from _gpu_helpers import factors_dev, mttkrp_error, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_00280_amd import spt as _spt
    return _spt


def _check(t, F, outs, label):
    for n in range(t.nmodes):
        for rc in (1, 0, 3, 2):
            err, bad = mttkrp_error(t, F, n, outs[rc][n])
            print(f"{label} mode {n} row_cache {rc}: err {err:.3e}", flush=True)
            assert bad == 0 and err <= TOL


def _both(spt, t, F, modes=None):
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    Fd = factors_dev(F)
    outs = {}
    for rc in (1, 0):
        h.set_plan(tile=4096, strategy=5, row_cache=rc)
        assert h.get_plan()["row_cache"] == rc
        # a mode's dictionary comes with its plan: after one sweep every mode has one
        first = [spt.mttkrp(h, Fd, n).cpu().numpy() for n in (modes or range(t.nmodes))]
        outs[rc] = [spt.mttkrp(h, Fd, n).cpu().numpy() for n in (modes or range(t.nmodes))]
        outs[2 + rc] = first
    return h, outs


def _uniform(seed, dims, n, rank):
    rng = np.random.default_rng(seed)
    coords = np.stack([rng.integers(0, d, size=n) for d in dims]).astype(np.uint32)
    t = synth.SparseCOO(dims, coords, rng.standard_normal(n).astype(np.float32))
    return t, synth.normal_factors(seed + 7, dims, rank)


@pytest.mark.parametrize("rank", [32, 5, 16, 64, 100])
def test_row_cache_ratings(spt, rank):
    # skewed 3-mode tensor: a few hundred distinct rows per tile, most cached
    t, _, _, _ = synth.config("ratings", nnz=1_000_003)
    F = synth.normal_factors(40 + rank, t.dims, rank)
    _, outs = _both(spt, t, F)
    _check(t, F, outs, f"ratings rank {rank}")


def test_row_cache_skewed4d_rank64(spt):
    # 4 modes at rank 64: the cache holds only a few rows per mode, most reads miss
    t, F, rank, _ = synth.config("skewed4d", nnz=300_001)
    _, outs = _both(spt, t, F)
    _check(t, F, outs, "skewed4d")


@pytest.mark.parametrize("dims,n", [((200_000, 150_000, 90_000), 500_000),   # nearly every row distinct
                                    ((64, 48, 40), 300_000),                  # every tile covers all rows
                                    ((5000, 3000), 200_000)])                 # a matrix
def test_row_cache_extremes(spt, dims, n):
    t, F = _uniform(len(dims) * 11 + n % 7, dims, n, 32)
    _, outs = _both(spt, t, F)
    _check(t, F, outs, f"dims {dims}")


@pytest.mark.parametrize("rank", [130, 256])
def test_row_cache_wide_ranks(spt, rank):
    # wide rows: a small cache (16 rows per mode at rank 256), several column blocks per lane
    t, F = _uniform(rank, (3000, 2000, 500), 150_000, rank)
    _, outs = _both(spt, t, F)
    _check(t, F, outs, f"rank {rank}")


def test_row_cache_five_modes_falls_back(spt):
    # more than 4 modes: no dictionaries, the uncached kernel runs under either setting
    t, F = _uniform(5, (40, 30, 20, 10, 8), 100_000, 16)
    _, outs = _both(spt, t, F)
    _check(t, F, outs, "five modes")


def test_row_cache_rebuilt_after_replan_and_single_tile(spt):
    # dictionaries are dropped with the plans and rebuilt; a tensor smaller than one tile
    t, F = _uniform(3, (300, 200, 100), 3000, 32)
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    Fd = factors_dev(F)
    for _ in range(2):
        h.set_plan(tile=4096, strategy=5, row_cache=1)
        for m in (0, 0, 1, 2, 1, 0):  # mode 0's second call builds the missing dictionaries itself
            out = spt.mttkrp(h, Fd, m).cpu().numpy()
            err, bad = mttkrp_error(t, F, m, out)
            assert bad == 0 and err <= TOL
