"""Seeded fuzz over tiny tensors against the oracle: 2 to 5 modes, mode
lengths 1..9 (modes of length 1 included, so outputs of one row and modes
with no key bits), 0..64 nonzeros with duplicate coordinates, ranks 1..20,
every strategy.  Encoding bit-exact, MTTKRP within 1e-4 of the row scale."""
import numpy as np
import pytest

import oracle
from paper_2509_00280_amd import synth
from _gpu_helpers import check_encoding, factors_dev, mttkrp_error, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_00280_amd import spt as _spt
    _spt.lib()
    return _spt


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    nm = int(rng.integers(2, 6))
    dims = tuple(int(x) for x in rng.integers(1, 10, size=nm))
    if seed % 5 == 0:
        dims = (1,) + dims[1:]       # an output mode of one row
    nnz = int(rng.integers(0, 65))
    coords = np.stack([rng.integers(0, d, size=nnz) for d in dims]).astype(np.uint32) if nnz else \
        np.zeros((nm, 0), np.uint32)
    if nnz > 4:
        k = nnz // 4
        coords[:, nnz - k:] = coords[:, :k]  # duplicates
    vals = rng.standard_normal(nnz).astype(np.float32)
    rank = int(rng.integers(1, 21))
    return synth.SparseCOO(dims, coords, vals), rank, rng


@pytest.mark.parametrize("strategy", [0, 1, 2, 3, 5])
def test_fuzz_tiny_tensors(spt, strategy):
    import torch
    for seed in range(40):
        t, rank, rng = _case(seed)
        print(f"seed {seed} dims {t.dims} nnz {t.nnz} rank {rank} strategy {strategy}", flush=True)
        c, v = to_dev(t)
        h = spt.encode(t.dims, c, v)
        check_encoding(h, t)
        h.set_plan(strategy=strategy)
        F = [rng.standard_normal((d, rank)).astype(np.float32) for d in t.dims]
        Fd = factors_dev(F)
        for n in range(t.nmodes):
            out = torch.full((t.dims[n], rank), float("nan"), device="cuda")
            spt.mttkrp(h, Fd, n, out=out)
            got = out.cpu().numpy()
            if t.nnz == 0:
                assert (got == 0).all()
                continue
            err, bad = mttkrp_error(t, F, n, got)
            assert bad == 0 and err <= 1e-4, (seed, n, err)
        h.free()
