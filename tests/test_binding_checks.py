"""The binding rejects malformed arguments before any library call (CPU only:
CPU tensors stand in for device tensors; the device check comes last)."""
import numpy as np
import pytest
import torch

from paper_2509_00280_amd import spt

DIMS = (6, 5, 4)


def _factors(R=3, dtype=torch.float32):
    return [torch.zeros((d, R), dtype=dtype) for d in DIMS]


def test_factor_dtype_shape_rank_contiguity_device():
    with pytest.raises(ValueError, match="float32"):
        spt.check_factors(_factors(dtype=torch.float64), DIMS)
    bad = _factors()
    bad[1] = torch.zeros((4, 3))
    with pytest.raises(ValueError, match="shape"):
        spt.check_factors(bad, DIMS)
    bad = _factors()
    bad[2] = torch.zeros((4, 5))           # a different rank
    with pytest.raises(ValueError, match="shape"):
        spt.check_factors(bad, DIMS)
    bad = _factors()
    bad[0] = torch.zeros((3, 6)).t()       # transposed view: right shape, not row-major
    with pytest.raises(ValueError, match="contiguous"):
        spt.check_factors(bad, DIMS)
    with pytest.raises(ValueError, match="expected 3"):
        spt.check_factors(_factors()[:2], DIMS)
    with pytest.raises(ValueError, match="None"):
        spt.check_factors([None] + _factors()[1:], DIMS)
    # the output mode's factor may be absent
    assert spt.check_factors([None] + _factors()[1:], DIMS, skip_mode=0, device="cpu") == 3
    assert spt.check_factors(_factors(R=7), DIMS, device="cpu") == 7
    with pytest.raises(ValueError, match="CUDA"):
        spt.check_factors(_factors(), DIMS)


def test_out_and_lambda_checks():
    with pytest.raises(ValueError, match="shape"):
        spt.check_matrix("out", torch.zeros((5, 3)), 6, 3)
    with pytest.raises(ValueError, match="float32"):
        spt.check_matrix("out", torch.zeros((6, 3), dtype=torch.float16), 6, 3)
    with pytest.raises(ValueError, match="CUDA"):
        spt.check_matrix("out", torch.zeros((6, 3)), 6, 3)
    with pytest.raises(ValueError, match="float64"):
        spt.check_vector("lambda", torch.zeros(3), 3, "float64")
    with pytest.raises(ValueError, match="shape"):
        spt.check_vector("lambda", torch.zeros(4, dtype=torch.float64), 3, "float64")
    with pytest.raises(ValueError, match="torch tensor"):
        spt.check_matrix("out", np.zeros((6, 3), np.float32), 6, 3)


def test_coo_checks():
    c = torch.zeros((3, 10), dtype=torch.int32)
    v = torch.zeros(10)
    assert spt.check_coo(c, v, 3, device="cpu") == 10
    with pytest.raises(ValueError, match="int32"):
        spt.check_coo(c.to(torch.int64), v, 3)
    with pytest.raises(ValueError, match="shape"):
        spt.check_coo(c, v, 4)
    with pytest.raises(ValueError, match="shape"):
        spt.check_coo(c, torch.zeros(9), 3)
    with pytest.raises(ValueError, match="float32"):
        spt.check_coo(c, torch.zeros(10, dtype=torch.float64), 3)
    with pytest.raises(ValueError, match="contiguous"):
        spt.check_coo(torch.zeros((10, 3), dtype=torch.int32).t(), v, 3, device="cpu")
    with pytest.raises(ValueError, match="CUDA"):
        spt.check_coo(c, v, 3)


def test_server_request_checks():
    coords = np.zeros((3, 10), np.uint32)
    vals = np.zeros(10, np.float32)
    init = [np.zeros((d, 4), np.float32) for d in DIMS]
    c, v, i, rank = spt.check_request(DIMS, coords, vals, init)
    assert rank == 4 and c.dtype == np.uint32
    with pytest.raises(ValueError, match="coords"):
        spt.check_request(DIMS, np.zeros((2, 10), np.uint32), vals, init)
    with pytest.raises(ValueError, match="coords"):
        spt.check_request(DIMS, coords.astype(np.int64), vals, init)
    with pytest.raises(ValueError, match="vals"):
        spt.check_request(DIMS, coords, np.zeros(11, np.float32), init)
    with pytest.raises(ValueError, match="vals"):
        spt.check_request(DIMS, coords, np.zeros(10, np.float64), init)
    bad = list(init)
    bad[2] = np.zeros((3, 4), np.float32)   # too few rows: the server would read past it
    with pytest.raises(ValueError, match="init 2"):
        spt.check_request(DIMS, coords, vals, bad)
    bad = list(init)
    bad[1] = np.zeros((5, 5), np.float32)   # another rank
    with pytest.raises(ValueError, match="init 1"):
        spt.check_request(DIMS, coords, vals, bad)
    with pytest.raises(ValueError, match="init"):
        spt.check_request(DIMS, coords, vals, init[:2])
