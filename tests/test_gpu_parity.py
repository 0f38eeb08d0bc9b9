"""GPU parity: encoding bit-exact, MTTKRP within 1e-4 (row abs-sum scale), CP-ALS fit within 1e-4.

Every call goes through the C-ABI library; the oracle is the FP64 CPU reference.
"""
import numpy as np
import pytest

import oracle
from paper_2509_00280_amd import synth
from _gpu_helpers import check_encoding, cpd_error, factors_dev, mttkrp_error, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_00280_amd import spt as _spt
    print("library", _spt.version(), flush=True)
    return _spt


@pytest.fixture(scope="module")
def small():
    return synth.config("small")


def test_encode_small_bit_exact(spt, small):
    t, _, _, _ = small
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    info = h.info()
    assert info["lp"] == 23 and info["key_words"] == 1
    assert abs(info["norm_x2"] - float((t.vals.astype(np.float64) ** 2).sum())) < 1e-9 * info["norm_x2"]
    check_encoding(h, t)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_encode_random_layouts_and_duplicates(spt, seed):
    rng = np.random.default_rng(seed)
    dims = (37, 1, 300, 9)
    n = 5000
    coords = np.stack([rng.integers(0, d, size=n) for d in dims]).astype(np.uint32)
    coords[:, 4000:4500] = coords[:, 0:500]  # duplicate coordinates keep input order
    vals = rng.standard_normal(n).astype(np.float32)
    t = synth.SparseCOO(dims, coords, vals)
    lb = oracle.bit_lengths(dims)
    multiset = [m for m in range(4) for _ in range(lb[m])]
    layout = [int(x) for x in rng.permutation(multiset)]
    c, v = to_dev(t)
    check_encoding(spt.encode(dims, c, v, layout=layout), t, layout)
    check_encoding(spt.encode(dims, c, v), t)


def test_encode_wide_keys(spt):
    rng = np.random.default_rng(3)
    dims = (3_000_000, 2_500_000, 1_000_000, 700)  # l(p) = 22 + 22 + 20 + 10 = 74 bits
    n = 20_000
    coords = np.stack([rng.integers(0, d, size=n) for d in dims]).astype(np.uint32)
    t = synth.SparseCOO(dims, coords, rng.random(n, dtype=np.float32))
    c, v = to_dev(t)
    h = spt.encode(dims, c, v)
    assert h.info()["key_words"] == 2
    check_encoding(h, t)


def test_encode_rejects_out_of_range(spt):
    import torch
    dims = (4, 5)
    coords = torch.tensor([[0, 1, 4], [0, 2, 3]], dtype=torch.int32, device="cuda")
    vals = torch.ones(3, device="cuda")
    with pytest.raises(spt.SptError) as e:
        spt.encode(dims, coords, vals)
    assert e.value.status == -2 and "nonzero 2" in e.value.message


def test_encode_bad_layout(spt):
    import torch
    coords = torch.zeros((2, 3), dtype=torch.int32, device="cuda")
    vals = torch.ones(3, device="cuda")
    with pytest.raises(spt.SptError) as e:
        spt.encode((4, 4), coords, vals, layout=[0, 0, 0, 1])
    assert e.value.status == -4


@pytest.mark.parametrize("rank", [16, 5, 32, 64])
@pytest.mark.parametrize("strategy", [0, 1, 2, 3, 4, 5])
def test_mttkrp_small_all_modes(spt, small, rank, strategy):
    t, _, _, _ = small
    F = synth.normal_factors(100 + rank, t.dims, rank)
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    h.set_plan(strategy=strategy)
    Fd = factors_dev(F)
    for n in range(3):
        out = spt.mttkrp(h, Fd, n).cpu().numpy()
        err, bad = mttkrp_error(t, F, n, out)
        print(f"rank {rank} strategy {strategy} mode {n}: err {err:.3e}", flush=True)
        assert bad == 0 and err <= TOL


@pytest.mark.parametrize("tile,strategy", [(256, 1), (512, 1), (1024, 1), (1024, 2), (4096, 4), (2048, 5), (4096, 5),
                                           (1024, 5)])
def test_mttkrp_skewed_tiles_ragged(spt, tile, strategy):
    # 4-mode power-law tensor with a ragged last tile, rank 64
    t, F, rank, _ = synth.config("skewed4d", nnz=300_001)
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    h.set_plan(tile=tile, strategy=strategy)
    Fd = factors_dev(F)
    for n in range(4):
        out = spt.mttkrp(h, Fd, n).cpu().numpy()
        err, bad = mttkrp_error(t, F, n, out)
        print(f"tile {tile} mode {n}: err {err:.3e}", flush=True)
        assert bad == 0 and err <= TOL


@pytest.mark.parametrize("strategy", [2, 3, 5])
def test_mttkrp_priv_column_passes_and_table_flushes(spt, strategy):
    # mode 0 (1000 rows x rank 64) needs two LDS column passes under PRIV;
    # under TABLE every mode flushes its accumulator many times
    rng = np.random.default_rng(8)
    dims = (1000, 300, 50)
    n = 400_000
    coords = np.stack([rng.integers(0, d, size=n) for d in dims]).astype(np.uint32)
    t = synth.SparseCOO(dims, coords, rng.standard_normal(n).astype(np.float32))
    F = synth.normal_factors(9, dims, 64)
    c, v = to_dev(t)
    h = spt.encode(dims, c, v)
    h.set_plan(strategy=strategy)
    Fd = factors_dev(F)
    for mode in range(3):
        out = spt.mttkrp(h, Fd, mode).cpu().numpy()
        err, bad = mttkrp_error(t, F, mode, out)
        print(f"strategy {strategy} mode {mode}: err {err:.3e}", flush=True)
        assert bad == 0 and err <= TOL


@pytest.mark.parametrize("strategy", [2, 4, 5])
def test_mttkrp_ratings_table_parity(spt, strategy):
    t, F, rank, _ = synth.config("ratings", nnz=2_000_000)
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    h.set_plan(strategy=strategy)
    Fd = factors_dev(F)
    for mode in range(3):
        out = spt.mttkrp(h, Fd, mode).cpu().numpy()
        err, bad = mttkrp_error(t, F, mode, out)
        print(f"ratings strategy {strategy} mode {mode}: err {err:.3e}", flush=True)
        assert bad == 0 and err <= TOL


def test_mttkrp_ratings_all_ones_gives_slice_sums(spt):
    t, _, _, _ = synth.config("ratings", nnz=1_000_000)
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    ones = [np.ones((d, 32), np.float32) for d in t.dims]
    Fd = factors_dev(ones)
    for n in range(3):
        out = spt.mttkrp(h, Fd, n).cpu().numpy()
        ref = np.bincount(t.coords[n], weights=t.vals.astype(np.float64), minlength=t.dims[n])
        # integer-valued sums below 2^24 are exact in FP32 whatever the order
        exact = ref < 2 ** 24
        np.testing.assert_array_equal(out[exact, 0], ref[exact])
        assert (out == out[:, :1]).all()


def test_mttkrp_empty_tensor(spt):
    import torch
    coords = torch.zeros((3, 0), dtype=torch.int32, device="cuda")
    vals = torch.zeros(0, device="cuda")
    h = spt.encode((5, 6, 7), coords, vals)
    F = factors_dev([np.ones((d, 8), np.float32) for d in (5, 6, 7)])
    out = torch.full((6, 8), 7.0, device="cuda")
    spt.mttkrp(h, F, 1, out=out)
    assert (out == 0).all()


def test_mttkrp_invalid_args(spt, small):
    import torch
    t, F, rank, _ = small
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    Fd = factors_dev(F)
    with pytest.raises(spt.SptError):
        spt.mttkrp(h, Fd, 3)
    bad = torch.empty(200 * 16 + 1, device="cuda")[1:].view(200, 16)  # misaligned output
    with pytest.raises(spt.SptError):
        spt.mttkrp(h, Fd, 0, out=bad)


def test_cp_als_small_matches_oracle(spt, small):
    t, F, rank, iters = small
    ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    Fd = factors_dev(F)
    lam, fit, its = spt.cp_als(h, Fd, iters)
    e, el = cpd_error(to_host(Fd), lam.cpu().numpy(), ref["factors"], ref["lam"])
    print(f"fit gpu {fit:.8f} oracle {ref['fit']:.8f} factor err {e:.2e} lambda err {el:.2e}", flush=True)
    assert its == iters
    assert abs(fit - ref["fit"]) <= TOL
    # lambda-scaled factors row by row (same trajectory from the same initial factors)
    assert e <= TOL and el <= TOL
    for n in range(3):
        got = Fd[n].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(np.linalg.norm(got, axis=0), 1.0, rtol=1e-5)


def test_cp_als_recovery_rank4(spt):
    dims = (30, 20, 10)
    rng = np.random.default_rng(2)
    R = 4
    true = [rng.random((d, R)) + 0.1 for d in dims]
    X = np.einsum("ir,jr,kr->ijk", *true)
    coords = np.stack(np.nonzero(np.ones(dims))).astype(np.uint32)
    t = synth.SparseCOO(dims, coords, X[tuple(coords)].astype(np.float32))
    F0 = [rng.standard_normal((d, R)).astype(np.float32) for d in dims]
    ref = oracle.cp_als(t.coords, t.vals, dims, F0, iters=200)
    c, v = to_dev(t)
    h = spt.encode(dims, c, v)
    Fd = factors_dev(F0)
    lam, fit, its = spt.cp_als(h, Fd, 200)
    print(f"recovery fit gpu {fit:.8f} oracle {ref['fit']:.8f}", flush=True)
    assert fit > 0.999 and ref["fit"] > 0.999
    assert abs(fit - ref["fit"]) <= TOL


def test_cp_als_tol_stops(spt, small):
    t, F, rank, _ = small
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    Fd = factors_dev(F)
    lam, fit, its = spt.cp_als(h, Fd, 500, tol=1e-3)
    ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=500, tol=1e-3)
    assert its < 500 and abs(its - ref["iters"]) <= 1
    if its == ref["iters"]:
        e, _ = cpd_error(to_host(Fd), lam.cpu().numpy(), ref["factors"], ref["lam"])
        assert abs(fit - ref["fit"]) <= TOL and e <= TOL
