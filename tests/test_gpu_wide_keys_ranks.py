"""GPU parity of 128-bit keys through MTTKRP, CP-ALS and the batched launch,
of CP-ALS at ranks 48 and 64 (single tensor, batched, served), and of the
normal-equation solve with its ridge retry, all against the FP64 oracle.

Tolerances: MTTKRP max row error 1e-4 of the |X|,|C| row scale; CP-ALS fit
within 1e-4 and lambda-scaled factors within 1e-4 of the factor's largest row
(FP32 rounding alone moves them ~3e-7 over 10 iterations of these tensors).
"""
import numpy as np
import pytest

import oracle
from paper_2509_00280_amd import synth
from _gpu_helpers import check_encoding, cpd_error, factors_dev, mttkrp_error, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_ROW = 1e-4
TOL_FIT = 1e-4
TOL_CPD = 1e-4
E_NOT_SPD = -6


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_00280_amd import spt as _spt
    _spt.lib()
    return _spt


@pytest.fixture(scope="module")
def wide():
    # l(p) = 19 + 18 + 17 + 13 = 67 bits: two-word keys
    dims = (300_000, 200_000, 100_000, 5_000)
    t = synth.distinct_coo(21, dims, 200_000, [("zipf", 1.2)] * 3 + ["uniform"], "lognormal")
    assert oracle.key_words(dims) == 2
    return t


@pytest.mark.parametrize("rank", [16, 64])
@pytest.mark.parametrize("name,strategy,row_cache", [
    ("segment_cached", 5, 1), ("segment_plain", 5, 0), ("direct", 0, 1), ("regroup", 1, 1),
    ("table", 2, 1), ("priv_small_mode", [5, 5, 5, 3], 1)])
def test_u128_mttkrp_every_mode(spt, wide, rank, name, strategy, row_cache):
    t = wide
    F = synth.normal_factors(22 + rank, t.dims, rank)
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    assert h.info()["key_words"] == 2
    h.set_plan(strategy=strategy, row_cache=row_cache)
    Fd = factors_dev(F)
    for n in range(4):
        out = spt.mttkrp(h, Fd, n).cpu().numpy()
        err, bad = mttkrp_error(t, F, n, out)
        print(f"u128 {name} rank {rank} mode {n}: err {err:.3e}", flush=True)
        assert bad == 0 and err <= TOL_ROW


def test_u128_encoding_and_cp_als(spt, wide):
    t = wide
    R, iters = 16, 8
    F = synth.normal_factors(30, t.dims, R)
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    check_encoding(h, t)
    ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
    Fd = factors_dev(F)
    lam, fit, its = spt.cp_als(h, Fd, iters)
    e, el = cpd_error(to_host(Fd), lam.cpu().numpy(), ref["factors"], ref["lam"])
    print(f"u128 cp_als fit {fit:.8f} oracle {ref['fit']:.8f} factor err {e:.2e} lambda err {el:.2e}", flush=True)
    assert its == iters and abs(fit - ref["fit"]) <= TOL_FIT
    assert e <= TOL_CPD and el <= TOL_CPD


def _mix_with_wide_member(ranks=(8, 16)):
    members = synth.batch_config(seed=44, count=4, nnz_range=(1500, 20_000), dim_range=(20, 3000), zipf_s=1.2,
                                 ranks=ranks)
    dims = (70_000, 70_000, 70_000, 70_000)  # 17 bits each: 68-bit keys
    t = synth.distinct_coo(45, dims, 20_000, [("zipf", 1.2)] * 4, "u01")
    members.insert(2, (t, synth.normal_factors(46, dims, 16), 16))
    return members


def test_u128_member_in_batched_mttkrp_and_cp_als(spt):
    import torch
    members = _mix_with_wide_member()
    hs = []
    for t, F, R in members:
        c, v = to_dev(t)
        hs.append(spt.encode(t.dims, c, v))
    assert hs[2].info()["key_words"] == 2
    Fd = [factors_dev(F) for _, F, _ in members]
    for mode in range(4):
        outs = [torch.empty((t.dims[mode] if t.nmodes > mode else 1, R), device="cuda") for t, _, R in members]
        spt.mttkrp_batched(hs, Fd, mode, outs)
        torch.cuda.synchronize()
        for (t, F, R), o in zip(members, outs):
            if t.nmodes <= mode:
                continue
            err, bad = mttkrp_error(t, F, mode, o.cpu().numpy())
            assert bad == 0 and err <= TOL_ROW, (t.dims, mode, err)
    iters = 6
    Fb = [factors_dev(F) for _, F, _ in members]
    lams, fits, its = spt.cp_als_batched(hs, Fb, iters)
    t, F, R = members[2]
    ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
    e, el = cpd_error(to_host(Fb[2]), lams[2].cpu().numpy(), ref["factors"], ref["lam"])
    print(f"u128 member batched fit {fits[2]:.8f} oracle {ref['fit']:.8f} factor err {e:.2e}", flush=True)
    assert abs(fits[2] - ref["fit"]) <= TOL_FIT and e <= TOL_CPD and el <= TOL_CPD


@pytest.fixture(scope="module")
def skewed_small():
    # the skewed 4-mode family at a size the oracle runs in seconds
    return synth.distinct_coo(11, (20_000, 5_000, 2_000, 24), 300_000, [("zipf", 1.3)] * 3 + ["uniform"],
                              "lognormal")


@pytest.mark.parametrize("rank", [48, 64])
def test_cp_als_rank_48_64_matches_oracle(spt, skewed_small, rank):
    t = skewed_small
    iters = 10
    F = synth.normal_factors(12 + rank, t.dims, rank)
    ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    Fd = factors_dev(F)
    lam, fit, its = spt.cp_als(h, Fd, iters)
    e, el = cpd_error(to_host(Fd), lam.cpu().numpy(), ref["factors"], ref["lam"])
    print(f"rank {rank}: fit {fit:.8f} oracle {ref['fit']:.8f} factor err {e:.2e} lambda err {el:.2e}", flush=True)
    assert its == iters and abs(fit - ref["fit"]) <= TOL_FIT
    assert e <= TOL_CPD and el <= TOL_CPD


def test_cp_als_batched_rank_48_64(spt):
    members = synth.batch_config(seed=47, count=6, nnz_range=(2000, 40_000), dim_range=(30, 4000), zipf_s=1.2,
                                 ranks=(48, 64))
    hs = []
    for t, F, R in members:
        c, v = to_dev(t)
        hs.append(spt.encode(t.dims, c, v))
    iters = 6
    Fb = [factors_dev(F) for _, F, _ in members]
    lams, fits, its = spt.cp_als_batched(hs, Fb, iters)
    assert sorted({R for _, _, R in members}) == [48, 64]
    for b, (t, F, R) in enumerate(members):
        ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
        e, el = cpd_error(to_host(Fb[b]), lams[b].cpu().numpy(), ref["factors"], ref["lam"])
        print(f"member {b} R {R}: fit {fits[b]:.8f} oracle {ref['fit']:.8f} factor err {e:.2e}", flush=True)
        assert its[b] == iters and abs(fits[b] - ref["fit"]) <= TOL_FIT
        assert e <= TOL_CPD and el <= TOL_CPD


def test_server_rank_48_64_alone_and_in_mix(spt):
    reqs = [synth.materialize(r) for r in synth.serving_requests(
        seed=48, count=5, rate_per_s=1000.0, ranks=(48, 64), nnz_range=(2000, 30_000), dim_range=(20, 3000))]
    iters = 6
    srv = spt.Server(8 << 30, 4)
    try:
        tickets = [srv.submit(t.dims, t.coords, t.vals, F, iters) for t, F, R in reqs]
        results = [srv.wait(k, timeout_s=120.0) for k in tickets]
    finally:
        srv.close()
    for (t, F, R), (res, Fo, lam) in zip(reqs, results):
        assert res["status"] == 0 and res["iters"] == iters
        # alone: the single-tensor path from the same initial factors
        c, v = to_dev(t)
        h = spt.encode(t.dims, c, v)
        Fs = factors_dev(F)
        lam_s, fit_s, _ = spt.cp_als(h, Fs, iters)
        e, el = cpd_error(Fo, lam, to_host(Fs), lam_s.cpu().numpy())
        ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
        eo, _ = cpd_error(Fo, lam, ref["factors"], ref["lam"])
        print(f"served R {R}: fit {res['fit']:.8f} alone {fit_s:.8f} oracle {ref['fit']:.8f} "
              f"mix-vs-alone {e:.2e} vs oracle {eo:.2e}", flush=True)
        assert abs(res["fit"] - fit_s) <= TOL_FIT and abs(res["fit"] - ref["fit"]) <= TOL_FIT
        assert e <= TOL_CPD and el <= TOL_CPD and eo <= TOL_CPD


# ---------------------------------------------------------------- the solve and its ridge
def _rotated(eigs, angle):
    c, s = np.cos(angle), np.sin(angle)
    Q = np.array([[c, -s], [s, c]])
    return Q @ np.diag(eigs) @ Q.T


def _grams_dev(grams):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.stack(grams))).cuda()


@pytest.mark.parametrize("neg_mult,k_expected,rtol", [(0.5, 1, 5e-3), (10.0, 2, 1e-5)])
def test_als_update_ridge_retry_matches_oracle(spt, neg_mult, k_expected, rtol):
    """V = Q diag(1, -neg_mult d_1) Q^T fails a plain Cholesky; the GPU solve must take
    the same retry as the oracle and give the same lambda-scaled update."""
    import torch
    R = 2
    d1 = 1e-12 / R
    for _ in range(5):
        d1 = 1e-12 * (1.0 - neg_mult * d1) / R
    V = _rotated([1.0, -neg_mult * d1], 0.6)
    grams = [np.eye(R), V]
    M = np.array([[1.0, 2.0], [-0.5, 0.25], [3.0, -1.0], [0.0, 0.0]], dtype=np.float32)
    C_ref, lam_ref = oracle.als_update(M.astype(np.float64), grams, 0)
    _, k_ref = oracle._cholesky_ridge(V)
    C, lam, retries = spt.als_update(_grams_dev(grams), 0, torch.from_numpy(M).cuda())
    got = C.cpu().numpy().astype(np.float64) * lam.cpu().numpy()[None, :]
    print(f"ridge retries gpu {retries} oracle {k_ref}", flush=True)
    assert retries == k_ref == k_expected
    np.testing.assert_allclose(got, C_ref * lam_ref[None, :], rtol=rtol, atol=rtol * np.abs(C_ref * lam_ref).max())
    assert (C.cpu().numpy()[3] == 0).all()  # a zero row of M stays zero


def test_als_update_not_spd_after_retries(spt):
    import torch
    R = 2
    V = _rotated([1.0, -1e-3], 0.3)
    M = torch.ones((3, R), dtype=torch.float32, device="cuda")
    C = torch.full((3, R), 7.0, device="cuda")
    with pytest.raises(spt.SptError) as e:
        spt.als_update(_grams_dev([np.eye(R), V]), 0, M, C=C)
    assert e.value.status == E_NOT_SPD
    assert (C == 7.0).all()  # outputs untouched on failure
    nan = np.eye(R)
    nan[0, 0] = np.nan
    with pytest.raises(spt.SptError) as e:
        spt.als_update(_grams_dev([np.eye(R), nan]), 0, M)
    assert e.value.status == E_NOT_SPD


@pytest.mark.parametrize("rank", [16, 48, 64])
def test_als_update_well_conditioned(spt, rank):
    import torch
    rng = np.random.default_rng(rank)
    rows = 5000
    grams = []
    for k in range(3):
        A = rng.standard_normal((40 + rank, rank))
        grams.append(A.T @ A / (40 + rank))
    M = rng.standard_normal((rows, rank)).astype(np.float32)
    C_ref, lam_ref = oracle.als_update(M.astype(np.float64), grams, 1)
    C, lam, retries = spt.als_update(_grams_dev(grams), 1, torch.from_numpy(M).cuda())
    e, el = cpd_error([C.cpu().numpy()], lam.cpu().numpy(), [C_ref], lam_ref)
    print(f"rank {rank}: update err {e:.2e} lambda {el:.2e}", flush=True)
    assert retries == 0 and e <= 1e-5 and el <= 1e-6
