"""Autotuner (measured search over bit layouts and per-mode plans, Section
III-C) and the continuous-batching server, on the GPU."""
import numpy as np
import pytest

import oracle
from paper_2509_00280_amd import synth
from _gpu_helpers import check_encoding, cpd_error, factors_dev, mttkrp_error, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_ROW = 1e-4
TOL_FIT = 1e-4
E_OOM, E_NOT_FOUND = -5, -9


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_00280_amd import spt as _spt
    _spt.lib()
    return _spt


def _check_after_tune(spt, h, t, F):
    import torch
    layout = h.info()["layout"]
    assert oracle.is_valid_layout(layout, t.dims)
    check_encoding(h, t, layout=layout)  # keys, values, perm (input order) and decode, bit for bit
    plan = h.get_plan()
    Fd = factors_dev(F)
    for n in range(t.nmodes):
        assert plan["strategy"][n] in (3, 5)
        out = torch.empty((t.dims[n], F[0].shape[1]), device="cuda")
        spt.mttkrp(h, Fd, n, out=out)
        torch.cuda.synchronize()
        err, bad = mttkrp_error(t, F, n, out.cpu().numpy())
        assert bad == 0 and err <= TOL_ROW


def test_autotune_small_keeps_exact_encoding(spt):
    t, F, R, _ = synth.config("small")
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v)
    res = spt.autotune(h, factors_dev(F), budget_ms=600.0, random_samples=3, seed=1)
    print(f"tune {res} layout {h.info()['layout']}", flush=True)
    assert res["best_ms"] > 0 and res["best_ms"] <= min(res["alto_ms"], res["start_ms"])
    assert res["random_samples"] <= 3 and res["candidates"] >= 1
    _check_after_tune(spt, h, t, F)
    # the winner is cached per (shape, nnz, rank, layout, content): a zero-budget call returns it
    again = spt.autotune(h, factors_dev(F), budget_ms=0.0, random_samples=0)
    assert again["best_ms"] == res["best_ms"] and again["cache_hits"] >= 1


def test_autotune_from_poor_layout(spt):
    """Start from a blocked layout (all bits of mode 0 lowest): moves are
    searched and whatever wins must still be an exact encoding."""
    t = synth.distinct_coo(7, (300, 200, 64), 30_000, [("zipf", 1.2), ("zipf", 1.2), "uniform"], "u01")
    F = synth.normal_factors(8, t.dims, 16)
    lb = oracle.bit_lengths(t.dims)
    blocked = [n for n in range(3) for _ in range(lb[n])]
    c, v = to_dev(t)
    h = spt.encode(t.dims, c, v, layout=blocked)
    res = spt.autotune(h, factors_dev(F), budget_ms=1500.0, random_samples=4, seed=2)
    print(f"tune {res}, layout moved: {h.info()['layout'] != blocked}", flush=True)
    assert res["start_ms"] >= res["best_ms"]
    _check_after_tune(spt, h, t, F)


def test_autotune_cache_distinguishes_contents(spt):
    """Two tensors of one shape and nnz (one the label-shuffled other) are measured separately."""
    t = synth.distinct_coo(17, (400, 300, 50), 40_000, [("zipf", 1.2), ("zipf", 1.2), "uniform"], "u01")
    ts = synth.shuffle_labels(t, 5)
    F = synth.normal_factors(18, t.dims, 16)
    r1 = spt.autotune(spt.encode(t.dims, *to_dev(t)), factors_dev(F), budget_ms=0.0, random_samples=0)
    r2 = spt.autotune(spt.encode(ts.dims, *to_dev(ts)), factors_dev(F), budget_ms=0.0, random_samples=0)
    assert r1["cache_hits"] == 0 and r2["cache_hits"] == 0


def _requests(count, seed=5, ranks=(8, 16, 32)):
    reqs = synth.serving_requests(seed=seed, count=count, rate_per_s=1000.0, ranks=ranks,
                                  nnz_range=(2000, 30_000), dim_range=(20, 3000))
    return [synth.materialize(r) for r in reqs]


def test_server_matches_single_tensor_cp_als(spt):
    iters = 8
    reqs = _requests(6)
    srv = spt.Server(8 << 30, 4)
    try:
        tickets = [srv.submit(t.dims, t.coords, t.vals, F, iters) for t, F, R in reqs]
        results = [srv.wait(k, timeout_s=60.0) for k in tickets]
    finally:
        srv.close()
    for (t, F, R), (res, Fo, lam) in zip(reqs, results):
        assert res["status"] == 0
        assert res["iters"] == iters
        assert res["t_arrive"] <= res["t_admit"] <= res["t_done"]
        c, v = to_dev(t)
        h = spt.encode(t.dims, c, v)
        Fs = factors_dev(F)
        lam_s, fit_s, _ = spt.cp_als(h, Fs, iters)
        e, el = cpd_error(Fo, lam, to_host(Fs), lam_s.cpu().numpy())
        print(f"nnz {t.nnz} R {R}: served fit {res['fit']:.8f} single {fit_s:.8f} factor err {e:.2e}", flush=True)
        assert abs(res["fit"] - fit_s) <= TOL_FIT
        assert e <= TOL_ROW and el <= TOL_ROW
        for n in range(t.nmodes):
            np.testing.assert_allclose(np.linalg.norm(Fo[n].astype(np.float64), axis=0), 1.0, rtol=1e-5)
    t, F, R = reqs[0]
    ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
    res, Fo, lam = results[0]
    e, el = cpd_error(Fo, lam, ref["factors"], ref["lam"])
    assert abs(res["fit"] - ref["fit"]) <= TOL_FIT
    assert e <= TOL_ROW and el <= TOL_ROW


def test_server_one_slot_tol_and_budget(spt):
    reqs = _requests(3, seed=6)
    srv = spt.Server(64 << 20, 1)
    try:
        big = synth.distinct_coo(9, (4000, 4000, 4000), 400_000, ["uniform"] * 3, "u01")
        Fb = synth.normal_factors(10, big.dims, 32)
        k_big = srv.submit(big.dims, big.coords, big.vals, Fb, 5)
        tickets = [srv.submit(t.dims, t.coords, t.vals, F, 50, tol=1e-3) for t, F, R in reqs]
        res_big, _, _ = srv.wait(k_big, timeout_s=60.0)
        results = [srv.wait(k, timeout_s=60.0)[0] for k in tickets]
        with pytest.raises(spt.SptError) as ei:
            srv.wait(123456, timeout_s=0.0)
        assert ei.value.status == E_NOT_FOUND
    finally:
        srv.close()
    assert res_big["status"] == E_OOM  # larger than the whole budget
    for (t, F, R), r in zip(reqs, results):
        assert r["status"] == 0
        ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=50, tol=1e-3)
        assert r["iters"] == ref["iters"]
        assert abs(r["fit"] - ref["fit"]) <= TOL_FIT
    # one slot: each request is admitted only after the previous one finished
    for a, b in zip(results, results[1:]):
        assert b["t_admit"] >= a["t_done"] - 1e-6


def test_server_isolates_failing_requests(spt):
    """A request with an out-of-range coordinate and one with a NaN initial factor
    retire with their errors; the requests beside them finish and match the
    single-tensor path and the oracle."""
    iters = 6
    reqs = _requests(4, seed=9)
    srv = spt.Server(8 << 30, 8)
    try:
        good = [srv.submit(t.dims, t.coords, t.vals, F, iters) for t, F, R in reqs[:2]]
        t, F, R = reqs[2]
        bad_c = t.coords.copy()
        bad_c[1, 5] = t.dims[1]  # one coordinate out of range
        k_range = srv.submit(t.dims, bad_c, t.vals, F, iters)
        t, F, R = reqs[3]
        Fn = [f.copy() for f in F]
        Fn[1][2, 1] = np.nan  # factor 0 is overwritten before it is read; factor 1 enters mode 0's solve
        k_nan = srv.submit(t.dims, t.coords, t.vals, Fn, iters)
        good += [srv.submit(t.dims, t.coords, t.vals, F, iters) for t, F, R in reqs[:2]]
        res_good = [srv.wait(k, timeout_s=60.0) for k in good]
        r_range, _, _ = srv.wait(k_range, timeout_s=60.0)
        r_nan, _, _ = srv.wait(k_nan, timeout_s=60.0)
    finally:
        srv.close()
    assert r_range["status"] == -2 and r_nan["status"] == -6
    for (t, F, R), (res, Fo, lam) in zip(reqs[:2] * 2, res_good):
        assert res["status"] == 0 and res["iters"] == iters
        h = spt.encode(t.dims, *to_dev(t))
        Fs = factors_dev(F)
        lam_s, fit_s, _ = spt.cp_als(h, Fs, iters)
        e, el = cpd_error(Fo, lam, to_host(Fs), lam_s.cpu().numpy())
        assert abs(res["fit"] - fit_s) <= TOL_FIT and e <= TOL_ROW and el <= TOL_ROW
    t, F, R = reqs[0]
    ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
    assert abs(res_good[0][0]["fit"] - ref["fit"]) <= TOL_FIT
