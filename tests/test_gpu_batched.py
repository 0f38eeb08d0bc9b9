"""Batched MTTKRP and lock-step CP-ALS over many tensors against the oracle
and against the single-tensor path (the batched launch of Section IV-D's
repeated decompositions)."""
import numpy as np
import pytest

import oracle
from paper_2509_00280_amd import synth
from _gpu_helpers import cpd_error, factors_dev, mttkrp_error, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_ROW = 1e-4
TOL_FIT = 1e-4


@pytest.fixture(scope="module")
def spt():
    import torch
    assert torch.cuda.is_available()
    from paper_2509_00280_amd import spt as _spt
    _spt.lib()
    return _spt


def _batch(ranks=(8, 16, 32), count=10, seed=41):
    return synth.batch_config(seed=seed, count=count, nnz_range=(1500, 40_000), dim_range=(20, 4000),
                              zipf_s=1.2, ranks=ranks)


@pytest.fixture(scope="module")
def mixed(spt):
    members = _batch()
    hs = []
    for t, F, R in members:
        c, v = to_dev(t)
        hs.append(spt.encode(t.dims, c, v))
    return members, hs


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_mttkrp_batched_matches_oracle(spt, mixed, mode):
    import torch
    members, hs = mixed
    Fd = [factors_dev(F) for _, F, _ in members]
    outs = [torch.full((t.dims[mode] if t.nmodes > mode else 1, R), float("nan"), device="cuda")
            for t, _, R in members]
    spt.mttkrp_batched(hs, Fd, mode, outs)
    torch.cuda.synchronize()
    seen = 0
    for (t, F, R), o in zip(members, outs):
        if t.nmodes <= mode:
            assert torch.isnan(o).all()  # skipped tensors are not written
            continue
        err, bad = mttkrp_error(t, F, mode, o.cpu().numpy())
        print(f"member {t.meta['member']} dims {t.dims} nnz {t.nnz} R {R} mode {mode}: err {err:.2e}", flush=True)
        assert bad == 0 and err <= TOL_ROW
        seen += 1
    assert seen > 0


def test_mttkrp_batched_equals_single(spt, mixed):
    import torch
    members, hs = mixed
    Fd = [factors_dev(F) for _, F, _ in members]
    outs = [torch.empty((t.dims[0], R), device="cuda") for t, _, R in members]
    spt.mttkrp_batched(hs, Fd, 0, outs)
    for (t, F, R), h, f, o in zip(members, hs, Fd, outs):
        ref = torch.empty_like(o)
        spt.mttkrp(h, f, 0, out=ref)
        torch.cuda.synchronize()
        scale = torch.abs(ref).max().item() + 1e-30
        assert torch.max(torch.abs(o - ref)).item() <= 1e-5 * scale


def test_mttkrp_batched_odd_ranks(spt):
    """Ranks that are not multiples of 4 take the one-column-per-lane path."""
    import torch
    members = _batch(ranks=(5, 7, 12), count=5, seed=43)
    hs, Fd = [], []
    for t, F, R in members:
        c, v = to_dev(t)
        hs.append(spt.encode(t.dims, c, v))
        Fd.append(factors_dev(F))
    for mode in range(3):
        outs = [torch.empty((t.dims[mode], R), device="cuda") for t, _, R in members]
        spt.mttkrp_batched(hs, Fd, mode, outs)
        torch.cuda.synchronize()
        for (t, F, R), o in zip(members, outs):
            err, bad = mttkrp_error(t, F, mode, o.cpu().numpy())
            assert bad == 0 and err <= TOL_ROW


def test_cp_als_batched_matches_single_and_oracle(spt, mixed):
    members, hs = mixed
    iters = 6
    Fb = [factors_dev(F) for _, F, _ in members]
    lams, fits, its = spt.cp_als_batched(hs, Fb, iters)
    assert its == [iters] * len(members)
    for b, ((t, F, R), h) in enumerate(zip(members, hs)):
        Fs = factors_dev(F)
        lam_s, fit_s, it_s = spt.cp_als(h, Fs, iters)
        e, el = cpd_error(to_host(Fb[b]), lams[b].cpu().numpy(), to_host(Fs), lam_s.cpu().numpy())
        print(f"member {b}: batched fit {fits[b]:.8f} single {fit_s:.8f} factor err {e:.2e}", flush=True)
        assert abs(fits[b] - fit_s) <= TOL_FIT
        assert e <= TOL_ROW and el <= TOL_ROW
    for b in (0, 1):
        t, F, R = members[b]
        ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
        e, el = cpd_error(to_host(Fb[b]), lams[b].cpu().numpy(), ref["factors"], ref["lam"])
        assert abs(fits[b] - ref["fit"]) <= TOL_FIT
        assert e <= TOL_ROW and el <= TOL_ROW


def test_cp_als_batched_alone_vs_in_mix(spt, mixed):
    members, hs = mixed
    iters = 5
    Fm = [factors_dev(F) for _, F, _ in members]
    lam_mix, fit_mix, _ = spt.cp_als_batched(hs, Fm, iters)
    for b in (0, 3):
        Fa = [factors_dev(members[b][1])]
        lam_a, fit_alone, _ = spt.cp_als_batched([hs[b]], Fa, iters)
        e, el = cpd_error(to_host(Fa[0]), lam_a[0].cpu().numpy(), to_host(Fm[b]), lam_mix[b].cpu().numpy())
        print(f"member {b}: alone vs in mix fit {abs(fit_alone[0] - fit_mix[b]):.2e} factor err {e:.2e}", flush=True)
        assert abs(fit_alone[0] - fit_mix[b]) <= TOL_FIT
        assert e <= TOL_ROW and el <= TOL_ROW


def test_cp_als_batched_members_stop_individually(spt, mixed):
    members, hs = mixed
    _, fits, its = spt.cp_als_batched(hs, [factors_dev(F) for _, F, _ in members], 60, tol=1e-3)
    assert all(1 <= i <= 60 for i in its)
    for b in (0, 2):
        t, F, R = members[b]
        ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=60, tol=1e-3)
        assert its[b] == ref["iters"]
        assert abs(fits[b] - ref["fit"]) <= TOL_FIT


def test_batched_empty_and_invalid(spt, mixed):
    import torch
    members, hs = mixed
    assert spt.cp_als_batched([], [], 3)[1] == []
    t, F, R = members[0]
    with pytest.raises(spt.SptError):
        spt.mttkrp_batched([hs[0]], [factors_dev(F)], 99, [torch.empty((1, R), device="cuda")])
