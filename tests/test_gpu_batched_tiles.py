"""Batched launches at every batch tile, the persistent work-pulling launch
over many tiles, and the batch autotuner (layouts of the members, then the
batch tile by measurement), against the oracle and the single-tensor path."""
import numpy as np
import pytest

import oracle
from paper_2509_00280_amd import synth
from _gpu_helpers import check_encoding, cpd_error, factors_dev, mttkrp_error, to_dev, to_host

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


def _members(count=6, seed=61, ranks=(8, 16, 32)):
    return synth.batch_config(seed=seed, count=count, nnz_range=(1500, 40_000), dim_range=(20, 4000),
                              zipf_s=1.2, ranks=ranks)


def _encode_all(spt, members):
    return [spt.encode(t.dims, *to_dev(t)) for t, _, _ in members]


@pytest.mark.parametrize("tile", [1024, 2048, 4096])
def test_mttkrp_batched_each_tile_matches_oracle(spt, tile):
    import torch
    members = _members()
    hs = _encode_all(spt, members)
    for h in hs:
        h.set_plan(batch_tile=tile)
        assert h.get_plan()["batch_tile"] == tile
    Fd = [factors_dev(F) for _, F, _ in members]
    for mode in range(4):
        outs = [torch.empty((t.dims[mode] if t.nmodes > mode else 1, R), device="cuda") for t, _, R in members]
        spt.mttkrp_batched(hs, Fd, mode, outs)
        torch.cuda.synchronize()
        for (t, F, R), o in zip(members, outs):
            if t.nmodes <= mode:
                continue
            err, bad = mttkrp_error(t, F, mode, o.cpu().numpy())
            print(f"tile {tile} mode {mode} dims {t.dims} nnz {t.nnz} R {R}: err {err:.2e}", flush=True)
            assert bad == 0 and err <= TOL_ROW


def test_persistent_launch_pulls_many_tiles(spt):
    """Enough tiles that every resident workgroup pulls several (about 2.5M
    nonzeros at 1024 per tile, over tensors of very different sizes)."""
    import torch
    big = [synth.distinct_coo(71 + i, dims, nnz, [("zipf", 1.2)] * len(dims), "u01")
           for i, (dims, nnz) in enumerate([((3000, 2000, 400), 1_500_000), ((900, 800, 300, 20), 1_000_000)])]
    small = [t for t, _, _ in _members(count=8, seed=73)]
    ts = big + small
    R = 16
    Fs = [synth.normal_factors(80 + i, t.dims, R) for i, t in enumerate(ts)]
    hs = [spt.encode(t.dims, *to_dev(t)) for t in ts]
    for h in hs:
        h.set_plan(batch_tile=1024)
    Fd = [factors_dev(F) for F in Fs]
    for mode in (0, 2):
        outs = [torch.empty((t.dims[mode], R), device="cuda") for t in ts]
        spt.mttkrp_batched(hs, Fd, mode, outs)
        torch.cuda.synchronize()
        for t, F, o in zip(ts, Fs, outs):
            err, bad = mttkrp_error(t, F, mode, o.cpu().numpy())
            assert bad == 0 and err <= TOL_ROW, (t.dims, mode, err, bad)
    # and the same members through the single-tensor path agree
    ref = torch.empty((ts[0].dims[1], R), device="cuda")
    spt.mttkrp(hs[0], Fd[0], 1, out=ref)
    outs = [torch.empty((t.dims[1], R), device="cuda") for t in ts]
    spt.mttkrp_batched(hs, Fd, 1, outs)
    torch.cuda.synchronize()
    assert torch.max(torch.abs(outs[0] - ref)).item() <= 1e-5 * (torch.abs(ref).max().item() + 1e-30)


def test_mixed_tiles_rejected_by_mttkrp_batched(spt):
    import torch
    members = _members(count=3, seed=62)
    hs = _encode_all(spt, members)
    hs[0].set_plan(batch_tile=1024)
    hs[1].set_plan(batch_tile=4096)
    for h in hs:
        h.prepare(1, batched=True)
    Fd = [factors_dev(F) for _, F, _ in members]
    outs = [torch.empty((t.dims[0], R), device="cuda") for t, _, R in members]
    with pytest.raises(spt.SptError):
        spt.mttkrp_batched(hs, Fd, 0, outs)


def test_cp_als_batched_replans_mixed_tiles(spt):
    """cp_als_batched runs every member at the first member's tile (re-planning the others)."""
    members = _members(count=4, seed=63)
    hs = _encode_all(spt, members)
    hs[0].set_plan(batch_tile=4096)
    hs[2].set_plan(batch_tile=1024)
    iters = 5
    Fb = [factors_dev(F) for _, F, _ in members]
    lams, fits, its = spt.cp_als_batched(hs, Fb, iters)
    assert its == [iters] * len(members)
    for b, ((t, F, R), h) in enumerate(zip(members, hs)):
        ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
        e, el = cpd_error(to_host(Fb[b]), lams[b].cpu().numpy(), ref["factors"], ref["lam"])
        print(f"member {b}: fit {fits[b]:.8f} oracle {ref['fit']:.8f} factor err {e:.2e}", flush=True)
        assert abs(fits[b] - ref["fit"]) <= TOL_FIT
        assert e <= TOL_ROW and el <= TOL_ROW


def test_autotune_batched_tile_and_layouts(spt):
    import torch
    members = _members(count=5, seed=64)
    hs = _encode_all(spt, members)
    Fd = [factors_dev(F) for _, F, _ in members]
    res = spt.autotune_batched(hs, Fd, layout_budget_ms=150.0, random_samples=2, seed=3)
    print(f"batch tune {res}", flush=True)
    ms = {k: v for k, v in res["ms"].items() if v > 0}
    assert res["best_tile"] in ms and ms[res["best_tile"]] == min(ms.values())
    assert res["layouts_tuned"] == len(members) and res["layout_speedup"] >= 1.0
    for (t, F, R), h in zip(members, hs):
        assert h.get_plan()["batch_tile"] == res["best_tile"]
        check_encoding(h, t, layout=h.info()["layout"])  # every re-encoding is exact
    for mode in range(3):
        outs = [torch.empty((t.dims[mode], R), device="cuda") for t, _, R in members]
        spt.mttkrp_batched(hs, Fd, mode, outs)
        torch.cuda.synchronize()
        for (t, F, R), o in zip(members, outs):
            err, bad = mttkrp_error(t, F, mode, o.cpu().numpy())
            assert bad == 0 and err <= TOL_ROW


def test_autotune_batched_tile_only_then_cp_als(spt):
    members = _members(count=4, seed=65)
    hs = _encode_all(spt, members)
    Fd = [factors_dev(F) for _, F, _ in members]
    layouts = [h.info()["layout"] for h in hs]
    res = spt.autotune_batched(hs, Fd)
    assert res["layouts_tuned"] == 0 and res["layout_speedup"] == 1.0
    assert [h.info()["layout"] for h in hs] == layouts
    iters = 4
    Fb = [factors_dev(F) for _, F, _ in members]
    lams, fits, _ = spt.cp_als_batched(hs, Fb, iters)
    for b, ((t, F, R), h) in enumerate(zip(members, hs)):
        Fs = factors_dev(F)
        lam_s, fit_s, _ = spt.cp_als(h, Fs, iters)
        e, el = cpd_error(to_host(Fb[b]), lams[b].cpu().numpy(), to_host(Fs), lam_s.cpu().numpy())
        assert abs(fits[b] - fit_s) <= TOL_FIT
        assert e <= TOL_ROW and el <= TOL_ROW


def _exact_rank(dims, R, seed):
    rng = np.random.default_rng(seed)
    true = [rng.random((d, R)) + 0.1 for d in dims]
    X = true[0]
    for f in true[1:]:
        X = np.einsum("...r,jr->...jr", X, f)
    X = X.sum(axis=-1)
    coords = np.stack(np.nonzero(np.ones(dims))).astype(np.uint32)
    t = synth.SparseCOO(tuple(dims), coords, X[tuple(coords)].astype(np.float32))
    F0 = [rng.standard_normal((d, R)).astype(np.float32) for d in dims]
    return t, F0, R


def test_cp_als_batched_direct_fit_recovery(spt):
    """Members that converge (1 - fit < 1e-2) take the direct FP64 residual, for
    the whole batch in one launch: exact rank-R tensors (3 and 4 modes, ranks
    4, 5 and 8, so both lane layouts) next to a member that stays far from it."""
    members = [_exact_rank((30, 20, 10), 4, 2), _exact_rank((12, 9, 8, 6), 5, 3), _exact_rank((25, 16, 12), 8, 4)]
    members.append(_members(count=1, seed=66, ranks=(8,))[0])
    hs = _encode_all(spt, members)
    iters = 120
    Fb = [factors_dev(F) for _, F, _ in members]
    lams, fits, its = spt.cp_als_batched(hs, Fb, iters)
    for b, ((t, F, R), h) in enumerate(zip(members, hs)):
        Fs = factors_dev(F)
        lam_s, fit_s, _ = spt.cp_als(h, Fs, iters)
        ref = oracle.cp_als(t.coords, t.vals, t.dims, F, iters=iters)
        print(f"member {b}: batched fit {fits[b]:.8f} single {fit_s:.8f} oracle {ref['fit']:.8f}", flush=True)
        assert abs(fits[b] - fit_s) <= TOL_FIT and abs(fits[b] - ref["fit"]) <= TOL_FIT
        if b < 3:
            assert fits[b] > 0.99  # the direct residual is in use
