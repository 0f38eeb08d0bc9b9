"""The continuous-batching server's admission policy (HBM budget, slots,
arrival order) driven on the host by a modelled executor: no GPU."""
import numpy as np
import pytest

from paper_2509_00280_amd import spt

GB = 1 << 30


def _replay(bytes_, adm, done, st):
    """Resource use over time from the admit/done log: max concurrent slots and bytes."""
    ev = []
    for b, a, d, s in zip(bytes_, adm, done, st):
        if s == 0:
            ev.append((a, 1, int(b)))
            ev.append((d, -1, -int(b)))
    ev.sort(key=lambda e: (e[0], e[1]))  # releases before admissions at equal times
    slots = used = ms = mu = 0
    for _, ds, db in ev:
        slots += ds
        used += db
        ms, mu = max(ms, slots), max(mu, used)
    return ms, mu


@pytest.fixture(scope="module")
def lib():
    if not __import__("os").path.exists(spt.LIB_PATH):
        from paper_2509_00280_amd import build
        build.build()
    return spt


def test_budget_bounds_concurrency_and_order_is_fifo(lib):
    n = 10
    bytes_ = [GB] * n
    arrive = np.zeros(n)
    service = np.arange(1, n + 1, dtype=float)
    adm, done, st = lib.server_simulate(3 * GB, 8, bytes_, arrive, service)
    assert (st == 0).all()
    ms, mu = _replay(bytes_, adm, done, st)
    assert ms == 3 and mu == 3 * GB               # the budget, not the slots, binds
    assert (np.diff(adm) >= 0).all()              # admitted in arrival order
    assert np.allclose(done, adm + service)
    # a waiting request is admitted exactly when an earlier one finishes (slot and bytes reuse)
    for i in range(3, n):
        assert np.isclose(adm[i], np.sort(done[:i])[i - 3])


def test_slots_bound_concurrency(lib):
    n = 7
    bytes_ = [1] * n
    adm, done, st = lib.server_simulate(100 * GB, 2, bytes_, np.zeros(n), np.full(n, 2.0))
    ms, _ = _replay(bytes_, adm, done, st)
    assert ms == 2 and np.isclose(done.max(), 8.0)  # 7 requests, 2 at a time, 2 s each


def test_over_budget_rejected_without_blocking_others(lib):
    bytes_ = [GB, 10 * GB, GB, GB]
    arrive = [0.0, 0.1, 0.2, 0.3]
    adm, done, st = lib.server_simulate(2 * GB, 4, bytes_, arrive, [1.0] * 4)
    assert st[1] == -5 and adm[1] == done[1]       # SPT_E_OOM at once
    assert (st[[0, 2, 3]] == 0).all()
    assert np.isclose(adm[2], 0.2) and np.isclose(adm[3], 1.0)  # the 4th waits for the 1st to free its bytes


def test_head_of_line_waits_in_arrival_order(lib):
    # a large request at the head waits for bytes; smaller later ones wait behind it
    bytes_ = [2 * GB, 3 * GB, GB]
    adm, done, st = lib.server_simulate(4 * GB, 4, bytes_, [0.0, 0.1, 0.2], [5.0, 1.0, 1.0])
    assert (st == 0).all()
    assert np.isclose(adm[1], 5.0) and np.isclose(adm[2], 5.0)
    ms, mu = _replay(bytes_, adm, done, st)
    assert mu <= 4 * GB


def test_random_streams_never_exceed_limits(lib):
    rng = np.random.default_rng(3)
    for _ in range(20):
        n = 200
        bytes_ = rng.integers(1, 5 * GB, size=n)
        arrive = np.cumsum(rng.exponential(0.01, size=n))
        service = rng.exponential(0.05, size=n)
        budget, slots = int(rng.integers(4, 12)) * GB, int(rng.integers(1, 16))
        adm, done, st = lib.server_simulate(budget, slots, bytes_, arrive, service)
        assert ((st == 0) | ((st == -5) & (bytes_ > budget))).all()
        assert (adm >= arrive - 1e-12).all() and (done >= adm).all()
        ms, mu = _replay(bytes_, adm, done, st)
        assert ms <= slots and mu <= budget
        ok = st == 0
        assert (np.diff(adm[ok]) >= -1e-12).all()  # arrival order kept


def test_simulate_rejects_bad_arguments(lib):
    with pytest.raises(lib.SptError):
        lib.server_simulate(GB, 0, [1], [0.0], [1.0])
    with pytest.raises(lib.SptError):
        lib.server_simulate(GB, 1, [1, 1], [1.0, 0.0], [1.0, 1.0])
