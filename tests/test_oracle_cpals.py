"""Pins of the oracle CP-ALS: least-squares optimality, dense residual, recovery, monotonicity."""
import numpy as np
import pytest

import oracle


def _full_coo(X):
    coords = np.stack(np.nonzero(np.ones(X.shape))).astype(np.uint32)
    return coords, X[tuple(coords)].astype(np.float32)


def _reconstruct(factors, lam):
    N = len(factors)
    letters = "abcdefgh"[:N]
    expr = ",".join(f"{l}r" for l in letters) + ",r->" + letters
    return np.einsum(expr, *factors, lam)


def _krp(mats):
    R = mats[0].shape[1]
    return np.stack([np.ravel(np.einsum(",".join("abcdefgh"[i] for i in range(len(mats))) + "->" +
                                        "abcdefgh"[:len(mats)], *[m[:, r] for m in mats])) for r in range(R)], axis=1)


def test_mode_update_is_the_least_squares_solution():
    dims = (6, 5, 4)
    rng = np.random.default_rng(0)
    X = rng.standard_normal(dims)
    coords, vals = _full_coo(X)
    Xd = vals.astype(np.float64).reshape(dims)
    F = [rng.standard_normal((d, 3)) for d in dims]
    grams = [f.T @ f for f in F]
    for n in range(3):
        M = oracle.mttkrp(coords, vals, dims, F, n)
        C, lam = oracle.als_update(M, grams, n)
        others = [F[k] for k in range(3) if k != n]
        K = _krp(others)
        Xn = np.moveaxis(Xd, n, 0).reshape(dims[n], -1)
        A, *_ = np.linalg.lstsq(K, Xn.T, rcond=None)
        np.testing.assert_allclose(C * lam, A.T, rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(np.linalg.norm(C, axis=0), 1.0, rtol=1e-12)
        assert (lam > 0).all()


def test_fit_matches_dense_residual_and_is_monotone():
    dims = (7, 6, 5)
    rng = np.random.default_rng(1)
    X = rng.random(dims) * (rng.random(dims) < 0.6)
    coords = np.stack(np.nonzero(X)).astype(np.uint32)
    vals = X[tuple(coords)].astype(np.float32)
    Xd = np.zeros(dims)
    Xd[tuple(coords)] = vals
    F0 = [rng.standard_normal((d, 3)).astype(np.float32) for d in dims]
    prev = -np.inf
    for it in range(1, 9):
        res = oracle.cp_als(coords, vals, dims, F0, iters=it)
        Xh = _reconstruct(res["factors"], res["lam"])
        dense_fit = 1 - np.linalg.norm(Xd - Xh) / np.linalg.norm(Xd)
        assert abs(res["fit"] - dense_fit) < 1e-9
        assert res["fit"] >= prev - 1e-12
        prev = res["fit"]
    # the recorded trajectory equals the sequence of restarted runs
    res = oracle.cp_als(coords, vals, dims, F0, iters=8)
    assert res["fits"] == sorted(res["fits"]) or np.all(np.diff(res["fits"]) > -1e-12)


def test_recovery_dense_rank4():
    dims = (30, 20, 10)
    rng = np.random.default_rng(2)
    R = 4
    true = [rng.random((d, R)) + 0.1 for d in dims]
    X = np.einsum("ir,jr,kr->ijk", *true)
    coords, vals = _full_coo(X)
    F0 = [rng.standard_normal((d, R)).astype(np.float32) for d in dims]
    res = oracle.cp_als(coords, vals, dims, F0, iters=200, tol=1e-10)
    assert res["fit"] > 0.999


def test_recovery_block_sparse():
    # R disjoint s^3 blocks, each an exact rank-one outer product: a rank-R sparse tensor
    R, s = 4, 6
    dims = (R * s + 3, R * s + 5, R * s + 1)
    rng = np.random.default_rng(3)
    cs, vs = [], []
    for r in range(R):
        a, b, c = (rng.random(s) + 0.5 for _ in range(3))
        blk = np.einsum("i,j,k->ijk", a, b, c)
        idx = np.stack(np.nonzero(np.ones((s, s, s))))
        cs.append(idx + r * s)
        vs.append(blk[tuple(idx)])
    coords = np.concatenate(cs, axis=1).astype(np.uint32)
    vals = np.concatenate(vs).astype(np.float32)
    F0 = [np.abs(rng.standard_normal((d, R))).astype(np.float32) + 0.1 for d in dims]
    res = oracle.cp_als(coords, vals, dims, F0, iters=300, tol=1e-12)
    assert res["fit"] > 0.999


def test_tol_stops_early_and_zero_norm_rejected():
    dims = (8, 7, 6)
    rng = np.random.default_rng(4)
    coords = np.stack([rng.integers(0, d, size=100) for d in dims]).astype(np.uint32)
    vals = rng.random(100).astype(np.float32)
    F0 = [rng.standard_normal((d, 2)).astype(np.float32) for d in dims]
    res = oracle.cp_als(coords, vals, dims, F0, iters=500, tol=1e-3)
    assert res["iters"] < 500
    assert abs(res["fits"][-1] - res["fits"][-2]) < 1e-3
    with pytest.raises(ValueError):
        oracle.cp_als(coords, np.zeros(100, np.float32), dims, F0, iters=2)


def _rotated(eigs, angle):
    """Symmetric 2x2 matrix Q diag(eigs) Q^T with Q the rotation by ``angle``."""
    c, s = np.cos(angle), np.sin(angle)
    Q = np.array([[c, -s], [s, c]])
    return Q @ np.diag(eigs) @ Q.T, Q


def _ridge_case(neg_mult, k_expected):
    """V with eigenvalues (1, -neg_mult * delta_1): plain Cholesky fails; the ridge
    delta_k = 1e-12 tr(V)/R * 1e3^(k-1) of retry k makes it positive definite first at
    k_expected.  Returns the update and the closed-form M (V + delta_k I)^-1."""
    R = 2
    # delta_1 depends on tr(V), which depends on the negative eigenvalue: solve the fixed point
    d1 = 1e-12 * 1.0 / R
    for _ in range(5):
        d1 = 1e-12 * (1.0 - neg_mult * d1) / R
    V, Q = _rotated([1.0, -neg_mult * d1], 0.6)
    base = 1e-12 * np.trace(V) / R
    grams = [np.eye(R), V]               # mode 0: V is the Hadamard product of the other Grams
    M = np.array([[1.0, 2.0], [-0.5, 0.25], [3.0, -1.0]])
    Lc, k = oracle._cholesky_ridge(V)
    assert k == k_expected
    dk = base * 1e3 ** (k - 1)
    # closed form of (V + dk I)^-1 through the eigen-decomposition
    w = np.array([1.0, -neg_mult * d1]) + dk
    inv = Q @ np.diag(1.0 / w) @ Q.T
    C, lam = oracle.als_update(M, grams, 0)
    return C * lam[None, :], M @ inv, w


def test_ridge_retry_first_ridge_closed_form():
    # eigenvalue -delta_1/2: fails plain, passes with delta_1 (the ridge is 1e-12 tr(V)/R)
    got, want, w = _ridge_case(0.5, 1)
    assert w.min() > 0
    # cond(V + delta_1 I) ~ 4e12, so the Cholesky solve carries ~1e-3 relative error;
    # a wrong ridge scale (factor 2 or 1e3) or sign is far outside it
    np.testing.assert_allclose(got, want, rtol=5e-3)


def test_ridge_retry_second_ridge_closed_form():
    # eigenvalue -10 delta_1: still indefinite with delta_1, positive with delta_2 = 1e3 delta_1
    got, want, _ = _ridge_case(10.0, 2)
    np.testing.assert_allclose(got, want, rtol=1e-5)


def test_ridge_gives_up_after_three_retries():
    R = 2
    V, _ = _rotated([1.0, -1e-3], 0.3)   # far below -delta_3 = -1e-6 tr(V)/R
    with pytest.raises(np.linalg.LinAlgError):
        oracle._cholesky_ridge(V)
    with pytest.raises(np.linalg.LinAlgError):
        oracle.als_update(np.ones((3, R)), [np.eye(R), V], 0)
    # a positive definite V takes no ridge
    _, k = oracle._cholesky_ridge(np.array([[2.0, 1.0], [1.0, 2.0]]))
    assert k == 0


def test_ridge_retry_on_singular_gram():
    # two identical columns make V singular; the ridge retry must still return a finite update
    dims = (5, 4, 3)
    rng = np.random.default_rng(5)
    F = [rng.standard_normal((d, 2)) for d in dims]
    for f in F:
        f[:, 1] = f[:, 0]
    grams = [f.T @ f for f in F]
    M = rng.standard_normal((5, 2))
    C, lam = oracle.als_update(M, grams, 0)
    assert np.isfinite(C).all() and np.isfinite(lam).all()
