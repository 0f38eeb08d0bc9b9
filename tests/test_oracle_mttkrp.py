"""Pins of the oracle MTTKRP: dense brute force, closed forms and invariants."""
import numpy as np
import pytest

import oracle


def _dense_random(dims, density, rng):
    X = rng.standard_normal(dims) * (rng.random(dims) < density)
    coords = np.stack(np.nonzero(X)).astype(np.uint32)
    vals = X[tuple(coords)].astype(np.float32)
    Xd = np.zeros(dims)
    Xd[tuple(coords)] = vals.astype(np.float64)
    return Xd, coords, vals


def _krp(mats):
    """Khatri-Rao product: column r is the Kronecker product of the columns r, second factor fastest."""
    R = mats[0].shape[1]
    cols = []
    for r in range(R):
        col = np.ones(1)
        for A in mats:
            col = np.kron(col, A[:, r])
        cols.append(col)
    return np.stack(cols, axis=1)


def _brute(X, factors, n):
    """X_(n) (C-order unfolding: remaining modes ascending, last fastest) times the forward KRP."""
    Xn = np.moveaxis(X, n, 0).reshape(X.shape[n], -1)
    K = _krp([factors[k].astype(np.float64) for k in range(X.ndim) if k != n])
    return Xn @ K


@pytest.mark.parametrize("dims,R", [((5, 4, 3), 3), ((3, 4, 2, 3), 4), ((7, 2), 5), ((2, 3, 2, 2, 3), 2)])
def test_brute_force_dense(dims, R):
    rng = np.random.default_rng(sum(dims) * 10 + R)
    X, c, v = _dense_random(dims, 0.5, rng)
    F = [rng.standard_normal((d, R)).astype(np.float32) for d in dims]
    for n in range(len(dims)):
        got = oracle.mttkrp(c, v, dims, F, n)
        ref = _brute(X, F, n)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_all_ones_gives_slice_sums():
    dims = (30, 20, 10, 4)
    rng = np.random.default_rng(1)
    c = np.stack([rng.integers(0, d, size=3000) for d in dims]).astype(np.uint32)
    v = rng.random(3000, dtype=np.float32)
    F = [np.ones((d, 6), np.float32) for d in dims]
    for n in range(4):
        got = oracle.mttkrp(c, v, dims, F, n)
        ref = np.bincount(c[n], weights=v.astype(np.float64), minlength=dims[n])
        for r in range(6):
            np.testing.assert_allclose(got[:, r], ref, rtol=1e-13, atol=0)


def test_duplicate_split_and_order_invariance():
    dims = (12, 9, 7)
    rng = np.random.default_rng(4)
    c = np.stack([rng.integers(0, d, size=500) for d in dims]).astype(np.uint32)
    v = rng.standard_normal(500).astype(np.float32)
    F = [rng.standard_normal((d, 8)).astype(np.float32) for d in dims]
    base = [oracle.mttkrp(c, v, dims, F, n) for n in range(3)]
    # split nonzero 17 into two halves with the same coordinate
    a = np.float32(0.25) * v[17]
    v2 = v.copy()
    v2[17] = v[17] - a
    c2 = np.concatenate([c, c[:, 17:18]], axis=1)
    v2 = np.concatenate([v2, [a]]).astype(np.float32)
    perm = rng.permutation(501)
    for n in range(3):
        np.testing.assert_allclose(oracle.mttkrp(c2, v2, dims, F, n), base[n], rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(oracle.mttkrp(c2[:, perm], v2[perm], dims, F, n), base[n], rtol=1e-6, atol=1e-6)


def test_rank_one_closed_form():
    dims = (6, 5, 4)
    rng = np.random.default_rng(9)
    a, b, cc = (rng.random(d) + 0.1 for d in dims)
    X = np.einsum("i,j,k->ijk", a, b, cc).astype(np.float32)
    coords = np.stack(np.nonzero(np.ones(dims))).astype(np.uint32)
    vals = X[tuple(coords)]
    U = [rng.standard_normal((d, 3)).astype(np.float32) for d in dims]
    M0 = oracle.mttkrp(coords, vals, dims, U, 0)
    Xd = vals.astype(np.float64).reshape(dims)
    # closed form for the exact FP32 values: M0[i,r] = sum_jk X[i,j,k] U1[j,r] U2[k,r]
    ref = np.einsum("ijk,jr,kr->ir", Xd, U[1].astype(np.float64), U[2].astype(np.float64))
    np.testing.assert_allclose(M0, ref, rtol=1e-12, atol=1e-12)
    # and, up to the FP32 rounding of X, the separable form a * (b.u1) * (c.u2)
    sep = np.outer(a, (b @ U[1].astype(np.float64)) * (cc @ U[2].astype(np.float64)))
    np.testing.assert_allclose(M0, sep, rtol=1e-5, atol=1e-5)


def test_empty_tensor_and_empty_rows():
    dims = (4, 3, 2)
    F = [np.ones((d, 2), np.float32) for d in dims]
    out = oracle.mttkrp(np.zeros((3, 0), np.uint32), np.zeros(0, np.float32), dims, F, 1)
    assert out.shape == (3, 2) and not out.any()
    c = np.array([[1], [2], [0]], np.uint32)
    out = oracle.mttkrp(c, np.array([2.0], np.float32), dims, F, 0)
    assert out[1, 0] == 2.0 and out[[0, 2, 3]].sum() == 0


def test_row_error_metric():
    ref = np.array([[1.0, -1.0], [0.0, 0.0]])
    scale = np.array([[2.0, 2.0], [0.0, 0.0]])
    err, bad = oracle.row_error(np.array([[1.0002, -1.0], [0.0, 0.0]]), ref, scale)
    assert abs(err - 1e-4) < 1e-12 and bad == 0
    _, bad = oracle.row_error(np.array([[1.0, -1.0], [0.0, 1e-30]]), ref, scale)
    assert bad == 1


def test_f64_values_brute_force_and_fp32_agreement():
    """The FP64-valued oracle: brute force (dense unfolding x Khatri-Rao) with
    values not representable in FP32, and equality with the FP32-valued routine
    when the values are FP32-exact."""
    rng = np.random.default_rng(12)
    dims = (5, 4, 3)
    X = rng.standard_normal(dims) / 3.0            # FP64 values, not FP32-exact
    X[rng.random(dims) < 0.4] = 0.0
    coords = np.stack(np.nonzero(X)).astype(np.uint32)
    vals = X[tuple(coords)]
    F = [rng.standard_normal((d, 3)) for d in dims]
    for mode in range(3):
        got = oracle.mttkrp_f64vals(coords, vals, dims, F, mode)
        others = [k for k in range(3) if k != mode]
        Xn = np.moveaxis(X, mode, 0).reshape(dims[mode], -1)       # C order: last mode fastest
        K = np.einsum("ir,jr->ijr", F[others[0]], F[others[1]]).reshape(-1, 3)  # forward KRP, second fastest
        np.testing.assert_allclose(got, Xn @ K, rtol=1e-12, atol=1e-13)
        v32 = vals.astype(np.float32)
        np.testing.assert_array_equal(oracle.mttkrp_f64vals(coords, v32.astype(np.float64), dims, F, mode),
                                      oracle.mttkrp(coords, v32, dims, F, mode))
