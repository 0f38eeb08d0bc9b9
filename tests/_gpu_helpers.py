"""Helpers shared by the GPU parity tests (upload, oracle comparison)."""
import numpy as np

import oracle


def to_dev(t):
    import torch
    coords = torch.from_numpy(np.ascontiguousarray(t.coords).view(np.int32)).cuda()
    vals = torch.from_numpy(np.ascontiguousarray(t.vals)).cuda()
    return coords, vals


def factors_dev(factors):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(f)).cuda() for f in factors]


def mttkrp_error(t, factors, mode, got):
    """Max row error of the GPU output against the FP64 oracle, relative to the |X|,|C| row scale."""
    ref = oracle.mttkrp(t.coords, t.vals, t.dims, factors, mode)
    scale = oracle.mttkrp(t.coords, np.abs(t.vals), t.dims, [np.abs(f) for f in factors], mode)
    return oracle.row_error(got, ref, scale)


def check_encoding(h, t, layout=None):
    """Keys, values, perm and decoded coordinates must equal the oracle bit for bit."""
    enc = oracle.encode(t.coords, t.vals, t.dims, layout)
    keys, vals, perm = h.export()
    assert keys.shape[1] == enc["key_words"]
    np.testing.assert_array_equal(keys[:, 0], enc["lo"])
    if enc["key_words"] == 2:
        np.testing.assert_array_equal(keys[:, 1], enc["hi"])
    np.testing.assert_array_equal(perm.astype(np.int64), enc["perm"])
    np.testing.assert_array_equal(vals.view(np.uint32), np.asarray(enc["vals"], np.float32).view(np.uint32))
    np.testing.assert_array_equal(h.decode(), enc["coords"])
    info = h.info()
    assert info["layout"] == enc["layout"]
    assert info["encoded_bytes"] == t.nnz * (8 * enc["key_words"] + 4)
    return enc


def cpd_error(F_got, lam_got, F_ref, lam_ref):
    """Largest per-factor error of two CP decompositions on the same trajectory.

    For every mode the lambda-scaled factor A = C diag(lambda) is compared row
    by row: max_i ||A_got[i] - A_ref[i]||_inf / max_i ||A_ref[i]||_inf (the
    row error relative to the factor's largest row).  Returns (max over
    modes, lambda error max_r |dlambda_r| / max_r lambda_r).
    """
    lg = np.asarray(lam_got, dtype=np.float64)
    lr = np.asarray(lam_ref, dtype=np.float64)
    errs = []
    for g, r in zip(F_got, F_ref):
        A = np.asarray(g, dtype=np.float64) * lg[None, :]
        B = np.asarray(r, dtype=np.float64) * lr[None, :]
        errs.append(float(np.abs(A - B).max(initial=0.0) / max(np.abs(B).max(initial=0.0), 1e-300)))
    return max(errs), float(np.abs(lg - lr).max() / lr.max())


def to_host(F):
    """Device factors to float32 numpy arrays."""
    return [f.detach().cpu().numpy() for f in F]


def mttkrp_error_compact(t, factors, mode, got):
    """mttkrp_error for tensors with huge modes: the oracle runs on the tensor with
    every mode relabelled to its touched rows (factor rows taken along), which
    gives the same rows; every untouched output row must be exactly zero."""
    coords = np.empty_like(t.coords)
    F = []
    for k in range(t.nmodes):
        u, inv = np.unique(t.coords[k], return_inverse=True)
        coords[k] = inv.astype(np.uint32)
        F.append(np.ascontiguousarray(factors[k][u]))
        if k == mode:
            rows = u
    dims = [f.shape[0] for f in F]
    ref = oracle.mttkrp(coords, t.vals, dims, F, mode)
    scale = oracle.mttkrp(coords, np.abs(t.vals), dims, [np.abs(f) for f in F], mode)
    err, bad = oracle.row_error(got[rows], ref, scale)
    mask = np.ones(got.shape[0], dtype=bool)
    mask[rows] = False
    bad += int(np.count_nonzero(np.abs(got[mask]).max(axis=1, initial=0.0) != 0)) if mask.any() else 0
    return err, bad
