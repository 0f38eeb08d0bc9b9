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
