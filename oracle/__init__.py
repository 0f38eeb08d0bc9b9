"""Oracle for the sparse MTTKRP / CP-ALS path — TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU reference of what the GPU library
computes.  Only ``tests/``, the package's smoke check and the benchmark's
CPU-baseline leg import it; the product path never does, and this package
imports nothing from the product (only the seeded generators are shared,
and they live in a module that holds none of the method's arithmetic).

Floating point is FP64 throughout (the paper's own precision, Section IV-A).
MTTKRP is the C routine in ``oracle.c`` (plain loops, -O2); everything else
is numpy/scipy written step by step from the definitions:

* bit lengths and the linear encoding: Section III-C (problem formulation);
* the default (ALTO) interleaving: Section III-C, the sentence on
  partitioning the longest mode first, pinned by the Fig. 5 example;
* the encoding-space count: Eq. (1);
* MTTKRP: Section II-B and Fig. 2;
* CP-ALS: Section II-B defers to Kolda and Bader; the steps below are the
  standard ALS with column 2-norm normalisation (readings listed in
  ``READINGS``).

Every function is pinned by ``tests/test_oracle_*.py`` against brute force,
closed forms, library routines or the paper's worked example; none is
"parity unpinned".
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import scipy.linalg

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

READINGS = {
    "alto_ties": "modes with equal bit length enter a level in ascending mode index",
    "unit_mode": "a mode of length 1 has 0 bits and contributes nothing to the key",
    "key_width": "64-bit keys when l(p) <= 64, two 64-bit words (low word first) up to 128, error beyond",
    "duplicates": "equal keys keep input order (stable sort); duplicates stay separate elements",
    "mttkrp_output": "a separate I_n x R output, zeroed then accumulated",
    "als": "Gauss-Seidel over modes 0..N-1, Cholesky of the Hadamard product of the other Grams, "
           "column 2-norm normalisation every iteration (lambda=1 kept for a zero column), "
           "ridge 1e-12*tr(V)/R*1e3^k on the k-th retry (3 retries) if V is not positive definite",
    "fit": "fit = 1 - sqrt(max(0, |X|^2 + |Xhat|^2 - 2<X,Xhat>)) / |X| with <X,Xhat> taken from the "
           "last mode's MTTKRP; stop when tol > 0 and |fit - previous fit| < tol (previous starts at 0)",
}


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        lib.oracle_mttkrp.restype = ctypes.c_int
        lib.oracle_mttkrp.argtypes = [
            ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.oracle_mttkrp_f64vals.restype = ctypes.c_int
        lib.oracle_mttkrp_f64vals.argtypes = lib.oracle_mttkrp.argtypes
        _LIB = lib
    return _LIB


# --------------------------------------------------------------------------
# Section III-C: bit lengths, layouts and the linear encoding
# --------------------------------------------------------------------------

def bit_lengths(dims) -> list:
    """l(n) = ceil(log2 I_n) for every mode (0 for a mode of length 1)."""
    out = []
    for d in dims:
        d = int(d)
        if d < 1:
            raise ValueError("mode length must be >= 1")
        out.append((d - 1).bit_length())
    return out


def key_words(dims) -> int:
    """Number of 64-bit words of a key: l(p) = sum l(n) bits, 1 word up to 64, 2 up to 128."""
    lp = sum(bit_lengths(dims))
    if lp > 128:
        raise ValueError("l(p) > 128 bits is not representable")
    return 1 if lp <= 64 else 2


def alto_layout(dims) -> list:
    """Default interleaving: level by level, shortest mode first.

    Partitioning the longest mode first is the same as interleaving bits
    starting with the shortest mode (Section III-C).  At level j every mode
    with l(n) > j contributes its j-th bit, modes taken in ascending
    (l(n), n) order.  Returns L with L[t] = the mode whose next low bit
    becomes key bit b^t.
    """
    lb = bit_lengths(dims)
    order = sorted(range(len(dims)), key=lambda n: (lb[n], n))
    L = []
    for j in range(max(lb, default=0)):
        for n in order:
            if j < lb[n]:
                L.append(n)
    return L


def is_valid_layout(L, dims) -> bool:
    """A terminal encoding: every mode n appears exactly l(n) times (action masking, Section III-D)."""
    lb = bit_lengths(dims)
    if len(L) != sum(lb):
        return False
    counts = [0] * len(dims)
    for m in L:
        if not (0 <= int(m) < len(dims)):
            return False
        counts[int(m)] += 1
    return counts == lb


def bit_positions(L, nmodes) -> list:
    """pos[n][j] = key bit that holds bit j of coordinate i_n (the "next low bit" rule of Fig. 5)."""
    pos = [[] for _ in range(nmodes)]
    for t, m in enumerate(L):
        pos[int(m)].append(t)
    return pos


def encode_keys(coords: np.ndarray, dims, L=None):
    """Positions p of every nonzero, in input order.

    Key bit b^t takes the next unused low bit of coordinate i_{L[t]}.
    Returns (lo, hi) uint64 arrays (hi is all zero when l(p) <= 64).
    Raises ValueError when a coordinate is out of range.
    """
    dims = [int(d) for d in dims]
    if L is None:
        L = alto_layout(dims)
    if not is_valid_layout(L, dims):
        raise ValueError("invalid layout")
    key_words(dims)
    coords = np.asarray(coords)
    nnz = coords.shape[1]
    for n, d in enumerate(dims):
        if nnz and int(coords[n].max()) >= d:
            raise ValueError(f"coordinate out of range in mode {n}")
    lo = np.zeros(nnz, dtype=np.uint64)
    hi = np.zeros(nnz, dtype=np.uint64)
    used = [0] * len(dims)
    for t, m in enumerate(L):
        m = int(m)
        bit = (coords[m].astype(np.uint64) >> np.uint64(used[m])) & np.uint64(1)
        used[m] += 1
        if t < 64:
            lo |= bit << np.uint64(t)
        else:
            hi |= bit << np.uint64(t - 64)
    return lo, hi


def decode_keys(lo: np.ndarray, hi: np.ndarray, dims, L=None) -> np.ndarray:
    """Inverse of ``encode_keys``: coordinates (nmodes x nnz, uint32) of each key."""
    dims = [int(d) for d in dims]
    if L is None:
        L = alto_layout(dims)
    nnz = lo.shape[0]
    out = np.zeros((len(dims), nnz), dtype=np.uint64)
    used = [0] * len(dims)
    for t, m in enumerate(L):
        m = int(m)
        word = lo if t < 64 else hi
        bit = (word >> np.uint64(t % 64)) & np.uint64(1)
        out[m] |= bit << np.uint64(used[m])
        used[m] += 1
    return out.astype(np.uint32)


def encode(coords: np.ndarray, vals: np.ndarray, dims, L=None) -> dict:
    """The linearized tensor: nonzeros ordered by position p (Section III-C).

    The sort is stable, so equal positions keep input order.  Returns the
    sorted key words, the values in that order, ``perm`` (original index of
    each sorted element) and the decoded coordinates.
    """
    lo, hi = encode_keys(coords, dims, L)
    perm = np.lexsort((lo, hi)).astype(np.int64)  # primary hi, then lo; ties stay in input order
    s_lo, s_hi = lo[perm], hi[perm]
    return {
        "lo": s_lo, "hi": s_hi, "vals": np.asarray(vals)[perm], "perm": perm,
        "coords": decode_keys(s_lo, s_hi, dims, L),
        "layout": list(alto_layout(dims) if L is None else L),
        "key_words": key_words(dims),
    }


# --------------------------------------------------------------------------
# Section II-B: MTTKRP (C routine) and CP-ALS
# --------------------------------------------------------------------------

def mttkrp(coords: np.ndarray, vals: np.ndarray, dims, factors, mode: int) -> np.ndarray:
    """FP64 mode-``mode`` MTTKRP of a COO tensor (see ``oracle.c``)."""
    dims_a = (ctypes.c_int64 * len(dims))(*[int(d) for d in dims])
    coords = np.ascontiguousarray(coords, dtype=np.uint32)
    vals = np.ascontiguousarray(vals, dtype=np.float32)
    f64 = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
    rank = int(f64[0].shape[1])
    for n, f in enumerate(f64):
        if f.shape != (int(dims[n]), rank):
            raise ValueError("factor shape mismatch")
    ptrs = (ctypes.c_void_p * len(f64))(*[f.ctypes.data for f in f64])
    out = np.empty((int(dims[mode]), rank), dtype=np.float64)
    nnz = int(vals.shape[0])
    rc = _lib().oracle_mttkrp(len(dims), dims_a, nnz, coords.ctypes.data if nnz else None,
                              vals.ctypes.data if nnz else None, ptrs, rank, int(mode),
                              out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_mttkrp failed ({rc})")
    return out


def mttkrp_f64vals(coords: np.ndarray, vals: np.ndarray, dims, factors, mode: int) -> np.ndarray:
    """``mttkrp`` with FP64 values (the paper's precision), see ``oracle.c``."""
    dims_a = (ctypes.c_int64 * len(dims))(*[int(d) for d in dims])
    coords = np.ascontiguousarray(coords, dtype=np.uint32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    f64 = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
    rank = int(f64[0].shape[1])
    for n, f in enumerate(f64):
        if f.shape != (int(dims[n]), rank):
            raise ValueError("factor shape mismatch")
    ptrs = (ctypes.c_void_p * len(f64))(*[f.ctypes.data for f in f64])
    out = np.empty((int(dims[mode]), rank), dtype=np.float64)
    nnz = int(vals.shape[0])
    rc = _lib().oracle_mttkrp_f64vals(len(dims), dims_a, nnz, coords.ctypes.data if nnz else None,
                                      vals.ctypes.data if nnz else None, ptrs, rank, int(mode), out.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_mttkrp_f64vals failed ({rc})")
    return out


def _cholesky_ridge(V: np.ndarray):
    """Cholesky factor of V, retrying with a growing ridge if V is not positive definite."""
    R = V.shape[0]
    base = 1e-12 * float(np.trace(V)) / R
    for k in range(4):
        W = V if k == 0 else V + (base * 1e3 ** (k - 1)) * np.eye(R)
        try:
            return scipy.linalg.cholesky(W, lower=True), k
        except np.linalg.LinAlgError:
            continue
    raise np.linalg.LinAlgError("normal-equation matrix is not positive definite")


def als_update(M: np.ndarray, grams, mode: int):
    """One ALS mode update: C = M V^-1 with V the Hadamard product of the other Grams,
    then column 2-norm normalisation.  Returns (C, lam)."""
    R = M.shape[1]
    V = np.ones((R, R))
    for k, G in enumerate(grams):
        if k != mode:
            V = V * G
    Lc, _ = _cholesky_ridge(V)
    # C V = M  <=>  V C^T = M^T  (V symmetric)
    Y = scipy.linalg.solve_triangular(Lc, M.T, lower=True)
    C = scipy.linalg.solve_triangular(Lc.T, Y, lower=False).T
    lam = np.sqrt((C * C).sum(axis=0))
    lam_safe = np.where(lam > 0, lam, 1.0)
    return C / lam_safe, lam_safe


def fit_value(normX2: float, grams, lam, M_last, C_last) -> float:
    """CP fit from the Grams and the last mode's MTTKRP (no dense reconstruction)."""
    R = lam.shape[0]
    V = np.ones((R, R))
    for G in grams:
        V = V * G
    normXhat2 = float(lam @ V @ lam)
    inner = float(((M_last * C_last).sum(axis=0) * lam).sum())
    resid2 = max(0.0, normX2 + normXhat2 - 2.0 * inner)
    return 1.0 - np.sqrt(resid2) / np.sqrt(normX2)


def cp_als(coords, vals, dims, factors0, iters: int, tol: float = 0.0, record=False):
    """CP-ALS from caller-supplied initial factors (FP32 values widened to FP64).

    Returns dict(factors, lam, fit, iters, fits).
    """
    vals64 = np.asarray(vals, dtype=np.float64)
    normX2 = float((vals64 * vals64).sum())
    if normX2 == 0.0:
        raise ValueError("tensor norm is zero")
    N = len(dims)
    C = [np.array(f, dtype=np.float64) for f in factors0]
    R = C[0].shape[1]
    grams = [c.T @ c for c in C]
    lam = np.ones(R)
    fit_prev = 0.0
    fits = []
    it = 0
    fit = 0.0
    while it < iters:
        M = None
        for n in range(N):
            M = mttkrp(coords, vals, dims, C, n)
            C[n], lam = als_update(M, grams, n)
            grams[n] = C[n].T @ C[n]
        fit = fit_value(normX2, grams, lam, M, C[N - 1])
        fits.append(fit)
        it += 1
        if tol > 0 and abs(fit - fit_prev) < tol:
            break
        fit_prev = fit
    return {"factors": C, "lam": lam, "fit": fit, "iters": it, "fits": fits}


def row_error(got: np.ndarray, ref: np.ndarray, scale: np.ndarray):
    """Max row error of ``got`` against ``ref`` relative to the row's absolute-sum scale.

    ``scale`` is the MTTKRP of |X| with |C^(k)| (same oracle routine).  Rows
    whose scale is 0 (no nonzeros, or all-zero factor rows) must be exactly
    zero in ``got``; they are reported separately.
    """
    got = np.asarray(got, dtype=np.float64)
    d = np.abs(got - ref).max(axis=1)
    s = np.abs(scale).max(axis=1)
    empty = s == 0
    rel = np.where(empty, 0.0, d / np.where(empty, 1.0, s))
    bad_empty = int(np.count_nonzero(np.abs(got[empty]).max(axis=1) != 0)) if empty.any() else 0
    return float(rel.max(initial=0.0)), bad_empty
