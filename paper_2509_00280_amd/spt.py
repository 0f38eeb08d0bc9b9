"""Thin ctypes binding of ``libspt.so`` (C-ABI in ``include/spt.h``).

Argument marshalling only: every step of MTTKRP / CP-ALS runs in the HIP
library.  Device buffers are torch CUDA tensors (PyTorch is used for device
memory and streams); their data pointers go straight to the library.  There
is no fallback: if the library is missing every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspt.so")
MAX_MODES = 8

STRATEGY_DIRECT = 0
STRATEGY_REGROUP = 1

STATUS = {0: "SPT_OK", -1: "SPT_E_INVALID_ARG", -2: "SPT_E_INDEX_RANGE", -3: "SPT_E_TOO_MANY_BITS",
          -4: "SPT_E_BAD_LAYOUT", -5: "SPT_E_OOM", -6: "SPT_E_NOT_SPD", -7: "SPT_E_DEVICE", -8: "SPT_E_BUSY",
          -9: "SPT_E_NOT_FOUND"}


class SptError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class TensorInfo(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("nmodes", ctypes.c_int), ("lp", ctypes.c_int),
                ("key_words", ctypes.c_int), ("dims", ctypes.c_int64 * MAX_MODES),
                ("lbits", ctypes.c_int * MAX_MODES), ("layout", ctypes.c_uint8 * 128),
                ("encoded_bytes", ctypes.c_size_t), ("norm_x2", ctypes.c_double)]


class Plan(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int * MAX_MODES), ("strategy", ctypes.c_int * MAX_MODES), ("row_cache", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("nmodes", ctypes.c_int), ("dims", ctypes.c_int64 * MAX_MODES), ("nnz", ctypes.c_int64),
                ("coords", ctypes.c_void_p), ("vals", ctypes.c_void_p), ("init", ctypes.POINTER(ctypes.c_void_p)),
                ("rank", ctypes.c_int), ("max_iters", ctypes.c_int), ("tol", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("fit", ctypes.c_double), ("iters", ctypes.c_int),
                ("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


_LIB = None
_VP = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)


def _sig(lib, name, restype, argtypes):
    try:
        f = getattr(lib, name)
    except AttributeError:
        return  # calling it raises AttributeError, naming the missing entry point
    f.restype = restype
    f.argtypes = argtypes


def lib():
    """The loaded library (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    i, i64, d, st = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    _sig(L, "spt_last_error", ctypes.c_char_p, [])
    _sig(L, "spt_version", ctypes.c_char_p, [])
    _sig(L, "spt_encode", st, [ctypes.POINTER(i64), i, _VP, _VP, i64, _VP, i, _VP, ctypes.POINTER(_VP)])
    _sig(L, "spt_tensor_get_info", st, [_VP, ctypes.POINTER(TensorInfo)])
    _sig(L, "spt_tensor_export", st, [_VP, _VP, _VP, _VP, _VP])
    _sig(L, "spt_tensor_decode", st, [_VP, _VP, _VP])
    _sig(L, "spt_tensor_get_plan", st, [_VP, ctypes.POINTER(Plan)])
    _sig(L, "spt_tensor_set_plan", st, [_VP, ctypes.POINTER(Plan)])
    _sig(L, "spt_tensor_free", None, [_VP])
    _sig(L, "spt_mttkrp", st, [_VP, _PP, i, i, _VP, _VP])
    _sig(L, "spt_cp_als", st, [_VP, i, i, d, _PP, _VP, ctypes.POINTER(d), ctypes.POINTER(i), _VP])
    _sig(L, "spt_mttkrp_batched", st, [_PP, i, ctypes.POINTER(_PP), ctypes.POINTER(i), i, _PP, _VP])
    _sig(L, "spt_cp_als_batched", st, [_PP, i, ctypes.POINTER(i), i, d, ctypes.POINTER(_PP), _PP,
                                       ctypes.POINTER(d), ctypes.POINTER(i), _VP])
    _sig(L, "spt_autotune", st, [ctypes.POINTER(_VP), _PP, i, d, ctypes.POINTER(d), _VP])
    _sig(L, "spt_server_create", st, [ctypes.c_size_t, i, ctypes.POINTER(_VP)])
    _sig(L, "spt_server_submit", st, [_VP, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)])
    _sig(L, "spt_server_wait", st, [_VP, ctypes.c_uint64, d, ctypes.POINTER(Result), _PP, _VP])
    _sig(L, "spt_server_now", d, [_VP])
    _sig(L, "spt_server_destroy", None, [_VP])
    _sig(L, "spt_profile_enable", st, [i])
    _sig(L, "spt_profile_read", st, [ctypes.POINTER(d), ctypes.POINTER(i64)])
    _LIB = L
    return L


def _check(status: int):
    if status != 0:
        raise SptError(status, lib().spt_last_error().decode(errors="replace"))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _ptr_array(tensors):
    return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() if t is not None else 0 for t in tensors])


class Tensor:
    """An encoded sparse tensor living on the GPU (owns an spt_tensor handle)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = TensorInfo()
        _check(lib().spt_tensor_get_info(self._h, ctypes.byref(inf)))
        nm = inf.nmodes
        return {"nnz": inf.nnz, "nmodes": nm, "lp": inf.lp, "key_words": inf.key_words,
                "dims": tuple(inf.dims[:nm]), "lbits": tuple(inf.lbits[:nm]),
                "layout": list(inf.layout[:inf.lp]), "encoded_bytes": inf.encoded_bytes,
                "norm_x2": inf.norm_x2}

    def export(self, stream=None):
        """(keys uint64 [nnz, key_words] numpy, vals float32, perm uint32) copied to the host."""
        import torch
        inf = self.info()
        n, kw = inf["nnz"], inf["key_words"]
        keys = torch.empty(max(n * kw, 1), dtype=torch.int64, device="cuda")
        vals = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        perm = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        _check(lib().spt_tensor_export(self._h, _ptr(keys), _ptr(vals), _ptr(perm), _stream(stream)))
        torch.cuda.synchronize()
        k = keys.cpu().numpy().view(np.uint64)[: n * kw].reshape(n, kw)
        return k, vals.cpu().numpy()[:n], perm.cpu().numpy().view(np.uint32)[:n]

    def decode(self, stream=None) -> np.ndarray:
        import torch
        inf = self.info()
        n, nm = inf["nnz"], inf["nmodes"]
        out = torch.empty(max(n * nm, 1), dtype=torch.int32, device="cuda")
        _check(lib().spt_tensor_decode(self._h, _ptr(out), _stream(stream)))
        torch.cuda.synchronize()
        return out.cpu().numpy().view(np.uint32)[: n * nm].reshape(nm, n)

    def get_plan(self) -> dict:
        p = Plan()
        _check(lib().spt_tensor_get_plan(self._h, ctypes.byref(p)))
        return {"tile": list(p.tile), "strategy": list(p.strategy), "row_cache": int(p.row_cache)}

    def set_plan(self, tile=None, strategy=None, row_cache=None):
        p = Plan()
        _check(lib().spt_tensor_get_plan(self._h, ctypes.byref(p)))
        for n in range(MAX_MODES):
            if tile is not None:
                p.tile[n] = tile[n] if isinstance(tile, (list, tuple)) and n < len(tile) else (
                    tile if isinstance(tile, int) else p.tile[n])
            if strategy is not None:
                p.strategy[n] = strategy[n] if isinstance(strategy, (list, tuple)) and n < len(strategy) else (
                    strategy if isinstance(strategy, int) else p.strategy[n])
        if row_cache is not None:
            p.row_cache = 1 if row_cache else 0
        _check(lib().spt_tensor_set_plan(self._h, ctypes.byref(p)))

    def free(self):
        if self._h is not None and self._h.value:
            lib().spt_tensor_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def encode(dims, coords, vals, layout=None, stream=None) -> Tensor:
    """Encode a COO tensor held in device memory.

    coords: torch CUDA int32/uint32 tensor of shape (nmodes, nnz) (bits are read as uint32).
    vals:   torch CUDA float32 tensor of shape (nnz,).
    """
    nm = len(dims)
    d = (ctypes.c_int64 * nm)(*[int(x) for x in dims])
    nnz = int(vals.numel())
    lay = None
    lay_len = 0
    if layout is not None:
        lay = (ctypes.c_uint8 * max(len(layout), 1))(*[int(x) for x in layout])
        lay_len = len(layout)
    h = ctypes.c_void_p()
    _check(lib().spt_encode(d, nm, _ptr(coords) if nnz else None, _ptr(vals) if nnz else None, nnz,
                            ctypes.cast(lay, ctypes.c_void_p) if lay is not None else None, lay_len,
                            _stream(stream), ctypes.byref(h)))
    return Tensor(h)


def mttkrp(t: Tensor, factors, mode: int, out=None, stream=None):
    """out[I_mode, R] = MTTKRP of mode ``mode`` (factors: list of CUDA float32 [I_k, R])."""
    import torch
    R = int(factors[0].shape[1] if factors[0] is not None else factors[1].shape[1])
    if out is None:
        dims = t.info()["dims"]
        rows = dims[mode] if 0 <= mode < len(dims) else 1  # an invalid mode is rejected by the library
        out = torch.empty((rows, R), dtype=torch.float32, device="cuda")
    _check(lib().spt_mttkrp(t.handle, _ptr_array(factors), R, int(mode), _ptr(out), _stream(stream)))
    return out


def cp_als(t: Tensor, factors, iters: int, tol: float = 0.0, lam=None, stream=None):
    """Run CP-ALS in place on ``factors``; returns (lambda tensor, fit, iterations)."""
    import torch
    R = int(factors[0].shape[1])
    if lam is None:
        lam = torch.empty(R, dtype=torch.float64, device="cuda")
    fit = ctypes.c_double()
    its = ctypes.c_int()
    _check(lib().spt_cp_als(t.handle, R, int(iters), float(tol), _ptr_array(factors), _ptr(lam),
                            ctypes.byref(fit), ctypes.byref(its), _stream(stream)))
    return lam, fit.value, its.value


def mttkrp_batched(tensors, factor_lists, mode: int, outs, stream=None):
    count = len(tensors)
    hs = (ctypes.c_void_p * count)(*[t.handle.value for t in tensors])
    farrs = [_ptr_array(fl) for fl in factor_lists]
    fptrs = (_PP * count)(*[ctypes.cast(a, _PP) for a in farrs])
    ranks = (ctypes.c_int * count)(*[int(fl[0].shape[1]) for fl in factor_lists])
    optrs = _ptr_array(outs)
    _check(lib().spt_mttkrp_batched(hs, count, fptrs, ranks, int(mode), optrs, _stream(stream)))
    return outs


def cp_als_batched(tensors, factor_lists, iters: int, tol: float = 0.0, lams=None, stream=None):
    import torch
    count = len(tensors)
    hs = (ctypes.c_void_p * count)(*[t.handle.value for t in tensors])
    farrs = [_ptr_array(fl) for fl in factor_lists]
    fptrs = (_PP * count)(*[ctypes.cast(a, _PP) for a in farrs])
    ranks = (ctypes.c_int * count)(*[int(fl[0].shape[1]) for fl in factor_lists])
    if lams is None:
        lams = [torch.empty(int(fl[0].shape[1]), dtype=torch.float64, device="cuda") for fl in factor_lists]
    lptrs = _ptr_array(lams)
    fits = (ctypes.c_double * count)()
    its = (ctypes.c_int * count)()
    _check(lib().spt_cp_als_batched(hs, count, ranks, int(iters), float(tol), fptrs, lptrs, fits, its,
                                    _stream(stream)))
    return lams, list(fits), list(its)


def autotune(t: Tensor, factors, budget_ms: float = 2000.0, stream=None):
    R = int(factors[0].shape[1])
    h = ctypes.c_void_p(t.handle.value)
    best = ctypes.c_double()
    _check(lib().spt_autotune(ctypes.byref(h), _ptr_array(factors), R, float(budget_ms), ctypes.byref(best),
                              _stream(stream)))
    t._h = h
    return best.value


class Server:
    """Continuous-batching CP-ALS server (one per process and GPU is typical).

    ``submit`` copies a COO tensor (host numpy arrays) and its initial factors
    and returns a ticket; ``wait`` returns the result and, on success, the
    normalised factors and lambda as numpy arrays.
    """

    def __init__(self, hbm_budget_bytes: int, max_slots: int):
        h = ctypes.c_void_p()
        _check(lib().spt_server_create(ctypes.c_size_t(int(hbm_budget_bytes)), int(max_slots), ctypes.byref(h)))
        self._h = h
        self._meta = {}

    def submit(self, dims, coords, vals, init, max_iters: int, tol: float = 0.0) -> int:
        import numpy as np
        nm = len(dims)
        coords = np.ascontiguousarray(coords, dtype=np.uint32)
        vals = np.ascontiguousarray(vals, dtype=np.float32)
        init = [np.ascontiguousarray(f, dtype=np.float32) for f in init]
        rank = int(init[0].shape[1])
        r = Request()
        r.nmodes = nm
        for k in range(nm):
            r.dims[k] = int(dims[k])
        r.nnz = int(vals.shape[0])
        r.coords = coords.ctypes.data
        r.vals = vals.ctypes.data
        iptr = (ctypes.c_void_p * nm)(*[f.ctypes.data for f in init])
        r.init = ctypes.cast(iptr, _PP)
        r.rank = rank
        r.max_iters = int(max_iters)
        r.tol = float(tol)
        ticket = ctypes.c_uint64()
        _check(lib().spt_server_submit(self._h, ctypes.byref(r), ctypes.byref(ticket)))
        self._meta[ticket.value] = (tuple(int(d) for d in dims), rank)
        return ticket.value

    def wait(self, ticket: int, timeout_s: float = -1.0, want_factors: bool = True):
        import numpy as np
        dims, rank = self._meta.get(ticket, ((), 0))
        want_factors = want_factors and rank > 0
        res = Result()
        outs = [np.empty((d, rank), np.float32) for d in dims] if want_factors else None
        lam = np.empty(rank, np.float64) if want_factors else None
        fptr = (ctypes.c_void_p * len(dims))(*[o.ctypes.data for o in outs]) if want_factors else None
        _check(lib().spt_server_wait(self._h, ctypes.c_uint64(ticket), float(timeout_s), ctypes.byref(res),
                                     ctypes.cast(fptr, _PP) if fptr is not None else None,
                                     lam.ctypes.data if lam is not None else None))
        self._meta.pop(ticket, None)
        out = {"status": res.status, "fit": res.fit, "iters": res.iters, "t_arrive": res.t_arrive,
               "t_admit": res.t_admit, "t_done": res.t_done}
        return out, outs, lam

    def now(self) -> float:
        return lib().spt_server_now(self._h)

    def close(self):
        if self._h is not None:
            lib().spt_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_reset(on: bool = True):
    """Clear recorded MTTKRP timings and (re)enable event timing."""
    _check(lib().spt_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """Per-mode summed MTTKRP GPU time (ms) and launch counts since the last reset."""
    ms = (ctypes.c_double * MAX_MODES)()
    n = (ctypes.c_int64 * MAX_MODES)()
    _check(lib().spt_profile_read(ms, n))
    return {"mttkrp_ms": list(ms), "mttkrp_launches": list(n)}


def version() -> str:
    return lib().spt_version().decode()
