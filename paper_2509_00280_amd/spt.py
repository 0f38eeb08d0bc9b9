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
    _fields_ = [("tile", ctypes.c_int * MAX_MODES), ("strategy", ctypes.c_int * MAX_MODES), ("row_cache", ctypes.c_int),
                ("batch_tile", ctypes.c_int)]


class BatchTuneResult(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 3), ("best_tile", ctypes.c_int), ("layouts_tuned", ctypes.c_int),
                ("layout_speedup", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("best_ms", ctypes.c_double), ("alto_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("candidates", ctypes.c_int), ("random_samples", ctypes.c_int), ("cache_hits", ctypes.c_int),
                ("pad", ctypes.c_int)]


PREPARE_SINGLE = 1
PREPARE_BATCHED = 2

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


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
    _sig(L, "spt_tensor_set_plan", st, [_VP, ctypes.POINTER(Plan), _VP])
    _sig(L, "spt_tensor_prepare", st, [_VP, i, i, _VP])
    _sig(L, "spt_tensor_free", None, [_VP, _VP])
    _sig(L, "spt_set_allocator", st, [ALLOC_FN, RELEASE_FN, _VP])
    _sig(L, "spt_mttkrp", st, [_VP, _PP, i, i, _VP, _VP])
    _sig(L, "spt_mttkrp_noalloc", st, [_VP, _PP, i, i, _VP, _VP])
    _sig(L, "spt_tensor_attach_f64", st, [_VP, _VP, _VP])
    _sig(L, "spt_mttkrp_f64", st, [_VP, _PP, i, i, _VP, _VP])
    _sig(L, "spt_cp_als", st, [_VP, i, i, d, _PP, _VP, ctypes.POINTER(d), ctypes.POINTER(i), _VP])
    _sig(L, "spt_als_update", st, [_VP, i, i, i, _VP, i64, _VP, _VP, ctypes.POINTER(i), _VP])
    _sig(L, "spt_mttkrp_batched", st, [_PP, i, ctypes.POINTER(_PP), ctypes.POINTER(i), i, _PP, _VP])
    _sig(L, "spt_cp_als_batched", st, [_PP, i, ctypes.POINTER(i), i, d, ctypes.POINTER(_PP), _PP,
                                       ctypes.POINTER(d), ctypes.POINTER(i), _VP])
    _sig(L, "spt_autotune", st, [ctypes.POINTER(_VP), _PP, i, d, i, ctypes.c_uint64, ctypes.POINTER(TuneResult),
                                 _VP])
    _sig(L, "spt_autotune_batched", st, [_PP, i, ctypes.POINTER(_PP), ctypes.POINTER(i), d, i, ctypes.c_uint64,
                                         ctypes.POINTER(BatchTuneResult), _VP])
    _sig(L, "spt_server_create", st, [ctypes.c_size_t, i, ctypes.POINTER(_VP)])
    _sig(L, "spt_server_submit", st, [_VP, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)])
    _sig(L, "spt_server_wait", st, [_VP, ctypes.c_uint64, d, ctypes.POINTER(Result), _PP, _VP])
    _sig(L, "spt_server_now", d, [_VP])
    _sig(L, "spt_server_simulate", st, [ctypes.c_size_t, i, i, _VP, _VP, _VP, _VP, _VP, _VP])
    _sig(L, "spt_server_destroy", None, [_VP])
    _sig(L, "spt_profile_enable", st, [i])
    _sig(L, "spt_profile_read", st, [ctypes.POINTER(d), ctypes.POINTER(i64)])
    _sig(L, "spt_memory_stats", st, [ctypes.POINTER(i64)])
    _sig(L, "spt_empty_cache", st, [])
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


# ---------------------------------------------------------------- argument checks
# The C side sees only pointers, so the binding checks what it can before a
# call: dtype, shape, one rank for every factor, contiguity and the device.
# A mismatch raises ValueError and nothing reaches the library.

def _is_torch(x) -> bool:
    try:
        import torch
    except ImportError:
        return False
    return isinstance(x, torch.Tensor)


def check_matrix(name: str, x, rows, cols, dtype: str = "float32", device: str = "cuda"):
    """A row-major (rows, cols) tensor of ``dtype`` on ``device`` (rows/cols None: any)."""
    if not _is_torch(x):
        raise ValueError(f"{name}: expected a torch tensor, got {type(x).__name__}")
    if str(x.dtype) != f"torch.{dtype}":
        raise ValueError(f"{name}: dtype must be {dtype}, got {x.dtype}")
    if x.dim() != 2 or (rows is not None and int(x.shape[0]) != int(rows)) or (
            cols is not None and int(x.shape[1]) != int(cols)):
        raise ValueError(f"{name}: shape must be ({rows}, {cols}), got {tuple(x.shape)}")
    if not x.is_contiguous():
        raise ValueError(f"{name}: must be contiguous (row-major)")
    if device == "cuda" and not x.is_cuda:
        raise ValueError(f"{name}: must be a CUDA tensor")
    return x


def check_vector(name: str, x, n, dtype: str, device: str = "cuda"):
    if not _is_torch(x):
        raise ValueError(f"{name}: expected a torch tensor, got {type(x).__name__}")
    if str(x.dtype) != f"torch.{dtype}":
        raise ValueError(f"{name}: dtype must be {dtype}, got {x.dtype}")
    if x.dim() != 1 or (n is not None and int(x.shape[0]) != int(n)):
        raise ValueError(f"{name}: shape must be ({n},), got {tuple(x.shape)}")
    if not x.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if device == "cuda" and not x.is_cuda:
        raise ValueError(f"{name}: must be a CUDA tensor")
    return x


def check_factors(factors, dims, skip_mode=None, device: str = "cuda") -> int:
    """Every factor k != skip_mode is float32 (dims[k], R), one R for all; returns R."""
    if len(factors) != len(dims):
        raise ValueError(f"factors: expected {len(dims)} matrices, got {len(factors)}")
    R = None
    for k, f in enumerate(factors):
        if f is None:
            if k == skip_mode:
                continue
            raise ValueError(f"factor {k} is None")
        if not _is_torch(f) or f.dim() != 2:
            raise ValueError(f"factor {k}: expected a 2-D torch tensor")
        if R is None:
            R = int(f.shape[1])
        check_matrix(f"factor {k}", f, dims[k], R, device="any")
    if R is None or R < 1:
        raise ValueError("factors: no rank")
    for k, f in enumerate(factors):  # the device last, once every shape is known good
        if f is not None and device == "cuda" and not f.is_cuda:
            raise ValueError(f"factor {k}: must be a CUDA tensor")
    return R


def check_coo(coords, vals, nmodes: int, device: str = "cuda") -> int:
    """coords int32/uint32 (nmodes, nnz), vals float32 (nnz,); returns nnz."""
    if not _is_torch(coords) or str(coords.dtype) not in ("torch.int32", "torch.uint32"):
        raise ValueError("coords: expected an int32 or uint32 torch tensor")
    if coords.dim() != 2 or int(coords.shape[0]) != nmodes:
        raise ValueError(f"coords: shape must be ({nmodes}, nnz), got {tuple(coords.shape)}")
    nnz = int(coords.shape[1])
    check_vector("vals", vals, nnz, "float32", device)
    if not coords.is_contiguous():
        raise ValueError("coords: must be contiguous")
    if device == "cuda" and not coords.is_cuda:
        raise ValueError("coords: must be a CUDA tensor")
    return nnz


def check_request(dims, coords, vals, init):
    """Host arrays of a server request: coords (nmodes, nnz), vals (nnz,),
    init[k] (dims[k], rank) with one rank.  Returns the converted arrays and rank."""
    nm = len(dims)
    if not 1 <= nm <= MAX_MODES:
        raise ValueError(f"nmodes must be in 1..{MAX_MODES}")
    coords = np.ascontiguousarray(coords)
    if coords.dtype not in (np.uint32, np.int32) or coords.ndim != 2 or coords.shape[0] != nm:
        raise ValueError(f"coords: expected int32/uint32 of shape ({nm}, nnz), got {coords.dtype} {coords.shape}")
    coords = coords.view(np.uint32)
    vals = np.ascontiguousarray(vals)
    if vals.dtype != np.float32 or vals.shape != (coords.shape[1],):
        raise ValueError(f"vals: expected float32 of shape ({coords.shape[1]},), got {vals.dtype} {vals.shape}")
    if len(init) != nm:
        raise ValueError(f"init: expected {nm} matrices, got {len(init)}")
    init = [np.ascontiguousarray(f) for f in init]
    rank = int(init[0].shape[1]) if init[0].ndim == 2 else 0
    for k, f in enumerate(init):
        if f.dtype != np.float32 or f.shape != (int(dims[k]), rank):
            raise ValueError(f"init {k}: expected float32 of shape ({int(dims[k])}, {rank}), got {f.dtype} {f.shape}")
    return coords, vals, init, rank


class Tensor:
    """An encoded sparse tensor living on the GPU (owns an spt_tensor handle)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        self._prepared_rank = None   # rank of the last SPT_PREPARE_SINGLE
        self._batched = False        # SPT_PREPARE_BATCHED done

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
        return {"tile": list(p.tile), "strategy": list(p.strategy), "row_cache": int(p.row_cache),
                "batch_tile": int(p.batch_tile)}

    def set_plan(self, tile=None, strategy=None, row_cache=None, batch_tile=None):
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
        if batch_tile is not None:
            p.batch_tile = int(batch_tile)
        _check(lib().spt_tensor_set_plan(self._h, ctypes.byref(p), _stream(None)))
        self._prepared_rank = None
        self._batched = False

    def prepare(self, rank: int, batched: bool = False, stream=None):
        """Build the per-mode MTTKRP state (plans, tile dictionaries) for ``rank``."""
        what = PREPARE_BATCHED if batched else PREPARE_SINGLE
        _check(lib().spt_tensor_prepare(self._h, int(rank), what, _stream(stream)))
        if batched:
            self._batched = True
        else:
            self._prepared_rank = int(rank)

    def ensure_prepared(self, rank: int, stream=None):
        if self._prepared_rank != int(rank):
            self.prepare(rank, stream=stream)

    def free(self, stream=None):
        if self._h is not None and self._h.value:
            lib().spt_tensor_free(self._h, _stream(stream))
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
    nnz = check_coo(coords, vals, nm)
    d = (ctypes.c_int64 * nm)(*[int(x) for x in dims])
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
    dims = t.info()["dims"]
    R = check_factors(factors, dims, skip_mode=mode)
    rows = dims[mode] if 0 <= mode < len(dims) else 1  # an invalid mode is rejected by the library
    if out is None:
        out = torch.empty((rows, R), dtype=torch.float32, device="cuda")
    elif 0 <= mode < len(dims):
        check_matrix("out", out, rows, R)
    t.ensure_prepared(R, stream)
    _check(lib().spt_mttkrp(t.handle, _ptr_array(factors), R, int(mode), _ptr(out), _stream(stream)))
    return out


def attach_f64(t: Tensor, vals, stream=None):
    """Attach FP64 values (CUDA float64, input order) for ``mttkrp_f64``."""
    nnz = t.info()["nnz"]
    check_vector("vals", vals, nnz, "float64")
    _check(lib().spt_tensor_attach_f64(t.handle, _ptr(vals), _stream(stream)))


def mttkrp_f64(t: Tensor, factors, mode: int, out=None, stream=None):
    """FP64 MTTKRP (FP64 values, factors and accumulation): factors CUDA float64 [I_k, R]."""
    import torch
    dims = t.info()["dims"]
    if len(factors) != len(dims):
        raise ValueError(f"factors: expected {len(dims)} matrices")
    R = None
    for k, f in enumerate(factors):
        if f is None and k == mode:
            continue
        if R is None:
            R = int(f.shape[1])
        check_matrix(f"factor {k}", f, dims[k], R, dtype="float64")
    rows = dims[mode] if 0 <= mode < len(dims) else 1
    if out is None:
        out = torch.empty((rows, R), dtype=torch.float64, device="cuda")
    elif 0 <= mode < len(dims):
        check_matrix("out", out, rows, R, dtype="float64")
    t.ensure_prepared(R, stream)
    _check(lib().spt_mttkrp_f64(t.handle, _ptr_array(factors), R, int(mode), _ptr(out), _stream(stream)))
    return out


def mttkrp_noalloc(t: Tensor, factors, mode: int, out, stream=None):
    """``mttkrp`` into a caller-given ``out`` through the entry point that allocates nothing
    (its workspace is the library's fixed per-GPU array; the tensor must be prepared)."""
    dims = t.info()["dims"]
    R = check_factors(factors, dims, skip_mode=mode)
    if 0 <= mode < len(dims):
        check_matrix("out", out, dims[mode], R)
    _check(lib().spt_mttkrp_noalloc(t.handle, _ptr_array(factors), R, int(mode), _ptr(out), _stream(stream)))
    return out


def cp_als(t: Tensor, factors, iters: int, tol: float = 0.0, lam=None, stream=None):
    """Run CP-ALS in place on ``factors``; returns (lambda tensor, fit, iterations)."""
    import torch
    R = check_factors(factors, t.info()["dims"])
    if lam is None:
        lam = torch.empty(R, dtype=torch.float64, device="cuda")
    check_vector("lambda", lam, R, "float64")
    fit = ctypes.c_double()
    its = ctypes.c_int()
    _check(lib().spt_cp_als(t.handle, R, int(iters), float(tol), _ptr_array(factors), _ptr(lam),
                            ctypes.byref(fit), ctypes.byref(its), _stream(stream)))
    t._prepared_rank = R  # cp_als prepares the tensor for its rank
    return lam, fit.value, its.value


def als_update(grams, mode: int, M, C=None, lam=None, stream=None):
    """One ALS mode update (FP64 solve with ridge retry) of a dense M.

    grams: CUDA float64 (nmodes, R, R); M: CUDA float32 (rows, R).
    Returns (C, lam, ridge retries)."""
    import torch
    if not _is_torch(grams) or str(grams.dtype) != "torch.float64" or grams.dim() != 3 or \
            grams.shape[1] != grams.shape[2] or not grams.is_contiguous() or not grams.is_cuda:
        raise ValueError("grams: expected a contiguous CUDA float64 tensor of shape (nmodes, R, R)")
    nm, R = int(grams.shape[0]), int(grams.shape[1])
    check_matrix("M", M, None, R)
    rows = int(M.shape[0])
    if C is not None:
        check_matrix("C", C, rows, R)
    if lam is not None:
        check_vector("lambda", lam, R, "float64")
    if C is None:
        C = torch.empty((rows, R), dtype=torch.float32, device="cuda")
    if lam is None:
        lam = torch.empty(R, dtype=torch.float64, device="cuda")
    retries = ctypes.c_int()
    _check(lib().spt_als_update(_ptr(grams), nm, int(mode), R, _ptr(M), rows, _ptr(C), _ptr(lam),
                                ctypes.byref(retries), _stream(stream)))
    return C, lam, retries.value


def mttkrp_batched(tensors, factor_lists, mode: int, outs, stream=None):
    count = len(tensors)
    if len(factor_lists) != count or len(outs) != count:
        raise ValueError("tensors, factor_lists and outs must have one entry per tensor")
    for t, fl, o in zip(tensors, factor_lists, outs):
        dims = t.info()["dims"]
        R = check_factors(fl, dims, skip_mode=mode)
        if 0 <= mode < len(dims):
            check_matrix("out", o, dims[mode], R)
    for t in tensors:
        if not t._batched:
            t.prepare(1, batched=True, stream=stream)
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
    if len(factor_lists) != count or (lams is not None and len(lams) != count):
        raise ValueError("tensors, factor_lists and lams must have one entry per tensor")
    for t, fl in zip(tensors, factor_lists):
        check_factors(fl, t.info()["dims"])
    hs = (ctypes.c_void_p * count)(*[t.handle.value for t in tensors])
    farrs = [_ptr_array(fl) for fl in factor_lists]
    fptrs = (_PP * count)(*[ctypes.cast(a, _PP) for a in farrs])
    ranks = (ctypes.c_int * count)(*[int(fl[0].shape[1]) for fl in factor_lists])
    if lams is None:
        lams = [torch.empty(int(fl[0].shape[1]), dtype=torch.float64, device="cuda") for fl in factor_lists]
    for fl, lam in zip(factor_lists, lams):
        check_vector("lambda", lam, int(fl[0].shape[1]), "float64")
    lptrs = _ptr_array(lams)
    fits = (ctypes.c_double * count)()
    its = (ctypes.c_int * count)()
    _check(lib().spt_cp_als_batched(hs, count, ranks, int(iters), float(tol), fptrs, lptrs, fits, its,
                                    _stream(stream)))
    return lams, list(fits), list(its)


def autotune(t: Tensor, factors, budget_ms: float = 2000.0, random_samples: int = 4, seed: int = 0, stream=None):
    """Measured layout and plan search; re-encodes ``t`` in place when another layout wins.

    Returns a dict: best_ms, alto_ms, start_ms (all-mode MTTKRP ms), candidates,
    random_samples, cache_hits."""
    R = check_factors(factors, t.info()["dims"])
    h = ctypes.c_void_p(t.handle.value)
    res = TuneResult()
    _check(lib().spt_autotune(ctypes.byref(h), _ptr_array(factors), R, float(budget_ms), int(random_samples),
                              ctypes.c_uint64(int(seed)), ctypes.byref(res), _stream(stream)))
    t._h = h
    t._prepared_rank = R
    t._batched = False
    return {"best_ms": res.best_ms, "alto_ms": res.alto_ms, "start_ms": res.start_ms,
            "candidates": res.candidates, "random_samples": res.random_samples, "cache_hits": res.cache_hits}


def autotune_batched(tensors, factor_lists, layout_budget_ms: float = 0.0, random_samples: int = 2, seed: int = 0,
                     stream=None):
    """Batch autotuner: optionally every member's layout (``layout_budget_ms`` > 0), then the batched
    tile by timing the all-mode batched MTTKRP at 1024, 2048 and 4096 nonzeros per tile.

    Returns a dict: ms (tile -> all-mode batched ms, 0 when the tile does not fit),
    best_tile, layouts_tuned, layout_speedup."""
    count = len(tensors)
    if len(factor_lists) != count or count == 0:
        raise ValueError("one factor list per tensor, at least one tensor")
    for t, fl in zip(tensors, factor_lists):
        R = check_factors(fl, t.info()["dims"])
        if R > 64:
            raise ValueError("batched launches take ranks 1..64")
    hs = (ctypes.c_void_p * count)(*[t.handle.value for t in tensors])
    farrs = [_ptr_array(fl) for fl in factor_lists]
    fptrs = (_PP * count)(*[ctypes.cast(a, _PP) for a in farrs])
    ranks = (ctypes.c_int * count)(*[int(fl[0].shape[1]) for fl in factor_lists])
    res = BatchTuneResult()
    _check(lib().spt_autotune_batched(hs, count, fptrs, ranks, float(layout_budget_ms), int(random_samples),
                                      ctypes.c_uint64(int(seed)), ctypes.byref(res), _stream(stream)))
    for t, h in zip(tensors, hs):
        t._h = ctypes.c_void_p(h)
        t._batched = True
        if layout_budget_ms > 0:
            t._prepared_rank = None
    return {"ms": {1024: res.ms[0], 2048: res.ms[1], 4096: res.ms[2]}, "best_tile": res.best_tile,
            "layouts_tuned": res.layouts_tuned, "layout_speedup": res.layout_speedup}


_ALLOC_HOOKS = None


def use_torch_allocator(on: bool = True):
    """Route every device allocation of the library through PyTorch's caching allocator.

    The hooks take and return memory on the stream the library passes; torch
    keeps freed blocks for reuse on their allocation stream."""
    global _ALLOC_HOOKS
    if not on:
        _check(lib().spt_set_allocator(ALLOC_FN(), RELEASE_FN(), None))
        _ALLOC_HOOKS = None
        return
    import torch

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0))
        except Exception:
            return None

    def _release(ptr, stream, ctx):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    hooks = (ALLOC_FN(_alloc), RELEASE_FN(_release))
    _check(lib().spt_set_allocator(hooks[0], hooks[1], None))
    _ALLOC_HOOKS = hooks  # keep the callbacks alive


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
        nm = len(dims)
        coords, vals, init, rank = check_request(dims, coords, vals, init)
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


def server_simulate(hbm_budget_bytes: int, max_slots: int, bytes_, arrive, service):
    """The server's admission policy against a modelled executor (host only).
    Returns (admit times, done times, statuses) as numpy arrays."""
    b = np.ascontiguousarray(bytes_, dtype=np.uint64)
    a = np.ascontiguousarray(arrive, dtype=np.float64)
    sv = np.ascontiguousarray(service, dtype=np.float64)
    n = int(b.shape[0])
    if a.shape != (n,) or sv.shape != (n,):
        raise ValueError("bytes, arrive and service must have one entry per request")
    adm = np.empty(n, np.float64)
    done = np.empty(n, np.float64)
    stt = np.empty(n, np.int32)
    _check(lib().spt_server_simulate(ctypes.c_size_t(int(hbm_budget_bytes)), int(max_slots), n,
                                     b.ctypes.data, a.ctypes.data, sv.ctypes.data, adm.ctypes.data,
                                     done.ctypes.data, stt.ctypes.data))
    return adm, done, stt


def profile_reset(on: bool = True):
    """Clear recorded MTTKRP timings and (re)enable event timing."""
    _check(lib().spt_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """Per-mode summed MTTKRP GPU time (ms) and launch counts since the last reset."""
    ms = (ctypes.c_double * MAX_MODES)()
    n = (ctypes.c_int64 * MAX_MODES)()
    _check(lib().spt_profile_read(ms, n))
    return {"mttkrp_ms": list(ms), "mttkrp_launches": list(n)}


def memory_stats() -> dict:
    """The library's device block cache: bytes in live buffers and in idle
    blocks, hipMalloc calls and requests served from idle blocks so far."""
    v = (ctypes.c_int64 * 4)()
    _check(lib().spt_memory_stats(v))
    return {"bytes_live": v[0], "bytes_idle": v[1], "device_allocs": v[2], "reuses": v[3]}


def empty_cache():
    """Return the idle blocks of the library's cache to the driver."""
    _check(lib().spt_empty_cache())


def version() -> str:
    return lib().spt_version().decode()
