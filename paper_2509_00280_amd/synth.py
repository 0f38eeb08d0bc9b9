"""Seeded synthetic sparse tensors, factor initialisations and request streams.

This module only draws random inputs.  It holds none of the method's
arithmetic (no encoding, no MTTKRP, no solve): both the GPU path and the
CPU oracle consume what it returns, so a parity test feeds the two sides the
same bytes.

Streams come from ``numpy.random.SeedSequence(seed).spawn``; every call with
the same arguments returns bit-identical arrays on any host.

The workloads stand in for the sparse tensors of the paper's evaluation
(Section IV-A, Table I), which are not available here: ratings-like 3-mode
tensors with power-law (Zipf) mode distributions, 4-mode tensors with a short
date-like mode, and batches of small tensors for many independent
decompositions (Section IV-D).  The per-mode label shuffle follows the
"shuffled" experiments of Section IV-A.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "SparseCOO", "zipf_cdf", "draw_labels", "distinct_coo", "uniform_distinct_coo",
    "normal_factors", "shuffle_labels", "config", "batch_config", "serving_requests",
    "CONFIG_NAMES", "DeviceCOO", "distinct_coo_device", "config_device",
]


@dataclass
class SparseCOO:
    """A sparse tensor in coordinate form, in draw (input) order.

    coords: uint32 array of shape (nmodes, nnz), 0-based coordinates (SoA).
    vals:   float32 array of shape (nnz,).
    dims:   tuple of mode lengths.
    """
    dims: tuple
    coords: np.ndarray
    vals: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nmodes(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.vals.shape[0])


def zipf_cdf(n: int, s: float) -> np.ndarray:
    """Cumulative FP64 weights of a bounded Zipf law on {0..n-1}: P(i) ~ (i+1)^-s."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(s))
    c = np.cumsum(w)
    c /= c[-1]
    return c


def draw_labels(rng: np.random.Generator, n: int, count: int, dist) -> np.ndarray:
    """Draw ``count`` labels in {0..n-1}.

    dist is ``"uniform"`` or ``("zipf", s)``; Zipf is sampled by inverse CDF
    (``searchsorted(side='right')``), so label 0 is the most frequent one.
    """
    if dist == "uniform":
        return rng.integers(0, n, size=count, dtype=np.int64).astype(np.uint32)
    kind, s = dist
    assert kind == "zipf"
    cdf = zipf_cdf(n, s)
    u = rng.random(count)
    idx = _searchsorted_right(cdf, u)
    np.minimum(idx, n - 1, out=idx)
    return idx.astype(np.uint32)


def _searchsorted_right(table: np.ndarray, x: np.ndarray) -> np.ndarray:
    """``np.searchsorted(table, x, side='right')`` (multi-threaded through torch when present)."""
    try:
        import torch
    except ImportError:
        return np.searchsorted(table, x, side="right")
    return torch.searchsorted(torch.from_numpy(table), torch.from_numpy(x), right=True).numpy()


def _first_occurrences(lin: np.ndarray) -> np.ndarray:
    """Indices of the first occurrence of every distinct value, in increasing index order.

    Same result as ``np.sort(np.unique(lin, return_index=True)[1])``; a stable
    sort keeps the earliest index first among equal values.
    """
    try:
        import torch
    except ImportError:
        return np.sort(np.unique(lin, return_index=True)[1])
    sv, si = torch.sort(torch.from_numpy(lin), stable=True)
    head = torch.ones(sv.shape[0], dtype=torch.bool)
    if sv.shape[0] > 1:
        head[1:] = sv[1:] != sv[:-1]
    first, _ = torch.sort(si[head])
    return first.numpy()


def _draw_values(rng: np.random.Generator, count: int, vdist) -> np.ndarray:
    if vdist == "u01":
        return rng.random(count, dtype=np.float32)
    if vdist == "int1to5":
        return rng.integers(1, 6, size=count, dtype=np.int64).astype(np.float32)
    if vdist == "lognormal":
        return rng.lognormal(0.0, 1.0, size=count).astype(np.float32)
    if vdist == "normal":
        return rng.standard_normal(count, dtype=np.float32)
    raise ValueError(vdist)


def _linear(coords: np.ndarray, dims) -> np.ndarray:
    """Mixed-radix C-order cell number of each coordinate (needs prod(dims) < 2^63)."""
    lin = np.zeros(coords.shape[1], dtype=np.int64)
    for n, d in enumerate(dims):
        lin *= int(d)
        lin += coords[n].astype(np.int64)
    return lin


def _mode_groups(dims, limit: int = 2 ** 63) -> list:
    """Consecutive runs of modes whose box size stays below ``limit``."""
    groups, cur, prod = [], [], 1
    for n, d in enumerate(dims):
        if cur and prod * int(d) >= limit:
            groups.append(cur)
            cur, prod = [], 1
        cur.append(n)
        prod *= int(d)
    groups.append(cur)
    return groups


def _cell_words(coords: np.ndarray, dims, groups) -> list:
    """C-order cell number of each coordinate as one int64 word per mode group."""
    return [_linear(coords[g], [dims[n] for n in g]) for g in groups]


def _first_occurrences_words(words: list) -> np.ndarray:
    """``_first_occurrences`` for keys made of several int64 words (first word most significant)."""
    if len(words) == 1:
        return _first_occurrences(words[0])
    order = np.lexsort(tuple(reversed(words)))  # stable: equal keys keep index order
    head = np.ones(order.shape[0], dtype=bool)
    if order.shape[0] > 1:
        diff = np.zeros(order.shape[0] - 1, dtype=bool)
        for w in words:
            ws = w[order]
            diff |= ws[1:] != ws[:-1]
        head[1:] = diff
    return np.sort(order[head])


def distinct_coo(seed: int, dims, nnz: int, mode_dists, vdist, max_rounds: int = 40) -> SparseCOO:
    """Draw coordinate+value pairs until ``nnz`` distinct coordinates exist.

    Rounds draw ceil(1.5 * deficit) pairs; the first occurrence of each
    coordinate (in draw order) is kept; the result is truncated to exactly
    ``nnz`` in draw order.  If the box cannot be filled within ``max_rounds``
    the realized count is smaller and recorded in ``meta['realized_nnz']``.
    """
    dims = tuple(int(d) for d in dims)
    # boxes of 2^63 cells or more are numbered with one word per group of modes
    groups = _mode_groups(dims)
    nm = len(dims)
    ss = np.random.SeedSequence(seed)
    s_coord, s_val = ss.spawn(2)
    rc = np.random.default_rng(s_coord)
    rv = np.random.default_rng(s_val)
    kept_c = np.zeros((nm, 0), dtype=np.uint32)
    kept_v = np.zeros(0, dtype=np.float32)
    kept_w = [np.zeros(0, dtype=np.int64) for _ in groups]
    rounds = 0
    while kept_v.shape[0] < nnz and rounds < max_rounds:
        deficit = nnz - kept_v.shape[0]
        m = int(math.ceil(1.5 * deficit))
        c = np.stack([draw_labels(rc, dims[n], m, mode_dists[n]) for n in range(nm)])
        v = _draw_values(rv, m, vdist)
        w = _cell_words(c, dims, groups)
        nk = kept_v.shape[0]
        first = _first_occurrences_words([np.concatenate([a, b]) for a, b in zip(kept_w, w)])
        first = first[first >= nk] - nk
        kept_c = np.concatenate([kept_c, c[:, first]], axis=1)
        kept_v = np.concatenate([kept_v, v[first]])
        kept_w = [np.concatenate([a, b[first]]) for a, b in zip(kept_w, w)]
        rounds += 1
    kept_c = np.ascontiguousarray(kept_c[:, :nnz])
    kept_v = np.ascontiguousarray(kept_v[:nnz])
    return SparseCOO(dims, kept_c, kept_v,
                     meta={"seed": seed, "rounds": rounds, "realized_nnz": int(kept_v.shape[0]),
                           "requested_nnz": int(nnz), "mode_dists": list(mode_dists), "vdist": vdist})


def uniform_distinct_coo(seed: int, dims, nnz: int, vdist="u01") -> SparseCOO:
    """``nnz`` distinct cells sampled uniformly without replacement from the box (C order)."""
    dims = tuple(int(d) for d in dims)
    ss = np.random.SeedSequence(seed)
    s_coord, s_val = ss.spawn(2)
    total = math.prod(dims)
    lin = np.random.default_rng(s_coord).choice(total, size=nnz, replace=False)
    coords = np.stack(np.unravel_index(lin, dims)).astype(np.uint32)
    vals = _draw_values(np.random.default_rng(s_val), nnz, vdist)
    return SparseCOO(dims, np.ascontiguousarray(coords), vals,
                     meta={"seed": seed, "realized_nnz": nnz, "requested_nnz": nnz, "vdist": vdist})


def normal_factors(seed: int, dims, rank: int) -> list:
    """Row-major FP32 ``I_n x rank`` matrices with N(0,1) entries, one stream per mode."""
    ss = np.random.SeedSequence(seed).spawn(len(dims))
    return [np.random.default_rng(s).standard_normal((int(d), rank), dtype=np.float32) for s, d in zip(ss, dims)]


def shuffle_labels(t: SparseCOO, seed: int) -> SparseCOO:
    """Apply an independent uniform permutation to the labels of every mode."""
    ss = np.random.SeedSequence(seed).spawn(t.nmodes)
    c = np.empty_like(t.coords)
    for n, (s, d) in enumerate(zip(ss, t.dims)):
        p = np.random.default_rng(s).permutation(d).astype(np.uint32)
        c[n] = p[t.coords[n]]
    return SparseCOO(t.dims, c, t.vals.copy(), meta=dict(t.meta, shuffled=seed))


CONFIG_NAMES = ("small", "ratings", "skewed4d")

# name -> (master seed, dims, nnz, per-mode distributions, value law, rank, iterations)
_CONFIGS = {
    "small": (1, (200, 150, 100), 20_000, None, "u01", 16, 10),
    "ratings": (2, (480_000, 18_000, 2_000), 100_000_000,
                (("zipf", 1.1), ("zipf", 1.1), "uniform"), "int1to5", 32, 20),
    "skewed4d": (3, (2_000_000, 100_000, 50_000, 24), 150_000_000,
                 (("zipf", 1.3), ("zipf", 1.3), ("zipf", 1.3), "uniform"), "lognormal", 64, 10),
}


def config(name: str, nnz: int | None = None, shuffle: bool = False):
    """One of the single-tensor workloads.

    Returns (tensor, factors, rank, iters).  ``nnz`` scales the tensor down
    (same shape and laws) for quick runs; ``shuffle`` permutes labels per mode.
    """
    seed, dims, full_nnz, dists, vdist, rank, iters = _CONFIGS[name]
    n = full_nnz if nnz is None else int(nnz)
    ss = np.random.SeedSequence(seed)
    s_t, s_f, s_sh = (int(x.generate_state(1)[0]) for x in ss.spawn(3))
    if dists is None:
        t = uniform_distinct_coo(s_t, dims, n, vdist)
    else:
        t = distinct_coo(s_t, dims, n, dists, vdist)
    if shuffle:
        t = shuffle_labels(t, s_sh)
    t.meta["config"] = name
    return t, normal_factors(s_f, dims, rank), rank, iters


def batch_config(seed: int = 4, count: int = 256, nnz_range=(10_000, 5_000_000),
                 dim_range=(50, 200_000), zipf_s: float = 1.2, ranks=(16, 32)):
    """Many small independent tensors (3 or 4 modes with p=1/2, log-uniform sizes).

    Returns a list of (tensor, factors, rank).
    """
    root = np.random.SeedSequence(seed)
    shape_rng = np.random.default_rng(root.spawn(1)[0])
    members = root.spawn(count + 1)[1:]
    out = []
    lo_n, hi_n = np.log(nnz_range[0]), np.log(nnz_range[1])
    lo_d, hi_d = np.log(dim_range[0]), np.log(dim_range[1])
    for b in range(count):
        nm = 3 if shape_rng.random() < 0.5 else 4
        nnz = int(np.floor(np.exp(shape_rng.uniform(lo_n, hi_n))))
        dims = tuple(int(np.floor(np.exp(shape_rng.uniform(lo_d, hi_d)))) for _ in range(nm))
        rank = int(ranks[int(shape_rng.integers(0, len(ranks)))])
        s_t, s_f = (int(x.generate_state(1)[0]) for x in members[b].spawn(2))
        t = distinct_coo(s_t, dims, nnz, [("zipf", zipf_s)] * nm, "u01")
        t.meta["member"] = b
        out.append((t, normal_factors(s_f, dims, rank), rank))
    return out


def serving_requests(seed: int = 5, count: int = 2100, rate_per_s: float = 100.0,
                     ranks=(16, 32, 48, 64), **batch_kw):
    """Poisson arrivals of decomposition requests drawn like ``batch_config``.

    Returns a list of dicts {t_arrive, tensor, factors, rank}.  Tensors are
    generated lazily by ``materialize(req)`` to bound host memory.
    """
    root = np.random.SeedSequence(seed)
    s_arr, s_shape = root.spawn(2)
    gaps = np.random.default_rng(s_arr).exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps)
    reqs = []
    shape_seed = int(s_shape.generate_state(1)[0])
    for i in range(count):
        reqs.append({"id": i, "t_arrive": float(t[i]), "shape_seed": shape_seed, "index": i,
                     "ranks": tuple(ranks), "batch_kw": batch_kw})
    return reqs


def materialize(req):
    """Generate the tensor and initial factors of one serving request."""
    kw = dict(req["batch_kw"])
    rng = np.random.default_rng(np.random.SeedSequence([req["shape_seed"], req["index"]]))
    lo_n, hi_n = np.log(kw.get("nnz_range", (10_000, 5_000_000))[0]), np.log(kw.get("nnz_range", (10_000, 5_000_000))[1])
    lo_d, hi_d = np.log(kw.get("dim_range", (50, 200_000))[0]), np.log(kw.get("dim_range", (50, 200_000))[1])
    nm = 3 if rng.random() < 0.5 else 4
    nnz = int(np.floor(np.exp(rng.uniform(lo_n, hi_n))))
    dims = tuple(int(np.floor(np.exp(rng.uniform(lo_d, hi_d)))) for _ in range(nm))
    ranks = req["ranks"]
    rank = int(ranks[int(rng.integers(0, len(ranks)))])
    s_t, s_f = (int(x) for x in rng.integers(0, 2 ** 63 - 1, size=2))
    t = distinct_coo(s_t, dims, nnz, [("zipf", kw.get("zipf_s", 1.2))] * nm, "u01")
    return t, normal_factors(s_f, dims, rank), rank


# --------------------------------------------------------------------------
# The same recipes drawn on a torch device (the GPU for the full-size
# workloads, which NumPy takes minutes to draw).  Same algorithm as
# ``distinct_coo`` (bounded Zipf by inverse CDF over FP64 weights, rounds of
# ceil(1.5 * deficit) draws, first occurrence in draw order kept, truncation
# to exactly nnz in draw order); the stream is torch's generator of the
# device, seeded, so the arrays are reproducible on one device type but are
# not the NumPy arrays of ``distinct_coo``.
# --------------------------------------------------------------------------

@dataclass
class DeviceCOO:
    """A sparse tensor in coordinate form held in torch tensors on one device.

    coords: int32 tensor (nmodes, nnz) (bits of uint32 coordinates); vals: float32 (nnz,).
    """
    dims: tuple
    coords: object
    vals: object
    meta: dict = field(default_factory=dict)

    @property
    def nmodes(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.vals.shape[0])

    def to_host(self) -> SparseCOO:
        return SparseCOO(self.dims, self.coords.cpu().numpy().view(np.uint32), self.vals.cpu().numpy(),
                         meta=dict(self.meta))


def _draw_labels_device(torch, gen, n: int, count: int, dist, cdf, device):
    if dist == "uniform":
        return torch.randint(0, n, (count,), generator=gen, device=device, dtype=torch.int64)
    u = torch.rand(count, generator=gen, device=device, dtype=torch.float64)
    idx = torch.searchsorted(cdf, u, right=True)
    return torch.clamp(idx, max=n - 1)


def _draw_values_device(torch, gen, count: int, vdist, device):
    if vdist == "u01":
        return torch.rand(count, generator=gen, device=device, dtype=torch.float32)
    if vdist == "int1to5":
        return torch.randint(1, 6, (count,), generator=gen, device=device, dtype=torch.int64).to(torch.float32)
    if vdist == "lognormal":
        return torch.exp(torch.randn(count, generator=gen, device=device, dtype=torch.float64)).to(torch.float32)
    if vdist == "normal":
        return torch.randn(count, generator=gen, device=device, dtype=torch.float32)
    raise ValueError(vdist)


def distinct_coo_device(seed: int, dims, nnz: int, mode_dists, vdist, device="cuda", max_rounds: int = 40):
    """``distinct_coo``'s recipe drawn with torch on ``device``.  Boxes of 2^63
    cells or more are numbered with one int64 word per group of modes."""
    import torch
    dims = tuple(int(d) for d in dims)
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    cdfs = [None if d == "uniform" else torch.from_numpy(zipf_cdf(n, d[1])).to(dev) for n, d in zip(dims, mode_dists)]
    groups = _mode_groups(dims)
    kept_c = torch.zeros((len(dims), 0), dtype=torch.int32, device=dev)
    kept_w = [torch.zeros(0, dtype=torch.int64, device=dev) for _ in groups]
    kept_v = torch.zeros(0, dtype=torch.float32, device=dev)
    rounds = 0
    while kept_v.shape[0] < nnz and rounds < max_rounds:
        deficit = nnz - kept_v.shape[0]
        m = int(math.ceil(1.5 * deficit))
        c = torch.stack([_draw_labels_device(torch, gen, d, m, mode_dists[n], cdfs[n], dev).to(torch.int32)
                         for n, d in enumerate(dims)])
        v = _draw_values_device(torch, gen, m, vdist, dev)
        w = []
        for g in groups:
            lin = torch.zeros(m, dtype=torch.int64, device=dev)
            for n in g:
                lin = lin * dims[n] + c[n].to(torch.int64)
            w.append(lin)
        nk = kept_v.shape[0]
        allw = [torch.cat([a, b]) for a, b in zip(kept_w, w)]
        # lexicographic order of the words, equal keys in index order (stable sorts, last word first)
        order = torch.arange(allw[0].shape[0], device=dev)
        for word in reversed(allw):
            order = order[torch.sort(word[order], stable=True).indices]
        head = torch.ones(order.shape[0], dtype=torch.bool, device=dev)
        if order.shape[0] > 1:
            diff = torch.zeros(order.shape[0] - 1, dtype=torch.bool, device=dev)
            for word in allw:
                ws = word[order]
                diff |= ws[1:] != ws[:-1]
            head[1:] = diff
        first = order[head]
        new = torch.sort(first[first >= nk] - nk).values
        kept_c = torch.cat([kept_c, c[:, new]], dim=1)
        kept_w = [torch.cat([a, b[new]]) for a, b in zip(kept_w, w)]
        kept_v = torch.cat([kept_v, v[new]])
        del allw, order, head, first, new, c, v, w
        rounds += 1
    coords = kept_c[:, :nnz].contiguous()
    return DeviceCOO(dims, coords, kept_v[:nnz].contiguous(),
                     meta={"seed": seed, "rounds": rounds, "realized_nnz": int(coords.shape[1]),
                           "requested_nnz": int(nnz), "mode_dists": list(mode_dists), "vdist": vdist,
                           "generator": f"torch {dev.type}"})


def shuffle_labels_device(t: DeviceCOO, seed: int) -> DeviceCOO:
    """``shuffle_labels`` with torch on the tensor's device: an independent uniform
    permutation of the labels of every mode (the shuffled experiments, Section IV-A)."""
    import torch
    dev = t.coords.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    c = torch.empty_like(t.coords)
    for n, d in enumerate(t.dims):
        p = torch.randperm(d, generator=gen, device=dev).to(torch.int32)
        c[n] = p[t.coords[n].long()]
    return DeviceCOO(t.dims, c, t.vals.clone(), meta=dict(t.meta, shuffled=seed))


def normal_factors_device(seed: int, dims, rank: int, device="cuda") -> list:
    """Row-major FP32 ``I_n x rank`` N(0,1) matrices drawn with torch on ``device``."""
    import torch
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    return [torch.randn((int(d), rank), generator=gen, device=dev, dtype=torch.float32) for d in dims]


# Shapes and nonzero counts of the sparse tensors of the paper's evaluation
# (Table I), for synthetic stand-ins: the data sets themselves are not used.
TABLE1 = {
    "darpa": ((22_500, 22_500, 23_800_000), 28_400_000),
    "fb-m": ((23_300_000, 23_300_000, 166), 99_600_000),
    "flickr-4d": ((319_700, 28_200_000, 1_600_000, 731), 112_900_000),
    "flickr-3d": ((319_700, 28_200_000, 1_600_000), 112_900_000),
    "deli-4d": ((532_900, 17_300_000, 2_500_000, 1_400), 140_100_000),
    "deli-3d": ((532_900, 17_300_000, 2_500_000), 140_100_000),
    "nell-1": ((2_900_000, 2_100_000, 25_500_000), 143_600_000),
    "amazon": ((4_800_000, 1_800_000, 1_800_000), 1_700_000_000),
    "patents": ((46, 239_200, 239_200), 3_600_000_000),
    "reddit": ((8_200_000, 177_000, 8_100_000), 4_700_000_000),
}
TABLE1_SEED = 11


def table1_config(name: str, nnz: int | None = None, rank: int = 16, zipf_s: float = 1.1, device=None,
                  shuffle: bool = False):
    """A synthetic stand-in for one Table I tensor: its mode lengths, ``nnz``
    distinct nonzeros (default: its count), Zipf(s) labels on every mode (the
    power-law mode distributions of such data; the paper gives shapes and
    counts only), U(0,1) values, rank-16 N(0,1) factors (the paper's rank).
    ``device`` None draws with NumPy; else with torch on that device.
    Returns (tensor, factors, rank)."""
    dims, full = TABLE1[name]
    n = full if nnz is None else int(nnz)
    idx = list(TABLE1).index(name)
    ss = np.random.SeedSequence([TABLE1_SEED, idx])
    s_t, s_f, s_sh = (int(x.generate_state(1)[0]) for x in ss.spawn(3))
    dists = [("zipf", zipf_s)] * len(dims)
    if device is None:
        t = distinct_coo(s_t, dims, n, dists, "u01")
        if shuffle:
            t = shuffle_labels(t, s_sh)
        F = normal_factors(s_f, dims, rank)
    else:
        t = distinct_coo_device(s_t, dims, n, dists, "u01", device)
        if shuffle:
            t = shuffle_labels_device(t, s_sh)
        F = normal_factors_device(s_f, dims, rank, device)
    t.meta["table1"] = name
    return t, F, rank


def config_device(name: str, device="cuda", nnz: int | None = None, shuffle: bool = False):
    """``config``'s workloads drawn with torch on ``device``.  Returns (DeviceCOO, factors, rank, iters)."""
    seed, dims, full_nnz, dists, vdist, rank, iters = _CONFIGS[name]
    if dists is None:
        raise ValueError("config_device: the small workload is drawn by ``config``")
    n = full_nnz if nnz is None else int(nnz)
    ss = np.random.SeedSequence(seed)
    s_t, s_f, s_sh = (int(x.generate_state(1)[0]) for x in ss.spawn(3))
    t = distinct_coo_device(s_t, dims, n, dists, vdist, device)
    if shuffle:
        t = shuffle_labels_device(t, s_sh)
    t.meta["config"] = name
    return t, normal_factors_device(s_f, dims, rank, device), rank, iters


def materialize_device(req, device="cuda"):
    """``materialize``'s recipe (same shape draw: modes, nnz, dims, rank) with the
    tensor and initial factors drawn by torch on ``device`` and returned on the host."""
    kw = dict(req["batch_kw"])
    rng = np.random.default_rng(np.random.SeedSequence([req["shape_seed"], req["index"]]))
    lo_n, hi_n = np.log(kw.get("nnz_range", (10_000, 5_000_000))[0]), np.log(kw.get("nnz_range", (10_000, 5_000_000))[1])
    lo_d, hi_d = np.log(kw.get("dim_range", (50, 200_000))[0]), np.log(kw.get("dim_range", (50, 200_000))[1])
    nm = 3 if rng.random() < 0.5 else 4
    nnz = int(np.floor(np.exp(rng.uniform(lo_n, hi_n))))
    dims = tuple(int(np.floor(np.exp(rng.uniform(lo_d, hi_d)))) for _ in range(nm))
    ranks = req["ranks"]
    rank = int(ranks[int(rng.integers(0, len(ranks)))])
    s_t, s_f = (int(x) for x in rng.integers(0, 2 ** 63 - 1, size=2))
    t = distinct_coo_device(s_t, dims, nnz, [("zipf", kw.get("zipf_s", 1.2))] * nm, "u01", device).to_host()
    F = [f.cpu().numpy() for f in normal_factors_device(s_f, dims, rank, device)]
    return t, F, rank
