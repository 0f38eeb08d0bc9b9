"""Pins of the oracle's layout / encoding / decoding against the paper and closed forms."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_alto_example_from_paper():
    g = _gold("alto_4x8x2.json")
    assert oracle.bit_lengths(g["dims"]) == g["bit_lengths"]
    L = oracle.alto_layout(g["dims"])
    assert len(L) == g["lp"]
    pos = oracle.bit_positions(L, 3)
    assert pos[0] == g["mode0_key_bits"]
    assert oracle.is_valid_layout(L, g["dims"])


def test_eq1_interleaving_count_by_enumeration():
    g = _gold("alto_4x8x2.json")
    dims = g["dims"]
    lp = sum(oracle.bit_lengths(dims))
    assert math.factorial(lp) == g["linear_formats"]
    valid = [L for L in itertools.product(range(3), repeat=lp) if oracle.is_valid_layout(list(L), dims)]
    assert len(valid) == g["interleavings"]
    # every valid layout gives a bijection on the box, all distinct
    grid = np.stack(np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")).reshape(3, -1).astype(np.uint32)
    seen = set()
    for L in valid:
        lo, _ = oracle.encode_keys(grid, dims, list(L))
        assert sorted(lo.tolist()) == list(range(2 ** lp))
        seen.add(tuple(lo.tolist()))
    assert len(seen) == len(valid)  # different interleavings give different encodings


def test_eq1_printed_magnitudes():
    g = _gold("eq1_counts.json")
    lin = math.factorial(g["N"] * g["l"])
    inter = lin // math.factorial(g["l"]) ** g["N"]
    assert abs(lin / g["linear_formats"] - 1) < g["rel_tol"]
    assert abs(inter / g["interleavings"] - 1) < g["rel_tol"]


@pytest.mark.parametrize("dims", [(3, 5, 2), (4, 8, 2), (1, 7, 3), (2, 2, 2, 2), (6, 1, 1, 5), (9, 4, 3, 2)])
def test_bijection_on_full_boxes(dims):
    rng = np.random.default_rng(7)
    nm = len(dims)
    grid = np.stack(np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")).reshape(nm, -1).astype(np.uint32)
    lb = oracle.bit_lengths(dims)
    lp = sum(lb)
    multiset = [n for n in range(nm) for _ in range(lb[n])]
    layouts = [oracle.alto_layout(dims)] + [list(rng.permutation(multiset)) for _ in range(4)]
    for L in layouts:
        lo, hi = oracle.encode_keys(grid, dims, L)
        assert not hi.any()
        assert len(set(lo.tolist())) == grid.shape[1]
        assert int(lo.max(initial=0)) < 2 ** lp
        back = oracle.decode_keys(lo, hi, dims, L)
        np.testing.assert_array_equal(back, grid)


def test_unit_modes_have_no_bits():
    dims = (1, 1, 1)
    assert oracle.alto_layout(dims) == []
    lo, hi = oracle.encode_keys(np.zeros((3, 4), np.uint32), dims)
    assert not lo.any() and not hi.any()


def _morton_textbook(coords, nbits):
    """Classic Morton code: bit j of coordinate n lands at position j*N + n (string construction)."""
    N = coords.shape[0]
    out = []
    for e in range(coords.shape[1]):
        bits = [format(int(coords[n, e]), f"0{nbits}b")[::-1] for n in range(N)]  # LSB first
        s = "".join(bits[n][j] for j in range(nbits) for n in range(N))
        out.append(int(s[::-1], 2))
    return np.array(out, dtype=np.uint64)


def test_round_robin_layout_is_morton():
    dims = (16, 16, 16)
    rng = np.random.default_rng(3)
    c = rng.integers(0, 16, size=(3, 200)).astype(np.uint32)
    L = [0, 1, 2] * 4
    lo, _ = oracle.encode_keys(c, dims, L)
    np.testing.assert_array_equal(lo, _morton_textbook(c, 4))


@pytest.mark.parametrize("dims", [(8, 4, 16), (2, 32, 4, 8)])
def test_concatenated_layout_is_c_order_index(dims):
    nm = len(dims)
    lb = oracle.bit_lengths(dims)
    L = [n for n in reversed(range(nm)) for _ in range(lb[n])]  # last mode in the lowest bits
    rng = np.random.default_rng(5)
    c = np.stack([rng.integers(0, d, size=300) for d in dims]).astype(np.uint32)
    lo, _ = oracle.encode_keys(c, dims, L)
    np.testing.assert_array_equal(lo, np.ravel_multi_index(c.astype(np.int64), dims).astype(np.uint64))


def test_wide_keys_use_two_words():
    dims = (2 ** 20, 2 ** 20, 2 ** 20, 2 ** 10)  # l(p) = 70
    assert oracle.key_words(dims) == 2
    rng = np.random.default_rng(11)
    c = np.stack([rng.integers(0, d, size=500) for d in dims]).astype(np.uint32)
    lo, hi = oracle.encode_keys(c, dims)
    assert int(hi.max()) < 2 ** 6 and hi.any()
    np.testing.assert_array_equal(oracle.decode_keys(lo, hi, dims), c)
    # the concatenated layout (mode 3 lowest) equals the big-integer C-order index
    lb = oracle.bit_lengths(dims)
    L = [n for n in reversed(range(4)) for _ in range(lb[n])]
    lo2, hi2 = oracle.encode_keys(c, dims, L)
    for e in range(50):
        big = ((int(c[0, e]) * dims[1] + int(c[1, e])) * dims[2] + int(c[2, e])) * dims[3] + int(c[3, e])
        assert (int(hi2[e]) << 64) | int(lo2[e]) == big


def test_key_width_limits():
    assert oracle.key_words((200, 150, 100)) == 1
    assert sum(oracle.bit_lengths((200, 150, 100))) == 23
    assert sum(oracle.bit_lengths((480_000, 18_000, 2_000))) == 45
    assert sum(oracle.bit_lengths((2_000_000, 100_000, 50_000, 24))) == 59
    assert oracle.key_words((2 ** 32, 2 ** 32, 2)) == 2
    with pytest.raises(ValueError):
        oracle.key_words((2 ** 32,) * 4 + (2,))


def test_out_of_range_rejected():
    with pytest.raises(ValueError):
        oracle.encode_keys(np.array([[0, 4], [0, 1]], np.uint32), (4, 2))


def test_stable_order_with_duplicates():
    dims = (5, 6, 3)
    rng = np.random.default_rng(2)
    c = np.stack([rng.integers(0, d, size=400) for d in dims]).astype(np.uint32)
    c[:, 100:150] = c[:, 0:50]  # duplicates
    v = rng.random(400, dtype=np.float32)
    enc = oracle.encode(c, v, dims)
    lo, hi = oracle.encode_keys(c, dims)
    expect = sorted(range(400), key=lambda e: (int(hi[e]), int(lo[e])))  # Python's sort is stable
    np.testing.assert_array_equal(enc["perm"], np.array(expect))
    np.testing.assert_array_equal(enc["vals"], v[expect])
    np.testing.assert_array_equal(enc["coords"], c[:, expect])


def test_storage_is_layout_independent():
    dims = (480_000, 18_000, 2_000)
    lb = oracle.bit_lengths(dims)
    multiset = [n for n in range(3) for _ in range(lb[n])]
    rng = np.random.default_rng(0)
    widths = {oracle.key_words(dims)}
    for _ in range(5):
        L = list(rng.permutation(multiset))
        assert oracle.is_valid_layout(L, dims)
        widths.add(oracle.key_words(dims))
    assert widths == {1}
