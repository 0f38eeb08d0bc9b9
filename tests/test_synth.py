"""Seeded generators: determinism, distinctness, marginal laws and sizes."""
import numpy as np
import scipy.stats

from paper_2509_00280_amd import synth


def test_small_config_is_deterministic_and_distinct():
    t1, f1, r1, it1 = synth.config("small")
    t2, f2, _, _ = synth.config("small")
    assert t1.dims == (200, 150, 100) and t1.nnz == 20_000 and r1 == 16 and it1 == 10
    np.testing.assert_array_equal(t1.coords, t2.coords)
    np.testing.assert_array_equal(t1.vals, t2.vals)
    for a, b in zip(f1, f2):
        np.testing.assert_array_equal(a, b)
    lin = np.ravel_multi_index(t1.coords.astype(np.int64), t1.dims)
    assert np.unique(lin).size == t1.nnz
    assert t1.vals.dtype == np.float32 and (t1.vals >= 0).all() and (t1.vals < 1).all()
    assert f1[0].shape == (200, 16) and f1[0].dtype == np.float32


def test_zipf_marginal_matches_exact_pmf():
    rng = np.random.default_rng(0)
    n, s, m = 40, 1.1, 200_000
    x = synth.draw_labels(rng, n, m, ("zipf", s))
    obs = np.bincount(x, minlength=n)
    p = np.arange(1, n + 1, dtype=np.float64) ** -s
    p /= p.sum()
    chi2, pval = scipy.stats.chisquare(obs, p * m)
    assert pval > 1e-4
    assert obs.argmax() == 0


def test_distinct_topup_scaled_ratings():
    t, f, rank, iters = synth.config("ratings", nnz=200_000)
    assert t.nnz == 200_000 and rank == 32 and iters == 20
    lin = np.ravel_multi_index(t.coords.astype(np.int64), t.dims)
    assert np.unique(lin).size == t.nnz
    assert set(np.unique(t.vals).tolist()) <= {1.0, 2.0, 3.0, 4.0, 5.0}
    # mode 0 skewed towards label 0, mode 2 roughly uniform
    assert np.bincount(t.coords[0])[0] > 50 * t.nnz / t.dims[0]
    assert np.bincount(t.coords[2], minlength=t.dims[2]).max() < 3 * t.nnz / t.dims[2]


def test_shuffle_keeps_values_and_shape():
    t, _, _, _ = synth.config("small")
    s = synth.shuffle_labels(t, 9)
    np.testing.assert_array_equal(s.vals, t.vals)
    for n, d in enumerate(t.dims):
        assert s.coords[n].max() < d
        assert sorted(np.bincount(s.coords[n], minlength=d)) == sorted(np.bincount(t.coords[n], minlength=d))


def test_batch_members_shapes():
    batch = synth.batch_config(count=6, nnz_range=(1000, 5000), dim_range=(20, 300))
    for t, f, r in batch:
        assert t.nmodes in (3, 4) and r in (16, 32)
        assert len(f) == t.nmodes and all(ff.shape == (d, r) for ff, d in zip(f, t.dims))
        assert 1000 * 0.5 <= t.nnz <= 5000


def test_multiword_dedup_matches_single_word():
    rng = np.random.default_rng(3)
    dims = (50, 40, 30, 20)
    c = np.stack([rng.integers(0, d, 5000) for d in dims]).astype(np.uint32)
    one = synth._first_occurrences(synth._linear(c, dims))
    words = synth._cell_words(c, dims, [[0, 1], [2, 3]])
    np.testing.assert_array_equal(synth._first_occurrences_words(words), one)


def test_distinct_coo_huge_box():
    dims = (200_000, 150_000, 190_000, 170_000)  # more than 2^63 cells
    assert len(synth._mode_groups(dims)) == 2
    t = synth.distinct_coo(3, dims, 20_000, [("zipf", 1.2)] * 4, "u01")
    assert t.nnz == 20_000
    assert len(set(map(tuple, t.coords.T))) == 20_000


def test_device_generator_recipe_on_cpu():
    """The torch recipe (run on the CPU here): exact distinct count, ranges,
    Zipf label 0 most frequent, value laws, reproducible for a seed."""
    import torch
    from paper_2509_00280_amd import synth
    dims = (500, 300, 24)
    dists = [("zipf", 1.3), ("zipf", 1.3), "uniform"]
    t = synth.distinct_coo_device(7, dims, 20_000, dists, "lognormal", device="cpu")
    assert t.nnz == 20_000 and t.coords.dtype == torch.int32
    c = t.coords.numpy()
    lin = (c[0].astype(np.int64) * 300 + c[1]) * 24 + c[2]
    assert np.unique(lin).size == t.nnz
    for n, d in enumerate(dims):
        assert c[n].min() >= 0 and c[n].max() < d
    for n in (0, 1):
        cnt = np.bincount(c[n], minlength=dims[n])
        assert cnt.argmax() == 0 and cnt[0] > cnt[10] > cnt[200]
    assert (t.vals.numpy() > 0).all()
    t2 = synth.distinct_coo_device(7, dims, 20_000, dists, "lognormal", device="cpu")
    assert torch.equal(t.coords, t2.coords) and torch.equal(t.vals, t2.vals)
    h = t.to_host()
    assert h.coords.dtype == np.uint32 and h.nnz == t.nnz
    r = synth.distinct_coo_device(8, (40, 30, 20), 3000, ["uniform"] * 3, "int1to5", device="cpu")
    assert set(np.unique(r.vals.numpy())) <= {1.0, 2.0, 3.0, 4.0, 5.0}


def test_device_generator_wide_box_and_shuffle_on_cpu():
    """Boxes of 2^63 cells or more dedup on two words; the shuffle is a per-mode bijection."""
    import torch
    from paper_2509_00280_amd import synth
    dims = (3_000_000, 2_500_000, 1_000_000, 4_000)  # 3e22 cells
    t = synth.distinct_coo_device(5, dims, 30_000, [("zipf", 1.2)] * 4, "u01", device="cpu")
    c = t.coords.numpy().astype(np.int64)
    keys = set(zip(*c))
    assert t.nnz == 30_000 and len(keys) == t.nnz
    s = synth.shuffle_labels_device(t, 9)
    cs = s.coords.numpy().astype(np.int64)
    for n in range(4):
        pairs = set(zip(c[n], cs[n]))
        assert len({a for a, _ in pairs}) == len(pairs) == len({b for _, b in pairs})  # a bijection on used labels
    assert torch.equal(s.vals, t.vals)


def test_table1_shapes():
    from paper_2509_00280_amd import synth
    assert len(synth.TABLE1) == 10
    t, F, R = synth.table1_config("flickr-4d", nnz=5000)
    assert t.dims == (319_700, 28_200_000, 1_600_000, 731) and t.nnz == 5000 and R == 16
    assert [f.shape for f in F] == [(d, 16) for d in t.dims]
    wide = [n for n, (d, _) in synth.TABLE1.items() if sum((x - 1).bit_length() for x in d) > 64]
    assert sorted(wide) == sorted(["flickr-4d", "flickr-3d", "deli-4d", "deli-3d", "nell-1", "amazon"])
