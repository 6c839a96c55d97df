"""Seeded input generators: determinism, thread independence, shapes."""
import numpy as np


def test_same_seed_same_bytes(inputs_mod):
    a = inputs_mod.log_uniform(7, 2, 1e-8, 1e6, 300001, threads=1)
    b = inputs_mod.log_uniform(7, 2, 1e-8, 1e6, 300001, threads=8)
    c = inputs_mod.log_uniform(8, 2, 1e-8, 1e6, 300001, threads=8)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 1e-8 and a.max() <= 1e6
    # log10 is uniform: mean near the midpoint of [-8, 6]
    assert abs(np.log10(a).mean() + 1.0) < 0.05


def test_offsets_are_counter_based(inputs_mod):
    a = inputs_mod.log_uniform(3, 2, 1.0, 10.0, 1000)
    b = inputs_mod.log_uniform(3, 2, 1.0, 10.0, 500, k0=500)
    assert np.array_equal(a[500:], b)


def test_smooth_walk(inputs_mod):
    w1 = inputs_mod.smooth_walk(11, 1e-8, 1e6, 200001, threads=1)
    w8 = inputs_mod.smooth_walk(11, 1e-8, 1e6, 200001, threads=8)
    assert np.array_equal(w1, w8)
    assert np.all(np.diff(w1) >= 0)
    assert w1[0] >= 1e-8 and w1[-1] <= 1e6 * (1 + 1e-12)


def test_tables(inputs_mod):
    t = inputs_mod.single64_table()
    assert t.shape == (64,) and np.all(np.diff(t) >= 0)
    assert 0.9e-6 <= t[0] and t[-1] <= 1.1e4
    for n in (100, 300, 1000):
        s = inputs_mod.single_table(n)
        assert s.shape == (n,) and s[0] == 1e-8 and s[-1] == 1e6 and np.all(np.diff(s) >= 0)
    p = inputs_mod.paper_shape_table()
    assert p.shape == (110,) and p[0] == 3e-6 and p[-1] == 5.4e4


def test_batched_layout(inputs_mod):
    b = inputs_mod.batched_layout()
    assert b.num_tables == 512
    sizes = np.diff(b.table_off)
    assert sizes.min() >= 20 and sizes.max() <= 2000
    counts = np.diff(b.query_off)
    assert counts.min() >= 10**4 - 1 and counts.max() <= 10**7
    # expected total about 7.4e8
    assert 5e8 < b.num_queries < 1e9
    for t in range(0, 512, 37):
        tab = b.table(t)
        assert np.all(np.diff(tab) >= 0) and np.log10(tab[-1] / tab[0]) >= 1.0 - 1e-9


def test_paired_layout(inputs_mod):
    p = inputs_mod.paired_layout(materials=64, total_pairs=10**6)
    assert p.num_pairs == 10**6 and p.num_materials == 64
    assert np.array_equal(p.rho.query_off, p.temp.query_off)
    assert np.diff(p.rho.table_off).min() >= 50 and np.diff(p.rho.table_off).max() <= 4000
    assert np.diff(p.temp.table_off).min() >= 20 and np.diff(p.temp.table_off).max() <= 1000
    r, t = inputs_mod.paired_targets(p)
    assert r.shape == (10**6,) and t.shape == (10**6,)
