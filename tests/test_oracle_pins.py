"""Pins the CPU oracle to things other than itself (no GPU needed).

* Library routines: Python's ``bisect.bisect_left`` and numpy's
  ``searchsorted(side="left")`` count the entries strictly below a target, so
  for non-NaN targets idx = bisect_left - 1.
* Brute force over every sorted table of length 0..4 drawn from a small
  alphabet with duplicates, crossed with exact hits, midpoints and specials.
* The bracket property a[i] < x <= a[i+1], and planted mistakes that it must
  catch (the mistakes are planted in oracle outputs, on the CPU).
* The exponent hash key (Sec. 3.5) through two independent routes: the
  IEEE-754 bit pattern (struct) and math.frexp / log2.
* The paper's closed-form binning numbers for its density axis (Sec. 5.2).
"""
import bisect
import itertools
import json
import math
import os
import struct

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

SPECIALS = [float("nan"), -float("nan"), float("inf"), -float("inf"), 0.0, -0.0, 5e-324,
            -5e-324, 2.2250738585072014e-308, 1e-300, 1.0, -1.0, 1.7976931348623157e308]


def lib_idx(table, x):
    """Reference through a library routine (non-NaN x only)."""
    return bisect.bisect_left(list(table), x) - 1


def test_tiny_tables_brute_force(oracle_mod):
    alphabet = [-2.0, -0.0, 0.0, 5e-324, 1e-310, 1.0, 1.5, 3.0, float("inf")]
    probes = sorted(set(alphabet + [(a + b) / 2 for a, b in zip(alphabet, alphabet[1:])
                                    if math.isfinite(a + b)] + [-float("inf"), 7.0, -7.0]))
    probes_arr = np.array(probes + [float("nan")])
    checked = 0
    for n in range(0, 5):
        for combo in itertools.combinations_with_replacement(alphabet, n):
            table = np.array(sorted(combo), dtype=np.float64)
            got = oracle_mod.search_lt(table, probes_arr, threads=1)
            for k, x in enumerate(probes_arr):
                if math.isnan(x):
                    assert got[k] == -1
                else:
                    assert got[k] == lib_idx(table, x), (table, x)
                checked += 1
    assert checked > 10000


def test_matches_numpy_on_log_tables(oracle_mod, inputs_mod):
    for n in (1, 2, 3, 63, 64, 65, 110, 1000):
        table = inputs_mod.sorted_log_table(n, n, 1e-8, 1e6)
        x = inputs_mod.log_uniform(n, 2, 0.5e-8, 2e6, 20000)
        x[::97] = table[np.arange(x[::97].shape[0]) % n]          # exact hits
        x[1::89] = np.nextafter(table[np.arange(x[1::89].shape[0]) % n], np.inf)
        x[2::83] = np.nextafter(table[np.arange(x[2::83].shape[0]) % n], -np.inf)
        want = np.searchsorted(table, x, side="left") - 1
        assert np.array_equal(oracle_mod.search_lt(table, x), want)


@settings(max_examples=60, deadline=None)
@given(st.lists(st.floats(min_value=1e-12, max_value=1e12), min_size=0, max_size=50),
       st.lists(st.floats(allow_nan=False), min_size=1, max_size=60))
def test_property_against_bisect(oracle_mod, raw_table, raw_x):
    table = np.array(sorted(raw_table), dtype=np.float64)
    x = np.array(raw_x, dtype=np.float64)
    got = oracle_mod.search_lt(table, x, threads=2)
    want = np.array([lib_idx(table, v) for v in x], dtype=np.int32)
    assert np.array_equal(got, want)


def test_specials(oracle_mod):
    table = np.array([0.0, 5e-324, 1e-310, 1.0, 2.0, 2.0, 1e300], dtype=np.float64)
    x = np.array([float("nan"), -float("nan"), -float("inf"), float("inf"), -0.0, 0.0, 5e-324,
                  2e-323, 2.0, np.nextafter(2.0, 3.0), 1e308], dtype=np.float64)
    got = oracle_mod.search_lt(table, x)
    # -0.0 == +0.0, so nothing is below either; a hit on a duplicate run gives
    # the entry before the run; +inf is above every finite entry.
    assert got.tolist() == [-1, -1, -1, 6, -1, -1, 0, 1, 3, 5, 6]
    tinf = np.array([1.0, float("inf")])
    assert oracle_mod.search_lt(tinf, np.array([float("inf")])).tolist() == [0]


def test_threads_do_not_change_results(oracle_mod, inputs_mod):
    table = inputs_mod.single_table(300)
    x = inputs_mod.table_targets(table, 100003, seed=5)
    a, used1 = oracle_mod.search_lt(table, x, threads=1, return_threads=True)
    b, used7 = oracle_mod.search_lt(table, x, threads=7, return_threads=True)
    assert used1 == 1 and used7 == 7
    assert np.array_equal(a, b)
    pos = np.array([0, 5, 99999, 100002, 17], dtype=np.int64)
    assert np.array_equal(oracle_mod.search_lt_at(table, x, pos), a[pos])


def test_segments_match_numpy(oracle_mod, inputs_mod):
    batch = inputs_mod.batched_layout(seed=3, num_tables=9, query_scale=1e-3)
    x = inputs_mod.batched_targets(batch, seed=3)
    got = oracle_mod.search_lt_segments(batch.tables, batch.table_off, x, batch.query_off)
    for t in range(batch.num_tables):
        q0, q1 = batch.query_off[t], batch.query_off[t + 1]
        want = np.searchsorted(batch.table(t), x[q0:q1], side="left") - 1
        assert np.array_equal(got[q0:q1], want)


def test_bracket_accepts_truth_and_catches_planted_mistakes(oracle_mod, inputs_mod):
    table = inputs_mod.single_table(100)
    x = inputs_mod.table_targets(table, 50000, seed=9)
    x[:100] = table[:100]                       # exact hits
    x[100] = np.nan
    idx = oracle_mod.search_lt(table, x)
    assert oracle_mod.check_bracket(table, x, idx) == (0, -1)
    # "<=" reading of the comparison (side="right") differs exactly at hits
    le = (np.searchsorted(table, x, side="right") - 1).astype(np.int32)
    le[100] = -1
    bad, first = oracle_mod.check_bracket(table, x, le)
    assert bad == 100 and first == 0
    for delta in (+1, -1):
        wrong = idx.copy()
        wrong[12345] += delta
        assert oracle_mod.check_bracket(table, x, wrong) == (1, 12345)
    nan_wrong = idx.copy()
    nan_wrong[100] = table.shape[0] - 1
    assert oracle_mod.check_bracket(table, x, nan_wrong) == (1, 100)
    out_of_range = idx.copy()
    out_of_range[7] = table.shape[0]
    assert oracle_mod.check_bracket(table, x, out_of_range)[0] == 1


def _bits_key(v, s):
    (u,) = struct.unpack("<Q", struct.pack("<d", v))
    return u >> (52 - s)


def test_exponent_key_two_routes(oracle_mod, inputs_mod):
    vals = list(inputs_mod.log_uniform(1, 11, 1e-300, 1e300, 3000))
    vals += [0.0, 5e-324, 1e-310, 2.2250738585072009e-308, 2.2250738585072014e-308, 1.0,
             np.nextafter(1.0, 2.0), 2.0, 1.7976931348623157e308, float("inf")]
    for s in (0, 1, 3, 5, 8, 13, 20):
        for v in vals:
            assert oracle_mod.exponent_key(v, s) == _bits_key(v, s), (v, s)
    # s = 0 is the biased base-2 exponent: floor(log2 v) + 1023 for normal v
    for v in vals:
        if 2.2250738585072014e-308 <= v < float("inf"):
            assert oracle_mod.exponent_key(v, 0) == math.frexp(v)[1] - 1 + 1023
    # monotone over sorted non-negative values
    sv = np.sort(np.array([v for v in vals if v >= 0]))
    for s in (0, 5, 20):
        keys = [oracle_mod.exponent_key(v, s) for v in sv]
        assert all(a <= b for a, b in zip(keys, keys[1:]))


def test_paper_binning_closed_form(oracle_mod, inputs_mod):
    with open(os.path.join(GOLDEN, "paper_binning.json")) as f:
        g = json.load(f)
    lo, hi, n = g["table_min"], g["table_max"], g["n"]
    # "about 34 powers of two" between the smallest and largest value
    assert round(math.log2(hi / lo)) == g["powers_of_two_spanned"]
    assert round(n / g["powers_of_two_spanned"], 3) == g["entries_per_bin"]
    table = inputs_mod.paper_shape_table()
    assert table.shape[0] == n and table[0] == lo and table[-1] == hi
    kmin, C = oracle_mod.exponent_bins(table, 0)
    nb = C.shape[0] - 1
    # the binades floor(log2 3e-6) = -19 .. floor(log2 5.4e4) = 15: 35 bins
    assert kmin == -19 + 1023 and nb == 35
    assert abs(n / nb - g["entries_per_bin"]) < 0.1
    assert C[0] == 0 and C[-1] == n and np.all(np.diff(C) >= 0)
    e = np.floor(np.log2(table)).astype(np.int64)   # library route to the exponent
    for b in range(nb):
        assert C[b + 1] - C[b] == np.count_nonzero(e == -19 + b)


@pytest.mark.parametrize("s", [0, 2, 5, 7])
def test_exponent_bins_brute_force(oracle_mod, inputs_mod, s):
    table = inputs_mod.single_table(300)
    kmin, C = oracle_mod.exponent_bins(table, s)
    keys = np.array([_bits_key(v, s) for v in table])
    assert kmin == keys[0]
    nb = C.shape[0] - 1
    assert nb == keys[-1] - keys[0] + 1
    for b in range(nb + 1):
        assert C[b] == np.count_nonzero(keys - kmin < b)


# ---------------------------------------------------------------------------
# Logarithm hash (Sec. 3.4, Eq. 1-3): pinned through the bin edges b^k
# computed with pow (a route that never takes a logarithm), Eq. 1's closed
# form and brute-force bin counts.
# ---------------------------------------------------------------------------

LOG_HASH_CASES = [(3e-6, 5.4e4, 110), (3e-6, 5.4e4, 34), (1e-8, 1e6, 1000), (1.0, 2.0, 64),
                  (0.5, 3e7, 4096), (1e-300, 1e300, 50)]


@pytest.mark.parametrize("xmin,xmax,H", LOG_HASH_CASES)
def test_log_hash_base_closed_form(oracle_mod, xmin, xmax, H):
    b = oracle_mod.log_hash_base(xmin, xmax, H)
    # Eq. 1: b^|H| = Xmax / Xmin (in logarithms where the power overflows)
    if xmax / xmin < 1e300:
        assert math.isclose(b ** H, xmax / xmin, rel_tol=1e-10)
    assert math.isclose(H * math.log(b), math.log(xmax) - math.log(xmin), rel_tol=1e-12)
    # Eq. 2 at the ends: Xmin hashes to 0; Xmax to |H| before the clamp
    # (its log lies exactly |H| bases above Xmin's), so into |H| - 1 after
    assert oracle_mod.log_hash_raw(xmin, xmin, b) == 0
    assert oracle_mod.log_hash_raw(xmax, xmin, b) in (H - 1, H)
    assert oracle_mod.log_hash_key(xmax, xmin, xmax, H)[0] == H - 1


@pytest.mark.parametrize("xmin,xmax,H", LOG_HASH_CASES)
def test_log_hash_key_against_pow_edges(oracle_mod, inputs_mod, xmin, xmax, H):
    """key(x) = i  <=>  b^(F+i) <= x < b^(F+i+1), F = floor(log_b Xmin), for x
    inside [Xmin, Xmax], except within rounding of an edge."""
    b = oracle_mod.log_hash_base(xmin, xmax, H)
    F = math.floor(math.log(xmin) / math.log(b))
    x = inputs_mod.log_uniform(77, 1, xmin, xmax, 20000)
    keys = oracle_mod.log_hash_key(x, xmin, xmax, H)
    checked = 0
    for xi, k in zip(x, keys):
        lo, hi = b ** (F + k), b ** (F + k + 1)
        near = min(abs(xi / lo - 1), abs(xi / hi - 1)) < 1e-9
        if k == H - 1:
            hi = math.inf   # the clamp folds the rest into the last bin
        if not near:
            assert lo <= xi < hi, (xi, k, lo, hi)
            checked += 1
    assert checked > 19000


def test_log_hash_specials_and_monotone(oracle_mod, inputs_mod):
    xmin, xmax, H = 1e-8, 1e6, 500
    k = oracle_mod.log_hash_key([float("nan"), -1.0, 0.0, 5e-324, 1e-20, float("inf"), 1e300],
                                xmin, xmax, H)
    assert list(k) == [0, 0, 0, 0, 0, H - 1, H - 1]
    x = np.sort(inputs_mod.log_uniform(5, 2, 1e-9, 1e7, 50000))
    assert np.all(np.diff(oracle_mod.log_hash_key(x, xmin, xmax, H)) >= 0)


@pytest.mark.parametrize("n,H", [(110, 110), (100, 400), (1000, 64), (2000, 8192)])
def test_log_hash_bins_brute_force(oracle_mod, inputs_mod, n, H):
    table = inputs_mod.single_table(n) if n != 110 else inputs_mod.paper_shape_table()
    C = oracle_mod.log_hash_bins(table, H)
    assert C.shape == (H + 1,) and C[0] == 0 and C[-1] == n and np.all(np.diff(C) >= 0)
    # route 1: per-entry keys, counted one bin at a time
    keys = oracle_mod.log_hash_key(table, table[0], table[-1], H)
    for i in range(H + 1):
        assert C[i] == int(np.count_nonzero(keys < i))
    # route 2: entries below each interior edge b^(F+i), by pow and a sorted
    # count; entries within rounding of an edge may sit on either side
    b = oracle_mod.log_hash_base(table[0], table[-1], H)
    F = math.floor(math.log(table[0]) / math.log(b))
    for i in range(1, H):
        edge = b ** (F + i)
        below = int(np.searchsorted(table, edge, side="left"))
        slack = int(np.count_nonzero(np.abs(table / edge - 1) < 1e-9))
        assert abs(int(C[i]) - below) <= slack, (i, C[i], below)


def test_log_hash_paper_table_shape(oracle_mod, inputs_mod):
    """The paper's density axis shape (110 log-spaced entries over
    3e-6..5.4e4) with one bin per entry: every bin holds at most a few
    entries, far fewer than the exponent hash's ~3.2 per binade."""
    table = inputs_mod.paper_shape_table()
    C = oracle_mod.log_hash_bins(table, 110)
    assert np.diff(C).max() <= 3


# ---------------------------------------------------------------------------
# The paper's convention (Sec. 3): last index with a[i] <= x, clamped to
# [0, n-1].  Pinned by bisect.bisect_right and by brute force on tiny tables.
# ---------------------------------------------------------------------------

def test_paper_convention_against_bisect_right(oracle_mod, inputs_mod):
    for n in (1, 2, 5, 110, 1000):
        table = inputs_mod.single_table(n) if n > 1 else np.array([3.0])
        x = inputs_mod.table_targets(table, 5000, seed=n)
        x[::7] = table[np.arange(0, 5000, 7) % n]
        got = oracle_mod.search_le_clamped(table, x)
        want = [min(max(bisect.bisect_right(list(table), v) - 1, 0), n - 1) for v in x]
        assert np.array_equal(got, want), n


def test_paper_convention_tiny_tables(oracle_mod):
    alphabet = [-2.0, -0.0, 0.0, 5e-324, 1.0, 3.0, float("inf")]
    probes = np.array(alphabet + [-float("inf"), 0.5, 2.0, 7.0, float("nan")])
    for n in range(0, 4):
        for tab in itertools.combinations_with_replacement(alphabet, n):
            table = np.array(tab, dtype=np.float64)
            got = oracle_mod.search_le_clamped(table, probes)
            for v, g in zip(probes, got):
                cnt = sum(1 for a in tab if a <= v)
                want = -1 if n == 0 else min(max(cnt - 1, 0), n - 1)
                assert g == want, (tab, v, g, want)
    # the relation to the strict definition: they differ only at exact hits
    # (x equal to an entry) and below the first entry (-1 versus 0)
    table = np.array([1.0, 2.0, 2.0, 5.0])
    x = np.array([0.5, 1.0, 1.5, 2.0, 4.0, 5.0, 9.0])
    assert list(oracle_mod.search_le_clamped(table, x)) == [0, 0, 0, 2, 2, 3, 3]
    assert list(oracle_mod.search_lt(table, x)) == [-1, -1, 0, 0, 2, 2, 3]
