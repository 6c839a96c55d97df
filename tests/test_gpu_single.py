"""GPU parity of the single-table kernels against the CPU oracle (bit-exact).

Every case compares int32 indices element by element with
``oracle.search_lt`` on the same host bytes, or, at full workload sizes,
checks every index with the bracket property and a seeded sample with the
oracle's definition.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

ALGOS = ["auto", "binary", "ballot", "exphash", "binary_global", "loghash", "skiplist"]
TILE = 512 * 8           # targets per workgroup tile at the default launch shape


def say(*a):
    print(*a, flush=True)


def run(binding, dev, table, x, algo="auto", bits=-1):
    t = torch.from_numpy(np.ascontiguousarray(table)).to(dev)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    out = binding.search_with(t, xt, algo, bits)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def mixed_targets(inputs_mod, table, m, seed):
    """Random log-uniform targets with exact hits, neighbours and specials."""
    x = inputs_mod.table_targets(table, m, seed=seed)
    n = table.shape[0]
    if n:
        k = np.arange(0, m, 7)
        x[k] = table[k % n]
        k = np.arange(3, m, 11)
        x[k] = np.nextafter(table[k % n], np.inf)
        k = np.arange(5, m, 13)
        x[k] = np.nextafter(table[k % n], -np.inf)
    sp = inputs_mod.special_values()
    x[1:1 + sp.shape[0]] = sp
    return x


@pytest.fixture(scope="module")
def binding(gpu):
    from paper_2112_03229_amd import binding as b
    return b


@pytest.mark.parametrize("n", [1, 2, 3, 7, 63, 64, 65, 100, 110, 300, 1000, 2000, 4000])
def test_parity_across_sizes(binding, gpu, oracle_mod, inputs_mod, n):
    table = inputs_mod.single_table(n) if n >= 2 else np.array([1.0])
    m = 20 * TILE + 77
    x = mixed_targets(inputs_mod, table, m, seed=n)
    want = oracle_mod.search_lt(table, x)
    for algo in ALGOS:
        say(f"case n={n} m={m} algo={algo}")
        got = run(binding, gpu, table, x, algo)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (algo, n, bad[:5], got[bad[:5]], want[bad[:5]], x[bad[:5]])


@pytest.mark.parametrize("kind", ["random", "smooth"])
def test_parity_smooth_and_random(binding, gpu, oracle_mod, inputs_mod, kind):
    table = inputs_mod.single_table(300)
    m = 64 * TILE + 5
    x = inputs_mod.table_targets(table, m, seed=2, kind=kind)
    want = oracle_mod.search_lt(table, x)
    for algo in ALGOS:
        say(f"case kind={kind} algo={algo}")
        assert np.array_equal(run(binding, gpu, table, x, algo), want), algo


def edge_tables():
    return {
        "zeros_denormals": np.array([0.0, 0.0, 5e-324, 1e-320, 1e-310, 2.2250738585072014e-308,
                                     1e-300, 1.0, 1.0, 1.0, 2.0, 1e300]),
        "duplicates": np.repeat(np.array([1e-3, 1.0, 7.0, 1e5]), [5, 17, 1, 30]),
        "all_equal": np.full(50, 3.25),
        "with_negatives": np.array([-1e10, -5.0, -1.0, -0.0, 0.0, 1e-5, 3.0, 1e20]),
        "negative_zero_first": np.array([-0.0, 0.0, 1.0, 2.0]),
        "with_inf": np.array([1e-3, 1.0, 10.0, np.inf]),
        "single_zero": np.array([0.0]),
        "huge_range": np.array([5e-324, 1e-200, 1e-100, 1.0, 1e100, 1e200, 1.7976931348623157e308]),
        "narrow": 1.0 + np.arange(200) * 2.0 ** -40,
    }


@pytest.mark.parametrize("name", list(edge_tables().keys()))
def test_edge_tables(binding, gpu, oracle_mod, inputs_mod, name):
    table = edge_tables()[name].astype(np.float64)
    assert np.all(table[:-1] <= table[1:])
    m = 3 * TILE + 19
    x = inputs_mod.log_uniform(17, 4, 1e-320, 1e305, m)
    x[::3] *= -1.0
    x[:table.shape[0]] = table
    x[table.shape[0]:2 * table.shape[0]] = np.nextafter(table, np.inf)
    sp = inputs_mod.special_values()
    x[-sp.shape[0]:] = sp
    want = oracle_mod.search_lt(table, x)
    for algo in ALGOS:
        say(f"case table={name} algo={algo}")
        got = run(binding, gpu, table, x, algo)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (algo, name, bad[:5], got[bad[:5]], want[bad[:5]], x[bad[:5]])


def test_empty_table_and_tiny_m(binding, gpu, oracle_mod, inputs_mod):
    empty = np.zeros(0)
    x = inputs_mod.log_uniform(1, 1, 1e-3, 1e3, 1000)
    for algo in ALGOS:
        say(f"case n=0 algo={algo}")
        assert np.all(run(binding, gpu, empty, x, algo) == -1)
    table = inputs_mod.single_table(100)
    for m in (1, 2, 63, 64, 65, 255, 256, 257, TILE - 1, TILE, TILE + 1):
        xm = inputs_mod.table_targets(table, m, seed=m)
        want = oracle_mod.search_lt(table, xm)
        for algo in ALGOS:
            assert np.array_equal(run(binding, gpu, table, xm, algo), want), (m, algo)
    # m == 0 is a no-op
    t = torch.from_numpy(table).to(gpu)
    out = binding.search_sorted_batch(t, torch.zeros(0, dtype=torch.float64, device=gpu))
    assert out.numel() == 0


def test_unaligned_views(binding, gpu, oracle_mod, inputs_mod):
    table = inputs_mod.single_table(1000)
    x = inputs_mod.table_targets(table, 5 * TILE + 3, seed=4)
    t = torch.from_numpy(table).to(gpu)
    xt = torch.from_numpy(x).to(gpu)
    for off in (1, 3):
        out = torch.full((xt.numel() - off + 1,), -9, dtype=torch.int32, device=gpu)
        binding.search_sorted_batch(t[1:], xt[off:], out[1:])
        torch.cuda.synchronize()
        want = oracle_mod.search_lt(table[1:], x[off:])
        got = out.cpu().numpy()
        assert got[0] == -9 and np.array_equal(got[1:], want)


@pytest.mark.parametrize("bits", list(range(0, 9)) + [12, 20])
def test_exphash_bucket_bits(binding, gpu, oracle_mod, inputs_mod, bits):
    table = inputs_mod.single_table(1000)
    x = mixed_targets(inputs_mod, table, 9 * TILE + 1, seed=bits)
    want = oracle_mod.search_lt(table, x)
    say(f"case bits={bits}")
    assert np.array_equal(run(binding, gpu, table, x, "exphash", bits), want)


def test_exphash_small_caps_force_bin_bisection(binding, gpu, oracle_mod, inputs_mod):
    table = inputs_mod.single_table(2000)
    x = mixed_targets(inputs_mod, table, 9 * TILE + 1, seed=3)
    want = oracle_mod.search_lt(table, x)
    try:
        for cap in (16, 64, 256):
            say(f"case cap={cap}")
            binding.set_option(binding.OPT_BUCKET_CAP, cap)
            assert np.array_equal(run(binding, gpu, table, x, "exphash"), want), cap
    finally:
        binding.set_option(binding.OPT_BUCKET_CAP, 0)


@pytest.mark.parametrize("block", [256, 512, 1024])
@pytest.mark.parametrize("q", [4, 8])
def test_launch_shapes(binding, gpu, oracle_mod, inputs_mod, block, q):
    """Every kernel at every workgroup size and both target counts per lane
    (SS_OPT_TARGETS_PER_LANE), with the default grid, one workgroup and
    seven (grid-stride loops over many tiles), on a ragged target count."""
    table = inputs_mod.single_table(300)
    x = mixed_targets(inputs_mod, table, 40 * 1024 + 9, seed=block)
    want = oracle_mod.search_lt(table, x)
    try:
        binding.set_option(binding.OPT_BLOCK_SIZE, block)
        binding.set_option(binding.OPT_TARGETS_PER_LANE, q)
        for grid in (0, 1, 7):
            binding.set_option(binding.OPT_GRID_BLOCKS, grid)
            for algo in ALGOS:
                say(f"case block={block} q={q} grid={grid} algo={algo}")
                assert np.array_equal(run(binding, gpu, table, x, algo), want)
    finally:
        binding.set_option(binding.OPT_BLOCK_SIZE, 0)
        binding.set_option(binding.OPT_TARGETS_PER_LANE, 0)
        binding.set_option(binding.OPT_GRID_BLOCKS, 0)


def test_paper_shape_every_kernel(binding, gpu, oracle_mod, inputs_mod):
    """The paper's measured configuration: the 110-entry stand-in for the
    density axis and 5e6 targets log-uniform on [1e-10, 1e10] (about half
    outside the table), every kernel bit for bit against the oracle."""
    table = inputs_mod.paper_shape_table()
    x = inputs_mod.paper_shape_targets(5 * 10**6)
    outside = np.mean((x < table[0]) | (x > table[-1]))
    assert 0.4 < outside < 0.6
    want = oracle_mod.search_lt(table, x)
    for algo in ALGOS:
        say(f"case paper shape algo={algo}")
        got = run(binding, gpu, table, x, algo)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (algo, bad[:5], got[bad[:5]], want[bad[:5]])


@pytest.mark.parametrize("s", [0, 3, 5, 8])
@pytest.mark.parametrize("n", [64, 110, 1000, 4000])
def test_exphash_bins_match_oracle(binding, gpu, oracle_mod, inputs_mod, n, s):
    table = inputs_mod.paper_shape_table() if n == 110 else inputs_mod.single_table(n)
    kmin, C = oracle_mod.exponent_bins(table, s)
    info, counts = binding.exphash_bins(torch.from_numpy(table).to(gpu), s, cap=1 << 16)
    assert info["bits"] == s and info["kmin"] == kmin and info["nb"] == C.shape[0] - 1
    assert np.array_equal(counts.cpu().numpy().astype(np.int64), C)
    assert info["max_occupancy"] == min(int(np.diff(C).max()), 9)


@pytest.mark.parametrize("n,nb", [(110, 110), (110, 34), (1000, 4096), (2000, 500), (4000, 16384),
                                  (300, 7)])
def test_loghash_bins_match_oracle(binding, gpu, oracle_mod, inputs_mod, n, nb):
    """Device bins against Eq. 1-3 in float64.  The device evaluates the key
    in FP32, so an entry whose exact log_b value lies within 2e-3 of a bin
    edge may land in the neighbouring bin; every other entry's bin must be
    the oracle's."""
    table = inputs_mod.paper_shape_table() if n == 110 else inputs_mod.single_table(n)
    info, counts = binding.loghash_bins(torch.from_numpy(table).to(gpu), nb)
    C = counts.cpu().numpy().astype(np.int64)
    assert info["nb"] == nb and C[0] == 0 and C[-1] == n and np.all(np.diff(C) >= 0)
    dev_key = np.searchsorted(C, np.arange(n), side="right") - 1
    b = oracle_mod.log_hash_base(table[0], table[-1], nb)
    lb0 = np.log(table[0]) / np.log(b)
    phi = lb0 - np.floor(lb0)
    if min(phi, 1 - phi) >= 1e-4:
        # the oracle's keys (Eq. 2 in float64), and its unfloored values
        want = oracle_mod.log_hash_key(table, table[0], table[-1], nb)
        t = np.log(table) / np.log(b) - np.floor(lb0)
        candidates = [(want, t)]
    else:
        # log_b Xmin within rounding of an integer (e.g. the 300-entry table
        # with 7 bins: b = 100 and Xmin = 1e-8 = b^-4): floor(log_b Xmin) is
        # ill-conditioned and either neighbour is a correct evaluation of
        # Eq. 2, so the keys floor(log_b x - log_b Xmin + phi) for phi just
        # above 0 and just below 1 are both accepted
        rel = np.log(table / table[0]) / np.log(b)
        candidates = []
        for ph in (0.0, 1.0 - 1e-12):
            t = rel + ph
            candidates.append((np.clip(np.floor(t), 0, nb - 1).astype(np.int64), t))
    ok = False
    for want, t in candidates:
        near = np.abs(t - np.rint(t)) < 2e-3
        diff = dev_key - want
        if np.all(diff[~near] == 0) and np.all(np.abs(diff[near]) <= 1):
            ok = True
            break
    assert ok, np.nonzero(diff[~near])[0][:5]
    say(f"loghash n={n} nb={nb}: {int(near.sum())} entries near an edge, "
        f"{int(np.count_nonzero(diff))} in the neighbouring bin, K={info['max_occupancy']}")
    # the FP32 parameters are Eq. 1's base and Eq. 2's offset
    assert abs(info["S"] * np.log2(b) - 1.0) < 1e-5
    dphi = abs(info["phi"] - phi)
    assert min(dphi, 1 - dphi) < 1e-3
    if not near.any():
        assert info["max_occupancy"] == min(int(np.diff(C).max()), 9)


@pytest.mark.parametrize("cap", [4, 16, 64, 4096, 65535])
def test_loghash_bin_counts(binding, gpu, oracle_mod, inputs_mod, cap):
    """Few bins (long bins: bisection inside the bin) to many."""
    table = inputs_mod.single_table(2000)
    x = mixed_targets(inputs_mod, table, 9 * TILE + 1, seed=cap)
    want = oracle_mod.search_lt(table, x)
    try:
        say(f"case loghash bins={cap}")
        binding.set_option(binding.OPT_BUCKET_CAP, cap)
        assert np.array_equal(run(binding, gpu, table, x, "loghash"), want), cap
    finally:
        binding.set_option(binding.OPT_BUCKET_CAP, 0)


def test_validate_table(binding, gpu, inputs_mod):
    table = inputs_mod.single_table(1000)
    t = torch.from_numpy(table).to(gpu)
    assert binding.validate_table(t) == -1
    bad = table.copy()
    bad[700], bad[701] = bad[701], bad[700]
    assert binding.validate_table(torch.from_numpy(bad).to(gpu)) == 700
    nan = table.copy()
    nan[33] = np.nan
    assert binding.validate_table(torch.from_numpy(nan).to(gpu)) in (32, 33)


def test_unsorted_table_stays_in_bounds(binding, gpu, inputs_mod):
    # precondition violated: results are unspecified but must lie in [-1, n-1]
    rng_tab = inputs_mod.log_uniform(5, 1, 1e-8, 1e6, 500)
    x = inputs_mod.log_uniform(6, 1, 1e-9, 1e7, 4 * TILE + 3)
    for algo in ALGOS:
        got = run(binding, gpu, rng_tab, x, algo)
        assert got.min() >= -1 and got.max() <= 499, algo


def test_non_default_stream_and_graph_replay(binding, gpu, oracle_mod, inputs_mod):
    table = inputs_mod.single_table(1000)
    x = inputs_mod.table_targets(table, 50 * TILE + 11, seed=8)
    want = oracle_mod.search_lt(table, x)
    t = torch.from_numpy(table).to(gpu)
    xt = torch.from_numpy(x).to(gpu)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = binding.search_sorted_batch(t, xt)
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    # capture one call in a graph and replay it, with eager work in between
    out2 = torch.full_like(out, -5)
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    with torch.cuda.stream(cs):
        binding.search_sorted_batch(t, xt, out2)  # warm-up outside capture
    cs.synchronize()
    out2.fill_(-5)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=cs):
        binding.search_sorted_batch(t, xt, out2)
    for r in range(3):
        out2.fill_(-5)
        _ = (xt * 2.0).sum()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out2.cpu().numpy(), want), r


@pytest.mark.parametrize("algo", ["exphash", "loghash", "skiplist", "ballot"])
def test_full_size_forced(binding, gpu, oracle_mod, inputs_mod, algo):
    """Each kernel the automatic choice does not take, forced on the
    1000-entry table with 1e8 targets in its default launch shape."""
    table = inputs_mod.single_table(1000)
    m = 10**8
    t = torch.from_numpy(table).to(gpu)
    host = torch.empty(m, dtype=torch.float64).pin_memory()
    inputs_mod.table_targets(table, m, seed=11, out=host.numpy())
    say(f"case full {algo} n=1000")
    out = binding.search_with(t, host.to(gpu), algo)
    got = out.cpu().numpy()
    x = host.numpy()
    bad, first = oracle_mod.check_bracket(table, x, got)
    assert bad == 0, first
    pos = (inputs_mod.uniform(1000, 98, 200000) * m).astype(np.int64)
    assert np.array_equal(got[pos], oracle_mod.search_lt_at(table, x, pos))


@pytest.mark.parametrize("n", [100, 300, 1000])
def test_full_size_single_tables(binding, gpu, oracle_mod, inputs_mod, n):
    """1e8 targets per table and order, in the benchmark's launch shape:
    every index passes the bracket check; a seeded sample equals the
    oracle's definition."""
    table = inputs_mod.single_table(n)
    m = 10**8
    t = torch.from_numpy(table).to(gpu)
    host = torch.empty(m, dtype=torch.float64).pin_memory()
    for kind in ("random", "smooth"):
        say(f"case full n={n} kind={kind}")
        inputs_mod.table_targets(table, m, seed=7, kind=kind, out=host.numpy())
        xt = host.to(gpu, non_blocking=True)
        out = binding.search_sorted_batch(t, xt)
        got = out.cpu().numpy()
        x = host.numpy()
        bad, first = oracle_mod.check_bracket(table, x, got)
        assert bad == 0, (kind, first)
        pos = (inputs_mod.uniform(n, 99, 200000) * m).astype(np.int64)
        assert np.array_equal(got[pos], oracle_mod.search_lt_at(table, x, pos))
        del xt, out


def test_full_size_single64(binding, gpu, oracle_mod, inputs_mod):
    table = inputs_mod.single64_table()
    x = inputs_mod.table_targets(table, 10**6, seed=64)
    want = oracle_mod.search_lt(table, x)
    for algo in ALGOS:
        say(f"case single64 algo={algo}")
        assert np.array_equal(run(binding, gpu, table, x, algo), want), algo


@pytest.mark.parametrize("algo", ["auto", "exphash"])
def test_more_than_2_31_targets(binding, gpu, oracle_mod, inputs_mod, algo):
    """m = 2^31 + 4111 targets in one call (64-bit target positions): target
    k is a[k mod n] for even k (idx = k mod n - 1) and the next double above
    it for odd k (idx = k mod n), checked on the device in chunks; positions
    around 2^31 and a seeded sample are compared with the oracle."""
    table = inputs_mod.single_table(100)
    assert np.all(np.diff(table) > 0)
    n = table.size
    m = 2**31 + 4111
    say(f"case m={m} algo={algo}")
    t = torch.from_numpy(table).to(gpu)
    x = torch.empty(m, dtype=torch.float64, device=gpu)
    chunk = 1 << 28
    for k0 in range(0, m, chunk):
        k = torch.arange(k0, min(m, k0 + chunk), device=gpu, dtype=torch.int64)
        v = t[k % n]
        x[k0:k0 + k.numel()] = torch.where(k % 2 == 1, torch.nextafter(v, torch.full_like(v, np.inf)), v)
    out = binding.search_with(t, x, algo)
    for k0 in range(0, m, chunk):
        k = torch.arange(k0, min(m, k0 + chunk), device=gpu, dtype=torch.int64)
        want = (k % n) - 1 + (k % 2)
        bad = int((out[k0:k0 + k.numel()].to(torch.int64) != want).sum())
        assert bad == 0, (k0, bad)
    pos = np.concatenate([np.arange(2**31 - 2048, m), (inputs_mod.uniform(77, 5, 4096) * m).astype(np.int64)])
    pt = torch.from_numpy(pos).to(gpu)
    xs = x[pt].cpu().numpy()
    assert np.array_equal(out[pt].cpu().numpy(), oracle_mod.search_lt(table, xs))
    del x, out


def fuzz_table(rng, n):
    """A sorted table of n entries from one of several distributions:
    log-spaced, with runs of duplicates, signed, with zeros and denormals,
    with infinities at the end, or clustered."""
    kind = rng.integers(0, 6)
    if kind == 0:
        t = 10.0 ** rng.uniform(-12, 12, n)
    elif kind == 1:
        t = np.repeat(10.0 ** rng.uniform(-3, 3, max(1, n // 4 + 1)), 4)[:n]
    elif kind == 2:
        t = rng.normal(0, 1e3, n)
    elif kind == 3:
        t = np.concatenate([np.zeros(n // 8), np.full(n // 8, 5e-324), 10.0 ** rng.uniform(-310, -300, n // 8),
                            10.0 ** rng.uniform(-5, 5, n - 3 * (n // 8))])
    elif kind == 4:
        t = 10.0 ** rng.uniform(-2, 2, n)
        t[-min(n, 2):] = np.inf
    else:
        t = 1.0 + rng.integers(0, 7, n) * 2.0 ** -52
    return np.sort(t.astype(np.float64))


def fuzz_targets(rng, table, m):
    n = table.size
    parts = [10.0 ** rng.uniform(-14, 14, m // 4) * rng.choice([-1.0, 1.0], m // 4)]
    if n:
        fin = table[np.isfinite(table)]
        if fin.size:
            pick = rng.choice(fin, m // 4)
            parts += [pick, np.nextafter(pick, np.inf), np.nextafter(pick, -np.inf)]
    x = np.concatenate(parts + [inputs_special()])
    rng.shuffle(x)
    return x


def inputs_special():
    return np.array([np.nan, -0.0, 0.0, 5e-324, -5e-324, np.inf, -np.inf, 1.7976931348623157e308])


@pytest.mark.parametrize("seed", range(6))
def test_random_tables_every_kernel(binding, gpu, oracle_mod, seed):
    """Seeded fuzzing: 40 random tables per seed (0..5000 entries, six
    distributions) and targets at, between and around their entries, every
    kernel bit for bit against the oracle."""
    rng = np.random.default_rng(1000 + seed)
    for case in range(40):
        n = int(rng.choice([0, 1, 2, 3, 7, 63, 64, 65, 130, 1000, 4095, 5000]))
        table = fuzz_table(rng, n)
        x = fuzz_targets(rng, table, int(rng.integers(1, 3 * TILE)))
        want = oracle_mod.search_lt(table, x)
        for algo in ALGOS:
            got = run(binding, gpu, table, x, algo)
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, (seed, case, n, algo, bad[:3], got[bad[:3]], want[bad[:3]], x[bad[:3]])


def test_random_batches(binding, gpu, oracle_mod):
    """A batched plan over 60 fuzzed tables (empty target slices and empty
    tables included) against the oracle."""
    rng = np.random.default_rng(77)
    tabs, xs, counts = [], [], []
    for t in range(60):
        n = int(rng.choice([0, 1, 5, 64, 300, 2000]))
        tab = fuzz_table(rng, n)
        m = int(rng.choice([0, 1, 100, 5000, 70000]))
        x = fuzz_targets(rng, tab, max(m, 1))[:m]
        tabs.append(tab)
        xs.append(x)
        counts.append(x.size)
    toff = np.concatenate([[0], np.cumsum([t.size for t in tabs])]).astype(np.int64)
    qoff = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    tables = np.concatenate(tabs)
    x = np.concatenate(xs)
    want = oracle_mod.search_lt_segments(tables, toff, x, qoff)
    plan = binding.MultiPlan(torch.from_numpy(tables).to(gpu), toff, qoff)
    got = plan.search(torch.from_numpy(x).to(gpu)).cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]])
