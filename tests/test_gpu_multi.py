"""GPU parity of the batched (many tables, one launch) and paired searches.

Each table's slice of the output must equal the oracle's definition applied
to that table alone (composition), bit for bit.  Full-size workloads (512
tables with ~7.4e8 targets; 4096 materials with 1e9 pairs) are checked on
every index with the bracket property and on a seeded sample with the
oracle's definition.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def binding(gpu):
    from paper_2112_03229_amd import binding as b
    return b


def odd_batch(inputs_mod, seed=5):
    """A batch mixing generated log tables with edge tables: a single entry,
    an empty table, negative entries, duplicates, and empty target slices."""
    base = inputs_mod.batched_layout(seed=seed, num_tables=24, query_scale=2e-3)
    tabs = [base.table(t) for t in range(base.num_tables)]
    counts = list(np.diff(base.query_off))
    extra = [
        (np.array([1.0]), 3001),
        (np.zeros(0), 777),
        (np.array([-5.0, -1.0, -0.0, 0.0, 2.0, 1e10]), 4096),
        (np.repeat(np.array([1e-3, 1.0, 7.0]), [30, 2, 40]), 5000),
        (inputs_mod.single_table(1000), 0),
        (inputs_mod.single_table(2000), 70001),
        (np.array([0.0, 5e-324, 1e-310, 1.0]), 999),
    ]
    for t, c in extra:
        tabs.append(t.astype(np.float64))
        counts.append(c)
    toff = np.zeros(len(tabs) + 1, dtype=np.int64)
    toff[1:] = np.cumsum([t.shape[0] for t in tabs])
    qoff = np.zeros(len(tabs) + 1, dtype=np.int64)
    qoff[1:] = np.cumsum(counts)
    tables = np.concatenate(tabs)
    # targets: log-uniform around each table, with exact hits and specials
    x = np.empty(qoff[-1])
    for t in range(len(tabs)):
        q0, q1 = qoff[t], qoff[t + 1]
        if q1 == q0:
            continue
        tab = tabs[t]
        lo, hi = (0.5 * abs(tab[0]) + 1e-300, 2.0 * abs(tab[-1]) + 1e-300) if tab.size else (1e-3, 1e3)
        lo, hi = min(lo, hi), max(lo, hi)
        seg = inputs_mod.log_uniform(seed + t, 3, lo, max(hi, lo * 10), q1 - q0)
        if tab.size:
            k = np.arange(0, q1 - q0, 5)
            seg[k] = tab[k % tab.size]
        seg[::7] *= -1.0 if tab.size and tab[0] < 0 else 1.0
        sp = inputs_mod.special_values()
        seg[:min(sp.size, seg.size)] = sp[:min(sp.size, seg.size)]
        x[q0:q1] = seg
    return tables, toff, qoff, x


def test_batched_composition(binding, gpu, oracle_mod, inputs_mod):
    tables, toff, qoff, x = odd_batch(inputs_mod)
    want = oracle_mod.search_lt_segments(tables, toff, x, qoff)
    say(f"case batched T={toff.size - 1} m={x.size}")
    plan = binding.MultiPlan(torch.from_numpy(tables).to(gpu), toff, qoff)
    xt = torch.from_numpy(x).to(gpu)
    out = plan.search(xt)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]], x[bad[:5]])
    info = plan.info()
    T = toff.size - 1
    assert info["tables"] == T and info["graph_uses"] == 1
    # generated log tables hash; the table with negative entries bisects
    assert info["algos"][0] == binding.ALGO_EXPHASH
    assert info["algos"][T - 5] == binding.ALGO_BINARY
    # repeat (graph replay), then new buffers (graph parameter update)
    out.fill_(-7)
    plan.search(xt, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    x2 = x.copy()
    x2[::3] = np.where(np.isfinite(x2[::3]), x2[::3] * 0.75, x2[::3])
    want2 = oracle_mod.search_lt_segments(tables, toff, x2, qoff)
    out2 = plan.search(torch.from_numpy(x2).to(gpu))
    torch.cuda.synchronize()
    assert np.array_equal(out2.cpu().numpy(), want2)
    assert plan.info()["graph_uses"] == 3
    plan.close()


@pytest.mark.parametrize("block", [256, 1024])
def test_plan_workgroup_sizes(binding, gpu, oracle_mod, inputs_mod, block):
    """Plans created with another workgroup size (SS_OPT_BLOCK_SIZE): the
    tile size, the tile cut and the tiles per workgroup all follow it.  The
    edge batch and a ragged paired layout in both forms, every index."""
    tables, toff, qoff, x = odd_batch(inputs_mod, seed=11)
    want = oracle_mod.search_lt_segments(tables, toff, x, qoff)
    pairs = ragged_pairs(inputs_mod, 23, 40, 300007)
    rho, temp = inputs_mod.paired_targets(pairs, seed=23)
    want_r = oracle_mod.search_lt_segments(pairs.rho.tables, pairs.rho.table_off, rho,
                                           pairs.rho.query_off)
    want_t = oracle_mod.search_lt_segments(pairs.temp.tables, pairs.temp.table_off, temp,
                                           pairs.temp.query_off)
    try:
        binding.set_option(binding.OPT_BLOCK_SIZE, block)
        say(f"case plan block={block} batched")
        plan = binding.MultiPlan(torch.from_numpy(tables).to(gpu), toff, qoff)
        assert np.array_equal(plan.search(torch.from_numpy(x).to(gpu)).cpu().numpy(), want)
        plan.close()
        for joint in (0, 1):
            binding.set_option(binding.OPT_PAIR_JOINT, joint)
            say(f"case plan block={block} paired joint={joint}")
            pp = binding.PairPlan(torch.from_numpy(pairs.rho.tables).to(gpu),
                                  pairs.rho.table_off, torch.from_numpy(pairs.temp.tables).to(gpu),
                                  pairs.temp.table_off, pairs.rho.query_off)
            o_r, o_t = pp.search(torch.from_numpy(rho).to(gpu), torch.from_numpy(temp).to(gpu))
            assert np.array_equal(o_r.cpu().numpy(), want_r)
            assert np.array_equal(o_t.cpu().numpy(), want_t)
            pp.close()
    finally:
        binding.set_option(binding.OPT_BLOCK_SIZE, 0)
        binding.set_option(binding.OPT_PAIR_JOINT, 0)


@pytest.mark.parametrize("xcd", [0, 1, 2, 3, 7, 1 << 24])
def test_xcd_mappings_cover_every_range(binding, gpu, oracle_mod, inputs_mod, xcd):
    """Every workgroup-to-XCD mapping (dispatch order, chunks of 2, 3, 7, the
    default, one contiguous part per XCD) searches every tile exactly once,
    with grids that are and are not multiples of the chunk."""
    tables, toff, qoff, x = odd_batch(inputs_mod, seed=17)
    want = oracle_mod.search_lt_segments(tables, toff, x, qoff)
    for k in (1, 3):
        try:
            binding.set_option(binding.OPT_PLAN_XCD, xcd)
            binding.set_option(binding.OPT_PLAN_TILES, k)
            say(f"case xcd={xcd} tiles={k}")
            plan = binding.MultiPlan(torch.from_numpy(tables).to(gpu), toff, qoff)
        finally:
            binding.set_option(binding.OPT_PLAN_XCD, 0)
            binding.set_option(binding.OPT_PLAN_TILES, 0)
        out = torch.full((x.size,), -9, dtype=torch.int32, device=gpu)
        plan.search(torch.from_numpy(x).to(gpu), out)
        got = out.cpu().numpy()
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (xcd, k, bad[:5], got[bad[:5]], want[bad[:5]])
        plan.close()


@pytest.mark.parametrize("order", [1, 2], ids=["contiguous", "strided"])
def test_tile_orders_cover_every_tile(binding, gpu, oracle_mod, inputs_mod, order):
    """Both tile orders (SS_OPT_PLAN_ORDER) at several tiles per workgroup,
    in every plan form (batched, learned batched, split and joint paired,
    interpolation): every index equal to the oracle's."""
    tables, toff, qoff, x = odd_batch(inputs_mod, seed=29)
    want = oracle_mod.search_lt_segments(tables, toff, x, qoff)
    pairs = ragged_pairs(inputs_mod, 31, 40, 400009)
    rho, temp = inputs_mod.paired_targets(pairs, seed=31)
    want_r = oracle_mod.search_lt_segments(pairs.rho.tables, pairs.rho.table_off, rho,
                                           pairs.rho.query_off)
    want_t = oracle_mod.search_lt_segments(pairs.temp.tables, pairs.temp.table_off, temp,
                                           pairs.temp.query_off)
    it = inputs_mod.interp_layout(seed=31, materials=24, total_pairs=300011)
    ri, ti = inputs_mod.paired_targets(it.pairs, seed=31)
    want_f, scale = oracle_mod.interp_pairs(it.pairs.rho.tables, it.pairs.rho.table_off,
                                            it.pairs.temp.tables, it.pairs.temp.table_off,
                                            it.pairs.rho.query_off, it.values, ri, ti)
    xt = torch.from_numpy(x).to(gpu)
    dr, dt = torch.from_numpy(rho).to(gpu), torch.from_numpy(temp).to(gpu)
    for k in (1, 3, 7):
        try:
            binding.set_option(binding.OPT_PLAN_ORDER, order)
            binding.set_option(binding.OPT_PLAN_TILES, k)
            for learned in (binding.PLAN_LEARNED_NONE, binding.PLAN_LEARNED_ALL):
                binding.set_option(binding.OPT_PLAN_LEARNED, learned)
                say(f"case order={order} tiles={k} batched learned={learned}")
                plan = binding.MultiPlan(torch.from_numpy(tables).to(gpu), toff, qoff)
                out = torch.full((x.size,), -9, dtype=torch.int32, device=gpu)
                got = plan.search(xt, out).cpu().numpy()
                bad = np.nonzero(got != want)[0]
                assert bad.size == 0, (order, k, learned, bad[:5], got[bad[:5]], want[bad[:5]])
                plan.close()
            binding.set_option(binding.OPT_PLAN_LEARNED, 0)
            for joint in (0, 1):
                binding.set_option(binding.OPT_PAIR_JOINT, joint)
                say(f"case order={order} tiles={k} paired joint={joint}")
                pp = binding.PairPlan(torch.from_numpy(pairs.rho.tables).to(gpu),
                                      pairs.rho.table_off,
                                      torch.from_numpy(pairs.temp.tables).to(gpu),
                                      pairs.temp.table_off, pairs.rho.query_off)
                o_r, o_t = pp.search(dr, dt)
                assert np.array_equal(o_r.cpu().numpy(), want_r)
                assert np.array_equal(o_t.cpu().numpy(), want_t)
                pp.close()
            binding.set_option(binding.OPT_PAIR_JOINT, 0)
            say(f"case order={order} tiles={k} interpolation")
            ip = binding.InterpPlan(torch.from_numpy(it.pairs.rho.tables).to(gpu),
                                    it.pairs.rho.table_off,
                                    torch.from_numpy(it.pairs.temp.tables).to(gpu),
                                    it.pairs.temp.table_off, it.pairs.rho.query_off,
                                    torch.from_numpy(it.values).to(gpu))
            f = ip.interpolate(torch.from_numpy(ri).to(gpu), torch.from_numpy(ti).to(gpu))
            f = f.cpu().numpy()
            ok = ~np.isnan(want_f)
            assert np.array_equal(np.isnan(f), ~ok)
            assert np.all(np.abs(f[ok] - want_f[ok]) <= 16 * np.finfo(np.float64).eps * scale[ok])
            ip.close()
        finally:
            binding.set_option(binding.OPT_PLAN_ORDER, 0)
            binding.set_option(binding.OPT_PLAN_TILES, 0)
            binding.set_option(binding.OPT_PLAN_LEARNED, 0)
            binding.set_option(binding.OPT_PAIR_JOINT, 0)


def test_batched_rejects_bad_arguments(binding, gpu, inputs_mod):
    t = torch.from_numpy(inputs_mod.single_table(100)).to(gpu)
    with pytest.raises(binding.SearchSortedError):
        binding.MultiPlan(t, [0, 50, 40], [0, 10, 20])       # decreasing table offsets
    with pytest.raises(binding.SearchSortedError):
        binding.MultiPlan(t, [1, 100], [0, 10])               # offsets must start at 0
    big = torch.zeros(70000, dtype=torch.float64, device=gpu)
    with pytest.raises(binding.SearchSortedError):
        binding.MultiPlan(big, [0, 70000], [0, 10])           # table over 65535 entries
    plan = binding.MultiPlan(t, [0, 100], [0, 10])
    with pytest.raises(ValueError):
        plan.search(torch.zeros(11, dtype=torch.float64, device=gpu))


def test_largest_stageable_tables(binding, gpu, oracle_mod, inputs_mod, pair_form):
    """A table of 6136 entries (48 KB staged with its padding) is the
    largest a plan takes: exact at that size; one entry more is refused
    with SS_ERR_UNSUPPORTED.  Paired plans: each table up to 6136 in the
    split form; in the joint form the two axes together up to 6128."""
    rng = np.random.default_rng(61)
    def table(n):
        return np.sort(np.exp(rng.uniform(np.log(1e-6), np.log(1e6), n)))
    big, small = table(6136), table(40)
    x = inputs_mod.table_targets(big, 50000, seed=3)
    tb = torch.from_numpy(np.concatenate([small, big])).to(gpu)
    plan = binding.MultiPlan(tb, [0, 40, 6176], [0, 1000, 51000])
    xs = np.concatenate([inputs_mod.table_targets(small, 1000, seed=4), x])
    got = plan.search(torch.from_numpy(xs).to(gpu)).cpu().numpy()
    want = np.concatenate([oracle_mod.search_lt(small, xs[:1000]), oracle_mod.search_lt(big, x)])
    assert np.array_equal(got, want)
    plan.close()
    over = torch.from_numpy(table(6137)).to(gpu)
    with pytest.raises(binding.SearchSortedError) as e:
        binding.MultiPlan(over, [0, 6137], [0, 10])
    assert e.value.code == -6
    rho, tt = table(6136) if pair_form == 0 else table(6000), table(128)
    r = inputs_mod.table_targets(rho, 20000, seed=5)
    tq = inputs_mod.table_targets(tt, 20000, seed=6)
    pp = binding.PairPlan(torch.from_numpy(rho).to(gpu), [0, rho.size],
                          torch.from_numpy(tt).to(gpu), [0, tt.size], [0, 20000])
    out_r, out_t = pp.search(torch.from_numpy(r).to(gpu), torch.from_numpy(tq).to(gpu))
    assert np.array_equal(out_r.cpu().numpy(), oracle_mod.search_lt(rho, r))
    assert np.array_equal(out_t.cpu().numpy(), oracle_mod.search_lt(tt, tq))
    pp.close()
    if pair_form == 1:
        with pytest.raises(binding.SearchSortedError) as e:
            binding.PairPlan(torch.from_numpy(rho).to(gpu), [0, rho.size],
                             torch.from_numpy(table(129)).to(gpu), [0, 129], [0, 10])
        assert e.value.code == -6


@pytest.fixture(params=[0, 1], ids=["split", "joint"])
def pair_form(request, binding):
    """Both launch forms of paired plans: the density and temperature
    searches as 2M independent segments (default), or one workgroup per tile
    of pairs with both tables staged."""
    binding.set_option(binding.OPT_PAIR_JOINT, request.param)
    yield request.param
    binding.set_option(binding.OPT_PAIR_JOINT, 0)


def ragged_pairs(inputs_mod, seed, materials, total_pairs):
    """A paired layout whose pair counts include empty and one-pair
    materials and whose total is not a multiple of any tile or line size."""
    from paper_2112_03229_amd.inputs import Batch, Paired
    pairs = inputs_mod.paired_layout(seed=seed, materials=materials, total_pairs=total_pairs)
    counts = np.diff(pairs.rho.query_off)
    counts[[0, 5, materials // 2]] = 0
    counts[[1, 6, materials - 1]] = [1, 3, 4099]
    poff = np.zeros(materials + 1, dtype=np.int64)
    poff[1:] = np.cumsum(counts)
    r, t = pairs.rho, pairs.temp
    return Paired(Batch(r.tables, r.table_off, poff, r.lo, r.hi),
                  Batch(t.tables, t.table_off, poff.copy(), t.lo, t.hi))


@pytest.mark.parametrize("layout", ["regular", "ragged"])
def test_paired_composition(binding, gpu, oracle_mod, inputs_mod, pair_form, layout):
    if layout == "regular":
        pairs = inputs_mod.paired_layout(seed=9, materials=96, total_pairs=2 * 10**6)
    else:
        pairs = ragged_pairs(inputs_mod, 19, 80, 10**6 + 13)
    rho, temp = inputs_mod.paired_targets(pairs, seed=9)
    rho[:4] = [np.nan, -1.0, np.inf, 0.0]
    temp[-3:] = [np.nan, -np.inf, 5e-324]
    want_r = oracle_mod.search_lt_segments(pairs.rho.tables, pairs.rho.table_off, rho,
                                           pairs.rho.query_off)
    want_t = oracle_mod.search_lt_segments(pairs.temp.tables, pairs.temp.table_off, temp,
                                           pairs.temp.query_off)
    say(f"case paired {layout} form={pair_form} M={pairs.num_materials} pairs={pairs.num_pairs}")
    plan = binding.PairPlan(torch.from_numpy(pairs.rho.tables).to(gpu), pairs.rho.table_off,
                            torch.from_numpy(pairs.temp.tables).to(gpu), pairs.temp.table_off,
                            pairs.rho.query_off)
    dr, dt = torch.from_numpy(rho).to(gpu), torch.from_numpy(temp).to(gpu)
    out_r, out_t = plan.search(dr, dt)
    torch.cuda.synchronize()
    assert np.array_equal(out_r.cpu().numpy(), want_r)
    assert np.array_equal(out_t.cpu().numpy(), want_t)
    info = plan.info()
    assert info["tables"] == 2 * pairs.num_materials
    algos = info["algos"]
    assert np.all((algos == binding.ALGO_EXPHASH) | (algos == binding.ALGO_BINARY))
    assert np.count_nonzero(algos == binding.ALGO_EXPHASH) > algos.size // 2
    assert np.all((info["bits"] >= 0) == (algos == binding.ALGO_EXPHASH))
    # graph replay into the same outputs, then new output buffers
    out_r.fill_(-7)
    out_t.fill_(-7)
    plan.search(dr, dt, out_r, out_t)
    assert np.array_equal(out_r.cpu().numpy(), want_r)
    assert np.array_equal(out_t.cpu().numpy(), want_t)
    o2r, o2t = plan.search(dr, dt)
    assert np.array_equal(o2r.cpu().numpy(), want_r)
    assert np.array_equal(o2t.cpu().numpy(), want_t)
    plan.close()


def test_tuner_calibration_roundtrip(binding, gpu, oracle_mod, inputs_mod, tmp_path):
    coeffs = binding.tuner_calibrate()
    say(f"tuner: {coeffs}")
    assert coeffs["calibrated"] == 1.0
    assert 1000 < coeffs["stream_gbs"] < 20000
    assert coeffs["bin_per_step_ns"] >= 0 and coeffs["hash_per_k_ns"] >= 0
    path = str(tmp_path / "tuner.json")
    binding.tuner_save(path)
    binding.tuner_load(path)
    assert binding.tuner_get() == coeffs
    # a plan tuned with the calibrated model is still exact
    batch = inputs_mod.batched_layout(seed=21, num_tables=16, query_scale=1e-3)
    x = inputs_mod.batched_targets(batch, seed=21)
    plan = binding.MultiPlan(torch.from_numpy(batch.tables).to(gpu), batch.table_off,
                             batch.query_off)
    got = plan.search(torch.from_numpy(x).to(gpu)).cpu().numpy()
    want = oracle_mod.search_lt_segments(batch.tables, batch.table_off, x, batch.query_off)
    assert np.array_equal(got, want)


def test_full_size_batched(binding, gpu, oracle_mod, inputs_mod):
    """512 tables, n uniform on 20..2000, ~7.4e8 targets, one launch."""
    batch = inputs_mod.batched_layout()
    m = batch.num_queries
    say(f"case full batched T=512 m={m}")
    host = torch.empty(m, dtype=torch.float64).pin_memory()
    x = inputs_mod.batched_targets(batch, out=host.numpy())
    plan = binding.MultiPlan(torch.from_numpy(batch.tables).to(gpu), batch.table_off,
                             batch.query_off)
    xt = host.to(gpu, non_blocking=True)
    out = plan.search(xt)
    got = out.cpu().numpy()
    del xt, out
    bad, first = oracle_mod.check_bracket_segments(batch.tables, batch.table_off, x,
                                                   batch.query_off, got)
    assert bad == 0, first
    # a seeded sample of 1e7 targets against the definition, every table
    pos = np.sort((inputs_mod.uniform(512, 97, 10**7) * m).astype(np.int64))
    seg = np.searchsorted(batch.query_off, pos, side="right") - 1
    bounds = np.searchsorted(seg, np.arange(batch.num_tables + 1))
    for t in range(batch.num_tables):
        p = pos[bounds[t]:bounds[t + 1]]
        if p.size:
            assert np.array_equal(got[p], oracle_mod.search_lt_at(batch.table(t), x, p)), t


def test_full_size_learned_batched(binding, gpu, oracle_mod, inputs_mod):
    """The 512-table batch with every table learned (500 Adam steps each,
    the configuration bench.py times): every index bracket-checked, a seeded
    2e6-target sample against the definition over every table."""
    batch = inputs_mod.batched_layout()
    m = batch.num_queries
    say(f"case full learned batched T=512 m={m}")
    host = torch.empty(m, dtype=torch.float64).pin_memory()
    x = inputs_mod.batched_targets(batch, out=host.numpy())
    try:
        binding.set_option(binding.OPT_PLAN_LEARNED, 1)
        plan = binding.MultiPlan(torch.from_numpy(batch.tables).to(gpu), batch.table_off,
                                 batch.query_off)
    finally:
        binding.set_option(binding.OPT_PLAN_LEARNED, 0)
    assert np.all(plan.info()["algos"] == binding.ALGO_LEARNED)
    xt = host.to(gpu, non_blocking=True)
    out = plan.search(xt)
    got = out.cpu().numpy()
    say(f"fallbacks {plan.fallbacks()} of {m}")
    del xt, out
    plan.close()
    bad, first = oracle_mod.check_bracket_segments(batch.tables, batch.table_off, x,
                                                   batch.query_off, got)
    assert bad == 0, first
    pos = np.sort((inputs_mod.uniform(512, 98, 2 * 10**6) * m).astype(np.int64))
    seg = np.searchsorted(batch.query_off, pos, side="right") - 1
    bounds = np.searchsorted(seg, np.arange(batch.num_tables + 1))
    for t in range(batch.num_tables):
        p = pos[bounds[t]:bounds[t + 1]]
        if p.size:
            assert np.array_equal(got[p], oracle_mod.search_lt_at(batch.table(t), x, p)), t


def test_full_size_paired(binding, gpu, oracle_mod, inputs_mod, pair_form):
    """4096 materials (density 50..4000 entries, temperature 20..1000), 1e9
    pairs, both searches in one launch."""
    pairs = inputs_mod.paired_layout()
    m = pairs.num_pairs
    say(f"case full paired form={pair_form} M=4096 pairs={m}")
    hr = torch.empty(m, dtype=torch.float64).pin_memory()
    ht = torch.empty(m, dtype=torch.float64).pin_memory()
    rho, temp = inputs_mod.paired_targets(pairs, out_rho=hr.numpy(), out_t=ht.numpy())
    plan = binding.PairPlan(torch.from_numpy(pairs.rho.tables).to(gpu), pairs.rho.table_off,
                            torch.from_numpy(pairs.temp.tables).to(gpu), pairs.temp.table_off,
                            pairs.rho.query_off)
    dr, dt = hr.to(gpu, non_blocking=True), ht.to(gpu, non_blocking=True)
    out_r, out_t = plan.search(dr, dt)
    got_r = out_r.cpu().numpy()
    got_t = out_t.cpu().numpy()
    del dr, dt, out_r, out_t
    for name, b, x, got in (("rho", pairs.rho, rho, got_r), ("temp", pairs.temp, temp, got_t)):
        say(f"check {name}")
        bad, first = oracle_mod.check_bracket_segments(b.tables, b.table_off, x, b.query_off, got)
        assert bad == 0, (name, first)
        # a seeded sample of 1e7 targets per axis against the definition,
        # every material
        pos = np.sort((inputs_mod.uniform(4096, 98, 10**7) * m).astype(np.int64))
        seg = np.searchsorted(b.query_off, pos, side="right") - 1
        M = b.query_off.size - 1
        bounds = np.searchsorted(seg, np.arange(M + 1))
        for t in range(M):
            p = pos[bounds[t]:bounds[t + 1]]
            if p.size:
                assert np.array_equal(got[p], oracle_mod.search_lt_at(b.table(t), x, p)), (name, t)


def test_full_size_learned_paired(binding, gpu, oracle_mod, inputs_mod):
    """The 1e9-pair workload with all 8192 tables learned (500 Adam steps
    each), split form as bench.py times it: every index bracket-checked on
    both axes, a seeded 2e6-target sample per axis against the definition."""
    pairs = inputs_mod.paired_layout()
    m = pairs.num_pairs
    say(f"case full learned paired M=4096 pairs={m}")
    hr = torch.empty(m, dtype=torch.float64).pin_memory()
    ht = torch.empty(m, dtype=torch.float64).pin_memory()
    rho, temp = inputs_mod.paired_targets(pairs, out_rho=hr.numpy(), out_t=ht.numpy())
    try:
        binding.set_option(binding.OPT_PLAN_LEARNED, 1)
        plan = binding.PairPlan(torch.from_numpy(pairs.rho.tables).to(gpu), pairs.rho.table_off,
                                torch.from_numpy(pairs.temp.tables).to(gpu),
                                pairs.temp.table_off, pairs.rho.query_off)
    finally:
        binding.set_option(binding.OPT_PLAN_LEARNED, 0)
    assert np.all(plan.info()["algos"] == binding.ALGO_LEARNED)
    dr, dt = hr.to(gpu, non_blocking=True), ht.to(gpu, non_blocking=True)
    out_r, out_t = plan.search(dr, dt)
    got_r = out_r.cpu().numpy()
    got_t = out_t.cpu().numpy()
    say(f"fallbacks {plan.fallbacks()} of {2 * m}")
    del dr, dt, out_r, out_t
    plan.close()
    for name, b, x, got in (("rho", pairs.rho, rho, got_r), ("temp", pairs.temp, temp, got_t)):
        bad, first = oracle_mod.check_bracket_segments(b.tables, b.table_off, x, b.query_off, got)
        assert bad == 0, (name, first)
        pos = np.sort((inputs_mod.uniform(4096, 99, 2 * 10**6) * m).astype(np.int64))
        seg = np.searchsorted(b.query_off, pos, side="right") - 1
        M = b.query_off.size - 1
        bounds = np.searchsorted(seg, np.arange(M + 1))
        for t in range(M):
            p = pos[bounds[t]:bounds[t + 1]]
            if p.size:
                assert np.array_equal(got[p], oracle_mod.search_lt_at(b.table(t), x, p)), (name, t)


def test_learned_batched_plan_is_exact(binding, gpu, oracle_mod, inputs_mod):
    """Every eligible table gets a device-trained model; ineligible ones
    (negative entries, a single entry, empty) keep the tuner's kernel."""
    tables, toff, qoff, x = odd_batch(inputs_mod, seed=12)
    want = oracle_mod.search_lt_segments(tables, toff, x, qoff)
    try:
        binding.set_option(binding.OPT_PLAN_LEARNED, 1)
        binding.set_option(binding.OPT_LEARNED_STEPS, 300)
        say(f"case learned batched T={toff.size - 1}")
        plan = binding.MultiPlan(torch.from_numpy(tables).to(gpu), toff, qoff)
    finally:
        binding.set_option(binding.OPT_PLAN_LEARNED, 0)
        binding.set_option(binding.OPT_LEARNED_STEPS, 0)
    out = plan.search(torch.from_numpy(x).to(gpu))
    got = out.cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]], x[bad[:5]])
    info = plan.info()
    T = toff.size - 1
    algos = info["algos"]
    assert algos[0] == binding.ALGO_LEARNED
    assert algos[T - 5] != binding.ALGO_LEARNED    # negative entries
    assert algos[T - 6] != binding.ALGO_LEARNED    # empty table
    assert algos[T - 7] != binding.ALGO_LEARNED    # single entry
    say(f"learned tables {int((algos == binding.ALGO_LEARNED).sum())} of {T}, "
        f"fallbacks {plan.fallbacks()} of {x.size}")
    # replay: still exact, fallback counter restarts
    out.fill_(-3)
    plan.search(torch.from_numpy(x).to(gpu), out)
    assert np.array_equal(out.cpu().numpy(), want)


def test_learned_paired_plan_is_exact(binding, gpu, oracle_mod, inputs_mod, pair_form):
    pairs = ragged_pairs(inputs_mod, 13, 48, 10**6 + 5)
    rho, temp = inputs_mod.paired_targets(pairs, seed=13)
    rho[:3] = [np.nan, 0.0, np.inf]
    want_r = oracle_mod.search_lt_segments(pairs.rho.tables, pairs.rho.table_off, rho,
                                           pairs.rho.query_off)
    want_t = oracle_mod.search_lt_segments(pairs.temp.tables, pairs.temp.table_off, temp,
                                           pairs.temp.query_off)
    try:
        binding.set_option(binding.OPT_PLAN_LEARNED, 1)
        binding.set_option(binding.OPT_LEARNED_STEPS, 300)
        plan = binding.PairPlan(torch.from_numpy(pairs.rho.tables).to(gpu), pairs.rho.table_off,
                                torch.from_numpy(pairs.temp.tables).to(gpu),
                                pairs.temp.table_off, pairs.rho.query_off)
    finally:
        binding.set_option(binding.OPT_PLAN_LEARNED, 0)
        binding.set_option(binding.OPT_LEARNED_STEPS, 0)
    out_r, out_t = plan.search(torch.from_numpy(rho).to(gpu), torch.from_numpy(temp).to(gpu))
    assert np.array_equal(out_r.cpu().numpy(), want_r)
    assert np.array_equal(out_t.cpu().numpy(), want_t)
    assert np.all(plan.info()["algos"] == binding.ALGO_LEARNED)
    say(f"paired learned form={pair_form} fallbacks {plan.fallbacks()} of {2 * pairs.num_pairs}")
