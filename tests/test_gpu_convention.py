"""GPU parity of the paper's convention (Sec. 3: the last index with
a[i] <= x, clamped to [0, n-1]) against ``oracle.search_le_clamped``, bit for
bit, for every single-table kernel, edge tables, batched and paired plans and
the learned index.  SS_OPT_CONVENTION is read per call by single-table and
learned searches and at creation by plans.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

ALGOS = ["auto", "binary", "ballot", "exphash", "binary_global", "loghash", "skiplist"]
TILE = 512 * 8


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def binding(gpu):
    from paper_2112_03229_amd import binding as b
    return b


@pytest.fixture
def paper_convention(binding):
    binding.set_option(binding.OPT_CONVENTION, 1)
    yield
    binding.set_option(binding.OPT_CONVENTION, 0)


def targets(inputs_mod, table, m, seed):
    x = inputs_mod.table_targets(table, m, seed=seed) if table.size and table[0] > 0 else \
        inputs_mod.log_uniform(seed, 4, 1e-12, 1e12, m)
    n = table.shape[0]
    if n:
        k = np.arange(0, m, 5)
        x[k] = table[k % n]
        k = np.arange(2, m, 9)
        x[k] = np.nextafter(table[k % n], np.inf)
        k = np.arange(4, m, 11)
        x[k] = np.nextafter(table[k % n], -np.inf)
    sp = inputs_mod.special_values()
    x[1:1 + sp.size] = sp
    x[::13] *= -1.0
    return x


def run(binding, dev, table, x, algo):
    t = torch.from_numpy(np.ascontiguousarray(table)).to(dev)
    out = binding.search_with(t, torch.from_numpy(x).to(dev), algo)
    return out.cpu().numpy()


TABLES = {
    "log300": None,
    "log2000": None,
    "single": np.array([2.5]),
    "pair_equal": np.array([1.0, 1.0]),
    "zeros_denormals": np.array([-0.0, 0.0, 5e-324, 1e-310, 1.0, 1.0, 3.0]),
    "with_inf": np.array([1e-3, 1.0, 10.0, np.inf, np.inf]),
    "negatives": np.array([-1e10, -5.0, -1.0, -0.0, 0.0, 1e-5, 3.0, 1e20]),
    "max_double": np.array([1.0, 1.7976931348623157e308]),
    "empty": np.zeros(0),
}


@pytest.mark.parametrize("name", list(TABLES))
def test_single_table_paper_convention(binding, gpu, oracle_mod, inputs_mod, paper_convention,
                                       name):
    table = TABLES[name]
    if table is None:
        table = inputs_mod.single_table(int(name[3:]))
    table = table.astype(np.float64)
    x = targets(inputs_mod, table, 5 * TILE + 37, seed=len(name))
    want = oracle_mod.search_le_clamped(table, x)
    try:
        for q in (8, 4):  # both targets-per-lane variants of every kernel
            binding.set_option(binding.OPT_TARGETS_PER_LANE, q)
            for algo in ALGOS:
                say(f"case convention table={name} q={q} algo={algo}")
                got = run(binding, gpu, table, x, algo)
                bad = np.nonzero(got != want)[0]
                assert bad.size == 0, (algo, q, name, bad[:5], got[bad[:5]], want[bad[:5]],
                                       x[bad[:5]])
    finally:
        binding.set_option(binding.OPT_TARGETS_PER_LANE, 0)


def test_convention_is_read_per_call(binding, gpu, oracle_mod, inputs_mod):
    table = inputs_mod.single_table(100)
    x = targets(inputs_mod, table, TILE + 3, seed=1)
    try:
        binding.set_option(binding.OPT_CONVENTION, 1)
        a = run(binding, gpu, table, x, "auto")
    finally:
        binding.set_option(binding.OPT_CONVENTION, 0)
    b = run(binding, gpu, table, x, "auto")
    assert np.array_equal(a, oracle_mod.search_le_clamped(table, x))
    assert np.array_equal(b, oracle_mod.search_lt(table, x))
    assert not np.array_equal(a, b)


def segments_le(oracle_mod, tables, toff, x, qoff):
    out = np.empty(x.shape[0], dtype=np.int32)
    for s in range(toff.shape[0] - 1):
        q0, q1 = qoff[s], qoff[s + 1]
        if q1 > q0:
            out[q0:q1] = oracle_mod.search_le_clamped(tables[toff[s]:toff[s + 1]], x[q0:q1])
    return out


def test_batched_plan_paper_convention(binding, gpu, oracle_mod, inputs_mod):
    batch = inputs_mod.batched_layout(seed=31, num_tables=40, query_scale=2e-3)
    x = inputs_mod.batched_targets(batch, seed=31)
    x[::6] = batch.tables[np.arange(0, x.size, 6) % batch.tables.size]
    x[:14] = inputs_mod.special_values()
    want = segments_le(oracle_mod, batch.tables, batch.table_off, x, batch.query_off)
    try:
        binding.set_option(binding.OPT_CONVENTION, 1)
        plan = binding.MultiPlan(torch.from_numpy(batch.tables).to(gpu), batch.table_off,
                                 batch.query_off)
    finally:
        binding.set_option(binding.OPT_CONVENTION, 0)
    # the plan keeps the convention it was created with
    got = plan.search(torch.from_numpy(x).to(gpu)).cpu().numpy()
    assert np.array_equal(got, want)
    strict = binding.MultiPlan(torch.from_numpy(batch.tables).to(gpu), batch.table_off,
                               batch.query_off)
    got2 = strict.search(torch.from_numpy(x).to(gpu)).cpu().numpy()
    assert np.array_equal(got2, oracle_mod.search_lt_segments(batch.tables, batch.table_off, x,
                                                              batch.query_off))


@pytest.mark.parametrize("joint", [0, 1])
def test_paired_plan_paper_convention(binding, gpu, oracle_mod, inputs_mod, joint):
    pairs = inputs_mod.paired_layout(seed=33, materials=40, total_pairs=600001)
    rho, temp = inputs_mod.paired_targets(pairs, seed=33)
    rho[::5] = pairs.rho.tables[np.arange(0, rho.size, 5) % pairs.rho.tables.size]
    temp[:14] = inputs_mod.special_values()
    want_r = segments_le(oracle_mod, pairs.rho.tables, pairs.rho.table_off, rho,
                         pairs.rho.query_off)
    want_t = segments_le(oracle_mod, pairs.temp.tables, pairs.temp.table_off, temp,
                         pairs.temp.query_off)
    try:
        binding.set_option(binding.OPT_CONVENTION, 1)
        binding.set_option(binding.OPT_PAIR_JOINT, joint)
        plan = binding.PairPlan(torch.from_numpy(pairs.rho.tables).to(gpu), pairs.rho.table_off,
                                torch.from_numpy(pairs.temp.tables).to(gpu),
                                pairs.temp.table_off, pairs.rho.query_off)
    finally:
        binding.set_option(binding.OPT_CONVENTION, 0)
        binding.set_option(binding.OPT_PAIR_JOINT, 0)
    o_r, o_t = plan.search(torch.from_numpy(rho).to(gpu), torch.from_numpy(temp).to(gpu))
    assert np.array_equal(o_r.cpu().numpy(), want_r)
    assert np.array_equal(o_t.cpu().numpy(), want_t)


def test_learned_paper_convention(binding, gpu, oracle_mod, inputs_mod, paper_convention):
    table = inputs_mod.single_table(500)
    li = binding.LearnedIndex(torch.from_numpy(table).to(gpu), steps=300, seed=5)
    x = targets(inputs_mod, table, 3 * TILE + 5, seed=9)
    got = li.search(torch.from_numpy(x).to(gpu)).cpu().numpy()
    assert np.array_equal(got, oracle_mod.search_le_clamped(table, x))


@pytest.mark.parametrize("seed", range(3))
def test_random_tables_paper_convention(binding, gpu, oracle_mod, paper_convention, seed):
    """Seeded fuzzing in the paper's convention: random tables (duplicates,
    signed entries, zeros, denormals, infinities) and targets at, between
    and around their entries, every kernel against search_le_clamped."""
    from test_gpu_single import fuzz_table, fuzz_targets
    rng = np.random.default_rng(2000 + seed)
    for case in range(30):
        n = int(rng.choice([0, 1, 2, 5, 64, 65, 300, 1000, 4000]))
        table = fuzz_table(rng, n)
        x = fuzz_targets(rng, table, int(rng.integers(1, 3 * TILE)))
        want = oracle_mod.search_le_clamped(table, x)
        for algo in ALGOS:
            got = run(binding, gpu, table, x, algo)
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, (seed, case, n, algo, bad[:3], got[bad[:3]], want[bad[:3]], x[bad[:3]])


@pytest.mark.parametrize("form", ["batched", "split", "joint"])
def test_learned_plans_paper_convention(binding, gpu, oracle_mod, inputs_mod, form):
    """Plans whose tables all have learned models, created in the paper's
    convention: the learned plan kernels' convention variants, against the
    oracle's clamped count."""
    say(f"case learned plan convention form={form}")
    opts = {binding.OPT_CONVENTION: 1, binding.OPT_PLAN_LEARNED: 1,
            binding.OPT_LEARNED_STEPS: 100, binding.OPT_PAIR_JOINT: int(form == "joint")}
    try:
        for k, v in opts.items():
            binding.set_option(k, v)
        if form == "batched":
            batch = inputs_mod.batched_layout(seed=35, num_tables=12, query_scale=1e-3)
            x = inputs_mod.batched_targets(batch, seed=35)
            x[::6] = batch.tables[np.arange(0, x.size, 6) % batch.tables.size]
            x[:14] = inputs_mod.special_values()
            plan = binding.MultiPlan(torch.from_numpy(batch.tables).to(gpu), batch.table_off,
                                     batch.query_off)
        else:
            pairs = inputs_mod.paired_layout(seed=37, materials=12, total_pairs=200001)
            rho, temp = inputs_mod.paired_targets(pairs, seed=37)
            rho[::5] = pairs.rho.tables[np.arange(0, rho.size, 5) % pairs.rho.tables.size]
            temp[:14] = inputs_mod.special_values()
            plan = binding.PairPlan(torch.from_numpy(pairs.rho.tables).to(gpu),
                                    pairs.rho.table_off,
                                    torch.from_numpy(pairs.temp.tables).to(gpu),
                                    pairs.temp.table_off, pairs.rho.query_off)
    finally:
        for k in opts:
            binding.set_option(k, 0)
    assert (plan.info()["algos"] == binding.ALGO_LEARNED).all()
    if form == "batched":
        got = plan.search(torch.from_numpy(x).to(gpu)).cpu().numpy()
        assert np.array_equal(got, segments_le(oracle_mod, batch.tables, batch.table_off, x,
                                               batch.query_off))
    else:
        o_r, o_t = plan.search(torch.from_numpy(rho).to(gpu), torch.from_numpy(temp).to(gpu))
        assert np.array_equal(o_r.cpu().numpy(),
                              segments_le(oracle_mod, pairs.rho.tables, pairs.rho.table_off, rho,
                                          pairs.rho.query_off))
        assert np.array_equal(o_t.cpu().numpy(),
                              segments_le(oracle_mod, pairs.temp.tables, pairs.temp.table_off,
                                          temp, pairs.temp.query_off))
    plan.close()
