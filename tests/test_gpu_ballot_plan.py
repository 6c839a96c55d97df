"""The ballot scan (Sec. 2.1's linear search, limited to each wave's bracket)
as a plan kernel, and the sampled plans that let the autotuner choose it.

Paper Sec. 5.2: the best method depends on the distribution of the data.
The ballot scan's cost is the number of table entries between the smallest
and the largest target of a wave, which only the targets show.  A sampled
plan measures that bracket per table on sample targets; the test recomputes
the same footprints in numpy and needs the same means, checks the choice
against the modelled costs, and every result against the oracle.
"""
import os
import sys

import numpy as np
import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_multi import odd_batch, ragged_pairs  # noqa: E402

pytestmark = pytest.mark.gpu

NT, Q, SAMPLES = 512, 8, 32  # batched and split plans: 512 threads, 8 targets per lane


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def binding(gpu):
    from paper_2112_03229_amd import binding as b
    return b


def with_opts(binding, opts, make):
    old = {k: binding.get_option(k) for k in opts}
    try:
        for k, v in opts.items():
            binding.set_option(k, v)
        return make()
    finally:
        for k, v in old.items():
            binding.set_option(k, v)


def expected_brackets(tables, toff, x, qoff, nt=NT, q=Q):
    """Mean #{a < max} - #{a < min} over the 32 wave footprints the plan samples."""
    per_tile = nt * q
    out = np.full(len(toff) - 1, -1.0)
    lanes = np.arange(64)
    for t in range(len(toff) - 1):
        q0, q1 = int(qoff[t]), int(qoff[t + 1])
        if q1 <= q0:
            continue
        tab = tables[toff[t]:toff[t + 1]]
        b0, b1 = q0 // per_tile, (q1 - 1) // per_tile
        tiles = b1 - b0 + 1
        total, count = 0, 0
        for f in range(SAMPLES):
            b = b0 + f * tiles // SAMPLES
            base = b * per_tile + (f % (nt // 64)) * 64
            idx = (base + lanes[:, None] + nt * np.arange(q)[None, :]).ravel()
            idx = idx[(idx >= q0) & (idx < q1)]
            v = x[idx]
            v = v[~np.isnan(v)]
            if v.size == 0:
                continue
            lo = np.searchsorted(tab, v.min(), side="left")
            hi = np.searchsorted(tab, v.max(), side="left")
            total += int(hi - lo)
            count += 1
        if count:
            out[t] = total / count
    return out


def sorted_within(x, qoff):
    y = x.copy()
    for t in range(len(qoff) - 1):
        a, b = qoff[t], qoff[t + 1]
        y[a:b] = np.sort(y[a:b])  # NaN last
    return y


@pytest.mark.parametrize("conv", [0, 1], ids=["strict", "paper"])
def test_forced_ballot_plan_is_exact(binding, gpu, oracle_mod, inputs_mod, conv):
    tables, toff, qoff, x = odd_batch(inputs_mod, seed=61)
    for name, xs in (("random", x), ("sorted", sorted_within(x, qoff))):
        say(f"case forced ballot batched plan, {name} targets, convention {conv}")
        plan = with_opts(binding, {binding.OPT_PLAN_ALGO: binding.ALGO_BALLOT,
                                   binding.OPT_CONVENTION: conv},
                         lambda: binding.MultiPlan(torch.from_numpy(tables).to(gpu), toff, qoff))
        algos = plan.info()["algos"]
        n = np.diff(toff)
        assert np.all(algos[n > 0] == binding.ALGO_BALLOT)
        got = plan.search(torch.from_numpy(xs).to(gpu)).cpu().numpy()
        plan.close()
        if conv:
            for t in range(len(toff) - 1):
                a, b = qoff[t], qoff[t + 1]
                want = oracle_mod.search_le_clamped(tables[toff[t]:toff[t + 1]], xs[a:b])
                assert np.array_equal(got[a:b], want), t
        else:
            assert np.array_equal(got, oracle_mod.search_lt_segments(tables, toff, xs, qoff))


@pytest.mark.parametrize("joint", [0, 1], ids=["split", "joint"])
def test_forced_ballot_paired_plan_is_exact(binding, gpu, oracle_mod, inputs_mod, joint):
    pairs = ragged_pairs(inputs_mod, 62, 40, 300007)
    rho, temp = inputs_mod.paired_targets(pairs, seed=62)
    rho[:3] = [np.nan, -np.inf, 0.0]
    temp[-2:] = [np.inf, 5e-324]
    say(f"case forced ballot paired plan joint={joint}")
    plan = with_opts(binding, {binding.OPT_PLAN_ALGO: binding.ALGO_BALLOT,
                               binding.OPT_PAIR_JOINT: joint},
                     lambda: binding.PairPlan(torch.from_numpy(pairs.rho.tables).to(gpu),
                                              pairs.rho.table_off,
                                              torch.from_numpy(pairs.temp.tables).to(gpu),
                                              pairs.temp.table_off, pairs.rho.query_off))
    assert np.all(plan.info()["algos"] == binding.ALGO_BALLOT)
    o_r, o_t = plan.search(torch.from_numpy(rho).to(gpu), torch.from_numpy(temp).to(gpu))
    plan.close()
    assert np.array_equal(o_r.cpu().numpy(), oracle_mod.search_lt_segments(
        pairs.rho.tables, pairs.rho.table_off, rho, pairs.rho.query_off))
    assert np.array_equal(o_t.cpu().numpy(), oracle_mod.search_lt_segments(
        pairs.temp.tables, pairs.temp.table_off, temp, pairs.temp.query_off))


def mixed_batch(inputs_mod):
    """Tables of 20..600 entries, some with negative entries (no exponent
    hash), each with many targets; half the segments sorted."""
    rng_tabs, counts = [], []
    for i in range(16):
        n = [20, 60, 150, 600][i % 4]
        t = inputs_mod.sorted_log_table(900 + i, n, 1e-4, 1e4)
        if i % 8 >= 4:
            t = np.concatenate([-t[::-1][: n // 3], t[n // 3:]])  # negative entries
        rng_tabs.append(np.ascontiguousarray(t, dtype=np.float64))
        counts.append(200000 + 9173 * i)
    toff = np.zeros(17, dtype=np.int64)
    toff[1:] = np.cumsum([t.size for t in rng_tabs])
    qoff = np.zeros(17, dtype=np.int64)
    qoff[1:] = np.cumsum(counts)
    tables = np.concatenate(rng_tabs)
    x = np.concatenate([inputs_mod.log_uniform(910 + i, 3, 1e-5, 2e4, c)
                        * np.where(inputs_mod.uniform(920 + i, 4, c) < 0.3, -1.0, 1.0)
                        for i, c in enumerate(counts)])
    sorted_seg = np.array([i % 8 in (0, 3, 5, 6) for i in range(16)])  # every size both ways
    for t in np.flatnonzero(sorted_seg):
        a, b = qoff[t], qoff[t + 1]
        x[a:b] = np.sort(x[a:b])
    return tables, toff, qoff, x, sorted_seg


# The exponent hash priced out, and a ballot scan that beats the bisection
# (1.05 ps per step) on narrow brackets only: on these tables sorted
# segments give brackets of at most ~0.02 n and i.i.d. targets about n.
BALLOT_MODEL = dict(hash_base_ns=1.0, hash_per_k_ns=1.0, ballot_base_ns=0.5e-3,
                    ballot_per_entry_ns=0.3e-3, bin_base_ns=0.0, bin_per_step_ns=1.05e-3)


def make_with_model(binding, make):
    saved = binding.tuner_get()
    try:
        binding.tuner_set(**BALLOT_MODEL)
        return with_opts(binding, {binding.OPT_PLAN_LEARNED: binding.PLAN_LEARNED_NONE}, make)
    finally:
        binding.tuner_set(**saved)


def test_sampled_plan_chooses_ballot_by_bracket(binding, gpu, oracle_mod, inputs_mod):
    tables, toff, qoff, x, sorted_seg = mixed_batch(inputs_mod)
    want = oracle_mod.search_lt_segments(tables, toff, x, qoff)
    d_tab, d_x = torch.from_numpy(tables).to(gpu), torch.from_numpy(x).to(gpu)
    model = dict(binding.tuner_get(), **BALLOT_MODEL)
    plain = make_with_model(binding, lambda: binding.MultiPlan(d_tab, toff, qoff))
    plain_info = plain.info()
    plain.close()
    say("case sampled batched plan: half the segments sorted")
    plan = make_with_model(binding, lambda: binding.MultiPlan(d_tab, toff, qoff, sample=d_x))
    info = plan.info()
    br = info["brackets"]
    assert np.array_equal(br, expected_brackets(tables, toff, x, qoff))
    assert np.all(plain_info["brackets"] == -1)
    n = np.diff(toff)
    say(f"brackets {np.round(br, 2).tolist()}")
    say(f"algos {info['algos'].tolist()}")
    for t in range(len(n)):
        ballot = model["ballot_base_ns"] + model["ballot_per_entry_ns"] * (br[t] + (n[t] + 64) // 64)
        if abs(ballot - plain_info["plain_ns"][t]) < 1e-9:
            continue
        assert (info["algos"][t] == binding.ALGO_BALLOT) == (ballot < plain_info["plain_ns"][t]), t
    # sorted segments have narrow brackets and take the ballot scan; i.i.d.
    # targets span most of the table and never do
    assert np.all(info["algos"][sorted_seg] == binding.ALGO_BALLOT)
    assert not np.any(info["algos"][~sorted_seg] == binding.ALGO_BALLOT)
    assert np.all(br[sorted_seg] < 0.2 * n[sorted_seg])
    got = plan.search(d_x).cpu().numpy()
    assert np.array_equal(got, want)
    # any later targets are still answered exactly
    y = x[::-1].copy()
    assert np.array_equal(plan.search(torch.from_numpy(y).to(gpu)).cpu().numpy(),
                          oracle_mod.search_lt_segments(tables, toff, y, qoff))
    plan.close()


def test_sampled_plan_save_load_keeps_ballot(binding, gpu, oracle_mod, inputs_mod, tmp_path):
    tables, toff, qoff, x, sorted_seg = mixed_batch(inputs_mod)
    d_tab, d_x = torch.from_numpy(tables).to(gpu), torch.from_numpy(x).to(gpu)
    plan = make_with_model(binding, lambda: binding.MultiPlan(d_tab, toff, qoff, sample=d_x))
    algos = plan.info()["algos"]
    assert (algos == binding.ALGO_BALLOT).sum() == sorted_seg.sum()
    path = str(tmp_path / "ballot.plan")
    plan.save(path)
    plan.close()
    say("case saved plan with ballot tables reloaded")
    again = binding.MultiPlan(d_tab, toff, qoff, saved=path)
    assert np.array_equal(again.info()["algos"], algos)
    assert np.array_equal(again.search(d_x).cpu().numpy(),
                          oracle_mod.search_lt_segments(tables, toff, x, qoff))
    again.close()


@pytest.mark.parametrize("joint", [0, 1], ids=["split", "joint"])
def test_sampled_paired_plan(binding, gpu, oracle_mod, inputs_mod, joint):
    pairs = inputs_mod.paired_layout(seed=63, materials=24, total_pairs=2 * 10**6)
    rho, temp = inputs_mod.paired_targets(pairs, seed=63)
    temp = sorted_within(temp, pairs.temp.query_off)  # T sorted per material, density i.i.d.
    d = {k: torch.from_numpy(v).to(gpu) for k, v in (("r", rho), ("t", temp))}
    rt, tt = torch.from_numpy(pairs.rho.tables).to(gpu), torch.from_numpy(pairs.temp.tables).to(gpu)
    args = (rt, pairs.rho.table_off, tt, pairs.temp.table_off, pairs.rho.query_off)
    say(f"case sampled paired plan joint={joint}")
    plain = make_with_model(binding, lambda: with_opts(
        binding, {binding.OPT_PAIR_JOINT: joint}, lambda: binding.PairPlan(*args)))
    plain_ns = plain.info()["plain_ns"]
    plain.close()
    plan = make_with_model(binding, lambda: with_opts(
        binding, {binding.OPT_PAIR_JOINT: joint},
        lambda: binding.PairPlan(*args, sample=(d["r"], d["t"]))))
    info = plan.info()
    M = pairs.num_materials
    q = 4 if joint else 8
    br_r = expected_brackets(pairs.rho.tables, pairs.rho.table_off, rho, pairs.rho.query_off,
                             q=q)
    br_t = expected_brackets(pairs.temp.tables, pairs.temp.table_off, temp,
                             pairs.temp.query_off, q=q)
    br = np.concatenate([br_r, br_t])
    assert np.array_equal(info["brackets"], br)
    n = np.concatenate([np.diff(pairs.rho.table_off), np.diff(pairs.temp.table_off)])
    for t in range(2 * M):
        if br[t] < 0:
            continue
        ballot = BALLOT_MODEL["ballot_base_ns"] + BALLOT_MODEL["ballot_per_entry_ns"] * (
            br[t] + (n[t] + 64) // 64)
        assert (info["algos"][t] == binding.ALGO_BALLOT) == (ballot < plain_ns[t]), t
    # sorted temperatures: the materials with many pairs per table entry take
    # the ballot scan (8-12 of 24 here); i.i.d. densities never do
    say(f"ballot temperature tables: {(info['algos'][M:] == binding.ALGO_BALLOT).sum()} of {M}")
    assert (info["algos"][M:] == binding.ALGO_BALLOT).sum() >= 4
    assert not np.any(info["algos"][:M] == binding.ALGO_BALLOT)
    o_r, o_t = plan.search(d["r"], d["t"])
    plan.close()
    assert np.array_equal(o_r.cpu().numpy(), oracle_mod.search_lt_segments(
        pairs.rho.tables, pairs.rho.table_off, rho, pairs.rho.query_off))
    assert np.array_equal(o_t.cpu().numpy(), oracle_mod.search_lt_segments(
        pairs.temp.tables, pairs.temp.table_off, temp, pairs.temp.query_off))
