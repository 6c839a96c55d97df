"""Saved plans (ss_plan_save / ss_multi_plan_load / ss_pair_plan_load).

A reloaded plan has the same per-table choices and gives the same indices as
the plan it was saved from, without tuning or training; on other tables of
the same sizes it is still exact (bin parameters are rebuilt and every
learned model's bound is measured again); tables of other sizes, a plan of
another form and interpolation plans are refused.  The saved convention,
tile order and tiles per workgroup win over the options in force.
"""
import os
import sys

import numpy as np
import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_multi import odd_batch, ragged_pairs  # noqa: E402

pytestmark = pytest.mark.gpu


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


def test_batched_plan_roundtrip(binding, gpu, oracle_mod, inputs_mod, tmp_path):
    tables, toff, qoff, x = odd_batch(inputs_mod, seed=41)
    want = oracle_mod.search_lt_segments(tables, toff, x, qoff)
    d_tab, xt = torch.from_numpy(tables).to(gpu), torch.from_numpy(x).to(gpu)
    say("case batched plan, every eligible table learned, saved and reloaded")
    plan = with_opts(binding, {binding.OPT_PLAN_LEARNED: binding.PLAN_LEARNED_ALL,
                               binding.OPT_PLAN_TILES: 3},
                     lambda: binding.MultiPlan(d_tab, toff, qoff))
    first = plan.search(xt).cpu().numpy()
    assert np.array_equal(first, want)
    fb = plan.fallbacks()
    info = plan.info()
    assert (info["algos"] == binding.ALGO_LEARNED).sum() > 10
    path = str(tmp_path / "batched.plan")
    plan.save(path)
    plan.close()
    # reloaded under other options: the saved choices and shape win
    again = with_opts(binding, {binding.OPT_PLAN_LEARNED: binding.PLAN_LEARNED_NONE,
                                binding.OPT_PLAN_TILES: 5},
                      lambda: binding.MultiPlan(d_tab, toff, qoff, saved=path))
    info2 = again.info()
    assert np.array_equal(info2["algos"], info["algos"])
    assert np.array_equal(info2["bits"], info["bits"])
    assert info2["tiles_per_wg"] == 3
    assert np.array_equal(again.search(xt).cpu().numpy(), first)
    assert again.fallbacks() == fb  # the same models, their bounds measured again
    again.close()
    # other tables of the same sizes (every entry scaled by 3): still exact
    other = np.ascontiguousarray(tables * 3.0)
    want3 = oracle_mod.search_lt_segments(other, toff, x, qoff)
    say("case batched plan reloaded on other tables of the same sizes")
    moved = binding.MultiPlan(torch.from_numpy(other).to(gpu), toff, qoff, saved=path)
    assert np.array_equal(moved.search(xt).cpu().numpy(), want3)
    moved.close()
    # tables of other sizes, and the file as a paired plan, are refused
    toff2 = toff.copy()
    toff2[1:-1] += 1
    with pytest.raises(binding.SearchSortedError) as e:
        binding.MultiPlan(d_tab, toff2, qoff, saved=path)
    assert e.value.code == -1
    pairs = ragged_pairs(inputs_mod, 3, 8, 10000)
    with pytest.raises(binding.SearchSortedError):
        binding.PairPlan(torch.from_numpy(pairs.rho.tables).to(gpu), pairs.rho.table_off,
                         torch.from_numpy(pairs.temp.tables).to(gpu), pairs.temp.table_off,
                         pairs.rho.query_off, saved=path)


@pytest.mark.parametrize("joint", [0, 1], ids=["split", "joint"])
def test_paired_plan_roundtrip(binding, gpu, oracle_mod, inputs_mod, tmp_path, joint):
    pairs = ragged_pairs(inputs_mod, 43, 60, 500003)
    rho, temp = inputs_mod.paired_targets(pairs, seed=43)
    want_r = oracle_mod.search_le_clamped
    dr, dt = torch.from_numpy(rho).to(gpu), torch.from_numpy(temp).to(gpu)
    rt = torch.from_numpy(pairs.rho.tables).to(gpu)
    tt = torch.from_numpy(pairs.temp.tables).to(gpu)
    say(f"case paired plan joint={joint}, paper convention, some tables learned, saved")
    opts = {binding.OPT_PAIR_JOINT: joint, binding.OPT_CONVENTION: 1,
            binding.OPT_PLAN_LEARNED: binding.PLAN_LEARNED_ALL, binding.OPT_PLAN_ORDER: 1}
    plan = with_opts(binding, opts, lambda: binding.PairPlan(rt, pairs.rho.table_off, tt,
                                                              pairs.temp.table_off,
                                                              pairs.rho.query_off))
    o_r, o_t = plan.search(dr, dt)
    first_r, first_t = o_r.cpu().numpy(), o_t.cpu().numpy()
    # the paper's convention, per material
    po = pairs.rho.query_off
    for j in range(pairs.num_materials):
        a, b = po[j], po[j + 1]
        assert np.array_equal(first_r[a:b], want_r(pairs.rho.table(j), rho[a:b]))
        assert np.array_equal(first_t[a:b], want_r(pairs.temp.table(j), temp[a:b]))
    info = plan.info()
    path = str(tmp_path / "paired.plan")
    plan.save(path)
    plan.close()
    say(f"case paired plan joint={joint} reloaded under the default options")
    again = binding.PairPlan(rt, pairs.rho.table_off, tt, pairs.temp.table_off,
                             pairs.rho.query_off, saved=path)
    assert np.array_equal(again.info()["algos"], info["algos"])
    r2, t2 = again.search(dr, dt)
    assert np.array_equal(r2.cpu().numpy(), first_r)
    assert np.array_equal(t2.cpu().numpy(), first_t)
    again.close()
    # a batched load of a paired file is refused
    with pytest.raises(binding.SearchSortedError):
        binding.MultiPlan(rt, pairs.rho.table_off, pairs.rho.query_off, saved=path)


def test_interp_plans_are_not_saved(binding, gpu, inputs_mod, tmp_path):
    it = inputs_mod.interp_layout(seed=45, materials=4, total_pairs=1000)
    p = it.pairs
    plan = binding.InterpPlan(torch.from_numpy(p.rho.tables).to(gpu), p.rho.table_off,
                              torch.from_numpy(p.temp.tables).to(gpu), p.temp.table_off,
                              p.rho.query_off, torch.from_numpy(it.values).to(gpu))
    with pytest.raises(binding.SearchSortedError) as e:
        plan.save(str(tmp_path / "x.plan"))
    assert e.value.code == -6
    plan.close()
