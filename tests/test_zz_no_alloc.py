"""The batched search that allocates nothing (ss_multi_search_noalloc),
called through the C ABI, against the plan-based ss_multi_search on the same
tables and targets, bit for bit -- two calls in a row, the second with fewer
tables and targets -- and against the oracle.  Also: tables longer than the
LDS budget (searched in place), the paper's convention, and an argument
error before any device work.
"""
import os
import sys

import numpy as np
import pytest
import torch

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_multi import odd_batch  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def binding(gpu):
    from paper_2112_03229_amd import binding as b
    return b


def run_both(binding, gpu, tables, toff, qoff, x):
    d_tab = torch.from_numpy(tables).to(gpu)
    xt = torch.from_numpy(x).to(gpu)
    plan = binding.MultiPlan(d_tab, toff, qoff)
    want = plan.search(xt)
    out = torch.full((x.size,), -7, dtype=torch.int32, device=gpu)
    got = binding.multi_search_noalloc(d_tab, torch.from_numpy(toff).to(gpu),
                                       torch.from_numpy(qoff).to(gpu), xt, out)
    torch.cuda.synchronize()
    plan.close()
    return got.cpu().numpy(), want.cpu().numpy()


def test_noalloc_matches_plan_two_calls(binding, gpu, oracle_mod, inputs_mod):
    big = odd_batch(inputs_mod, seed=5)
    small = odd_batch(inputs_mod, seed=9)
    # the second call: fewer tables and targets (the first 11 tables)
    tables, toff, qoff, x = small
    k = 11
    small = (tables[:toff[k]], toff[:k + 1].copy(), qoff[:k + 1].copy(), x[:qoff[k]])
    assert small[1].size < big[1].size and small[3].size < big[3].size
    for name, (tables, toff, qoff, x) in (("first", big), ("second, smaller", small)):
        say(f"case noalloc {name}: T={toff.size - 1} m={x.size}")
        got, want = run_both(binding, gpu, tables, toff, qoff, x)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]], x[bad[:5]])
        ref = oracle_mod.search_lt_segments(tables, toff, x, qoff)
        assert np.array_equal(got, ref)


def test_noalloc_long_tables_and_convention(binding, gpu, oracle_mod, inputs_mod):
    # tables past the LDS budget (6136 entries) are searched in global memory
    tabs = [inputs_mod.single_table(n) for n in (50, 6136, 6137, 20000, 1)]
    counts = [10001, 4096 * 3 + 5, 777, 65536 + 3, 9]
    toff = np.zeros(len(tabs) + 1, dtype=np.int64)
    toff[1:] = np.cumsum([t.size for t in tabs])
    qoff = np.zeros(len(tabs) + 1, dtype=np.int64)
    qoff[1:] = np.cumsum(counts)
    tables = np.concatenate(tabs)
    x = np.concatenate([inputs_mod.table_targets(t, c, seed=31 + i)
                        for i, (t, c) in enumerate(zip(tabs, counts))])
    x[::97] = tables[np.arange(0, x.size, 97) % tables.size]
    d_tab = torch.from_numpy(tables).to(gpu)
    d_toff, d_qoff = torch.from_numpy(toff).to(gpu), torch.from_numpy(qoff).to(gpu)
    xt = torch.from_numpy(x).to(gpu)
    say(f"case noalloc long tables: T={len(tabs)} m={x.size}")
    got = binding.multi_search_noalloc(d_tab, d_toff, d_qoff, xt).cpu().numpy()
    assert np.array_equal(got, oracle_mod.search_lt_segments(tables, toff, x, qoff))
    say("case noalloc paper convention")
    binding.set_option(binding.OPT_CONVENTION, 1)
    try:
        got = binding.multi_search_noalloc(d_tab, d_toff, d_qoff, xt).cpu().numpy()
    finally:
        binding.set_option(binding.OPT_CONVENTION, 0)
    want = np.concatenate([oracle_mod.search_le_clamped(tabs[i], x[qoff[i]:qoff[i + 1]])
                           for i in range(len(tabs))])
    assert np.array_equal(got, want)


def test_noalloc_rejects_too_many_tables(binding, gpu):
    L = binding.lib()
    z = torch.zeros(70000, dtype=torch.int64, device=gpu)
    x = torch.zeros(4, dtype=torch.float64, device=gpu)
    o = torch.zeros(4, dtype=torch.int32, device=gpu)
    rc = L.ss_multi_search_noalloc(x.data_ptr(), 4, z.data_ptr(), 65537, z.data_ptr(),
                                   x.data_ptr(), 4, o.data_ptr())
    assert rc == -1 and b"65536" in L.ss_last_error()
