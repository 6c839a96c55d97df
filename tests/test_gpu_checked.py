"""The device-checked library (built with -DSS_DEVICE_CHECKS=1 into
_lib/checked/): every kernel path -- each single-table kernel, every plan
form and forced kernel, learned searches, interpolation and the
no-allocation search -- runs on edge and regular inputs with every LDS index
of the search routines, every full tile's target range and every plan
workgroup's staged layout checked on the device.  The results must equal the
oracle and the kernels must count no violation; the self-test (one clamped
index in a one-thread kernel) shows that the counter counts.  Runs in a
child process that loads the checked build through SS_LIBRARY.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECKED = os.path.join(REPO, "paper_2112_03229_amd", "_lib", "checked", "libsearchsorted.so")

CHILD = r"""
import sys
sys.path[:0] = [{repo!r}, {tests!r}]
import numpy as np, torch
from paper_2112_03229_amd import binding as b, inputs
import oracle
from test_gpu_multi import odd_batch, ragged_pairs
from test_gpu_ballot_plan import mixed_batch

def say(*a):
    print(*a, flush=True)

def same(got, want, what):
    if not np.array_equal(got, want):
        k = int(np.flatnonzero(got != want)[0])
        raise AssertionError(f"{{what}}: first mismatch at {{k}}: {{got[k]}} != {{want[k]}}")

dev = torch.device("cuda:0")
say("case self-test")
b.debug_selftest()
v = b.debug_violations()
assert v == 1, v

def opts(d, make):
    old = {{k: b.get_option(k) for k in d}}
    try:
        for k, val in d.items():
            b.set_option(k, val)
        return make()
    finally:
        for k, val in old.items():
            b.set_option(k, val)

# single tables: every kernel, edge sizes, both conventions
tables = [np.zeros(0), np.array([1.0]), np.array([-2.0, 3.0]), inputs.single64_table(),
          inputs.single_table(100), inputs.single_table(1000), inputs.single_table(3000),
          np.array([-5.0, -1.0, -0.0, 0.0, 2.0, 1e10]), inputs.single_table(9000)]
for ti, table in enumerate(tables):
    lo = abs(table[0]) if table.size else 1.0
    x = inputs.log_uniform(70 + ti, 3, 1e-12, 1e12, 50021)
    x[::3] *= -1
    if table.size:
        x[1::7] = table[np.arange(1, x.size, 7) % table.size]
    x[:14] = inputs.special_values()
    want = oracle.search_lt(table, x)
    want_le = oracle.search_le_clamped(table, x)
    t, xt = torch.from_numpy(table).to(dev), torch.from_numpy(x).to(dev)
    algos = ("auto", "binary", "ballot", "exphash", "binary_global", "loghash", "skiplist")
    if table.size > 6000:  # not staged: the automatic choice reads it in place
        algos = ("auto", "binary_global")
    for algo in algos:
        say(f"case single n={{table.size}} algo={{algo}}")
        same(b.search_with(t, xt, algo).cpu().numpy(), want, algo)
        got = opts({{b.OPT_CONVENTION: 1}}, lambda: b.search_with(t, xt, algo).cpu().numpy())
        same(got, want_le, algo + " paper convention")

# plans: the odd batch, tuned and every forced kernel, learned models
tabs, toff, qoff, x = odd_batch(inputs, seed=71)
want = oracle.search_lt_segments(tabs, toff, x, qoff)
dt, dx = torch.from_numpy(tabs).to(dev), torch.from_numpy(x).to(dev)
for name, d in (("tuned", {{}}), ("binary", {{b.OPT_PLAN_ALGO: b.ALGO_BINARY}}),
                ("exphash", {{b.OPT_PLAN_ALGO: b.ALGO_EXPHASH}}),
                ("ballot", {{b.OPT_PLAN_ALGO: b.ALGO_BALLOT}}),
                ("learned", {{b.OPT_PLAN_LEARNED: b.PLAN_LEARNED_ALL, b.OPT_LEARNED_STEPS: 200}}),
                ("contiguous", {{b.OPT_PLAN_ORDER: 1}}), ("xcd8", {{b.OPT_PLAN_XCD: 8}})):
    say(f"case batched plan {{name}}")
    plan = opts(d, lambda: b.MultiPlan(dt, toff, qoff))
    same(plan.search(dx).cpu().numpy(), want, "batched " + name)
    plan.close()
say("case sampled plan")
mt, mo, mq, mx, _ = mixed_batch(inputs)
plan = b.MultiPlan(torch.from_numpy(mt).to(dev), mo, mq, sample=torch.from_numpy(mx).to(dev))
same(plan.search(torch.from_numpy(mx).to(dev)).cpu().numpy(),
     oracle.search_lt_segments(mt, mo, mx, mq), "sampled")
plan.close()

# paired forms
pairs = ragged_pairs(inputs, 72, 40, 200003)
rho, temp = inputs.paired_targets(pairs, seed=72)
rho[:3] = [np.nan, -1.0, np.inf]
wr = oracle.search_lt_segments(pairs.rho.tables, pairs.rho.table_off, rho, pairs.rho.query_off)
wt = oracle.search_lt_segments(pairs.temp.tables, pairs.temp.table_off, temp,
                               pairs.temp.query_off)
args = (torch.from_numpy(pairs.rho.tables).to(dev), pairs.rho.table_off,
        torch.from_numpy(pairs.temp.tables).to(dev), pairs.temp.table_off, pairs.rho.query_off)
dr, dtp = torch.from_numpy(rho).to(dev), torch.from_numpy(temp).to(dev)
for joint in (0, 1):
    for learned in (b.PLAN_LEARNED_NONE, b.PLAN_LEARNED_ALL):
        say(f"case paired joint={{joint}} learned={{learned}}")
        plan = opts({{b.OPT_PAIR_JOINT: joint, b.OPT_PLAN_LEARNED: learned,
                     b.OPT_LEARNED_STEPS: 200}}, lambda: b.PairPlan(*args))
        o_r, o_t = plan.search(dr, dtp)
        same(o_r.cpu().numpy(), wr, "paired rho")
        same(o_t.cpu().numpy(), wt, "paired T")
        plan.close()

# interpolation (staged grids and grids read from global memory: axes up
# to 250 x 120 points, grids over the 15360 values staged)
it = inputs.interp_layout(seed=73, materials=24, total_pairs=300007, n_rho=(100, 250),
                          n_t=(60, 120))
assert np.diff(it.value_off).max() > 15360 and np.diff(it.value_off).min() <= 15360
ip = it.pairs
ir, itp = inputs.paired_targets(ip, seed=73)
say("case interpolation")
plan = b.InterpPlan(torch.from_numpy(ip.rho.tables).to(dev), ip.rho.table_off,
                    torch.from_numpy(ip.temp.tables).to(dev), ip.temp.table_off,
                    ip.rho.query_off, torch.from_numpy(it.values).to(dev))
o_r = torch.empty(ip.num_pairs, dtype=torch.int32, device=dev)
o_t = torch.empty_like(o_r)
plan.interpolate(torch.from_numpy(ir).to(dev), torch.from_numpy(itp).to(dev), out_rho=o_r,
                 out_t=o_t)
same(o_r.cpu().numpy(), oracle.search_lt_segments(ip.rho.tables, ip.rho.table_off, ir,
                                                  ip.rho.query_off), "interp rho")
plan.close()

# learned single-table search, staged and in place
for n in (300, 2000):
    say(f"case learned n={{n}}")
    table = inputs.learned_table(n=n)
    tt = torch.from_numpy(table).to(dev)
    li = b.LearnedIndex(tt, steps=400)
    x = inputs.table_targets(table, 100003, seed=74)
    x[:14] = inputs.special_values()
    same(li.search(torch.from_numpy(x).to(dev)).cpu().numpy(), oracle.search_lt(table, x),
         "learned")
    li.set_error_bound(0)
    same(li.search(torch.from_numpy(x).to(dev)).cpu().numpy(), oracle.search_lt(table, x),
         "learned E=0")
    li.close()

# the no-allocation batched search
say("case no-allocation search")
got = b.multi_search_noalloc(dt, torch.from_numpy(toff).to(dev), torch.from_numpy(qoff).to(dev),
                             dx).cpu().numpy()
same(got, want, "noalloc")

torch.cuda.synchronize()
v = b.debug_violations()
say(f"violations {{v}}")
assert v == 0, v
say("checked: ok")
"""


def test_checked_build_counts_no_violation(gpu):
    if not os.path.exists(CHECKED):
        pytest.fail(f"{CHECKED} is missing: run __graft_entry__.build()")
    env = dict(os.environ, SS_LIBRARY=CHECKED)
    r = subprocess.run([sys.executable, "-u", "-c",
                        CHILD.format(repo=REPO, tests=os.path.join(REPO, "tests"))],
                       env=env, capture_output=True, text=True, timeout=280)
    print(r.stdout[-4000:], flush=True)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "checked: ok" in r.stdout


def test_normal_build_has_no_checks(gpu):
    """The library the package loads by default is the unchecked one."""
    from paper_2112_03229_amd import binding as b
    if os.environ.get("SS_LIBRARY"):
        pytest.skip("another build selected")
    with pytest.raises(b.SearchSortedError) as e:
        b.debug_violations()
    assert e.value.code == -6
