"""The autotuner on the GPU: the learned index as a per-table candidate, and
the SS_TUNER_CACHE calibrate-once cache.

The learned candidate is decided per table by the cost model (paper Sec. 5.1
and 5.2: the best method depends on the array size and the data's
distribution).  With coefficients that price out the exponent hash and put
the learned index's fixed cost between a short and a long bisection, the
choice turns on the table's size: short tables keep the bisection (they are
not even trained), long tables go to the learned index, and a table with
negative entries (no model possible) keeps the bisection.  The plan reports
both modelled costs of every table, and the choice must follow them.  Every
result must still equal the oracle.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def binding(gpu):
    from paper_2112_03229_amd import binding as b
    return b


def geometric(n, lo, hi):
    return lo * (hi / lo) ** (np.arange(n) / (n - 1))


def test_tuner_chooses_learned_per_table(binding, gpu, oracle_mod, inputs_mod):
    saved = binding.tuner_get()
    tabs = [geometric(20, 1e-3, 1e2), geometric(5000, 1e-6, 1e6), geometric(24, 2.0, 9.0),
            geometric(6000, 1e-2, 1e9), inputs_mod.single_table(30), geometric(16, 1e5, 1e7),
            np.array([-1.0, 0.5, 3.0] * 1 + list(geometric(3000, 4.0, 1e6)))]
    counts = [50001, 120003, 7777, 90000, 4096, 333, 20000]
    toff = np.zeros(len(tabs) + 1, dtype=np.int64)
    toff[1:] = np.cumsum([t.size for t in tabs])
    qoff = np.zeros(len(tabs) + 1, dtype=np.int64)
    qoff[1:] = np.cumsum(counts)
    tables = np.concatenate(tabs)
    x = np.concatenate([inputs_mod.table_targets(np.abs(t) + 1e-9, c, seed=40 + i)
                        for i, (t, c) in enumerate(zip(tabs, counts))])
    x[::13] = tables[np.arange(0, x.size, 13) % tables.size]
    x[:14] = inputs_mod.special_values()
    want = oracle_mod.search_lt_segments(tables, toff, x, qoff)
    # the exponent hash priced out, bisection steps ten times a learned
    # step, and a learned fixed cost between a short and a long bisection
    try:
        binding.tuner_set(hash_base_ns=1.0, hash_per_k_ns=1.0, bin_base_ns=0.0,
                          bin_per_step_ns=0.1e-3, learned_base_ns=0.6e-3,
                          learned_per_step_ns=0.01e-3)
        plan = binding.MultiPlan(torch.from_numpy(tables).to(gpu), toff, qoff)
    finally:
        binding.tuner_set(**saved)
    info = plan.info()
    algos, plain, learned = info["algos"], info["plain_ns"], info["learned_ns"]
    say(f"tuner choices: {algos.tolist()}")
    say(f"plain ns: {plain.tolist()}")
    say(f"learned ns: {learned.tolist()}")
    # the decision rule on every table
    for t in range(len(tabs)):
        if learned[t] >= 0:
            assert (algos[t] == binding.ALGO_LEARNED) == (learned[t] < plain[t])
        else:
            assert algos[t] == binding.ALGO_BINARY
    # long tables go to the learned index; short ones, and the table with
    # negative entries (no model), keep the bisection
    long_tab = [t.size >= 5000 for t in tabs[:6]]
    assert all(a == binding.ALGO_LEARNED for a, lg in zip(algos[:6], long_tab) if lg)
    assert all(a == binding.ALGO_BINARY for a, lg in zip(algos[:6], long_tab) if not lg)
    assert algos[6] == binding.ALGO_BINARY and learned[6] == -1
    got = plan.search(torch.from_numpy(x).to(gpu)).cpu().numpy()
    assert np.array_equal(got, want)
    say(f"fallbacks {plan.fallbacks()}")
    plan.close()
    # with the model as it was, the same batch is searched exactly whatever it picks
    plan = binding.MultiPlan(torch.from_numpy(tables).to(gpu), toff, qoff)
    assert np.array_equal(plan.search(torch.from_numpy(x).to(gpu)).cpu().numpy(), want)
    plan.close()


CHILD = r"""
import json, sys
sys.path.insert(0, {repo!r})
import numpy as np, torch
from paper_2112_03229_amd import binding
t = torch.from_numpy(np.geomspace(1e-3, 1e3, 100)).cuda()
plan = binding.MultiPlan(t, np.array([0, 100]), np.array([0, 1000]))
plan.search(torch.ones(1000, dtype=torch.float64, device="cuda"))
print(json.dumps(binding.tuner_get()))
"""


def run_child(path):
    env = dict(os.environ, SS_TUNER_CACHE=str(path))
    r = subprocess.run([sys.executable, "-c", CHILD.format(repo=REPO)], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1]), r.stderr


def test_env_cache_calibrates_once(gpu, tmp_path):
    path = tmp_path / "tuner.json"
    say("case SS_TUNER_CACHE: missing file -> calibrate and write")
    first, _ = run_child(path)
    assert first["calibrated"] == 1.0 and path.exists()
    rec = json.loads(path.read_text())
    assert rec["arch"].startswith("gfx950") and rec["calibrated"] == 1
    say(f"calibrated model: {first}")
    say("case SS_TUNER_CACHE: valid file -> loaded, not recalibrated")
    mtime = path.stat().st_mtime_ns
    second, _ = run_child(path)
    assert second == first and path.stat().st_mtime_ns == mtime
    say("case SS_TUNER_CACHE: file from another arch -> refused, recalibrated")
    path.write_text(json.dumps(dict(rec, arch="gfx942", stream_gbs=1.5)))
    third, err = run_child(path)
    assert "refused" in err and third["stream_gbs"] != 1.5 and third["calibrated"] == 1.0
    assert json.loads(path.read_text())["arch"].startswith("gfx950")


LOG_CHILD = r"""
import sys
sys.path.insert(0, {repo!r})
import numpy as np, torch
from paper_2112_03229_amd import binding
t = torch.from_numpy(np.geomspace(1e-3, 1e3, 100)).cuda()
x = torch.from_numpy(np.sort(np.geomspace(2e-3, 5e2, 100000))).cuda()
plan = binding.MultiPlan(t, np.array([0, 100]), np.array([0, 100000]), sample=x)
plan.search(x)
torch.cuda.synchronize()
"""


def test_log_reports_plan_decisions(gpu, tmp_path):
    env = dict(os.environ, SS_LOG="1", SS_TUNER_CACHE=str(tmp_path / "tuner.json"))
    say("case SS_LOG=1: plan and tuner decisions on stderr")
    r = subprocess.run([sys.executable, "-c", LOG_CHILD.format(repo=REPO)], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stderr.splitlines() if ln.startswith("[ss] ")]
    say("\n".join(lines))
    assert any(ln.startswith("[ss] tuner calibrated on gfx950") for ln in lines)
    assert any(ln.startswith("[ss] plan batched: 1 tables") and "100000 targets" in ln
               for ln in lines)
    assert any(ln.startswith("[ss] plan sample: mean ballot bracket") for ln in lines)
