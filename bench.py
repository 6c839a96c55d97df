"""Benchmark of the batched sorted search on one MI355X.

Headline workload (one "step"): the paired lookup of 4096 materials.  Each
material has a density table (50..4000 float64 entries) and a temperature
table (20..1000 entries), log-distributed within seeded ranges; 1e9 (rho, T)
float64 pairs, unevenly spread over the materials, are searched in both
tables -- 2e9 searches -- in one plan launch with the autotuner's per-table
choice of kernel (exponent hash, bisection or learned index).  Inputs are
generated on the host, copied to HBM before timing, and stay resident.

Output: one JSON line with whole-job throughput in Gqueries/s (one query is
one search: 12 algorithmic bytes, an 8-byte target read and a 4-byte index
written), the HBM roofline fraction of the plan kernel (its average launch
duration from HIP events on the launch stream around the timed region), the
metric's comparison of learned+batched against plain search on the same
pairs, the other workloads measured after the timed region, and the CPU
oracle timed on the host's cores over a bounded sample of the same pairs.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-kernels]
                       [--no-systems]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

METRIC = "Gqueries/s and % HBM roofline, bit-exact idx; learned+batched vs plain search"
HBM_PEAK_GBS = 8000.0
BYTES_PER_QUERY = 12
TABLE_SIZES = (100, 300, 1000)
ORDERS = ("random", "smooth")
M = 10**8
# Untimed load before any timed region, whatever the warm-up step count:
# after an idle period (host-side input generation) MI355X takes about 20 ms
# of load to reach steady clocks.
WARM_FLOOR_MS = 200.0
TRIALS = 20  # the paper reports the mean of 20 trials (Sec. 4)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources each profiled kernel and its launch are built from: a counter
# record in profiles/traffic.json is used only while their code is
# unchanged.  Comments and blank space do not count (the digest is taken
# over the text with comments removed and space collapsed), so a record
# survives edits of wording but not of code.
KERNEL_SOURCES = {
    "single": ("csrc/ss_single.hip", "csrc/ss_device.h", "csrc/ss_host.h", "csrc/ss_loghash.h",
               "csrc/ss_skiplist.h", "../include/searchsorted.h"),
    "plan": ("csrc/ss_plan.hip", "csrc/ss_device.h", "csrc/ss_host.h", "csrc/ss_mlp.h",
             "csrc/ss_learned.h", "csrc/ss_tuner.h", "csrc/ss_tuner.hip",
             "../include/searchsorted.h"),
    "learned": ("csrc/ss_learned.hip", "csrc/ss_device.h", "csrc/ss_host.h", "csrc/ss_mlp.h",
                "csrc/ss_learned.h", "../include/searchsorted.h"),
}


def _code_only(text: str) -> str:
    """C/C++ source without comments, runs of white space collapsed (string
    and character literals kept as they are)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == "/" and text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif c == "/" and text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_digest(group: str) -> str:
    h = hashlib.sha256()
    pkg = os.path.join(HERE, "paper_2112_03229_amd")
    for name in KERNEL_SOURCES[group]:
        with open(os.path.normpath(os.path.join(pkg, name)), encoding="utf-8") as f:
            h.update(name.encode())
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current sources of that kernel; else None."""
    path = os.path.join(HERE, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get(key)
    if not ent or ent.get("source_digest") != kernel_source_digest(ent.get("sources", "single")):
        return None
    return ent.get("bytes_per_launch")


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on the headline's own pairs, and the paper's numbers
# ---------------------------------------------------------------------------

def paper_cpu_speedups() -> list:
    """The paper's CPU results, quoted with their hardware (none is re-run here;
    its figures are not in the text, so only the numbers it states are given)."""
    cpus = "one core of an AMD EPYC 7551 (AVX2, 256-bit), an Intel Xeon Phi 7250 (AVX-512) " \
           "or an Intel Xeon Gold 6152 (AVX-512) (Table 1); which CPU gave the best case is " \
           "not stated"
    work = "the 110-entry density axis of SESAME table 301, material 3720; 5e6 targets on " \
           "1e-10..1e10; mean of 20 trials (Sec. 4, Sec. 5)"
    return [
        {"what": "vectorised (OpenMP SIMD) exponent hash search vs EOSPAC's hunt-and-locate",
         "speedup": "up to 8x (the conclusion words it as 800%)",
         "hardware": cpus, "compiler": "Intel 20.0.2 (gcc 9.3.0 showed no significant "
                                       "vectorisation gain)", "workload": work,
         "source": "Abstract; Sec. 6"},
        {"what": "unvectorised exponent hash search vs hunt-and-locate",
         "speedup": "more than 2x (over 100% faster)", "hardware": cpus,
         "compiler": "gcc 9.3.0 / Intel 20.0.2, vectorisation disabled", "workload": work,
         "source": "Sec. 6"},
        {"what": "explicit OpenMP SIMD plus auto-vectorisation flags vs auto-vectorisation alone",
         "speedup": "up to 4.8x (worded as 480%)", "hardware": cpus,
         "compiler": "Intel 20.0.2", "workload": work, "source": "Sec. 6"},
    ]


def _pair_sample(pairs, host_r, host_t, frac: float):
    """The first ceil(frac * count) pairs of every material (both axes)."""
    po = pairs.rho.query_off
    counts = np.diff(po)
    k = np.minimum(counts, np.ceil(counts * frac).astype(np.int64))
    off = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    off[1:] = np.cumsum(k)
    idx = np.concatenate([np.arange(po[j], po[j] + k[j]) for j in range(counts.shape[0])])
    return off, np.ascontiguousarray(host_r[idx]), np.ascontiguousarray(host_t[idx])


def cpu_baseline(pairs, host_r, host_t, budget_s: float = 20.0) -> dict:
    """The CPU oracle (plain linear count) on all host cores, on a bounded
    sample of the headline workload: the first pairs of every material,
    both axes."""
    import oracle

    def run(frac, threads):
        off, xr, xt = _pair_sample(pairs, host_r, host_t, frac)
        t0 = time.perf_counter()
        _, u1 = oracle.search_lt_segments(pairs.rho.tables, pairs.rho.table_off, xr, off,
                                          threads=threads, return_threads=True)
        _, u2 = oracle.search_lt_segments(pairs.temp.tables, pairs.temp.table_off, xt, off,
                                          threads=threads, return_threads=True)
        return int(off[-1]), time.perf_counter() - t0, max(u1, u2)

    total = pairs.num_pairs
    threads = oracle.default_threads()
    # calibration on 1% of the pairs (per-material thread start-up included,
    # which makes it pessimistic: the sample is enlarged once if short)
    n_cal, s_cal, _ = run(1e-2, threads)
    frac = min(1.0, max(1e7 / total, budget_s / (s_cal / n_cal) / total))
    n, sec, used = run(frac, threads)
    if sec < 0.5 * budget_s and frac < 1.0:
        frac = min(1.0, frac * 0.8 * budget_s / sec)
        n, sec, used = run(frac, threads)
    # the paper's own setting: one core (a third of the time budget)
    frac1 = min(1.0, max(1e5 / total, budget_s / 3 / (s_cal * threads / n_cal) / total))
    n1, sec1, _ = run(frac1, 1)
    return {
        "value": 2 * n / sec / 1e9,
        "unit": "Gqueries/s",
        "cores": int(used),
        "kind": "oracle",
        "sample": f"the first {frac:.2%} of every material's pairs of the headline workload "
                  f"({n} pairs = {2 * n} searches, both axes, {sec:.1f} s); plain linear "
                  f"count scan, {used} threads",
        "single_core": {"value": 2 * n1 / sec1 / 1e9, "unit": "Gqueries/s",
                        "sample": f"the first {frac1:.3%} of every material's pairs ({n1} "
                                  f"pairs), {sec1:.1f} s, 1 thread"},
        "host_cpu": _cpu_model(),
        "paper_cpu_speedups": paper_cpu_speedups(),
    }


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# Timing helpers
# ---------------------------------------------------------------------------

def copy_calibration(torch) -> None:
    """A plain 1 GiB device-to-device copy, launched 3 times: under rocprofv3
    --pmc its FETCH_SIZE / WRITE_SIZE per dispatch give the scale between the
    counters and true HBM bytes (1 GiB read and 1 GiB written per dispatch)."""
    n = (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 8, "dispatches": 3}), flush=True)


def warm(torch, fn, steps: int, floor_ms: float) -> dict:
    """Runs fn `steps` times, then keeps running it until at least floor_ms of
    wall time has passed since the first call (synchronised)."""
    t0 = time.perf_counter()
    done = 0
    for _ in range(steps):
        fn()
        done += 1
    torch.cuda.synchronize()
    while (time.perf_counter() - t0) * 1e3 < floor_ms:
        for _ in range(4):
            fn()
            done += 1
        torch.cuda.synchronize()
    return {"steps_run": done, "ms": round((time.perf_counter() - t0) * 1e3, 1)}


def time_call(torch, fn, reps: int = 5, warm_ms: float = 50.0) -> float:
    """Average milliseconds of fn() over reps calls on the current stream,
    after untimed calls that keep the GPU busy for at least warm_ms (first
    passes over freshly allocated multi-GB buffers also run slower)."""
    warm(torch, fn, 1, warm_ms)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def trials(torch, fn, queries: int, stream, count: int = TRIALS) -> dict:
    """count more calls, each bracketed by its own event pair."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(count)]
    for e0, e1 in ev:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    return {"count": count, "mean_ms": round(float(ms.mean()), 4),
            "median_ms": round(float(np.median(ms)), 4), "min_ms": round(float(ms.min()), 4),
            "mean_gqps": round(queries / (ms.mean() * 1e-3) / 1e9, 2),
            "median_gqps": round(queries / (np.median(ms) * 1e-3) / 1e9, 2),
            "max_gqps": round(queries / (ms.min() * 1e-3) / 1e9, 2)}


def roof(queries: int, ms: float) -> dict:
    gbs = queries * BYTES_PER_QUERY / (ms * 1e-3) / 1e9
    return {"gqps": round(queries / (ms * 1e-3) / 1e9, 2), "ms": round(ms, 4),
            "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}


def plan_counts(binding, info) -> dict:
    algos = info["algos"]
    return {"learned_tables": int((algos == binding.ALGO_LEARNED).sum()),
            "exphash_tables": int((algos == binding.ALGO_EXPHASH).sum()),
            "bisection_tables": int((algos == binding.ALGO_BINARY).sum()),
            "ballot_tables": int((algos == binding.ALGO_BALLOT).sum())}


def with_options(binding, opts: dict, make):
    """make() with the given library options set, restoring them afterwards."""
    old = {k: binding.get_option(k) for k in opts}
    for k, v in opts.items():
        binding.set_option(k, v)
    try:
        return make()
    finally:
        for k, v in old.items():
            binding.set_option(k, v)


def compare_plans(torch, binding, make, run, queries: int, tuned_counts: dict,
                  reps: int = 3) -> dict:
    """The metric's comparison on one workload: plans with the tuner's choice
    excluding learned models ("plain"), with every eligible table learned,
    with every table forced to bisection and to the exponent hash."""
    res = {}
    variants = (
        ("plain", {binding.OPT_PLAN_LEARNED: binding.PLAN_LEARNED_NONE}),
        ("learned_forced", {binding.OPT_PLAN_LEARNED: binding.PLAN_LEARNED_ALL}),
        ("bisection_forced", {binding.OPT_PLAN_ALGO: binding.ALGO_BINARY}),
        ("exphash_forced", {binding.OPT_PLAN_ALGO: binding.ALGO_EXPHASH}),
    )
    for name, opts in variants:
        if name == "plain" and tuned_counts["learned_tables"] == 0:
            res[name] = {"same_plan_as": "tuned",
                         "note": "the tuner chose no learned table, so the tuned plan is "
                                 "the plain one"}
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = with_options(binding, opts, make)
        build_s = time.perf_counter() - t0
        ms = time_call(torch, lambda: run(plan), reps=reps)
        row = {**roof(queries, ms), **plan_counts(binding, plan.info()),
               "build_s": round(build_s, 2)}
        if name == "learned_forced":
            row["fallbacks"] = plan.fallbacks()
        plan.close()
        res[name] = row
    return res


# ---------------------------------------------------------------------------
# The headline: paired lookup, 4096 materials, 1e9 pairs
# ---------------------------------------------------------------------------

def paired_headline(torch, binding, inputs, dev, args) -> tuple:
    pairs = inputs.paired_layout()
    m = pairs.num_pairs
    log(f"bench: generating {m} pairs")
    hr = torch.empty(m, dtype=torch.float64).pin_memory()
    ht = torch.empty(m, dtype=torch.float64).pin_memory()
    inputs.paired_targets(pairs, out_rho=hr.numpy(), out_t=ht.numpy())
    r, t = hr.to(dev), ht.to(dev)
    o_r = torch.empty(m, dtype=torch.int32, device=dev)
    o_t = torch.empty(m, dtype=torch.int32, device=dev)
    d_rt = torch.from_numpy(pairs.rho.tables).to(dev)
    d_tt = torch.from_numpy(pairs.temp.tables).to(dev)

    def make():
        return binding.PairPlan(d_rt, pairs.rho.table_off, d_tt, pairs.temp.table_off,
                                pairs.rho.query_off)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = make()
    build_s = time.perf_counter() - t0
    info = plan.info()
    counts = plan_counts(binding, info)
    stream = torch.cuda.current_stream()

    def step():
        plan.search(r, t, o_r, o_t)

    log(f"bench: warmup {args.warmup} (+ a {WARM_FLOOR_MS:.0f} ms floor)")
    warmed = warm(torch, step, args.warmup, WARM_FLOOR_MS)
    log(f"bench: timing {args.steps} steps")
    # One pair of HIP events on the launch stream around the whole timed
    # region: the launches (one graph launch holding the plan's kernel per
    # step) run back to back, so the average launch duration is the region's
    # event time over the step count.
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avg_launch_ms = ev0.elapsed_time(ev1) / args.steps
    searches = 2 * m
    value = searches * args.steps / wall / 1e9
    achieved = searches * BYTES_PER_QUERY / (avg_launch_ms * 1e-3) / 1e9
    kernel = (f"ss::multi_kernel<2, {info['targets_per_lane']}, {info['learned_form']}, 0> "
              "(split paired plan)")
    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gqueries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "paired lookup: 4096 materials, density tables of 50..4000 and "
                        "temperature tables of 20..1000 float64 entries (sorted log-uniform "
                        "draws within seeded ranges in [1e-10,1e8]); 1e9 (rho,T) float64 "
                        "pairs = 2e9 searches per step, pair counts per material "
                        "proportional to 10^U(0,3); one plan launch with the autotuner's "
                        "per-table kernel (learned index, exponent hash or bisection)",
            "materials": pairs.num_materials,
            "pairs_per_step": m,
            "searches_per_step": searches,
            "bytes_per_query": BYTES_PER_QUERY,
            "plan_form": "split (density and temperature searches as 2M segments)",
            **counts,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("multi_kernel<paired>|paired-4096"),
            "kernel": kernel,
            "algorithmic_bytes_per_launch": searches * BYTES_PER_QUERY,
            "avg_launch_ms": round(avg_launch_ms, 4),
        },
        "warmup_run": warmed,
        "plan": {"build_s": round(build_s, 2), "tiles": info["tiles"],
                 "tiles_per_wg": info["tiles_per_wg"], "grid": info["grid"],
                 "lds_bytes": info["lds_bytes"]},
    }
    # the paper reports the mean of 20 trials; each trial here is one step
    # bracketed by its own event pair (context beside `value`, not part of it)
    result["trials"] = trials(torch, step, searches, stream)

    # A practical ceiling beside the 8 TB/s peak: the single-table kernel
    # streaming the same two target arrays with a one-entry table (two
    # launches, each search one compare), i.e. the rate this access pattern
    # (8 bytes read and 4 written per search over the same 24 GB) reaches here.
    log("bench: stream ceiling (one-entry table over the same arrays)")
    one = torch.ones(1, dtype=torch.float64, device=dev)
    ceil_ms = time_call(torch, lambda: (binding.search_sorted_batch(one, r, o_r),
                                        binding.search_sorted_batch(one, t, o_t)), reps=5)
    ceiling = searches * BYTES_PER_QUERY / (ceil_ms * 1e-3) / 1e9
    # the plan kernel itself with one-entry tables (context: with no search
    # work its loads arrive in bursts, and it runs below the real tables)
    M_ = pairs.num_materials
    ones = torch.ones(M_, dtype=torch.float64, device=dev)
    off1 = np.arange(M_ + 1, dtype=np.int64)
    one_plan = binding.PairPlan(ones, off1, ones, off1, pairs.rho.query_off)
    one_ms = time_call(torch, lambda: one_plan.search(r, t, o_r, o_t), reps=5)
    one_plan.close()
    result["roofline"]["stream_ceiling"] = {
        "achieved": round(ceiling, 1), "unit": "GB/s",
        "frac_of_peak": round(ceiling / HBM_PEAK_GBS, 4),
        "kernel_frac_of_ceiling": round(achieved / ceiling, 4),
        "how": "the single-table kernel over the same rho and T arrays with a one-entry table",
        "plan_with_one_entry_tables_gbs": round(searches * BYTES_PER_QUERY / (one_ms * 1e-3)
                                                / 1e9, 1)}

    if not args.no_systems:
        log("bench: learned+batched vs plain on the headline pairs")
        comp = {"tuned": {**roof(searches, avg_launch_ms), **counts,
                          "build_s": round(build_s, 2)}}
        comp.update(compare_plans(torch, binding, make,
                                  lambda pl: pl.search(r, t, o_r, o_t), searches, counts))
        # the other launch form: both axes of a tile of pairs in one workgroup
        joint = with_options(binding, {binding.OPT_PAIR_JOINT: 1}, make)
        comp["joint_form"] = {**roof(searches, time_call(
            torch, lambda: joint.search(r, t, o_r, o_t), reps=3)), **plan_counts(binding,
                                                                              joint.info())}
        joint.close()
        # plain search without batching: one single-table launch per table
        po = pairs.rho.query_off
        tr = [d_rt[pairs.rho.table_off[j]:pairs.rho.table_off[j + 1]] for j in range(M_)]
        tt = [d_tt[pairs.temp.table_off[j]:pairs.temp.table_off[j + 1]] for j in range(M_)]

        def per_table():
            for j in range(M_):
                a, b = int(po[j]), int(po[j + 1])
                if b > a:
                    binding.search_sorted_batch(tr[j], r[a:b], o_r[a:b])
                    binding.search_sorted_batch(tt[j], t[a:b], o_t[a:b])
        comp["per_table_launches"] = roof(searches, time_call(torch, per_table, reps=1))
        result["comparison"] = comp
    plan.close()
    del r, t, o_r, o_t, d_rt, d_tt
    return result, pairs, hr.numpy(), ht.numpy()


# ---------------------------------------------------------------------------
# Other workloads, measured after the timed region
# ---------------------------------------------------------------------------

def measure_single_tables(torch, binding, inputs, dev, no_kernels: bool) -> dict:
    """Single tables of 100, 300 and 1000 entries, 1e8 targets per launch in
    two orders (i.i.d. log-uniform and a smooth sorted walk): six launches of
    the library's automatic kernel choice (the staged bisection)."""
    tables = [inputs.single_table(n) for n in TABLE_SIZES]
    host = {}
    for order in ORDERS:
        buf = torch.empty(M, dtype=torch.float64).pin_memory()
        # the three tables share the range [1e-8, 1e6], hence one target array per order
        inputs.table_targets(tables[0], M, seed=2112, kind=order, out=buf.numpy())
        host[order] = buf
    d_tables = [torch.from_numpy(t).to(dev) for t in tables]
    d_x = {o: host[o].to(dev) for o in ORDERS}
    d_out = {(n, o): torch.empty(M, dtype=torch.int32, device=dev)
             for n in TABLE_SIZES for o in ORDERS}
    pairs = [(i, o) for i in range(len(TABLE_SIZES)) for o in ORDERS]
    stream = torch.cuda.current_stream()

    def step():
        for i, o in pairs:
            binding.search_sorted_batch(d_tables[i], d_x[o], d_out[(TABLE_SIZES[i], o)])

    warm(torch, step, 5, 50.0)
    reps = 30
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    step_ms = ev0.elapsed_time(ev1) / reps
    avg_launch_ms = step_ms / len(pairs)
    achieved = M * BYTES_PER_QUERY / (avg_launch_ms * 1e-3) / 1e9
    one = torch.ones(1, dtype=torch.float64, device=dev)
    ceil_ms = min(time_call(torch, lambda: binding.search_sorted_batch(
        one, d_x[o], d_out[(TABLE_SIZES[0], o)]), reps=10) for o in ORDERS)
    ceiling = M * BYTES_PER_QUERY / (ceil_ms * 1e-3) / 1e9
    res = {"workload": "single tables n=100,300,1000 (log-uniform on [1e-8,1e6]); 1e8 "
                       "float64 targets per table and order (i.i.d. log-uniform and smooth "
                       "sorted walk); six launches of the automatic kernel (staged bisection)",
           **roof(len(pairs) * M, step_ms),
           "roofline": {"kernel": "ss::single_kernel<1, 8, 0>", "avg_launch_ms":
                        round(avg_launch_ms, 4), "achieved": round(achieved, 1),
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic("single_kernel<binary>|single-1e8"),
                        "stream_ceiling_gbs": round(ceiling, 1),
                        "kernel_frac_of_ceiling": round(achieved / ceiling, 4)},
           "trials": trials(torch, step, len(pairs) * M, stream)}
    if not no_kernels:
        log("bench: per-kernel comparison")
        comp = {}
        for (i, o) in pairs:
            row = {}
            for algo in ("binary", "ballot", "exphash", "loghash", "skiplist"):
                out = d_out[(TABLE_SIZES[i], o)]
                ms = time_call(torch, lambda: binding.search_with(d_tables[i], d_x[o], algo, -1,
                                                                  out), reps=5, warm_ms=20.0)
                row[algo] = round(M / (ms * 1e-3) / 1e9, 2)
            comp[f"n={TABLE_SIZES[i]}/{o}"] = row
        res["kernels_gqps"] = comp
    del d_x, d_out, host
    return res


def measure_batched(torch, binding, inputs, dev) -> dict:
    """512 tables (n uniform on 20..2000), ~7.4e8 targets, one plan launch."""
    batch = inputs.batched_layout()
    m = batch.num_queries
    host = torch.empty(m, dtype=torch.float64).pin_memory()
    inputs.batched_targets(batch, out=host.numpy())
    x = host.to(dev)
    out = torch.empty(m, dtype=torch.int32, device=dev)
    d_tab = torch.from_numpy(batch.tables).to(dev)

    def make():
        return binding.MultiPlan(d_tab, batch.table_off, batch.query_off)

    t0 = time.perf_counter()
    plan = make()
    build_s = time.perf_counter() - t0
    ms = time_call(torch, lambda: plan.search(x, out))
    info = plan.info()
    counts = plan_counts(binding, info)
    res = {"workload": "512 tables, n uniform on 20..2000, ranges within [1e-10,1e8], "
                       f"{m} targets (query counts log-uniform on 1e4..1e7)",
           "tuned": {**roof(m, ms), **counts, "build_s": round(build_s, 2)},
           "tiles": info["tiles"], "tiles_per_wg": info["tiles_per_wg"],
           "grid": info["grid"], "lds_bytes": info["lds_bytes"],
           "traffic": measured_traffic("multi_kernel<batched>|batched-512")}
    plan.close()
    res.update(compare_plans(torch, binding, make, lambda pl: pl.search(x, out), m, counts))
    # plain search without batching: one single-table launch per table
    tabs = [d_tab[batch.table_off[t]:batch.table_off[t + 1]] for t in range(batch.num_tables)]
    qo = batch.query_off

    def per_table():
        for t in range(batch.num_tables):
            binding.search_sorted_batch(tabs[t], x[qo[t]:qo[t + 1]], out[qo[t]:qo[t + 1]])
    res["per_table_launches"] = roof(m, time_call(torch, per_table, reps=2))
    # the same tables with targets that arrive sorted (a smooth walk per
    # table): the sampled plan measures each table's wave brackets on them
    # and weighs the ballot scan
    inputs.batched_smooth_targets(batch, out=host.numpy())
    x.copy_(host)
    smooth = {}
    for name, mk, opts in (
            ("tuned", make, {}),
            ("sampled", lambda: binding.MultiPlan(d_tab, batch.table_off, batch.query_off,
                                                  sample=x), {}),
            ("ballot_forced", make, {binding.OPT_PLAN_ALGO: binding.ALGO_BALLOT})):
        t0 = time.perf_counter()
        plan = with_options(binding, opts, mk)
        build_s = time.perf_counter() - t0
        ms = time_call(torch, lambda: plan.search(x, out))
        row = {**roof(m, ms), **plan_counts(binding, plan.info()), "build_s": round(build_s, 2)}
        if name == "sampled":
            br = plan.info()["brackets"]
            row["mean_bracket"] = round(float(br[br >= 0].mean()), 2)
        plan.close()
        smooth[name] = row
    res["smooth_targets"] = {"workload": "the same 512 tables; each table's targets one smooth "
                                         "increasing walk over its range", **smooth}
    del x, out, host
    return res


SMALL_M = 10**6
SMALL_BUFFERS = 48
SMALL_CALLS = 192
SMALL_STREAMS = 4


def measure_small(torch, binding, inputs, dev) -> dict:
    """A 64-entry table with 1e6 targets per call.  (i) Latency of one call:
    host clock from the call to the end of the synchronisation, and the
    kernel alone by HIP events.  (ii) Steady throughput of back-to-back calls
    replayed from one captured HIP graph that rotates over 48 distinct target
    buffers (48 x 12 MB = 576 MB, more than twice the 256 MB last-level
    cache), so that no call finds its targets left in cache by the previous
    one.  Every call is the same single-table call; the graph's outputs are
    compared with eager calls on the same buffers."""
    table = inputs.single64_table()
    t = torch.from_numpy(table).to(dev)
    host = torch.empty(SMALL_BUFFERS * SMALL_M, dtype=torch.float64).pin_memory()
    inputs.table_targets(table, host.numel(), seed=64, out=host.numpy())
    x = host.to(dev).view(SMALL_BUFFERS, SMALL_M)
    del host
    out = torch.empty(SMALL_BUFFERS, SMALL_M, dtype=torch.int32, device=dev)
    ref = torch.empty_like(out)
    for b in range(SMALL_BUFFERS):
        binding.search_sorted_batch(t, x[b], ref[b])
    torch.cuda.synchronize()

    lat = []
    for k in range(200):
        b = k % SMALL_BUFFERS
        t0 = time.perf_counter()
        binding.search_sorted_batch(t, x[b], out[b])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(SMALL_BUFFERS)]
    for b in range(SMALL_BUFFERS):
        ev[b][0].record()
        binding.search_sorted_batch(t, x[b], out[b])
        ev[b][1].record()
        torch.cuda.synchronize()
    kern_us = [e0.elapsed_time(e1) * 1e3 for e0, e1 in ev]

    # eager back-to-back calls, for comparison with the graph
    ms_eager = time_call(torch, lambda: [binding.search_sorted_batch(t, x[b], out[b])
                                         for b in range(SMALL_BUFFERS)], reps=4) / SMALL_BUFFERS

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        binding.search_sorted_batch(t, x[0], out[0])
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        for k in range(SMALL_CALLS):
            b = k % SMALL_BUFFERS
            binding.search_sorted_batch(t, x[b], out[b])
    replays_ok = True
    for _ in range(2):
        out.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        replays_ok &= bool(torch.equal(out, ref))
    ms_graph = time_call(torch, g.replay, reps=10) / SMALL_CALLS
    del g

    # the same calls as SMALL_STREAMS independent chains of one graph (the
    # calls write distinct buffers, so the chains may overlap on the device)
    g = torch.cuda.CUDAGraph()
    chains = [torch.cuda.Stream() for _ in range(SMALL_STREAMS)]
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        main = torch.cuda.current_stream()
        for c, s in enumerate(chains):
            s.wait_stream(main)
            with torch.cuda.stream(s):
                for k in range(c, SMALL_CALLS, SMALL_STREAMS):
                    b = k % SMALL_BUFFERS
                    binding.search_sorted_batch(t, x[b], out[b])
        for s in chains:
            main.wait_stream(s)
    chains_ok = True
    for _ in range(2):
        out.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        chains_ok &= bool(torch.equal(out, ref))
    ms_chains = time_call(torch, g.replay, reps=10) / SMALL_CALLS
    del g
    return {"workload": "one 64-entry table (jittered log grid on [1e-6,1e4]), 1e6 targets "
                        "per call, 48 rotating target buffers",
            "latency_us": {"call_to_sync_median": round(float(np.median(lat)) * 1e6, 1),
                           "call_to_sync_min": round(float(np.min(lat)) * 1e6, 1),
                           "kernel_median": round(float(np.median(kern_us)), 2)},
            "eager_back_to_back": roof(SMALL_M, ms_eager),
            "graph_back_to_back": {**roof(SMALL_M, ms_graph), "calls": SMALL_CALLS,
                                   "buffers": SMALL_BUFFERS, "matches_eager": replays_ok},
            "graph_independent_chains": {**roof(SMALL_M, ms_chains), "chains": SMALL_STREAMS,
                                         "calls": SMALL_CALLS, "matches_eager": chains_ok}}


PAPER_M = 5 * 10**6
PAPER_BUFFERS = 8


def measure_paper_shape(torch, binding, inputs, dev) -> dict:
    """The paper's own measured configuration, for context: a 110-entry
    table on [3e-6, 5.4e4] (stand-in for the SESAME density axis) and 5e6
    targets log-uniform on [1e-10, 1e10], about half outside it.  Each
    kernel: 64 calls replayed from a HIP graph, rotating over 8 target
    buffers (320 MB, more than the 256 MB last-level cache)."""
    table = inputs.paper_shape_table()
    t = torch.from_numpy(table).to(dev)
    host = torch.empty(PAPER_BUFFERS * PAPER_M, dtype=torch.float64).pin_memory()
    inputs.paper_shape_targets(host.numel(), out=host.numpy())
    x = host.to(dev).view(PAPER_BUFFERS, PAPER_M)
    del host
    out = torch.empty(PAPER_BUFFERS, PAPER_M, dtype=torch.int32, device=dev)
    res = {"workload": "one 110-entry table on [3e-6, 5.4e4], 5e6 targets log-uniform on "
                       "[1e-10, 1e10] per call (about half outside the table), 8 rotating "
                       "target buffers, 64 graph-replayed calls"}
    for algo in ("auto", "binary", "ballot", "exphash", "loghash", "skiplist"):
        def call(b):
            binding.search_with(t, x[b], algo, -1, out[b])
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            call(0)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, capture_error_mode="relaxed"):
            for k in range(64):
                call(k % PAPER_BUFFERS)
        res[algo] = roof(PAPER_M, time_call(torch, g.replay, reps=5) / 64)
        del g
    # the automatic choice's calls as SMALL_STREAMS independent chains (chain
    # c takes calls k = c mod SMALL_STREAMS, whose buffers no other chain
    # writes), so that the device may overlap them
    g = torch.cuda.CUDAGraph()
    chains = [torch.cuda.Stream() for _ in range(SMALL_STREAMS)]
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        main = torch.cuda.current_stream()
        for c, s in enumerate(chains):
            s.wait_stream(main)
            with torch.cuda.stream(s):
                for k in range(c, 64, SMALL_STREAMS):
                    binding.search_sorted_batch(t, x[k % PAPER_BUFFERS], out[k % PAPER_BUFFERS])
        for s in chains:
            main.wait_stream(s)
    ref = torch.empty_like(out)
    for b in range(PAPER_BUFFERS):
        binding.search_sorted_batch(t, x[b], ref[b])
    out.fill_(-7)
    g.replay()
    torch.cuda.synchronize()
    res["auto_independent_chains"] = {**roof(PAPER_M, time_call(torch, g.replay, reps=5) / 64),
                                      "chains": SMALL_STREAMS,
                                      "matches_eager": bool(torch.equal(out, ref))}
    del ref
    del g
    del x, out
    return res


def measure_small_m(torch, binding, inputs, dev) -> dict:
    """Per-call time in the small-m regime (m = 1e2..1e4 targets per call),
    where the per-workgroup setup decides: 64 calls replayed from a HIP
    graph, for the automatic choice and for each kernel forced, on a
    110-entry and a 4000-entry table."""
    res = {}
    for n, table in ((110, inputs.paper_shape_table()), (4000, inputs.single_table(4000))):
        t = torch.from_numpy(table).to(dev)
        for m in (100, 1000, 10000):
            x = torch.from_numpy(inputs.table_targets(table, m, seed=m)).to(dev)
            out = torch.empty(m, dtype=torch.int32, device=dev)
            row = {}
            for algo in ("auto", "binary", "exphash", "loghash"):
                def call():
                    binding.search_with(t, x, algo, -1, out)
                side = torch.cuda.Stream()
                side.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(side):
                    call()
                torch.cuda.current_stream().wait_stream(side)
                torch.cuda.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, capture_error_mode="relaxed"):
                    for _ in range(64):
                        call()
                row[algo] = round(time_call(torch, g.replay, reps=5) / 64 * 1e3, 2)
                del g
            res[f"n={n}/m={m}"] = row
    return {"unit": "us per call (graph-replayed)", **res}


def measure_interp(torch, binding, inputs, dev) -> dict:
    """1024 materials with SESAME-sized axes (50..150 x 20..100 points) and
    value grids; 1e9 (rho, T) pairs searched and interpolated in one launch.
    Algorithmic bytes: 24 per pair (two float64 targets in, one float64
    value out); with the two int32 indices also written, 32."""
    it = inputs.interp_layout()
    p = it.pairs
    m = p.num_pairs
    hr = torch.empty(m, dtype=torch.float64).pin_memory()
    ht = torch.empty(m, dtype=torch.float64).pin_memory()
    inputs.paired_targets(p, out_rho=hr.numpy(), out_t=ht.numpy())
    r, t = hr.to(dev), ht.to(dev)
    del hr, ht
    f = torch.empty(m, dtype=torch.float64, device=dev)
    plan = binding.InterpPlan(torch.from_numpy(p.rho.tables).to(dev), p.rho.table_off,
                              torch.from_numpy(p.temp.tables).to(dev), p.temp.table_off,
                              p.rho.query_off, torch.from_numpy(it.values).to(dev))
    ms = time_call(torch, lambda: plan.interpolate(r, t, f), reps=3)
    gbs = 24 * m / (ms * 1e-3) / 1e9
    o_r = torch.empty(m, dtype=torch.int32, device=dev)
    o_t = torch.empty(m, dtype=torch.int32, device=dev)
    ms_i = time_call(torch, lambda: plan.interpolate(r, t, f, o_r, o_t), reps=3)
    gbs_i = 32 * m / (ms_i * 1e-3) / 1e9
    info = plan.info()
    plan.close()
    del r, t, f, o_r, o_t
    return {"workload": f"1024 materials (axes 50..150 x 20..100), {m} pairs, bilinear "
                        "interpolation of each material's value grid",
            "gpairs_per_s": round(m / (ms * 1e-3) / 1e9, 2), "ms": round(ms, 4),
            "bytes_per_pair": 24, "achieved_gbs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "with_indices": {"gpairs_per_s": round(m / (ms_i * 1e-3) / 1e9, 2),
                             "ms": round(ms_i, 4), "bytes_per_pair": 32,
                             "achieved_gbs": round(gbs_i, 1),
                             "frac": round(gbs_i / HBM_PEAK_GBS, 4)},
            "value_grid_mb": round(it.values.nbytes / 1e6, 1),
            "tiles_per_wg": info["tiles_per_wg"], "lds_bytes": info["lds_bytes"],
            "block": info["block"],
            "traffic": measured_traffic("multi_kernel<interp>|interp-1024"),
            "traffic_with_indices": measured_traffic("multi_kernel<interp-indices>|interp-1024")}


def measure_learned(torch, binding, inputs, dev) -> dict:
    """One 2000-entry table, 1e8 log-uniform targets: the learned index
    (trained on the device) against the plain search on the same data.  The
    search evaluates the model in its compiled piecewise-linear form: one
    fused multiply-add per query, after the lookup of the piece holding the
    input; the window search that follows is LDS reads and compares."""
    table = inputs.learned_table()
    t = torch.from_numpy(table).to(dev)
    host = torch.empty(M, dtype=torch.float64).pin_memory()
    inputs.table_targets(table, M, seed=2000, out=host.numpy())
    x = host.to(dev)
    out = torch.empty(M, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    li = binding.LearnedIndex(t, steps=3000, lr=0.01, seed=1)
    build_s = time.perf_counter() - t0
    ms_l = time_call(torch, lambda: li.search(x, out), reps=3)
    fallbacks = li.fallbacks()
    ms_p = time_call(torch, lambda: binding.search_sorted_batch(t, x, out), reps=5)
    info = li.info()
    res = {"workload": "one 2000-entry table (log-uniform on [1e-8,1e6]), 1e8 targets",
           "learned": {**roof(M, ms_l), "E": info["E"], "fallbacks": fallbacks,
                       "train_loss": info["loss"], "build_s": round(build_s, 3),
                       "pieces": info.get("pieces"), "cells": info.get("cells"),
                       "executed_model_flops_per_query": 2},
           "plain": roof(M, ms_p)}
    li.close()
    del x, out, host
    return res


ONLY = {
    "single_tables": lambda torch, b, i, d: measure_single_tables(torch, b, i, d, True),
    "small": measure_small,
    "small_m": measure_small_m,
    "paper_shape": measure_paper_shape,
    "batched": measure_batched,
    "interp": measure_interp,
    "learned": measure_learned,
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-kernels", action="store_true",
                    help="skip the single-table per-kernel comparison")
    ap.add_argument("--no-systems", action="store_true",
                    help="skip the comparisons and every workload after the headline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of known size (HBM counter calibration)")
    ap.add_argument("--no-calibrate", action="store_true",
                    help="plan with the tuner's built-in coefficients instead of calibrating "
                         "them on this device first")
    ap.add_argument("--only", choices=sorted(ONLY),
                    help="run one of the other workloads alone and print its record (for "
                         "profiling); no headline")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}, "
              f"WORLD_SIZE={world}); the search shards by target ranges with no exchange "
              "step, so per-GPU throughput is the single-GPU figure.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2112_03229_amd import binding, inputs

    if args.copy_calibration:
        copy_calibration(torch)
        return

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    binding.lib()

    if args.only:
        log(f"bench: {args.only} alone")
        rec = ONLY[args.only](torch, binding, inputs, dev)
        print(json.dumps({"only": args.only, **rec}), flush=True)
        return

    tuner = {"calibrated": False, "model": binding.tuner_get()}
    if not args.no_calibrate:
        # the autotuner's cost model measured on this device before any plan
        log("bench: tuner calibration")
        t0 = time.perf_counter()
        tuner = {"calibrated": True, "model": binding.tuner_calibrate(),
                 "seconds": round(time.perf_counter() - t0, 2)}
    result, pairs, host_r, host_t = paired_headline(torch, binding, inputs, dev, args)
    result["tuner"] = tuner
    torch.cuda.empty_cache()

    if not args.no_systems:
        log("bench: single tables (n = 100, 300, 1000; 1e8 targets)")
        result["single_tables"] = measure_single_tables(torch, binding, inputs, dev,
                                                        args.no_kernels)
        torch.cuda.empty_cache()
        log("bench: small table, graph-replayed calls")
        result["small"] = measure_small(torch, binding, inputs, dev)
        result["small"]["small_m"] = measure_small_m(torch, binding, inputs, dev)
        torch.cuda.empty_cache()
        log("bench: the paper's configuration (n = 110, 5e6 targets)")
        result["paper_shape"] = measure_paper_shape(torch, binding, inputs, dev)
        torch.cuda.empty_cache()
        log("bench: batched plan")
        result["batched"] = measure_batched(torch, binding, inputs, dev)
        torch.cuda.empty_cache()
        log("bench: interpolation after the paired search")
        result["interp"] = measure_interp(torch, binding, inputs, dev)
        torch.cuda.empty_cache()
        log("bench: learned index")
        result["learned"] = measure_learned(torch, binding, inputs, dev)
        torch.cuda.empty_cache()

    if not args.no_cpu:
        log("bench: CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(pairs, host_r, host_t)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
