"""GPU tests of the learned index.

* Indices: bit-exact against the oracle's definition, for trained models,
  for deliberately useless models (zero, huge and NaN weights force the
  fallback), and at the full 1e8-target size (bracket check on every index
  plus an oracle sample).
* Model arithmetic: the device forward pass against the float64 oracle
  forward on the same weights; the training kernel's gradient against the
  oracle's back-propagation.
* Error bound: every table entry's prediction lies within E - 1 of its index.
"""
import numpy as np
import pytest
import torch

from oracle import learned as OL

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def binding(gpu):
    from paper_2112_03229_amd import binding as b
    return b


@pytest.fixture(scope="module")
def trained(binding, gpu, inputs_mod):
    table = inputs_mod.learned_table()
    t = torch.from_numpy(table).to(gpu)
    say("case build n=2000 steps=3000")
    li = binding.LearnedIndex(t, steps=3000, lr=0.01, seed=1)
    return table, t, li


def targets_for(inputs_mod, table, m, seed):
    x = inputs_mod.table_targets(table, m, seed=seed)
    n = table.shape[0]
    k = np.arange(0, m, 9)
    x[k] = table[k % n]
    k = np.arange(4, m, 13)
    x[k] = np.nextafter(table[k % n], np.inf)
    sp = inputs_mod.special_values()
    x[1:1 + sp.size] = sp
    return x


def test_trained_model_is_exact(binding, gpu, oracle_mod, inputs_mod, trained):
    table, t, li = trained
    info = li.info()
    say(f"learned: {info}")
    assert info["n"] == 2000 and info["E"] >= 1 and info["loss"] < 1e-3
    assert info["cells"] > 0  # a trained model's pieces are found through cells
    x = targets_for(inputs_mod, table, 300001, seed=3)
    want = oracle_mod.search_lt(table, x)
    got = li.search(torch.from_numpy(x).to(gpu)).cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]], x[bad[:5]])
    fb = li.fallbacks()
    say(f"fallbacks {fb} of {x.size}")
    # only the special values (NaN, non-positive, outside FP32) should miss
    assert fb <= 64


def test_error_bound_covers_every_entry(binding, gpu, oracle_mod, trained):
    table, t, li = trained
    E = li.info()["E"]
    pos = li.predict(t).cpu().numpy().astype(np.float64)
    g = np.clip(np.floor(pos), -1, table.size - 1)
    idx = oracle_mod.search_lt(table, table)
    assert np.max(np.abs(g - idx)) <= E - 1


def test_forward_matches_oracle(binding, gpu, inputs_mod, trained):
    table, t, li = trained
    w = li.weights().astype(np.float64)
    x = inputs_mod.table_targets(table, 20000, seed=5)
    pos = li.predict(torch.from_numpy(x).to(gpu)).cpu().numpy().astype(np.float64)
    want = OL.forward(w, OL.model_input(x, table)) * (table.size - 1)
    # FP32 compiled forward (FP32 log2 of x rounded to FP32) vs the float64
    # layered forward: agreement to a small fraction of one table position
    err = np.abs(pos - want)
    say(f"forward max abs err (positions): {err.max():.3e}")
    assert err.max() < 0.05


def compiled_vs_layered(li, gpu, table, w, extra_z):
    """Largest |compiled - layered| / tolerance over inputs spread on
    [-0.2, 1.2] plus extra_z (model inputs; |z| < 2 keeps x inside the FP32
    range the model input is formed in): the compiled FP32 output against
    the float64 layered forward pass, to FP32 rounding of the terms'
    magnitudes and of the input."""
    wd = w.astype(np.float64)
    w1, b1 = wd[0:32], wd[32:64]
    W2 = wd[64:64 + 1024].reshape(32, 32)
    b2, w3, b3 = wd[1088:1120], wd[1120:1152], wd[1152]
    extra_z = np.asarray(extra_z, dtype=np.float64)
    z = np.concatenate([np.linspace(-0.2, 1.2, 20001), extra_z[np.abs(extra_z) < 2]])
    u0, u1 = np.log2(table[0]), np.log2(table[-1])
    x = np.exp2(u0 + z * (u1 - u0))
    p = li.predict(torch.from_numpy(x).to(gpu)).cpu().numpy().astype(np.float64)
    p /= table.size - 1
    zr = OL.model_input(x, table)
    want = OL.forward(wd, zr)
    mag = np.abs(w3) @ (np.abs(W2) @ (np.outer(np.abs(w1), np.abs(zr)) + np.abs(b1)[:, None])
                        + np.abs(b2)[:, None]) + abs(b3)
    slope = np.abs(w3) @ (np.abs(W2) @ np.abs(w1))
    tol = 4e-6 * mag + 4e-6 * slope * np.maximum(1.0, np.abs(zr))
    return np.abs(p - want) / tol


@pytest.mark.parametrize("crowded", [False, True], ids=["cells", "bisection"])
def test_compiled_model_matches_layered_oracle(binding, gpu, inputs_mod, crowded):
    """The search evaluates a compiled form of the model: its pieces as a
    continuous piecewise-linear function of z (bounded by layer 1's
    breakpoints and by the sign changes of layer 2's pre-activations), each
    one (slope, intercept).  On weights built to stress it -- units with
    w1 = 0 (always on, always off), three units sharing one breakpoint (one
    with a negative slope), a breakpoint near 1e30, breakpoints inside and
    outside [0, 1] -- and inputs on both sides of every breakpoint, its
    output must equal the float64 layered forward pass to FP32 rounding of
    the terms' magnitudes.  The piece is found through the cell table; with
    twelve more units sharing one breakpoint (crowded) no cell table can
    hold them within the scan length, and it is found by bisection."""
    table = inputs_mod.learned_table()
    t = torch.from_numpy(table).to(gpu)
    rng = np.random.default_rng(7)
    w1 = rng.normal(0, 3, 32)
    b1 = rng.normal(0, 1, 32)
    w1[0:3], b1[0:3] = 0.0, [0.5, -0.5, 0.0]
    w1[3:6], b1[3:6] = [2.0, 4.0, -2.0], [-1.0, -2.0, 1.0]
    w1[6], b1[6] = 1e-30, 1.0
    if crowded:
        w1[7:19] = 1.0 + 0.25 * np.arange(12)
        b1[7:19] = -0.375 * w1[7:19]  # breakpoint exactly 0.375 for all twelve
    W2 = rng.normal(0, 0.3, (32, 32))
    b2 = rng.normal(0, 0.1, 32)
    w3 = rng.normal(0, 0.3, 32)
    b3 = 0.1
    w = np.concatenate([w1, b1, W2.reshape(-1), b2, w3, [b3]]).astype(np.float32)
    li = binding.LearnedIndex(t, weights=w)
    wd = w.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        bp = -wd[32:64] / wd[0:32]
    bp = bp[np.isfinite(bp)]
    r = compiled_vs_layered(li, gpu, table, w, np.concatenate([bp - 1e-6, bp + 1e-6, bp]))
    info = li.info()
    say(f"compiled vs layered: worst err / tol {r.max():.2e}, pieces {info['pieces']}, "
        f"cells {info['cells']}")
    assert np.all(r <= 1.0), (np.argmax(r), r.max())
    # the breakpoint near -1e30 is trimmed from the cells' range; twelve
    # equal boundaries always share a cell
    assert (info["cells"] == 0) == crowded


def test_compiled_model_with_the_most_pieces(binding, gpu, oracle_mod, inputs_mod):
    """A model with as many pieces as the compiled form holds.  Layer 1's
    breakpoints are j / 32 (w1 = 1, b1 = -j / 32).  Every layer-2 unit's
    pre-activation is a zigzag between -1 + d_k and 1 + d_k (slope +-64 on
    alternate segments, |d_k| < 0.4 distinct), so it changes sign once in
    each of the 32 segments right of z = 0 and never left of it.  That gives
    32 + 32 * 32 = 1056 piece boundaries: 1057 pieces and 2048 boundary
    slots, the largest padding.  The compiled output must match the layered
    forward pass on both sides of every boundary, and the search, whose
    model is useless for this table, must still return exact indices."""
    table = inputs_mod.learned_table()
    t = torch.from_numpy(table).to(gpu)
    j = np.arange(32)
    w1 = np.ones(32)
    b1 = -j / 32.0
    row = np.where(j == 0, 64.0, 128.0 * (-1.0) ** j)
    W2 = np.tile(row, (32, 1))
    d = (j - 15.5) / 40.0
    b2 = -1.0 + d
    w3 = np.random.default_rng(11).normal(0, 0.3, 32)
    w = np.concatenate([w1, b1, W2.reshape(-1), b2, w3, [0.05]]).astype(np.float32)
    li = binding.LearnedIndex(t, weights=w)
    info = li.info()
    say(f"most pieces: {info}")
    assert info["pieces"] == 1057 and info["bound_slots"] == 2048
    # 1056 boundaries over [0, 1.03): 2048 cells, a few boundaries each
    assert info["cells"] == 2048 and 1 <= info["cell_scan"] <= 8
    # probes around every boundary, located from the layered weights: layer
    # 1's breakpoints and, in each segment s (units 0..s-1 active), where
    # unit k's line P z + Q crosses zero
    wd = w.astype(np.float64)
    w1d, b1d = wd[0:32], wd[32:64]
    W2d, b2d = wd[64:1088].reshape(32, 32), wd[1088:1120]
    probes = [-b1d / w1d]
    for s_ in range(1, 33):
        P = W2d[:, :s_] @ w1d[:s_]
        Q = b2d + W2d[:, :s_] @ b1d[:s_]
        probes.append(-Q / P)
    bz = np.concatenate(probes)
    r = compiled_vs_layered(li, gpu, table, w, np.concatenate([bz - 2e-6, bz + 2e-6, bz]))
    say(f"most pieces: worst err / tol {r.max():.2e}")
    assert np.all(r <= 1.0), (np.argmax(r), r.max())
    x = targets_for(inputs_mod, table, 100003, seed=17)
    want = oracle_mod.search_lt(table, x)
    got = li.search(torch.from_numpy(x).to(gpu)).cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]])


@pytest.mark.parametrize("which", ["init", "trained"])
def test_training_gradient_matches_oracle(binding, gpu, inputs_mod, trained, which):
    table, t, li = trained
    if which == "init":
        w = binding.LearnedIndex(t, steps=0, seed=7).weights()
    else:
        w = li.weights()
    loss_dev, g_dev = binding.mlp_gradient(t, w)
    w64 = w.astype(np.float64)
    loss_ref, g_ref = OL.loss_and_grad(w64, table)
    say(f"{which}: loss dev {loss_dev:.6e} ref {loss_ref:.6e}")
    assert abs(loss_dev - loss_ref) <= 1e-4 * loss_ref + 1e-9
    # tolerance from the arithmetic: FP32 forward and backward (about 1e3
    # dependent operations per point, eps 6e-8) plus the FP32 log2 of the
    # input, relative to the cancellation-free size of each gradient term
    scale = OL.grad_scale(w64, table)
    err = np.abs(g_dev - g_ref)
    say(f"{which}: worst err/scale {np.max(err / np.maximum(scale, 1e-30)):.3e}")
    assert np.all(err <= 1e-3 * scale + 1e-12), int(np.argmax(err - 1e-3 * scale))


def test_training_is_deterministic(binding, gpu, inputs_mod):
    table = inputs_mod.single_table(300)
    t = torch.from_numpy(table).to(gpu)
    a = binding.LearnedIndex(t, steps=200, seed=3).weights()
    b = binding.LearnedIndex(t, steps=200, seed=3).weights()
    c = binding.LearnedIndex(t, steps=200, seed=4).weights()
    assert np.array_equal(a, b) and not np.array_equal(a, c)


@pytest.mark.parametrize("kind", ["zero", "huge", "nan", "untrained"])
def test_useless_models_stay_exact(binding, gpu, oracle_mod, inputs_mod, kind):
    table = inputs_mod.learned_table()
    t = torch.from_numpy(table).to(gpu)
    if kind == "untrained":
        li = binding.LearnedIndex(t, steps=0, seed=2)
    else:
        w = np.zeros(binding.MLP_PARAMS, dtype=np.float32)
        if kind == "huge":
            w[:] = np.random.default_rng(0).normal(0, 1e6, w.size).astype(np.float32)
        if kind == "nan":
            w[::7] = np.nan
        li = binding.LearnedIndex(t, weights=w)
    x = targets_for(inputs_mod, table, 100003, seed=11)
    want = oracle_mod.search_lt(table, x)
    got = li.search(torch.from_numpy(x).to(gpu)).cpu().numpy()
    assert np.array_equal(got, want), kind
    say(f"{kind}: E={li.info()['E']} fallbacks={li.fallbacks()}")


def test_small_tables_and_ragged_sizes(binding, gpu, oracle_mod, inputs_mod):
    for n in (2, 3, 17, 100, 1000):
        table = inputs_mod.single_table(n) if n > 2 else np.array([1e-3, 5.0])
        t = torch.from_numpy(table).to(gpu)
        li = binding.LearnedIndex(t, steps=300, seed=n)
        for m in (1, 511, 512, 513, 4099):
            x = targets_for(inputs_mod, table, max(m, 32), seed=m)[:m]
            want = oracle_mod.search_lt(table, x)
            assert np.array_equal(li.search(torch.from_numpy(x).to(gpu)).cpu().numpy(), want)


@pytest.mark.parametrize("n", [8200, 65535])
def test_tables_too_large_to_stage(binding, gpu, oracle_mod, inputs_mod, n):
    """Tables whose staged copy and model exceed the 64 KB staging limit are
    read in place from global memory: exact in both conventions, with a
    trained model (n = 8200) and with one that is useless for the table (the
    largest n, from given weights, so every window is wide or fails)."""
    rng = np.random.default_rng(n)
    table = np.sort(np.exp(rng.uniform(np.log(1e-8), np.log(1e6), n)))
    table[0], table[-1] = 1e-8, 1e6
    t = torch.from_numpy(table).to(gpu)
    say(f"case learned global table n={n}")
    if n <= 10000:
        li = binding.LearnedIndex(t, steps=300, seed=3)
    else:
        w = np.random.default_rng(5).normal(0, 0.5, 1153).astype(np.float32)
        li = binding.LearnedIndex(t, weights=w)
    x = targets_for(inputs_mod, table, 200003, seed=n)
    xd = torch.from_numpy(x).to(gpu)
    got = li.search(xd).cpu().numpy()
    want = oracle_mod.search_lt(table, x)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]])
    say(f"E {li.info()['E']} fallbacks {li.fallbacks()}")
    binding.set_option(binding.OPT_CONVENTION, 1)
    try:
        got = li.search(xd).cpu().numpy()
    finally:
        binding.set_option(binding.OPT_CONVENTION, 0)
    want = oracle_mod.search_le_clamped(table, x)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (bad[:5], got[bad[:5]], want[bad[:5]])


def test_rejects_bad_tables(binding, gpu):
    neg = torch.tensor([-1.0, 2.0, 3.0], dtype=torch.float64, device=gpu)
    with pytest.raises(binding.SearchSortedError):
        binding.LearnedIndex(neg, steps=1)
    one = torch.tensor([1.0], dtype=torch.float64, device=gpu)
    with pytest.raises(binding.SearchSortedError):
        binding.LearnedIndex(one, steps=1)


def test_full_size_learned(binding, gpu, oracle_mod, inputs_mod, trained):
    """n = 2000, 1e8 log-uniform targets: every index bracket-checked, a
    seeded sample compared with the definition."""
    table, t, li = trained
    m = 10**8
    host = torch.empty(m, dtype=torch.float64).pin_memory()
    x = inputs_mod.table_targets(table, m, seed=2000, out=host.numpy())
    say("case full learned n=2000 m=1e8")
    got = li.search(host.to(gpu)).cpu().numpy()
    bad, first = oracle_mod.check_bracket(table, x, got)
    assert bad == 0, first
    pos = (inputs_mod.uniform(2000, 96, 200000) * m).astype(np.int64)
    assert np.array_equal(got[pos], oracle_mod.search_lt_at(table, x, pos))
    say(f"fallbacks {li.fallbacks()} of {m}")


def test_save_and_load(binding, gpu, oracle_mod, inputs_mod, trained, tmp_path):
    """A saved model reads back bit-exactly; loaded onto its own table it
    searches exactly with the same bound, and loaded onto another table of
    the same size E is measured again and the search is still exact."""
    table, t, li = trained
    path = str(tmp_path / "model.json")
    li.save(path)
    back = binding.LearnedIndex.load(t, path)
    assert np.array_equal(back.weights().view(np.uint32), li.weights().view(np.uint32))
    info, info2 = li.info(), back.info()
    assert info2["E"] == info["E"] and info2["steps"] == info["steps"]
    x = targets_for(inputs_mod, table, 50001, seed=21)
    want = oracle_mod.search_lt(table, x)
    assert np.array_equal(back.search(torch.from_numpy(x).to(gpu)).cpu().numpy(), want)
    other = inputs_mod.single_table(2000, seed=77)
    on_other = binding.LearnedIndex.load(torch.from_numpy(other).to(gpu), path)
    xo = targets_for(inputs_mod, other, 50001, seed=22)
    got = on_other.search(torch.from_numpy(xo).to(gpu)).cpu().numpy()
    assert np.array_equal(got, oracle_mod.search_lt(other, xo))
    say(f"E on its table {info['E']}, on another table {on_other.info()['E']}")
    with pytest.raises(binding.SearchSortedError):
        binding.LearnedIndex.load(torch.from_numpy(table[:1000].copy()).to(gpu), path)
    bad = tmp_path / "bad.json"
    bad.write_text('{"format": "searchsorted-learned-1", "n": 2000, "weights": [1, 2]}')
    with pytest.raises(binding.SearchSortedError):
        binding.LearnedIndex.load(t, str(bad))


def plan_tiles(query_off, per_tile):
    """Tiles of a batched plan: each segment's aligned blocks of per_tile."""
    q0, q1 = np.asarray(query_off[:-1]), np.asarray(query_off[1:])
    return int(np.where(q1 > q0, (q1 - 1) // per_tile - q0 // per_tile + 1, 0).sum())


def test_plan_targets_per_lane_follow_learned_share(binding, gpu, oracle_mod, inputs_mod):
    """A batched plan whose learned tables carry at least 15% of the targets
    searches 4 targets per lane (tiles of 2048 targets at 512 threads), one
    with fewer learned targets keeps 8 (tiles of 4096), like a plain plan;
    the indices are exact either way."""
    batch = inputs_mod.batched_layout(seed=37, num_tables=6, query_scale=0.1)
    tt = torch.from_numpy(batch.tables).to(gpu)
    off, qoff = batch.table_off, np.asarray(batch.query_off)
    x = np.empty(batch.num_queries)
    inputs_mod.batched_targets(batch, out=x)
    want = oracle_mod.search_lt_segments(batch.tables, off, x, qoff)
    xd = torch.from_numpy(x).to(gpu)
    counts = np.diff(qoff)
    small = int(np.argmin(counts))
    assert counts[small] / counts.sum() < 0.15 and plan_tiles(qoff, 2048) > plan_tiles(qoff, 4096)
    plain = binding.MultiPlan(tt, off, qoff)
    info = plain.info()
    assert info["targets_per_lane"] == 8 and info["learned_form"] == 0
    assert info["tiles"] == plan_tiles(qoff, 4096)
    plain.close()
    for learned in ([small], list(range(6))):
        share = counts[learned].sum() / counts.sum()
        say(f"case learned tables {learned} share {share:.3f}")
        models = [None] * 6
        for t in learned:
            models[t] = binding.LearnedIndex(tt[off[t]:off[t + 1]], steps=300, seed=t)
        plan = binding.MultiPlan(tt, off, qoff, models=models)
        for m in models:
            if m is not None:
                m.close()
        q = 4 if share >= 0.15 else 8
        info = plan.info()
        assert info["targets_per_lane"] == q and info["learned_form"] in (1, 2)
        assert info["tiles"] == plan_tiles(qoff, 512 * q)
        assert np.array_equal(plan.search(xd).cpu().numpy(), want)
        plan.close()


def test_learned_plan_ragged_segments(binding, gpu, oracle_mod, inputs_mod):
    """Every table learned, so 4 targets per lane (tiles of 2048), with
    segments of 0, 1, 7, 2047, 2049 and 4097 targets starting at unaligned
    positions: the short first and last tiles of each segment, the empty
    one and the single-target one are exact, in both conventions."""
    counts = [1, 7, 0, 2047, 2049, 4097]
    batch = inputs_mod.batched_layout(seed=41, num_tables=6, query_scale=1e-3)
    tt = torch.from_numpy(batch.tables).to(gpu)
    off = batch.table_off
    qoff = np.zeros(7, dtype=np.int64)
    qoff[1:] = np.cumsum(counts)
    x = np.empty(int(qoff[-1]))
    for j in range(6):
        tab = batch.tables[off[j]:off[j + 1]]
        if counts[j]:
            x[qoff[j]:qoff[j + 1]] = inputs_mod.table_targets(tab, counts[j], seed=j)
    x[3] = np.nan
    xd = torch.from_numpy(x).to(gpu)
    models = [binding.LearnedIndex(tt[off[j]:off[j + 1]], steps=200, seed=j) for j in range(6)]
    try:
        for conv in (0, 1):
            binding.set_option(binding.OPT_CONVENTION, conv)
            say(f"case ragged learned plan convention={conv}")
            plan = binding.MultiPlan(tt, off, qoff, models=models)
            info = plan.info()
            assert info["targets_per_lane"] == 4 and info["learned_form"] in (1, 2)
            if conv:
                want = np.empty(x.size, dtype=np.int32)
                for j in range(6):
                    if counts[j]:
                        want[qoff[j]:qoff[j + 1]] = oracle_mod.search_le_clamped(
                            batch.tables[off[j]:off[j + 1]], x[qoff[j]:qoff[j + 1]])
            else:
                want = oracle_mod.search_lt_segments(batch.tables, off, x, qoff)
            assert np.array_equal(plan.search(xd).cpu().numpy(), want)
            plan.close()
    finally:
        binding.set_option(binding.OPT_CONVENTION, 0)
        for m in models:
            m.close()


def test_plan_with_attached_models(binding, gpu, oracle_mod, inputs_mod):
    """Learned handles built on tables of a batch are attached to a batched
    plan (ss_multi_plan_create_learned): those tables are searched through
    the copied models (the plan reports them learned) and every index is
    exact; the plan keeps working after the handles are destroyed; a handle
    built on a copy of a table, not on the table's own memory, is refused."""
    batch = inputs_mod.batched_layout(seed=31, num_tables=6, query_scale=1e-3)
    tt = torch.from_numpy(batch.tables).to(gpu)
    off = batch.table_off
    say("case attached models T=6")
    models = [None] * 6
    for t in (0, 2, 5):
        models[t] = binding.LearnedIndex(tt[off[t]:off[t + 1]], steps=300, seed=t)
    assert all(models[t].error_bound() >= 1 for t in (0, 2, 5))
    plan = binding.MultiPlan(tt, off, batch.query_off, models=models)
    algos = plan.info()["algos"]
    assert [int(a) == binding.ALGO_LEARNED for a in algos] == [True, False, True, False, False,
                                                                True]
    x = np.empty(batch.num_queries)
    inputs_mod.batched_targets(batch, out=x)
    want = oracle_mod.search_lt_segments(batch.tables, off, x, batch.query_off)
    xd = torch.from_numpy(x).to(gpu)
    assert np.array_equal(plan.search(xd).cpu().numpy(), want)
    for t in (0, 2, 5):
        models[t].close()
    assert np.array_equal(plan.search(xd).cpu().numpy(), want)
    plan.close()
    copy = binding.LearnedIndex(tt[off[1]:off[2]].clone(), steps=50, seed=1)
    with pytest.raises(binding.SearchSortedError):
        binding.MultiPlan(tt, off, batch.query_off, models=[None, copy, None, None, None, None])
    copy.close()


def test_error_bound_forced_below_measured(binding, gpu, oracle_mod, inputs_mod, trained):
    """E forced to 0 (and to 1): the verification rejects every window that
    misses, the fallback answers those targets, and every index stays exact;
    a wide bound verifies every window.  A plan built with a reduced bound
    counts its fallbacks the same way."""
    table, t, li = trained
    E0 = li.error_bound()
    x = targets_for(inputs_mod, table, 200003, seed=17)
    want = oracle_mod.search_lt(table, x)
    xd = torch.from_numpy(x).to(gpu)
    try:
        seen = {}
        for E in (0, 1, E0, 4 * E0 + 100):
            say(f"case learned E forced to {E} (measured {E0})")
            li.set_error_bound(E)
            assert li.error_bound() == E
            got = li.search(xd).cpu().numpy()
            assert np.array_equal(got, want), E
            seen[E] = li.fallbacks()
        say(f"fallbacks by E: {seen}")
        # NaN targets fail every window check whatever E, and so does -inf
        # in the staged search (its window's lower check meets the -inf
        # placed before the table); every other target verifies once E
        # reaches the measured bound
        nan = int((np.isnan(x) | (x == -np.inf)).sum())
        assert seen[E0] == nan and seen[4 * E0 + 100] == nan
        assert seen[0] >= seen[1] > seen[E0]
        # a plan attached while the bound is 0 takes it
        li.set_error_bound(0)
        plan = binding.MultiPlan(t, np.array([0, table.size]), np.array([0, x.size]),
                                 models=[li])
        assert np.array_equal(plan.search(xd).cpu().numpy(), want)
        assert plan.fallbacks() > 0
        plan.close()
        with pytest.raises(binding.SearchSortedError):
            li.set_error_bound(-1)
    finally:
        li.set_error_bound(E0)
    assert li.error_bound() == E0
