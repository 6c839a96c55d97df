"""GPU parity of the interpolation after the paired search against
``oracle.interp_pairs``.

The cell indices are integer decisions made by exact comparisons, so they
must equal the oracle's (and the optional index outputs equal
``oracle.search_lt`` per axis).  The interpolated values are float64
arithmetic in another order (and with fused multiply-adds): they must agree
within 16 units of rounding of the oracle's bound ``scale`` = sum of the
four terms' magnitudes |w_ij F_ij| (weights from the rounded u, 1-u, v and
1-v), and equal the grid exactly at grid nodes.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def binding(gpu):
    from paper_2112_03229_amd import binding as b
    return b


def make_plan(binding, gpu, it):
    p = it.pairs
    return binding.InterpPlan(torch.from_numpy(p.rho.tables).to(gpu), p.rho.table_off,
                              torch.from_numpy(p.temp.tables).to(gpu), p.temp.table_off,
                              p.rho.query_off, torch.from_numpy(it.values).to(gpu))


def check(oracle_mod, it, rho, temp, got):
    p = it.pairs
    want, scale = oracle_mod.interp_pairs(p.rho.tables, p.rho.table_off, p.temp.tables,
                                          p.temp.table_off, p.rho.query_off, it.values, rho, temp)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    err = np.abs(got[~nan] - want[~nan])
    tol = 16 * EPS * scale[~nan]
    worst = np.max(err / np.maximum(tol, 1e-300)) if err.size else 0.0
    say(f"worst error / tolerance {worst:.3f}")
    assert np.all(err <= tol), np.argmax(err - tol)


def test_interp_matches_oracle(binding, gpu, oracle_mod, inputs_mod):
    it = inputs_mod.interp_layout(seed=5, materials=64, total_pairs=2 * 10**6 + 7)
    p = it.pairs
    rho, temp = inputs_mod.paired_targets(p, seed=5)
    rho[:5] = [np.nan, 0.0, -1.0, np.inf, 1e300]
    temp[5:9] = [np.nan, 1e-300, -np.inf, 0.0]
    say(f"case interp M=64 pairs={p.num_pairs}")
    plan = make_plan(binding, gpu, it)
    dr, dt = torch.from_numpy(rho).to(gpu), torch.from_numpy(temp).to(gpu)
    o_r = torch.empty(p.num_pairs, dtype=torch.int32, device=gpu)
    o_t = torch.empty_like(o_r)
    f = plan.interpolate(dr, dt, out_rho=o_r, out_t=o_t).cpu().numpy()
    check(oracle_mod, it, rho, temp, f)
    want_r = oracle_mod.search_lt_segments(p.rho.tables, p.rho.table_off, rho, p.rho.query_off)
    want_t = oracle_mod.search_lt_segments(p.temp.tables, p.temp.table_off, temp,
                                           p.temp.query_off)
    assert np.array_equal(o_r.cpu().numpy(), want_r)
    assert np.array_equal(o_t.cpu().numpy(), want_t)
    # without index outputs (and a graph replay with new output buffers)
    f2 = plan.interpolate(dr, dt).cpu().numpy()
    assert np.array_equal(f2, f, equal_nan=True)


@pytest.mark.parametrize("axes,block", [(((20, 60), (10, 40)), 512),
                                        (((100, 250), (60, 120)), 1024)])
def test_interp_grid_staging_forms(binding, gpu, oracle_mod, inputs_mod, axes, block):
    """Small grids (all under 72 KB: two 512-thread workgroups per CU) and
    large ones (up to 30000 values: those over 15360 are read from L2, the
    rest staged by one 1024-thread workgroup per CU) in one plan each,
    against the oracle, with the index outputs."""
    n_rho, n_t = axes
    it = inputs_mod.interp_layout(seed=7, materials=32, total_pairs=10**6 + 3, n_rho=n_rho,
                                  n_t=n_t)
    p = it.pairs
    sizes = np.diff(it.value_off)
    if block == 1024:
        assert sizes.max() > 15360 and np.any((sizes > 9216) & (sizes <= 15360))
    else:
        assert sizes.max() <= 9216
    rho, temp = inputs_mod.paired_targets(p, seed=7)
    say(f"case interp staging block={block} largest grid {sizes.max()}")
    plan = make_plan(binding, gpu, it)
    assert plan.info()["block"] == block
    o_r = torch.empty(p.num_pairs, dtype=torch.int32, device=gpu)
    o_t = torch.empty_like(o_r)
    f = plan.interpolate(torch.from_numpy(rho).to(gpu), torch.from_numpy(temp).to(gpu),
                         out_rho=o_r, out_t=o_t).cpu().numpy()
    check(oracle_mod, it, rho, temp, f)
    assert np.array_equal(o_r.cpu().numpy(), oracle_mod.search_lt_segments(
        p.rho.tables, p.rho.table_off, rho, p.rho.query_off))
    assert np.array_equal(o_t.cpu().numpy(), oracle_mod.search_lt_segments(
        p.temp.tables, p.temp.table_off, temp, p.temp.query_off))
    plan.close()


def test_grid_nodes_are_exact(binding, gpu, inputs_mod):
    it = inputs_mod.interp_layout(seed=6, materials=8, total_pairs=8)
    p = it.pairs
    # one material at a time: every node of its grid
    for j in range(8):
        R, T = p.rho.table(j), p.temp.table(j)
        a, b = np.meshgrid(np.arange(R.size), np.arange(T.size), indexing="ij")
        from paper_2112_03229_amd.inputs import Batch, Interp, Paired
        npairs = a.size
        poff = np.array([0, npairs], dtype=np.int64)
        sub = Interp(Paired(Batch(R.copy(), np.array([0, R.size]), poff),
                            Batch(T.copy(), np.array([0, T.size]), poff.copy())),
                     it.values[it.value_off[j]:it.value_off[j + 1]].copy(),
                     np.array([0, R.size * T.size]))
        plan = make_plan(binding, gpu, sub)
        f = plan.interpolate(torch.from_numpy(R[a.ravel()]).to(gpu),
                             torch.from_numpy(T[b.ravel()]).to(gpu)).cpu().numpy()
        assert np.array_equal(f, sub.values), j


def test_interp_rejects_bad_axes(binding, gpu):
    d = lambda a: torch.tensor(a, dtype=torch.float64, device=gpu)
    vals = d(np.zeros(16))
    with pytest.raises(binding.SearchSortedError):   # a one-entry axis has no cell
        binding.InterpPlan(d([1.0]), [0, 1], d([1.0, 2.0]), [0, 2], [0, 5], vals)
    with pytest.raises(binding.SearchSortedError):   # repeated entry: zero-width cell
        binding.InterpPlan(d([1.0, 1.0, 2.0]), [0, 3], d([1.0, 2.0]), [0, 2], [0, 5], vals)
    plan = binding.InterpPlan(d([1.0, 2.0]), [0, 2], d([1.0, 2.0]), [0, 2], [0, 3], vals)
    with pytest.raises(TypeError):
        plan.search(d([1.0, 1.5, 2.0]), d([1.0, 1.5, 2.0]))


def test_full_size_interp(binding, gpu, oracle_mod, inputs_mod):
    """1024 SESAME-sized materials, 1e9 pairs in one launch; a seeded sample
    of 2e5 pairs against the oracle."""
    it = inputs_mod.interp_layout()
    p = it.pairs
    m = p.num_pairs
    say(f"case full interp M=1024 pairs={m}")
    hr = torch.empty(m, dtype=torch.float64).pin_memory()
    ht = torch.empty(m, dtype=torch.float64).pin_memory()
    rho, temp = inputs_mod.paired_targets(p, out_rho=hr.numpy(), out_t=ht.numpy())
    plan = make_plan(binding, gpu, it)
    f = plan.interpolate(hr.to(gpu, non_blocking=True), ht.to(gpu, non_blocking=True))
    got = f.cpu().numpy()
    del f
    pos = np.sort((inputs_mod.uniform(1024, 99, 200000) * m).astype(np.int64))
    seg = np.searchsorted(p.rho.query_off, pos, side="right") - 1
    counts = np.bincount(seg, minlength=p.num_materials)
    poff = np.zeros(p.num_materials + 1, dtype=np.int64)
    poff[1:] = np.cumsum(counts)
    want, scale = oracle_mod.interp_pairs(p.rho.tables, p.rho.table_off, p.temp.tables,
                                          p.temp.table_off, poff, it.values, rho[pos], temp[pos])
    err = np.abs(got[pos] - want)
    assert np.all(err <= 16 * EPS * scale)
