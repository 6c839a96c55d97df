"""Pins the oracle's bilinear interpolation after the paired search (no GPU).

* scipy's RegularGridInterpolator (method "linear", extrapolating) on single
  materials: inside and outside the axes;
* grid nodes return the stored value exactly;
* a bilinear function of (rho, T) is reproduced everywhere, extrapolation
  included, since bilinear interpolation is exact for it;
* NaN gives NaN.
"""
import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator


def one_material(inputs_mod, nr=40, nt=25, seed=3):
    R = inputs_mod.sorted_log_table(seed, nr, 1e-3, 1e3)
    T = inputs_mod.sorted_log_table(seed + 1, nt, 10.0, 1e5)
    F = np.cos(np.log10(R))[:, None] * np.log10(T)[None, :] + np.log10(R)[:, None]
    return R, T, F


def run(oracle_mod, R, T, F, rho, temp):
    f, scale = oracle_mod.interp_pairs(R, [0, R.size], T, [0, T.size], [0, rho.size],
                                       F.reshape(-1), rho, temp)
    return f, scale


def test_matches_scipy_inside_and_outside(oracle_mod, inputs_mod):
    R, T, F = one_material(inputs_mod)
    rho = inputs_mod.log_uniform(5, 1, 2e-4, 5e3, 20000)     # also below and above the axis
    temp = inputs_mod.log_uniform(5, 2, 2.0, 5e5, 20000)
    f, scale = run(oracle_mod, R, T, F, rho, temp)
    ref = RegularGridInterpolator((R, T), F, method="linear", bounds_error=False,
                                  fill_value=None)(np.stack([rho, temp], axis=1))
    assert np.all(np.abs(f - ref) <= 1e-12 * np.maximum(scale, 1.0))


def test_nodes_are_exact(oracle_mod, inputs_mod):
    R, T, F = one_material(inputs_mod)
    a, b = np.meshgrid(np.arange(R.size), np.arange(T.size), indexing="ij")
    f, _ = run(oracle_mod, R, T, F, R[a.ravel()], T[b.ravel()])
    assert np.array_equal(f, F.reshape(-1))


def test_bilinear_functions_are_reproduced(oracle_mod, inputs_mod):
    R, T, _ = one_material(inputs_mod, seed=9)
    c = (0.3, -1.5, 2e-4, 7e-3)
    F = c[0] + c[1] * R[:, None] + c[2] * T[None, :] + c[3] * R[:, None] * T[None, :]
    rho = inputs_mod.log_uniform(6, 1, 1e-4, 1e4, 5000)
    temp = inputs_mod.log_uniform(6, 2, 1.0, 1e6, 5000)
    f, scale = run(oracle_mod, R, T, F, rho, temp)
    exact = c[0] + c[1] * rho + c[2] * temp + c[3] * rho * temp
    assert np.all(np.abs(f - exact) <= 1e-11 * np.maximum(scale, 1.0))


def test_nan_and_segments(oracle_mod, inputs_mod):
    it = inputs_mod.interp_layout(seed=7, materials=6, total_pairs=3000)
    p = it.pairs
    rho, temp = inputs_mod.paired_targets(p, seed=7)
    rho[5] = np.nan
    temp[9] = np.nan
    f, _ = oracle_mod.interp_pairs(p.rho.tables, p.rho.table_off, p.temp.tables,
                                   p.temp.table_off, p.rho.query_off, it.values, rho, temp)
    assert np.isnan(f[5]) and np.isnan(f[9])
    assert np.isfinite(np.delete(f, [5, 9])).all()
    # each material's slice equals that material interpolated alone
    for j in range(6):
        q0, q1 = p.rho.query_off[j], p.rho.query_off[j + 1]
        R, T = p.rho.table(j), p.temp.table(j)
        F = it.values[it.value_off[j]:it.value_off[j + 1]].reshape(R.size, T.size)
        g, _ = run(oracle_mod, R, T, F, rho[q0:q1], temp[q0:q1])
        assert np.array_equal(g, f[q0:q1], equal_nan=True)
