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


# ---------------------------------------------------------------------------
# The rounding bound `scale` (the tolerance of the GPU parity test): the sum
# of the four terms' magnitudes |w_ij F_ij|, pinned on hand-computed cells in
# exact rational arithmetic.

EPS = np.finfo(np.float64).eps


def _exact_cell(R, T, F, r, t):
    """Exact (f, scale) for one pair in rational arithmetic.  The inputs are
    chosen so that u, 1-u, v and 1-v are exact in float64."""
    from fractions import Fraction as Q
    u = (Q(r) - Q(R[0])) / (Q(R[1]) - Q(R[0]))
    v = (Q(t) - Q(T[0])) / (Q(T[1]) - Q(T[0]))
    terms = [(1 - u) * (1 - v) * Q(F[0][0]), u * (1 - v) * Q(F[1][0]),
             (1 - u) * v * Q(F[0][1]), u * v * Q(F[1][1])]
    return sum(terms), sum(abs(x) for x in terms)


@pytest.mark.parametrize("case", ["large_corner_tiny_weight", "extrapolated_cancelling"])
def test_scale_is_the_termwise_magnitude(oracle_mod, case):
    R, T = np.array([1.0, 2.0]), np.array([10.0, 20.0])
    if case == "large_corner_tiny_weight":
        # u = 1 - 2^-30 and v = 1 - 2^-20 (both exact): the 1e18 corner
        # carries the weight (1-u)(1-v) = 2^-50, so its term is about 888
        F = np.array([[1e18, 1.0], [3.0, -2.0]])
        r, t = 2.0 - 2.0**-30, 20.0 - 10.0 * 2.0**-20
    else:
        # u = -3 (outside the axis), v = 1/2: terms 10, -16.5, 14, -19.5
        F = np.array([[5.0, 7.0], [11.0, 13.0]])
        r, t = -2.0, 15.0
    f, scale = run(oracle_mod, R, T, F, np.array([r]), np.array([t]))
    want_f, want_scale = _exact_cell(R, T, F, r, t)
    assert abs(scale[0] - float(want_scale)) <= 4 * EPS * float(want_scale)
    assert abs(f[0] - float(want_f)) <= 8 * EPS * float(want_scale)
    if case == "large_corner_tiny_weight":
        # the bound follows the terms, not the corners: (1+|u|)(1+|v|) sum |F|
        # would be about 4e18 here
        assert 880.0 < scale[0] < 900.0
    else:
        assert scale[0] == 60.0 and f[0] == -12.0


def test_scale_bounds_another_evaluation_order(oracle_mod, inputs_mod):
    """Three one-dimensional interpolations with fused multiply-adds (another
    order of the same terms) stay within a few eps * scale of the oracle,
    also outside the axes where the terms cancel."""
    R, T, F = one_material(inputs_mod, nr=30, nt=20, seed=11)
    rho = inputs_mod.log_uniform(8, 1, 1e-5, 1e5, 20000)
    temp = inputs_mod.log_uniform(8, 2, 1.0, 1e6, 20000)
    f, scale = run(oracle_mod, R, T, F, rho, temp)
    i = np.clip(np.searchsorted(R, rho, side="left") - 1, 0, R.size - 2)
    k = np.clip(np.searchsorted(T, temp, side="left") - 1, 0, T.size - 2)
    u = (rho - R[i]) / (R[i + 1] - R[i])
    v = (temp - T[k]) / (T[k + 1] - T[k])
    g0 = u * F[i + 1, k] + (1 - u) * F[i, k]
    g1 = u * F[i + 1, k + 1] + (1 - u) * F[i, k + 1]
    other = v * g1 + (1 - v) * g0
    assert np.all(np.abs(other - f) <= 16 * EPS * scale)
