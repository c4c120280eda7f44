"""Pins for the oracle's quantiser and its chi-squared gradient.

Quantiser cases are worked by hand from the rounding rules (nearest 1/O cell,
ties rounded up, floor division for the cell); property tests check the
rounding error bound and index ranges on random input.  The chi-squared
gradient is checked against central finite differences, which are exact for a
quadratic misfit, and the operator pair against the adjoint identity.
"""
import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import chi2, pswf, quantise, tables

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# --------------------------------------------------------------- hand cases
# fov = 1/16 rad so that u * fov is exact for the u values below; N = 64, O = 8
# x = u/16 + 32 (continuous cell coordinate), t = 8 x, q = floor(t + 1/2),
# cell = floor((q + 4) / 8), fi = q - 8 cell + 4.
HAND = [
    # u (wavelengths), cell, fi      derivation
    (0.0, 32, 4),      # x = 32,      t = 256,   q = 256, cell = 260 // 8 = 32, f = 0
    (16.0, 33, 4),     # x = 33,      t = 264,   q = 264, cell = 33, f = 0
    (8.0, 33, 0),      # x = 32.5,    t = 260,   q = 260, cell = 264 // 8 = 33, f = -4 (tie goes up)
    (7.0, 33, 0),      # x = 32.4375, t = 259.5, q = floor(260.0) = 260 (tie goes up), as above
    (6.0, 32, 7),      # x = 32.375,  t = 259,   q = 259, cell = 263 // 8 = 32, f = 3
    (-8.0, 32, 0),     # x = 31.5,    t = 252,   q = 252, cell = 256 // 8 = 32, f = -4
    (-10.0, 31, 7),    # x = 31.375,  t = 251,   q = 251, cell = 255 // 8 = 31, f = 3
    # left of the grid: the cell division must floor towards -infinity
    (-520.0, 0, 0),    # x = -0.5,    t = -4,    q = floor(-3.5) = -4, cell = 0 // 8 = 0, f = -4
    (-523.0, -1, 7),   # x = -0.6875, t = -5.5,  q = floor(-5.0) = -5, cell = -1 // 8 = -1, f = 3
    (-528.0, -1, 4),   # x = -1,      t = -8,    q = -8, cell = -4 // 8 = -1, f = 0
]


@pytest.mark.parametrize("u,cell,fi", HAND)
def test_hand_worked_cases(u, cell, fi):
    c, f, ok = quantise.axis_quantise(np.array([u]), 64, 1.0 / 16, 8)
    assert ok[0] and c[0] == cell and f[0] == fi


def test_channel_coordinates_order_and_rounding():
    # visibility row * nchan + ch; u = u_m * (f / c) with the division first
    rng = np.random.default_rng(77)
    uvw = rng.uniform(-5e3, 5e3, (40, 3))
    f = 1e9 + 7.3e6 * np.arange(5)
    u, v, w = quantise.channel_coordinates(uvw, f)
    c = 299792458.0
    for r in (0, 17, 39):
        for ch in range(5):
            i = r * 5 + ch
            s = f[ch] / c
            assert (u[i], v[i], w[i]) == (uvw[r, 0] * s, uvw[r, 1] * s, uvw[r, 2] * s)
    # the order is observable: find a row where u_m f / c rounds differently
    diff = [(x, ff) for x in uvw[:, 0] for ff in f if (x * ff) / c != x * (ff / c)]
    assert diff, "no case separates the two orders"
    x, ff = diff[0]
    got, _, _ = quantise.channel_coordinates([[x, 0.0, 0.0]], [ff])
    assert got[0] == x * (ff / c) and got[0] != (x * ff) / c
    # at f = c the scale is exactly 1
    uc, vc, wc = quantise.channel_coordinates(uvw[:3], [c])
    assert np.array_equal(np.stack([uc, vc, wc], 1), uvw[:3])


def test_plane_index_rules():
    w = np.array([-100.0, -99.999, -50.0, -0.001, 0.0, 49.999, 50.0, 99.999, 100.0, 1e9, -1e9, np.nan])
    k, ok = quantise.plane_index(w, 4, -100.0, 100.0)
    # planes of width 50: [-100,-50) [-50,0) [0,50) [50,100], clamped outside
    assert list(k[:11]) == [0, 0, 1, 1, 2, 2, 3, 3, 3, 3, 0]
    assert list(ok) == [True] * 11 + [False]


def test_drop_rules():
    N, S, O, fov = 32, 7, 4, 0.05
    h = S // 2
    # cells h and N-1-h are the extreme kept cells
    x = np.array([h, h - 1, N - 1 - h, N - h]) - N / 2
    u = x / fov
    q = quantise.quantise(u, 0 * u, 0 * u, N, fov, O, S, 2, -1.0, 1.0, 4)
    assert list(q['dropped']) == [False, True, False, True]
    q = quantise.quantise(np.array([np.nan, 0.0, np.inf]), np.array([0.0, 0.0, 0.0]),
                          np.array([0.0, np.nan, 0.0]), N, fov, O, S, 2, -1.0, 1.0, 4)
    assert list(q['dropped']) == [True, True, True]


def test_tile_index():
    N, S, O, fov, c = 40, 5, 2, 0.1, 6
    ntx = 7  # ceil(40 / 6)
    cells = np.array([[2, 2], [5, 6], [37, 3], [20, 37]])  # (cu, cv)
    u = (cells[:, 0] - N / 2) / fov
    v = (cells[:, 1] - N / 2) / fov
    q = quantise.quantise(u, v, 0 * u, N, fov, O, S, 1, -1.0, 1.0, c)
    assert list(q['cell_u']) == list(cells[:, 0]) and list(q['cell_v']) == list(cells[:, 1])
    assert list(q['tile']) == [0, 1 * ntx + 0, 0 * ntx + 6, 6 * ntx + 3]


@settings(max_examples=300, deadline=None)
@given(st.floats(-3000.0, 3000.0, allow_nan=False), st.sampled_from([1, 2, 4, 8, 16]),
       st.sampled_from([16, 64, 4096]))
def test_rounding_error_bound(u, O, N):
    fov = math.radians(2.0)
    cell, fi, ok = quantise.axis_quantise(np.array([u]), N, fov, O)
    assert ok[0]
    assert 0 <= fi[0] < O
    x = u * fov + N / 2
    xhat = cell[0] + (fi[0] - O // 2) / O
    assert abs(x - xhat) <= 1 / (2 * O) + 1e-12


@settings(max_examples=200, deadline=None)
@given(st.integers(-5000, 5000), st.sampled_from([1, 2, 8, 32]))
def test_exact_oversample_points_round_trip(m, O):
    # x on the oversample lattice: x = m / O -> t = m, q = m exactly
    N, fov = 64, 1.0 / 64  # u * fov exact for u = (x - N/2) * 64
    u = (m / O - N / 2) * 64.0
    cell, fi, ok = quantise.axis_quantise(np.array([u]), N, fov, O)
    assert cell[0] * O + fi[0] - O // 2 == m


# --------------------------------------------------------------- chi2
def _op(seed, N=16, S=5, O=4, P=3, nvis=80):
    fov = math.radians(2.0)
    rng = np.random.default_rng(seed)
    u, v = rng.uniform(-5, 5, (2, nvis)) / fov
    w = rng.uniform(-300, 300, nvis)
    q = quantise.quantise(u, v, w, N, fov, O, S, P, -300.0, 300.0, 2)
    c1 = pswf.taper_c1(N, fov, S)
    T = tables.separable_table(tables.w_plane_centres(P, -300.0, 300.0), N, fov, S, O, c1)
    return chi2.SeparableOperator(q, T, c1, N, S, fov), rng


def test_operator_adjoint_identity():
    op, rng = _op(70)
    x = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    r = rng.standard_normal(80) + 1j * rng.standard_normal(80)
    r[op.q['dropped']] = 0
    lhs = np.vdot(r, op.forward(x))
    rhs = np.vdot(op.adjoint(r), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_chi2_gradient_equals_central_differences():
    op, rng = _op(71)
    N = 16
    x = rng.standard_normal((N, N))
    Vt = rng.standard_normal(80) + 1j * rng.standard_normal(80)
    W = rng.uniform(0.5, 2.0, 80)
    g = chi2.chi2_grad(op, x, Vt, W)
    for (qq, pp) in [(3, 4), (8, 8), (0, 15), (11, 2)]:
        e = np.zeros((N, N))
        e[qq, pp] = 1.0                          # chi2 is quadratic: any step is exact
        fd = (chi2.chi2(op, x + e, Vt, W) - chi2.chi2(op, x - e, Vt, W)) / 2.0
        assert fd == pytest.approx(g[qq, pp], rel=1e-9, abs=1e-9 * np.abs(g).max())
