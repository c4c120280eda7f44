"""Pins for the factor n of the dirty-image and prediction equations (Section 2).

The dirty-image equation gives I_D(l)/n as a sum over visibilities, and the
prediction equation integrates I(l)/n.  Composing the two for a point source
of flux F at a pixel centre l0 (with n0 = n(l0) != 1) fixes values that do not
depend on how the oracle is written:

* prediction:  V_i = (F / n0) exp(-2 pi i (u_i l0 + v_i m0 + w_i (n0 - 1)))
  (the pixel sum of a delta picks out its pixel);
* dirty image of those visibilities at the source pixel:
  I_D(l0) = n0 * sum_i W_i V_i exp(+2 pi i (...)) = F * sum_i W_i.

At full support (S = N taps, wrap mode) with the exact 2D tables, gridding +
F+ + taper correction and its adjoint reproduce the direct sums exactly at
the quantised uv and the plane's w (pinned in test_oracle_gridding.py), so
these closed forms pin the ``n_power`` branches of the oracle's image <->
grid steps: image_from_grid(n_power=+1) for the dirty image and
grid_from_image(n_power=-1) for the model of a prediction.  A source far from
the phase centre (n0 ~ 0.95) makes a dropped or inverted factor n fail by
about 5 %, far above the 1e-10 tolerance; the last tests plant exactly those
mistakes in the oracle and check that the pins catch them.
"""
import math

import numpy as np
import pytest

from oracle import geometry, gridder, imaging, pswf, quantise, tables

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

N, O, P, FOV, WMAX, WIDTH = 16, 4, 3, 0.8, 40.0, 5.0
P0, Q0 = 13, 4            # source pixel: l0 = 0.25, m0 = -0.2, n0 = 0.9474
FLUX = 0.7


def _setup(seed=31, nvis=60):
    rng = np.random.default_rng(seed)
    cells = N / 2 - 1
    u = rng.uniform(-cells, cells, nvis) / FOV
    v = rng.uniform(-cells, cells, nvis) / FOV
    w = rng.uniform(-WMAX, WMAX, nvis)
    W = rng.uniform(0.5, 1.5, nvis)
    q = quantise.quantise(u, v, w, N, FOV, O, 1, P, -WMAX, WMAX, 1)
    q['dropped'] = np.zeros_like(q['dropped'])      # wrap mode: nothing is off-grid
    uh, vh = quantise.dequantised(q, N, FOV, O)
    wc = tables.w_plane_centres(P, -WMAX, WMAX)
    c1 = pswf.taper_c1(N, FOV, WIDTH)
    T2 = tables.exact_table_2d(wc, N, FOV, N, O, c1)
    return q, uh, vh, wc[q['k']], W, c1, T2


def _source():
    l0 = (P0 - N / 2) * FOV / N
    m0 = (Q0 - N / 2) * FOV / N
    n0 = math.sqrt(1.0 - l0 * l0 - m0 * m0)
    return l0, m0, n0


def _point_source_vis(uh, vh, wk):
    l0, m0, n0 = _source()
    return FLUX / n0 * np.exp(-2j * np.pi * (uh * l0 + vh * m0 + wk * (n0 - 1.0)))


def _dirty_peak(n_power=1):
    q, uh, vh, wk, W, c1, T2 = _setup()
    V = _point_source_vis(uh, vh, wk)
    G = gridder.grid_exact(q, W * V, T2, N, N, wrap=True)
    D = imaging.image_from_grid(G, c1, FOV, n_power=n_power)
    return D[Q0, P0], FLUX * np.sum(W)


def _predicted(n_power=-1):
    q, uh, vh, wk, W, c1, T2 = _setup()
    img = np.zeros((N, N), dtype=np.complex128)
    img[Q0, P0] = FLUX
    G = imaging.grid_from_image(img, c1, FOV, n_power=n_power)
    return gridder.degrid_exact(q, G, T2, N, N, wrap=True), _point_source_vis(uh, vh, wk)


def test_source_is_off_centre():
    l0, m0, n0 = _source()
    assert (l0, m0) == pytest.approx((0.25, -0.2)) and n0 < 0.95


def test_dirty_image_peak_is_flux_times_weight_sum():
    got, want = _dirty_peak()
    assert abs(got - want) <= 1e-10 * abs(want)


def test_dirty_image_is_n_times_dirty_sum_everywhere():
    # away from the source pixel: I_D = n * sum_i W_i V_i exp(+...), with n
    # evaluated as sqrt(1 - l^2 - m^2) at every pixel
    q, uh, vh, wk, W, c1, T2 = _setup()
    V = _point_source_vis(uh, vh, wk)
    D = imaging.image_from_grid(gridder.grid_exact(q, W * V, T2, N, N, wrap=True), c1, FOV, n_power=1)
    l = (np.arange(N) - N / 2) * FOV / N
    L, M = l[None, :], l[:, None]
    n = np.sqrt(1.0 - L * L - M * M)
    ph = uh[:, None, None] * L + vh[:, None, None] * M + wk[:, None, None] * (n - 1.0)
    ref = n * np.einsum('i,iqp->qp', W * V, np.exp(2j * np.pi * ph))
    amp = 1.0 / (c1[None, :] * c1[:, None])
    assert np.all(np.abs(D - ref) <= 1e-11 * np.max(np.abs(ref)) * amp)


def test_prediction_of_point_source_matches_closed_form():
    got, want = _predicted()
    assert np.max(np.abs(got - want)) <= 1e-10 * FLUX


def test_adjoint_pair_uses_one_over_n_on_both_sides():
    # <degrid(grid_from_image(X, -1)), y> = <X, image_from_grid(grid(y), -1)>
    q, uh, vh, wk, W, c1, T2 = _setup()
    rng = np.random.default_rng(4)
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    y = rng.standard_normal(len(uh)) + 1j * rng.standard_normal(len(uh))
    A = gridder.degrid_exact(q, imaging.grid_from_image(X, c1, FOV, n_power=-1), T2, N, N, wrap=True)
    B = imaging.image_from_grid(gridder.grid_exact(q, y, T2, N, N, wrap=True), c1, FOV, n_power=-1)
    lhs, rhs = np.vdot(y, A), np.vdot(B, X)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(y)


# ---- planted mistakes: each must make one of the pins above fail


@pytest.mark.parametrize("mutation", ["drop_n", "invert_n"])
def test_pins_catch_a_wrong_factor_n(monkeypatch, mutation):
    real = geometry.n_image
    if mutation == "drop_n":
        monkeypatch.setattr(imaging, "n_image", lambda n, fov: np.ones((n, n)))
    else:
        monkeypatch.setattr(imaging, "n_image", lambda n, fov: 1.0 / real(n, fov))
    got, want = _dirty_peak()
    assert abs(got - want) > 1e-2 * abs(want)
    got, want = _predicted()
    assert np.max(np.abs(got - want)) > 1e-2 * FLUX


@pytest.mark.parametrize("n_power", [0, -1])
def test_pins_catch_a_wrong_exponent(n_power):
    got, want = _dirty_peak(n_power=n_power)
    assert abs(got - want) > 1e-2 * abs(want)
    got, want = _predicted(n_power=-n_power if n_power else 0)
    assert np.max(np.abs(got - want)) > 1e-2 * FLUX
