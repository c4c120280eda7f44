"""Pins for the oracle's W-stacking hybrid (Section 4.3).

* Visibilities exactly at slice centres, full support (S = N, indices modulo
  N), one residual plane at 0: the hybrid must reproduce the direct DFT of the
  dirty-image equation with the exact w term at the quantised uv, since the
  whole w term is then the exact image-space phase of the slice.
* General w, full support: the image must equal the sum over slices of the
  exact phase exp(2 pi i w_s (n - 1)) (written with oracle.dft's exact screen,
  not the hybrid's own form of n - 1) times the DFT with the separable screen
  at the residual plane centre.
* Gridding and prediction are adjoint (FP64).
* One slice over a symmetric range is the plain separable path.
* The expected relative amplitude loss for residuals uniform in
  [-w_max, w_max] matches Section 4.3's (2/3) pi^2 eps^2 w_max^2.
"""
import math

import numpy as np
import pytest

from oracle import dft, gridder, imaging, phase_error, pswf, quantise, tables, wstack

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _full_bins(u, v, w, N, fov, O, S, P, w_lo, w_hi):
    q = quantise.quantise(u, v, w, N, fov, O, 1, P, w_lo, w_hi, 1)
    q['dropped'] = np.zeros_like(q['dropped'])   # wrap mode: nothing is off-grid
    return q


def _close(D, ref, c1, rel=1e-12):
    amp = 1.0 / (c1[None, :] * c1[:, None])
    return np.all(np.abs(D - ref) <= rel * np.max(np.abs(ref)) * amp)


def _vis(seed, N, fov, nvis, cells):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-cells, cells, nvis) / fov
    v = rng.uniform(-cells, cells, nvis) / fov
    y = rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)
    return rng, u, v, y


@pytest.mark.parametrize("N,O,ns", [(16, 4, 5), (18, 8, 3)])
def test_slice_centred_full_support_equals_exact_dft(N, O, ns):
    fov, w_lo, w_hi = math.radians(9.0), -1500.0, 1500.0
    rng, u, v, y = _vis(31 + N, N, fov, 40, N / 2 - 1)
    k = rng.integers(0, ns, len(u))
    w = w_lo + (k + 0.5) * (w_hi - w_lo) / ns          # exactly at the slice centres
    c1 = pswf.taper_c1(N, fov, 5.0)
    D = wstack.image(u, v, w, y, N, fov, N, O, 1, ns, w_lo, w_hi, c1, bins=_full_bins, wrap=True)
    q = _full_bins(u, v, w, N, fov, O, N, 1, -1.0, 1.0)
    uh, vh = quantise.dequantised(q, N, fov, O)
    ref = dft.dirty(uh, vh, w, y, N, fov, dft.phase_screen(N, fov, 'exact'))
    assert _close(D, ref, c1)


def test_residual_planes_use_the_separable_screen():
    N, O, P, ns, fov = 16, 4, 3, 4, math.radians(8.0)
    w_lo, w_hi = -2000.0, 2000.0
    rng, u, v, y = _vis(37, N, fov, 60, N / 2 - 1)
    w = rng.uniform(w_lo, w_hi, len(u))
    c1 = pswf.taper_c1(N, fov, 6.0)
    D = wstack.image(u, v, w, y, N, fov, N, O, P, ns, w_lo, w_hi, c1, bins=_full_bins, wrap=True)
    # reference: per slice, exact phase of the slice centre times the
    # separable-screen DFT at the residual plane centre
    h = (w_hi - w_lo) / (2 * ns)
    wc = tables.w_plane_centres(P, -h, h)
    exact = dft.phase_screen(N, fov, 'exact')
    sep = dft.phase_screen(N, fov, 'sep')
    ref = np.zeros((N, N), complex)
    for s in range(ns):
        ws = w_lo + (s + 0.5) * (w_hi - w_lo) / ns
        m = (w >= w_lo + s * 2 * h) & (w < w_lo + (s + 1) * 2 * h)
        q = _full_bins(u[m], v[m], w[m] - ws, N, fov, O, N, P, -h, h)
        uh, vh = quantise.dequantised(q, N, fov, O)
        ref += np.exp(2j * np.pi * ws * exact) * dft.dirty(uh, vh, wc[q['k']], y[m], N, fov, sep)
    assert _close(D, ref, c1)


@pytest.mark.parametrize("n_power", [0, -1])
def test_image_and_predict_are_adjoint(n_power):
    N, O, P, S, ns, fov = 32, 8, 4, 7, 3, math.radians(6.0)
    w_lo, w_hi = -900.0, 900.0
    rng, u, v, y = _vis(41, N, fov, 300, N / 2 - 5)
    w = rng.uniform(w_lo, w_hi, len(u))
    c1 = pswf.taper_c1(N, fov, S)
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    D = wstack.image(u, v, w, y, N, fov, S, O, P, ns, w_lo, w_hi, c1, n_power=n_power)
    V = wstack.predict(u, v, w, X, N, fov, S, O, P, ns, w_lo, w_hi, c1, n_power=n_power)
    lhs = np.vdot(X, D)               # <X, G y>
    rhs = np.vdot(V, y)               # <G^H X, y>
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(D) * np.linalg.norm(X)


def test_one_slice_is_the_plain_separable_path():
    N, O, P, S, fov = 32, 8, 5, 7, math.radians(5.0)
    W = 700.0
    rng, u, v, y = _vis(43, N, fov, 250, N / 2 - 5)
    w = rng.uniform(-W, W, len(u))
    c1 = pswf.taper_c1(N, fov, S)
    D = wstack.image(u, v, w, y, N, fov, S, O, P, 1, -W, W, c1, n_power=1)
    q = quantise.quantise(u, v, w, N, fov, O, S, P, -W, W, 1)
    T = tables.separable_table(tables.w_plane_centres(P, -W, W), N, fov, S, O, c1)
    ref = imaging.image_from_grid(gridder.grid_separable(q, y, T, N, S), c1, fov, n_power=1)
    assert np.linalg.norm(D - ref) <= 1e-14 * np.linalg.norm(ref)


def test_expected_amplitude_loss_matches_section_4_3():
    # a point source at (l, m): the residual phase error 2 pi dw eps(l, m) with
    # dw uniform in [-w_max, w_max] costs 1 - <cos> of the amplitude
    l, m, gamma = 0.06, -0.04, 5.0 / 24.0
    eps = phase_error.eps_exact(l, m, gamma)
    w_max = 0.01 / (2 * math.pi * abs(eps))
    dw = np.linspace(-w_max, w_max, 200001)
    loss = 1.0 - np.trapezoid(np.cos(2 * np.pi * dw * eps), dw) / (2 * w_max)
    assert loss == pytest.approx(2.0 / 3.0 * math.pi ** 2 * eps ** 2 * w_max ** 2, rel=1e-4)
