"""Pins for the oracle's correction table F_w - F~_w (Section 6).

* Full size (S_c = S, O_c = O): separable outer product plus correction is
  the exact 2D table of ``tables.exact_table_2d`` (itself pinned against the
  exact DFT), for plain and asymmetric axis coefficients.
* Full support (S = S_c = N, indices modulo N): separable gridding plus the
  correction reproduces the direct DFT of the dirty-image equation with the
  exact w term (``dft``, written independently).
* The coarse sample of each visibility is, by brute force over the 1/O_c
  lattice, the nearest one to its quantised position (ties towards +), and
  its cell is the visibility's cell or the next one.
* The w = 0 plane has no correction (both screens are 1).
* Truncated to S_c < S, the correction moves the image towards the exact DFT
  (the error falls with S_c and at S_c = S - 2 is within 2x of the exact 2D
  kernel's; with O_c = 2 it still removes most of the separable error), which
  is what the correction is for.
* Gridding and degridding with the correction are adjoint (FP64), and the
  per-cell evaluation used for full-size checks equals the full grid.
"""
import math

import numpy as np
import pytest

from oracle import correction, dft, gridder, imaging, pswf, quantise, tables

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _vis(seed, N, fov, nvis, cells, wmax):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-cells, cells, nvis) / fov
    v = rng.uniform(-cells, cells, nvis) / fov
    w = rng.uniform(-wmax, wmax, nvis)
    y = rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)
    return rng, u, v, w, y


@pytest.mark.parametrize("N,S,O,coef", [(16, 5, 4, None), (24, 7, 8, None), (20, 5, 2, (0.43, 0.1, 0.61, 0.3))])
def test_full_size_correction_completes_the_separable_table(N, S, O, coef):
    fov, P = math.radians(30.0), 3
    wc = tables.w_plane_centres(P, -60.0, 60.0)
    c1 = pswf.taper_c1(N, fov, S)
    a_u, b_u, a_v, b_v = coef or (0.5, 5.0 / 24.0, 0.5, 5.0 / 24.0)
    Tu = tables.separable_table(wc, N, fov, S, O, c1, a=a_u, b=b_u)
    Tv = tables.separable_table(wc, N, fov, S, O, c1, a=a_v, b=b_v)
    C = correction.correction_table(wc, N, fov, S, O, c1, a_u, b_u, a_v, b_v)
    T2 = tables.exact_table_2d(wc, N, fov, S, O, c1)
    sep = Tu[:, :, None, :, None] * Tv[:, None, :, None, :]     # [k][fu][fv][su][sv]
    assert np.max(np.abs(sep + C - T2)) <= 1e-13 * np.max(np.abs(T2))
    assert np.max(np.abs(C)) > 1e-6 * np.max(np.abs(T2))        # the correction is not trivially 0


@pytest.mark.parametrize("N,O", [(12, 4), (16, 2)])
def test_full_support_corrected_gridding_equals_exact_dft(N, O):
    fov, P, wmax = math.radians(12.0), 2, 500.0
    _, u, v, w, y = _vis(51 + N, N, fov, 30, N / 2 - 1, wmax)
    q = quantise.quantise(u, v, w, N, fov, O, 1, P, -wmax, wmax, 1)
    q['dropped'] = np.zeros_like(q['dropped'])                # wrap mode: nothing is off-grid
    wc = tables.w_plane_centres(P, -wmax, wmax)
    c1 = pswf.taper_c1(N, fov, 5.0)
    T = tables.separable_table(wc, N, fov, N, O, c1)
    C = correction.correction_table(wc, N, fov, N, O, c1)
    D = imaging.image_from_grid(correction.grid(q, y, T, C, N, N, O, N, O, wrap=True), c1, fov)
    uh, vh = quantise.dequantised(q, N, fov, O)
    ref = dft.dirty(uh, vh, wc[q['k']], y, N, fov, dft.phase_screen(N, fov, 'exact'))
    amp = 1.0 / (c1[None, :] * c1[:, None])
    assert np.all(np.abs(D - ref) <= 1e-12 * np.max(np.abs(ref)) * amp)
    # without the correction the separable screen's error remains
    D0 = imaging.image_from_grid(gridder.grid_separable(q, y, T, N, N, wrap=True), c1, fov)
    assert np.max(np.abs(D0 - ref)) > 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("O,Oc", [(8, 8), (8, 4), (8, 2), (8, 1), (4, 1), (16, 4), (1, 1)])
def test_coarse_sample_is_the_nearest_lattice_point(O, Oc):
    rng = np.random.default_rng(O * 31 + Oc)
    cell = rng.integers(-50, 50, 4000)
    fi = rng.integers(0, O, 4000)
    cc, fc = correction.coarse_axis(cell, fi, O, Oc)
    x = cell + (fi - O // 2) / O                               # quantised position (cells)
    # brute force: every lattice point m / Oc within two cells, nearest, ties to +
    m = np.floor(x * Oc)[:, None] + np.arange(-2 * Oc - 2, 2 * Oc + 3)[None, :]
    dist = np.abs(m / Oc - x[:, None])
    best = np.array([mm[np.flatnonzero(d == d.min()).max()] for mm, d in zip(m, dist)])
    got = cc * Oc + (fc - Oc // 2)
    assert np.array_equal(got, best.astype(np.int64))
    assert np.all((fc >= 0) & (fc < Oc))
    assert np.all((cc == cell) | (cc == cell + 1))
    if Oc in (1, O):
        assert np.array_equal(cc, cell)


def test_w_zero_plane_has_no_correction():
    N, fov = 32, math.radians(20.0)
    c1 = pswf.taper_c1(N, fov, 7)
    C = correction.correction_table(tables.w_plane_centres(1, -5.0, 5.0), N, fov, 5, 4, c1)
    assert np.all(C == 0)


def test_truncated_correction_moves_towards_the_exact_dft():
    N, fov, S, O, P, wmax = 64, 0.4, 15, 8, 4, 20.0
    _, u, v, w, y = _vis(3, N, fov, 300, N / 2 - S, wmax)
    c1 = pswf.taper_c1(N, fov, S)
    q = quantise.quantise(u, v, w, N, fov, O, S, P, -wmax, wmax, 1)
    wc = tables.w_plane_centres(P, -wmax, wmax)
    T = tables.separable_table(wc, N, fov, S, O, c1)
    keep = ~q['dropped']
    uh, vh = quantise.dequantised(q, N, fov, O)
    ref = dft.dirty(uh[keep], vh[keep], wc[q['k'][keep]], y[keep], N, fov,
                    dft.phase_screen(N, fov, 'exact'))
    inner = slice(N // 4, 3 * N // 4)

    def err(G):
        D = imaging.image_from_grid(G, c1, fov)
        return np.linalg.norm((D - ref)[inner, inner]) / np.linalg.norm(ref[inner, inner])

    e_sep = err(gridder.grid_separable(q, y, T, N, S))
    e_2d = err(gridder.grid_exact(q, y, tables.exact_table_2d(wc, N, fov, S, O, c1), N, S))
    e = {}
    for Sc, Oc in [(5, 8), (9, 8), (13, 8), (13, 2)]:
        C = correction.correction_table(wc, N, fov, Sc, Oc, c1)
        e[Sc, Oc] = err(correction.grid(q, y, T, C, N, S, O, Sc, Oc))
    assert e[5, 8] < e_sep and e[9, 8] < e[5, 8] and e[13, 8] < e[9, 8]
    assert e[13, 8] < 2.0 * e_2d and e[13, 8] < e_sep / 30
    assert e[13, 2] < e_sep / 3                                 # a coarser correction table keeps most of it


@pytest.mark.parametrize("n_power", [0, -1])
def test_corrected_gridding_and_degridding_are_adjoint(n_power):
    N, S, O, P, wmax, fov = 32, 9, 8, 3, 150.0, 0.3
    rng, u, v, w, y = _vis(57, N, fov, 300, N / 2 - 5, wmax)
    c1 = pswf.taper_c1(N, fov, S)
    q = quantise.quantise(u, v, w, N, fov, O, S, P, -wmax, wmax, 1)
    wc = tables.w_plane_centres(P, -wmax, wmax)
    T = tables.separable_table(wc, N, fov, S, O, c1)
    C = correction.correction_table(wc, N, fov, 7, 4, c1)
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    D = imaging.image_from_grid(correction.grid(q, y, T, C, N, S, O, 7, 4), c1, fov, n_power)
    V = correction.degrid(q, imaging.grid_from_image(X, c1, fov, n_power), T, C, N, S, O, 7, 4)
    assert abs(np.vdot(X, D) - np.vdot(V, y)) <= 1e-12 * np.linalg.norm(D) * np.linalg.norm(X)


def test_grid_cells_match_the_full_corrected_grid():
    N, fov, S, O, P, Sc, Oc = 48, 0.5, 7, 8, 3, 5, 4
    _, u, v, w, y = _vis(61, N, fov, 500, 18, 50.0)
    c1 = pswf.taper_c1(N, fov, S)
    q = quantise.quantise(u, v, w, N, fov, O, S, P, -50.0, 50.0, 1)
    wc = tables.w_plane_centres(P, -50.0, 50.0)
    T = tables.separable_table(wc, N, fov, S, O, c1)
    C = correction.correction_table(wc, N, fov, Sc, Oc, c1)
    G = correction.grid(q, y, T, C, N, S, O, Sc, Oc)
    cells = [(24, 24), (10, 30), (33, 7), (20, 21), (0, 0)]
    got = correction.grid_cells(q, y, T, C, N, S, O, Sc, Oc, cells)
    assert np.max(np.abs(got - np.array([G[a, b] for a, b in cells]))) <= 1e-13 * np.max(np.abs(G))
