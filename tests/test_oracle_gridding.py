"""Pins for the oracle's tables, quantiser, gridder and degridder.

The central pin is the full-support identity: with S = N taps (indices taken
modulo N), gridding followed by F+ and division by the taper reproduces the
direct DFT of the dirty-image equation at the quantised uv coordinates and the
plane's w exactly, because the N taps of every table row sum one period of a
discrete Fourier series.  The DFT side is written independently (oracle.dft),
so a wrong sign, index, offset or normalisation in the tables or the gridder
fails it.
"""
import math

import numpy as np
import pytest

from oracle import dft, facet, geometry, gridder, imaging, pswf, quantise, tables

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _setup(seed, N, fov, nvis, O, P, wmax, cells, width=None):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-cells, cells, nvis) / fov
    v = rng.uniform(-cells, cells, nvis) / fov
    w = rng.uniform(-wmax, wmax, nvis)
    y = rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)
    c1 = np.ones(N) if width is None else pswf.taper_c1(N, fov, width)
    return u, v, w, y, c1


def _close(D, ref, c1, rel=1e-12):
    """|D - ref| <= rel * max|ref| / (c1(l) c1(m)) per pixel: the taper
    correction amplifies rounding by 1/(c1 c1) towards the image edges."""
    amp = 1.0 / (c1[None, :] * c1[:, None])
    return np.all(np.abs(D - ref) <= rel * np.max(np.abs(ref)) * amp)


def _full_support_bins(u, v, w, N, fov, O, P, w_lo, w_hi):
    q = quantise.quantise(u, v, w, N, fov, O, 1, P, w_lo, w_hi, 1)
    q['dropped'] = np.zeros_like(q['dropped'])   # wrap mode: nothing is off-grid
    return q


@pytest.mark.parametrize("N,O,width", [(16, 4, None), (16, 8, 5.0), (20, 2, 7.0)])
def test_full_support_separable_gridding_equals_sep_dft(N, O, width):
    fov, P, wmax = math.radians(8.0), 3, 400.0
    u, v, w, y, c1 = _setup(10 + N + O, N, fov, 40, O, P, wmax, N / 2 - 1, width)
    q = _full_support_bins(u, v, w, N, fov, O, P, -wmax, wmax)
    wc = tables.w_plane_centres(P, -wmax, wmax)
    T = tables.separable_table(wc, N, fov, N, O, c1)
    D = imaging.image_from_grid(gridder.grid_separable(q, y, T, N, N, wrap=True), c1, fov)
    uh, vh = quantise.dequantised(q, N, fov, O)
    ref = dft.dirty(uh, vh, wc[q['k']], y, N, fov, dft.phase_screen(N, fov, 'sep'))
    assert _close(D, ref, c1)


def test_full_support_exact_gridding_equals_exact_dft():
    N, O, P, wmax, fov = 12, 4, 2, 600.0, math.radians(10.0)
    u, v, w, y, c1 = _setup(21, N, fov, 30, O, P, wmax, N / 2 - 1, 5.0)
    q = _full_support_bins(u, v, w, N, fov, O, P, -wmax, wmax)
    wc = tables.w_plane_centres(P, -wmax, wmax)
    T2 = tables.exact_table_2d(wc, N, fov, N, O, c1)
    D = imaging.image_from_grid(gridder.grid_exact(q, y, T2, N, N, wrap=True), c1, fov)
    uh, vh = quantise.dequantised(q, N, fov, O)
    ref = dft.dirty(uh, vh, wc[q['k']], y, N, fov, dft.phase_screen(N, fov, 'exact'))
    assert _close(D, ref, c1)


def test_full_support_degridding_equals_sep_predict():
    N, O, P, wmax, fov = 16, 8, 3, 300.0, math.radians(6.0)
    u, v, w, y, c1 = _setup(22, N, fov, 50, O, P, wmax, N / 2 - 1, 6.0)
    q = _full_support_bins(u, v, w, N, fov, O, P, -wmax, wmax)
    wc = tables.w_plane_centres(P, -wmax, wmax)
    T = tables.separable_table(wc, N, fov, N, O, c1)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    V = gridder.degrid_separable(q, imaging.grid_from_image(X, c1, fov), T, N, N, wrap=True)
    uh, vh = quantise.dequantised(q, N, fov, O)
    ref = dft.predict(uh, vh, wc[q['k']], X, N, fov, dft.phase_screen(N, fov, 'sep'))
    # rounding scale: the pre-corrected image X / (c1 c1) is what gets summed
    scale = np.sum(np.abs(X) / (c1[None, :] * c1[:, None]))
    assert np.max(np.abs(V - ref)) <= 1e-13 * scale


def test_full_support_facet_gridding_equals_facet_dft():
    # Section 4.1: rotated, shifted visibilities gridded with the facet tables
    N, O, P, fov = 16, 4, 3, math.radians(2.0)
    l0, m0 = math.radians(3.5), math.radians(-2.0)
    u, v, w, y, c1 = _setup(23, N, fov, 40, O, P, 800.0, N / 2 - 2, 5.0)
    u2, v2, w2, y2 = facet.facet_rotate(u, v, w, y, l0, m0)
    n0, a_l, a_m = facet.facet_coefficients(l0, m0)
    wlo, whi = -800.0, 800.0
    q = _full_support_bins(u2, v2, w2, N, fov, O, P, wlo, whi)
    wc = tables.w_plane_centres(P, wlo, whi)
    Tl = tables.separable_table(wc, N, fov, N, O, c1, a=a_l, b=0.0)
    Tm = tables.separable_table(wc, N, fov, N, O, c1, a=a_m, b=0.0)
    D = imaging.image_from_grid(gridder.grid_separable(q, y2, Tl, N, N, Tv=Tm, wrap=True), c1, fov)
    uh, vh = quantise.dequantised(q, N, fov, O)
    phi = dft.phase_screen(N, fov, 'facet', a=a_l, b=0.0, a_m=a_m, b_m=0.0)
    ref = dft.dirty(uh, vh, wc[q['k']], y2, N, fov, phi)
    assert _close(D, ref, c1)


def test_facet_rotation_sign_point_source():
    # a point source of flux 1 at the facet centre (prediction equation, X = I/n)
    # predicts V = exp(-2 pi i (u l0 + v m0 + w (n0-1))) / n0; rotating to the
    # facet centre must make it the constant 1/n0
    rng = np.random.default_rng(8)
    l0, m0 = 0.05, -0.03
    n0 = math.sqrt(1 - l0 * l0 - m0 * m0)
    u, v, w = rng.uniform(-3e4, 3e4, (3, 100))
    V = np.exp(-2j * np.pi * (u * l0 + v * m0 + w * (n0 - 1))) / n0
    _, _, _, V2 = facet.facet_rotate(u, v, w, V, l0, m0)
    assert np.max(np.abs(V2 - 1 / n0)) < 1e-12


def test_facet_coefficients_reduce_to_plain_at_centre():
    n0, a_l, a_m = facet.facet_coefficients(0.0, 0.0)
    assert (n0, a_l, a_m) == (1.0, 0.5, 0.5)
    # Hessian of h at l0: -1/n0 I - l0 l0^T / n0^3 ; a_l is minus half its ll entry
    l0, m0 = 0.1, 0.2
    n0, a_l, a_m = facet.facet_coefficients(l0, m0)
    e = 1e-4
    hfun = lambda a, b: math.sqrt(1 - a * a - b * b)  # noqa: E731
    hll = (hfun(l0 + e, m0) - 2 * hfun(l0, m0) + hfun(l0 - e, m0)) / e ** 2
    hmm = (hfun(l0, m0 + e) - 2 * hfun(l0, m0) + hfun(l0, m0 - e)) / e ** 2
    assert a_l == pytest.approx(-0.5 * hll, rel=1e-6)
    assert a_m == pytest.approx(-0.5 * hmm, rel=1e-6)


@pytest.mark.parametrize("kind", ['sep', 'exact'])
def test_gridding_degridding_adjoint(kind):
    N, S, O, P, wmax, fov = 32, 7, 8, 4, 200.0, math.radians(2.0)
    u, v, w, y, c1 = _setup(30, N, fov, 300, O, P, wmax, 14, 7.0)
    q = quantise.quantise(u, v, w, N, fov, O, S, P, -wmax, wmax, 2)
    wc = tables.w_plane_centres(P, -wmax, wmax)
    rng = np.random.default_rng(31)
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    if kind == 'sep':
        T = tables.separable_table(wc, N, fov, S, O, c1)
        Gy, Vg = gridder.grid_separable(q, y, T, N, S), gridder.degrid_separable(q, G, T, N, S)
    else:
        T2 = tables.exact_table_2d(wc, N, fov, S, O, c1)
        Gy, Vg = gridder.grid_exact(q, y, T2, N, S), gridder.degrid_exact(q, G, T2, N, S)
    lhs = np.vdot(G, Gy)
    rhs = np.vdot(Vg, y)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Gy) * np.linalg.norm(G)


def test_separable_equals_exact_at_w_zero():
    # one plane with centre w = 0: g_0 = 1, both tables are the taper's transform
    N, S, O, fov = 24, 7, 4, math.radians(3.0)
    u, v, w, y, c1 = _setup(40, N, fov, 200, O, 1, 100.0, 9, 7.0)
    q = quantise.quantise(u, v, w, N, fov, O, S, 1, -100.0, 100.0, 3)
    wc = tables.w_plane_centres(1, -100.0, 100.0)
    assert wc[0] == 0.0
    T = tables.separable_table(wc, N, fov, S, O, c1)
    T2 = tables.exact_table_2d(wc, N, fov, S, O, c1)
    a = gridder.grid_separable(q, y, T, N, S)
    b = gridder.grid_exact(q, y, T2, N, S)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_table_conjugate_symmetry():
    # c1 real and even about the centre pixel except the unpaired edge pixel
    # p = 0; with taper width chosen so that c1(edge) is negligible the
    # identity T_{-w}(Delta) = conj(T_w(-Delta)) holds to that level.  With no
    # taper it holds after removing the p = 0 term exactly: check the formula
    # on the paired entries fi >= 1, where -Delta is again a table entry.
    N, S, O, fov = 32, 7, 8, math.radians(4.0)
    c1 = pswf.taper_c1(N, fov, 7)
    wc = np.array([-350.0, 350.0])
    T = tables.separable_table(wc, N, fov, S, O, c1)
    edge = c1[0]
    for fi in range(1, O):
        fj = O - fi                      # f -> -f
        for s in range(S):
            sj = S - 1 - s               # s - h -> -(s - h)
            assert abs(T[0, fi, s] - np.conj(T[1, fj, sj])) <= 2 * edge / N + 1e-15


def test_table_w0_real_up_to_edge_pixel():
    N, S, O, fov = 32, 7, 8, math.radians(4.0)
    c1 = pswf.taper_c1(N, fov, 7)
    T = tables.separable_table(np.array([0.0]), N, fov, S, O, c1)
    assert np.max(np.abs(T.imag)) <= c1[0] / N + 1e-16


def test_grid_cells_matches_full_grid():
    N, S, O, P, fov = 32, 7, 8, 4, math.radians(2.0)
    u, v, w, y, c1 = _setup(50, N, fov, 500, O, P, 200.0, 14, 7.0)
    q = quantise.quantise(u, v, w, N, fov, O, S, P, -200.0, 200.0, 2)
    T = tables.separable_table(tables.w_plane_centres(P, -200.0, 200.0), N, fov, S, O, c1)
    G = gridder.grid_separable(q, y, T, N, S)
    cells = [(16, 16), (3, 29), (20, 5), (0, 0), (31, 12)]
    got = gridder.grid_cells(q, y, T, N, S, cells)
    assert np.allclose(got, [G[a, b] for a, b in cells], rtol=0, atol=1e-12)


def test_separable_error_scales_as_fov_to_the_fourth():
    # Abstract / Section 6: the separable error grows as the fourth power of
    # the field of view.  Fix u in cells (so the u.l phase is the same in
    # pixel units) and w in wavelengths; the relative image difference between
    # exact and separable phase must follow fov^4.
    N, nvis = 32, 150
    rng = np.random.default_rng(60)
    xu, xv = rng.uniform(-12, 12, (2, nvis))
    w = rng.uniform(-200, 200, nvis)
    y = rng.standard_normal(nvis) + 1j * rng.standard_normal(nvis)
    fovs = np.radians([0.5, 1.0, 2.0, 4.0])
    r = []
    for fov in fovs:
        ex = dft.dirty(xu / fov, xv / fov, w, y, N, fov, dft.phase_screen(N, fov, 'exact'))
        sp = dft.dirty(xu / fov, xv / fov, w, y, N, fov, dft.phase_screen(N, fov, 'sep'))
        r.append(np.linalg.norm(ex - sp) / np.linalg.norm(ex))
    slope = np.polyfit(np.log(fovs), np.log(r), 1)[0]
    assert slope == pytest.approx(4.0, abs=0.05)


def test_truncated_gridding_tracks_dft_at_64():
    # Truncation to S taps + taper aliasing: no closed form (the paper states
    # no number).  Guard only against gross breakage: on the 64^2 accuracy
    # workload the inner-half image must agree with the separable DFT at the
    # quantised coordinates to better than 1e-2 relative RMS.
    from paper_1511_07152_amd import synth
    d = synth.accuracy_64()
    N, fov, S, O, P = d['N'], d['fov'], d['S'], d['O'], d['P']
    c1 = pswf.taper_c1(N, fov, S)
    q = quantise.quantise(d['u'], d['v'], d['w'], N, fov, O, S, P, d['w_lo'], d['w_hi'], 10)
    assert not q['dropped'].any()
    wc = tables.w_plane_centres(P, d['w_lo'], d['w_hi'])
    T = tables.separable_table(wc, N, fov, S, O, c1)
    y = d['V'] * d['W']
    D = imaging.image_from_grid(gridder.grid_separable(q, y, T, N, S), c1, fov)
    uh, vh = quantise.dequantised(q, N, fov, O)
    ref = dft.dirty(uh, vh, wc[q['k']], y, N, fov, dft.phase_screen(N, fov, 'sep'))
    inner = slice(N // 4, 3 * N // 4)
    err = np.linalg.norm((D - ref)[inner, inner]) / np.linalg.norm(ref[inner, inner])
    assert err < 1e-2
