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


# ---- non-uniform slices (Section 4.3: narrow slices where w is dense)

EDGES = np.array([-1500.0, -400.0, -50.0, 0.0, 30.0, 700.0, 1500.0])


def test_nonuniform_slice_centred_full_support_equals_exact_dft():
    N, O, fov = 16, 4, math.radians(9.0)
    ns = len(EDGES) - 1
    rng, u, v, y = _vis(53, N, fov, 40, N / 2 - 1)
    k = rng.integers(0, ns, len(u))
    w = (EDGES[k] + EDGES[k + 1]) * 0.5           # exactly at the slice centres
    c1 = pswf.taper_c1(N, fov, 5.0)
    D = wstack.image(u, v, w, y, N, fov, N, O, 1, ns, EDGES[0], EDGES[-1], c1, bins=_full_bins,
                     wrap=True, edges=EDGES)
    q = _full_bins(u, v, w, N, fov, O, N, 1, -1.0, 1.0)
    uh, vh = quantise.dequantised(q, N, fov, O)
    ref = dft.dirty(uh, vh, w, y, N, fov, dft.phase_screen(N, fov, 'exact'))
    assert _close(D, ref, c1)


def test_nonuniform_residual_planes_use_each_slices_range():
    N, O, P, fov = 16, 4, 3, math.radians(8.0)
    ns = len(EDGES) - 1
    rng, u, v, y = _vis(59, N, fov, 80, N / 2 - 1)
    w = rng.uniform(-1600.0, 1600.0, len(u))      # some below e_0 and above e_ns
    c1 = pswf.taper_c1(N, fov, 6.0)
    D = wstack.image(u, v, w, y, N, fov, N, O, P, ns, EDGES[0], EDGES[-1], c1, bins=_full_bins,
                     wrap=True, edges=EDGES)
    # reference: per slice, the exact phase of its centre times the
    # separable-screen DFT at the centre of its residual plane, the planes
    # spanning that slice's own half-width
    exact = dft.phase_screen(N, fov, 'exact')
    sep = dft.phase_screen(N, fov, 'sep')
    ref = np.zeros((N, N), complex)
    for s in range(ns):
        lo = -np.inf if s == 0 else EDGES[s]
        hi = np.inf if s == ns - 1 else EDGES[s + 1]
        ws = (EDGES[s] + EDGES[s + 1]) / 2
        h = (EDGES[s + 1] - EDGES[s]) / 2
        wc = tables.w_plane_centres(P, -h, h)
        m = (w >= lo) & (w < hi)
        q = _full_bins(u[m], v[m], w[m] - ws, N, fov, O, N, P, -h, h)
        uh, vh = quantise.dequantised(q, N, fov, O)
        ref += np.exp(2j * np.pi * ws * exact) * dft.dirty(uh, vh, wc[q['k']], y[m], N, fov, sep)
    assert _close(D, ref, c1)


def test_nonuniform_image_and_predict_are_adjoint():
    N, O, P, S, fov = 32, 8, 4, 7, math.radians(6.0)
    ns = len(EDGES) - 1
    rng, u, v, y = _vis(61, N, fov, 300, N / 2 - 5)
    w = rng.uniform(-1500.0, 1500.0, len(u))
    c1 = pswf.taper_c1(N, fov, S)
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    D = wstack.image(u, v, w, y, N, fov, S, O, P, ns, -1500.0, 1500.0, c1, n_power=-1,
                     edges=EDGES)
    V = wstack.predict(u, v, w, X, N, fov, S, O, P, ns, -1500.0, 1500.0, c1, n_power=-1,
                       edges=EDGES)
    assert abs(np.vdot(X, D) - np.vdot(V, y)) <= 1e-12 * np.linalg.norm(D) * np.linalg.norm(X)


def test_uniform_edges_are_the_uniform_slices():
    N, O, P, S, ns, fov = 32, 8, 4, 7, 5, math.radians(6.0)
    w_lo, w_hi = -900.0, 900.0
    rng, u, v, y = _vis(67, N, fov, 300, N / 2 - 5)
    w = rng.uniform(w_lo, w_hi, len(u))
    c1 = pswf.taper_c1(N, fov, S)
    e = w_lo + np.arange(ns + 1) * (w_hi - w_lo) / ns
    s0, _, _ = wstack.slice_of(w, ns, w_lo, w_hi)
    s1, _, _ = wstack.slice_of(w, ns, w_lo, w_hi, e)
    assert np.array_equal(s0, s1)
    D0 = wstack.image(u, v, w, y, N, fov, S, O, P, ns, w_lo, w_hi, c1)
    D1 = wstack.image(u, v, w, y, N, fov, S, O, P, ns, w_lo, w_hi, c1, edges=e)
    assert np.linalg.norm(D1 - D0) <= 1e-12 * np.linalg.norm(D0)


def _density_edges_brute(w, ns, w_lo, w_hi, nfine):
    # every candidate boundary tried in turn, counts by direct comparison of
    # the fine-bin indices
    fin = [x for x in w if math.isfinite(x)]
    n = len(fin)
    d = (w_hi - w_lo) / nfine
    idx = []
    for x in fin:
        t = math.floor((x - w_lo) * (nfine / (w_hi - w_lo)))
        idx.append(min(max(t, 0), nfine - 1))
    e = [w_lo]
    prev = 0
    for k in range(1, ns):
        j = 0
        while sum(1 for t in idx if t < j) * ns < k * n:
            j += 1
        j = min(max(j, prev + 1), nfine - (ns - k))
        e.append(w_lo + j * d)
        prev = j
    e.append(w_hi)
    return np.array(e)


@pytest.mark.parametrize("ns", [1, 2, 5, 9])
def test_density_edges_match_brute_force(ns):
    rng = np.random.default_rng(71 + ns)
    w = np.r_[rng.laplace(0.0, 40.0, 300), rng.uniform(-1000, 1000, 40), np.nan, np.inf]
    e = wstack.density_edges(w, ns, -1000.0, 1000.0, nfine=64)
    assert np.array_equal(e, _density_edges_brute(w, ns, -1000.0, 1000.0, 64))
    assert np.all(np.diff(e) > 0)


def test_density_edges_balance_counts_and_narrow_where_dense():
    rng = np.random.default_rng(73)
    w = rng.laplace(0.0, 300.0, 200_000)
    w = w[np.abs(w) < 5000]
    ns, nfine = 8, 4096
    e = wstack.density_edges(w, ns, -5000.0, 5000.0, nfine)
    s, _, _ = wstack.slice_of(w, ns, -5000.0, 5000.0, e)
    counts = np.bincount(s, minlength=ns)
    # each slice within one fine bin's worth of the equal share (density is
    # at most ~ n / (2 * 300) per unit w, a fine bin is 10000 / 4096 wide)
    slack = len(w) / (2 * 300.0) * (10000.0 / nfine) + 1
    assert np.all(np.abs(counts - len(w) / ns) <= slack)
    widths = np.diff(e)
    # narrowest slices straddle w = 0, widest at the ends
    assert widths[ns // 2 - 1] < widths[0] / 5 and widths[ns // 2] < widths[-1] / 5


def test_slice_of_edges_at_the_boundaries():
    # a w equal to an edge belongs to the slice above it; w = e_ns to the last
    ns = len(EDGES) - 1
    s, ws, dw = wstack.slice_of(EDGES, ns, EDGES[0], EDGES[-1], EDGES)
    assert list(s) == list(range(ns)) + [ns - 1]
    assert np.array_equal(dw, EDGES - ws[s])
    s, _, dw = wstack.slice_of(np.array([-2e4, 2e4, np.nan, -np.inf]), ns, EDGES[0], EDGES[-1], EDGES)
    assert list(s) == [0, ns - 1, 0, 0] and not np.isfinite(dw[2:]).any()


def test_density_edges_on_exact_shares():
    # 10 visibilities in each of fine bins 5, 10, 20 and 40 of 64 over [0, 64):
    # with 4 slices each share (10) is reached exactly at the boundary after
    # each occupied bin, which is where the edges go
    w = np.repeat([5.5, 10.5, 20.5, 40.5], 10)
    e = wstack.density_edges(w, 4, 0.0, 64.0, nfine=64)
    assert list(e) == [0.0, 6.0, 11.0, 21.0, 64.0]
