"""Pins for the oracle's W snapshots (Section 4.2).

* The plane fit recovers an exactly planar w = u . d (and returns 0 for a
  degenerate snapshot); the residuals then vanish.
* Keys' cubic convolution reproduces quadratics exactly, sums to one and is
  the identity at whole pixels.
* A snapshot whose w is 0 reprojects by the identity: the hybrid equals the
  plain separable path.
* A point source seen by a coplanar array lands, after reprojection, on its own
  pixel, while the snapshot image before reprojection is displaced by
  d0 (n - 1) (full support, so the snapshot image is the exact DFT in l^s).
* Imaging and prediction are adjoint (FP64).
"""
import math

import numpy as np
import pytest

from oracle import geometry, gridder, imaging, pswf, quantise, tables, wsnap

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_plane_fit_recovers_a_plane_and_degenerate_cases():
    rng = np.random.default_rng(3)
    u, v = rng.uniform(-2e3, 2e3, (2, 500))
    d = (0.73, -1.9)
    w = d[0] * u + d[1] * v
    du, dv = wsnap.fit_plane(u, v, w)
    assert abs(du - d[0]) < 1e-12 and abs(dv - d[1]) < 1e-12
    d0, wr, h = wsnap.residuals(u, v, w, [0, 200, 500])
    assert np.max(np.abs(wr)) < 1e-9 and np.allclose(d0, [d, d], atol=1e-12)
    assert wsnap.fit_plane(u[:1], v[:1], w[:1]) == (0.0, 0.0)             # one point
    assert wsnap.fit_plane(u[:9], 2 * u[:9], w[:9]) == (0.0, 0.0)          # collinear uv
    # non-finite coordinates are left out of the fit
    u2, w2 = u.copy(), w.copy()
    u2[7], w2[9] = np.nan, np.inf
    du2, dv2 = wsnap.fit_plane(u2, v, w2)
    assert abs(du2 - d[0]) < 1e-12 and abs(dv2 - d[1]) < 1e-12


def test_keys_kernel_properties():
    rng = np.random.default_rng(5)
    N = 40
    x = rng.uniform(2, N - 3, 300)
    idx, wts = wsnap._taps(x, N)
    assert np.allclose(wts.sum(axis=1), 1.0, atol=1e-14)
    for c in ([1.0, 0, 0], [0.3, -2.0, 0], [-1.0, 0.7, 0.05]):
        g = lambda t: c[0] + c[1] * t + c[2] * t * t  # noqa: E731
        assert np.allclose(np.sum(wts * g(idx), axis=1), g(x), rtol=0, atol=1e-11)
    idx, wts = wsnap._taps(np.arange(2.0, 10.0), N)
    assert np.array_equal(wts, np.tile([0.0, 1.0, 0.0, 0.0], (8, 1)))
    assert wsnap.keys(2.0) == 0 and wsnap.keys(1.0) == 0 and wsnap.keys(0.0) == 1


def test_zero_w_reprojects_by_the_identity():
    N, fov, S, O, P = 48, 0.4, 7, 8, 3
    rng = np.random.default_rng(9)
    u, v = rng.uniform(-18, 18, (2, 400)) / fov
    w = np.zeros(400)
    y = rng.standard_normal(400) + 1j * rng.standard_normal(400)
    c1 = pswf.taper_c1(N, fov, S)
    D = wsnap.image(u, v, w, y, [0, 150, 400], N, fov, S, O, P, c1)
    T = tables.separable_table(tables.w_plane_centres(P, -1.0, 1.0), N, fov, S, O, c1)
    q = quantise.quantise(u, v, w, N, fov, O, S, P, -1.0, 1.0, 1)
    ref = imaging.image_from_grid(gridder.grid_separable(q, y, T, N, S), c1, fov)
    # the taper correction amplifies FP64 rounding by 1 / (c1 c1) towards the edges
    amp = 1.0 / (c1[None, :] * c1[:, None])
    assert np.all(np.abs(D - ref) <= 1e-12 * np.max(np.abs(ref)) * amp)


def test_point_source_lands_on_its_pixel():
    N, fov, O = 64, 0.6, 8
    rng = np.random.default_rng(11)
    u, v = rng.uniform(-N / 2 + 1, N / 2 - 1, (2, 3000)) / fov
    d = (3.0, -2.0)
    w = d[0] * u + d[1] * v                   # coplanar snapshot: w' = 0
    p0, q0 = N // 2 + 14, N // 2 - 11         # the source's pixel
    l0, m0 = geometry.pixel_l(N, fov)[p0], geometry.pixel_l(N, fov)[q0]
    n0 = math.sqrt(1 - l0 * l0 - m0 * m0)
    y = np.exp(-2j * np.pi * (u * l0 + v * m0 + w * (n0 - 1)))
    c1 = np.ones(N)
    # full support (S = N, indices modulo N): the snapshot image is the exact
    # DFT in the coordinate l^s
    d0, wr, h = wsnap.residuals(u, v, w, [0, len(u)])
    q = quantise.quantise(u, v, wr, N, fov, O, 1, 1, -h, h, 1)
    q['dropped'] = np.zeros_like(q['dropped'])
    T = tables.separable_table(tables.w_plane_centres(1, -h, h), N, fov, N, O, c1)
    Ds = imaging.image_from_grid(gridder.grid_separable(q, y, T, N, N, wrap=True), c1, fov)
    R = wsnap.reproject(Ds, N, fov, d0[0])
    assert np.unravel_index(np.argmax(np.abs(R)), R.shape) == (q0, p0)
    assert np.unravel_index(np.argmax(np.abs(Ds)), Ds.shape) != (q0, p0)
    # the peak is sampled between pixels of the snapshot image, so cubic
    # interpolation keeps most but not all of its height
    assert abs(R[q0, p0]) > 0.6 * len(u)


@pytest.mark.parametrize("n_power", [0, 1])
def test_image_and_predict_are_adjoint(n_power):
    N, fov, S, O, P = 32, 0.5, 7, 8, 4
    rng = np.random.default_rng(13)
    u, v = rng.uniform(-10, 10, (2, 600)) / fov
    w = 0.8 * u - 0.5 * v + rng.normal(0, 3.0, 600)
    y = rng.standard_normal(600) + 1j * rng.standard_normal(600)
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    c1 = pswf.taper_c1(N, fov, S)
    offs = [0, 250, 250, 600]                  # an empty snapshot in the middle
    D = wsnap.image(u, v, w, y, offs, N, fov, S, O, P, c1, n_power)
    V = wsnap.predict(u, v, w, X, offs, N, fov, S, O, P, c1, n_power)
    assert abs(np.vdot(X, D) - np.vdot(V, y)) <= 1e-12 * np.linalg.norm(D) * np.linalg.norm(X)
