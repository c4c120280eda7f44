"""Pins for the oracle's geometry, taper, DFT and phase-error pieces.

Each test checks the oracle against something other than itself: a brute-force
sum, an independent library routine, a closed form, or a number the paper
prints (tests/golden/paper_values.json).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import dft, geometry, phase_error, pswf

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---------------------------------------------------------------- geometry
@pytest.mark.parametrize("N", [8, 16, 30])
def test_fplus_matches_brute_force(N):
    rng = np.random.default_rng(1)
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    assert np.allclose(geometry.fplus(G), geometry.fplus_direct(G), rtol=0, atol=1e-10 * N * N)
    assert np.allclose(geometry.fminus(G), geometry.fminus_direct(G), rtol=0, atol=1e-10 * N * N)


def test_fplus_single_cell_is_plane_wave():
    # one unit cell at (jv, ju) gives exp(+2 pi i [(ju-N/2)(p-N/2) + (jv-N/2)(q-N/2)]/N)
    N, ju, jv = 16, 11, 3
    G = np.zeros((N, N), complex)
    G[jv, ju] = 1
    p = np.arange(N) - N / 2
    want = np.exp(2j * np.pi * ((ju - N / 2) * p[None, :] + (jv - N / 2) * p[:, None]) / N)
    assert np.allclose(geometry.fplus(G), want, atol=1e-12)


def test_fminus_is_adjoint_of_fplus():
    rng = np.random.default_rng(2)
    N = 24
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    lhs = np.vdot(X, geometry.fplus(G))
    rhs = np.vdot(geometry.fminus(X), G)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(G) * np.linalg.norm(X) * N


# ---------------------------------------------------------------- taper
@pytest.mark.parametrize("W", [7, 11, 15])
def test_pswf_matches_scipy(W):
    from scipy.special import pro_ang1
    c = math.pi * W / 2
    x = np.array([0.0, 0.1, 0.25, 0.5, 0.75, 0.9, 0.99, 0.999, -0.3])
    mine = pswf.psi0(c, x)
    ref = np.array([pro_ang1(0, 0, c, xx)[0] for xx in x]) / pro_ang1(0, 0, c, 0.0)[0]
    assert np.max(np.abs(mine - ref)) < 1e-9


@pytest.mark.parametrize("W", [7, 15])
def test_pswf_is_finite_fourier_eigenfunction(W):
    # psi_0 satisfies  int_{-1}^{1} exp(i c x t) psi_0(t) dt = lambda_0 psi_0(x)
    c = math.pi * W / 2
    t, wts = np.polynomial.legendre.leggauss(200)
    psi_t = pswf.psi0(c, t)
    x = np.array([0.0, 0.2, 0.45, 0.7, 0.9])
    lhs = np.array([np.sum(wts * np.exp(1j * c * xx * t) * psi_t) for xx in x])
    lam = lhs / pswf.psi0(c, x)
    assert np.allclose(lam, lam[0], rtol=1e-9)
    assert abs(lam[0].imag) < 1e-12


def test_pswf_even_and_normalised():
    c = math.pi * 11 / 2
    x = np.linspace(0, 1, 17)
    assert np.allclose(pswf.psi0(c, x), pswf.psi0(c, -x), rtol=1e-13, atol=1e-15)
    assert pswf.psi0(c, np.array([0.0]))[0] == pytest.approx(1.0, abs=1e-15)
    c1 = pswf.taper_c1(64, 0.03, 7)
    assert c1[32] == pytest.approx(1.0, abs=1e-15)
    assert np.all(np.diff(c1[32:]) < 0) and np.all(c1 > 0)


# ---------------------------------------------------------------- DFT
def _random_uvw(rng, n, fov, cells, wmax):
    return (rng.uniform(-cells, cells, n) / fov, rng.uniform(-cells, cells, n) / fov,
            rng.uniform(-wmax, wmax, n))


def test_point_source_at_phase_centre_gives_constant_visibilities():
    # prediction equation, Section 2: l = 0, n = 1 -> V_i = flux for every i
    N, fov = 32, math.radians(2.0)
    rng = np.random.default_rng(3)
    u, v, w = _random_uvw(rng, 300, fov, 14, 500)
    X = np.zeros((N, N))
    X[N // 2, N // 2] = 1.0
    V = dft.predict(u, v, w, X, N, fov, dft.phase_screen(N, fov, 'exact'))
    assert np.max(np.abs(V - 1.0)) < 1e-15


def test_point_source_off_centre_closed_form():
    # X = I/n at one pixel (l0, m0): V_i = exp(-2 pi i (u l0 + v m0 + w (n0 - 1))) / n0
    N, fov = 32, math.radians(4.0)
    rng = np.random.default_rng(4)
    u, v, w = _random_uvw(rng, 200, fov, 14, 2000)
    p, q = 27, 5
    l0, m0 = geometry.pixel_l(N, fov)[p], geometry.pixel_l(N, fov)[q]
    n0 = math.sqrt(1 - l0 * l0 - m0 * m0)
    X = np.zeros((N, N))
    X[q, p] = 1.0 / n0
    V = dft.predict(u, v, w, X, N, fov, dft.phase_screen(N, fov, 'exact'))
    want = np.exp(-2j * np.pi * (u * l0 + v * m0 + w * (n0 - 1))) / n0
    assert np.max(np.abs(V - want)) < 1e-13


def test_hermitian_symmetry():
    N, fov = 16, math.radians(3.0)
    rng = np.random.default_rng(5)
    u, v, w = _random_uvw(rng, 60, fov, 7, 300)
    X = rng.standard_normal((N, N))               # real image
    phi = dft.phase_screen(N, fov, 'exact')
    Vp = dft.predict(u, v, w, X, N, fov, phi)
    Vm = dft.predict(-u, -v, -w, X, N, fov, phi)
    assert np.max(np.abs(Vm - np.conj(Vp))) < 1e-12
    # Hermitian-symmetrised visibilities give a real dirty image
    y = rng.standard_normal(60) + 1j * rng.standard_normal(60)
    D = dft.dirty(np.r_[u, -u], np.r_[v, -v], np.r_[w, -w], np.r_[y, np.conj(y)], N, fov, phi)
    assert np.max(np.abs(D.imag)) < 1e-12 * np.max(np.abs(D.real))


@pytest.mark.parametrize("mode", ['exact', 'sep', 'none'])
def test_dft_adjoint_identity(mode):
    N, fov = 16, math.radians(3.0)
    rng = np.random.default_rng(6)
    u, v, w = _random_uvw(rng, 80, fov, 7, 300)
    phi = dft.phase_screen(N, fov, mode)
    y = rng.standard_normal(80) + 1j * rng.standard_normal(80)
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    lhs = np.vdot(X, dft.dirty(u, v, w, y, N, fov, phi))
    rhs = np.vdot(dft.predict(u, v, w, X, N, fov, phi), y)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(y) * np.linalg.norm(X) * N


def test_sep_screen_matches_taylor_of_exact():
    # Section 3: n - 1 = -(l^2+m^2)/2 - (l^2+m^2)^2/8 + O(l^6); the separable
    # screen with gamma = 1/8 keeps everything except the 1/4 l^2 m^2 cross term
    N, fov = 32, math.radians(6.0)
    l = geometry.pixel_l(N, fov)
    L, M = l[None, :], l[:, None]
    diff = dft.phase_screen(N, fov, 'sep', b=0.125) - dft.phase_screen(N, fov, 'exact')
    assert np.allclose(diff, 0.25 * L ** 2 * M ** 2, rtol=0, atol=2 * (fov / 2) ** 6)


# ---------------------------------------------------------------- epsilon
def _golden(golden_dir):
    with open(os.path.join(golden_dir, "paper_values.json")) as f:
        return json.load(f)


def test_eps_minimax_value(golden_dir):
    g = _golden(golden_dir)
    gamma = g["gamma_minimax"]["value"]
    mmax = math.radians(g["fig2_field_deg"]["m_max_deg"])
    want = g["max_eps_over_mmax4"]["value"] * mmax ** 4
    got = phase_error.max_abs_eps(math.radians(g["fig2_field_deg"]["value"]), gamma)
    assert got == pytest.approx(want, rel=0.02)
    # gamma = 5/24 beats gamma = 1/8 on the maximum
    assert got < phase_error.max_abs_eps(math.radians(4.0), g["gamma_axis"]["value"])


def test_eps_gamma_axis_is_sixth_order_on_axis(golden_dir):
    g = _golden(golden_dir)
    l = np.linspace(0.005, 0.05, 10)
    e = phase_error.eps_exact(l, 0 * l, g["gamma_axis"]["value"])
    assert np.allclose(e, l ** 6 / 16, rtol=0.01)


def test_eps_10deg_bound(golden_dir):
    g = _golden(golden_dir)
    got = phase_error.max_abs_eps(math.radians(g["eps_bound_10deg"]["field_deg"]),
                                  g["gamma_minimax"]["value"])
    assert got < g["eps_bound_10deg"]["value"]


def test_eps_quartic_is_leading_term():
    rng = np.random.default_rng(7)
    l, m = rng.uniform(-0.02, 0.02, (2, 100))
    for gamma in (0.125, 5 / 24):
        e = phase_error.eps_exact(l, m, gamma)
        assert np.allclose(e, phase_error.eps_quartic(l, m, gamma), rtol=0, atol=(2 * 0.02 ** 2) ** 3)
