"""Prolate spheroidal wave function taper (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2 combines W projection with an anti-aliasing kernel C whose inverse
transform c divides the image; Section 3 assumes c separable, c(l,m) =
c1(l) c1(m).  The paper does not name the taper.  Reading used here (the usual
choice in radio imaging): c1 is the zeroth prolate spheroidal wave function
psi_0(c, x) with x = 2 l / fov in [-1, 1) and bandwidth parameter
c = pi * W / 2, where W is the width of the anti-aliasing kernel in grid cells
(default: the GCF support S).  c1 is normalised so that c1(0) = 1.

psi_0 is computed by the Legendre-series method: expand psi in normalised
Legendre functions; the prolate differential operator
    L psi = -d/dx[(1 - x^2) dpsi/dx] + c^2 x^2 psi
is symmetric tridiagonal in that basis (even degrees couple only to even
degrees), and psi_0 is the eigenvector of its smallest eigenvalue.
"""
import numpy as np


def _n_terms(c):
    # The coefficients decay faster than geometrically once the degree passes
    # about c; 2c + 40 even degrees (up to degree 4c + 78) is ample.
    return int(2 * c + 40)


def legendre_coefficients(c):
    """Coefficients d_k (k = 0, 2, 4, ...) of psi_0 in normalised Legendre functions.

    Matrix of L in the basis Pbar_k = sqrt(k + 1/2) P_k restricted to even k:
      diag:   k(k+1) + c^2 (2k(k+1) - 1) / ((2k+3)(2k-1))
      off:    c^2 (k+1)(k+2) / ((2k+3) sqrt((2k+1)(2k+5)))   between k and k+2
    (from x^2 P_k expanded by the three-term Legendre recurrence).
    """
    m = _n_terms(c)
    k = 2.0 * np.arange(m)
    diag = k * (k + 1) + c * c * (2 * k * (k + 1) - 1) / ((2 * k + 3) * (2 * k - 1))
    kk = k[:-1]
    off = c * c * (kk + 1) * (kk + 2) / ((2 * kk + 3) * np.sqrt((2 * kk + 1) * (2 * kk + 5)))
    A = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    evals, evecs = np.linalg.eigh(A)
    d = evecs[:, 0]
    # fix the sign so that psi_0(0) > 0
    if _series(d, np.array([0.0]))[0] < 0:
        d = -d
    return d


def _series(d, x):
    """sum_k d_k Pbar_{2k}(x) via the Legendre three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)  # P_0
    p_cur = x.copy()          # P_1
    out = d[0] * np.sqrt(0.5) * p_prev
    nmax = 2 * (len(d) - 1)
    for n in range(1, nmax):
        # P_{n+1} = ((2n+1) x P_n - n P_{n-1}) / (n+1)
        p_next = ((2 * n + 1) * x * p_cur - n * p_prev) / (n + 1)
        p_prev, p_cur = p_cur, p_next
        deg = n + 1
        if deg % 2 == 0:
            out = out + d[deg // 2] * np.sqrt(deg + 0.5) * p_cur
    return out


def psi0(c, x):
    """psi_0(c, x), normalised so that psi_0(c, 0) = 1."""
    d = legendre_coefficients(c)
    return _series(d, x) / _series(d, np.array([0.0]))[0]


def taper_c1(N, fov, width):
    """c1(l_p) = psi_0(c, 2 l_p / fov) with c = pi * width / 2, at every pixel p."""
    p = np.arange(N, dtype=np.float64)
    x = 2.0 * (p - N / 2) / N          # = 2 l_p / fov exactly
    return psi0(np.pi * width / 2.0, x)
