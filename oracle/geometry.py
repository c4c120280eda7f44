"""Image/uv geometry and the centred transforms between grid and image (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (readings of the paper, Section 2, where it only names F^-1):

* The field of view ``fov`` is the full image width in direction cosines, so
  ``l`` runs over [-fov/2, fov/2) (Section 3 quotes m = 2 deg for a 4 deg field).
* Pixel p (0 <= p < N) sits at l_p = (p - N/2) * fov / N.
* Grid cell j sits at u_j = (j - N/2) / fov, so the cell size is 1/fov.
* Arrays are row-major with rows along m (image) or v (grid): D[q][p], G[jv][ju].
* Grid to image uses the sign of the dirty-image equation, e^{+2 pi i u.l},
  unnormalised:  F+[G](p,q) = sum_j G[jv][ju] exp(+2 pi i [(ju-N/2)(p-N/2) +
  (jv-N/2)(q-N/2)] / N).  F- is its conjugate transpose (sign -, unnormalised).
"""
import numpy as np


def pixel_l(N, fov):
    """Direction cosine of each pixel centre, l_p = (p - N/2) fov / N."""
    p = np.arange(N, dtype=np.float64)
    return (p - N / 2) * (fov / N)


def cell_u(N, fov):
    """uv coordinate (wavelengths) of each grid cell centre, u_j = (j - N/2)/fov."""
    j = np.arange(N, dtype=np.float64)
    return (j - N / 2) / fov


def n_of_lm(l, m):
    """n = sqrt(1 - l^2 - m^2) (Section 2)."""
    return np.sqrt(1.0 - l * l - m * m)


def n_image(N, fov):
    """n(l_p, m_q) on the image grid, indexed [q][p]."""
    l = pixel_l(N, fov)
    return n_of_lm(l[None, :], l[:, None])


def fplus(G):
    """F+ : grid -> image, exp(+2 pi i ...), unnormalised, centred at N/2.

    Uses the FFT library as a primitive; ``fplus_direct`` is the same sum
    written out and is used to pin this one on small N.
    """
    N = G.shape[0]
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(G))) * (N * N)


def fminus(X):
    """F- : image -> grid, exp(-2 pi i ...), unnormalised; adjoint of F+."""
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(X)))


def _centred_dft_matrix(N, sign):
    j = np.arange(N) - N / 2
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / N)


def fplus_direct(G):
    """F+ by an explicit double sum (brute force, small N only)."""
    N = G.shape[0]
    E = _centred_dft_matrix(N, +1.0)  # E[j][p]
    # D[q][p] = sum_{jv, ju} E[jv][q] G[jv][ju] E[ju][p]
    return E.T @ G @ E


def fminus_direct(X):
    """F- by an explicit double sum (brute force, small N only)."""
    N = X.shape[0]
    E = _centred_dft_matrix(N, -1.0)
    return E.T @ X @ E
