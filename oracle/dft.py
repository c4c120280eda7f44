"""Direct evaluation of the dirty-image and prediction equations (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2, dirty image:  I_D(l)/n = sum_i W_i V_i exp(2 pi i (u_i . l + w_i (n - 1))).
Section 2, prediction:   V_i = integral of I(l)/n exp(-2 pi i (u_i . l + w_i (n - 1))) dl.

On the N x N pixel grid the integral is a pixel sum; the pixel area is dropped
(reading, consistent with the unnormalised F- between image and grid).  The
phase function phi replaces (n - 1):

* 'exact':  phi = n - 1                                   (Section 2)
* 'sep':    phi = -(a l^2 + b l^4) - (a m^2 + b m^4)       (Section 3, g~_w)
* 'facet':  phi = -a_l l^2 - a_m m^2                        (Section 4.1)
* 'none':   phi = 0  (no w correction; Section 3's closing remark)

``D`` below is I_D / n, i.e. the quantity gridding + F+ + taper correction
approximates.
"""
import numpy as np

from .geometry import pixel_l


def phase_screen(N, fov, mode, a=0.5, b=5.0 / 24.0, a_m=None, b_m=None):
    """phi(l_p, m_q) indexed [q][p]."""
    l = pixel_l(N, fov)
    L, M = l[None, :], l[:, None]
    if a_m is None:
        a_m = a
    if b_m is None:
        b_m = b
    if mode == 'exact':
        return np.sqrt(1.0 - L * L - M * M) - 1.0
    if mode in ('sep', 'facet'):
        return -(a * L ** 2 + b * L ** 4) - (a_m * M ** 2 + b_m * M ** 4)
    if mode == 'none':
        return np.zeros((N, N))
    raise ValueError(mode)


def dirty(u, v, w, y, N, fov, phi, chunk=512):
    """D[q][p] = sum_i y_i exp(2 pi i (u_i l_p + v_i m_q + w_i phi[q][p]))."""
    l = pixel_l(N, fov)
    D = np.zeros((N, N), dtype=np.complex128)
    for c0 in range(0, len(u), chunk):
        sl = slice(c0, c0 + chunk)
        ph = (u[sl, None, None] * l[None, None, :] + v[sl, None, None] * l[None, :, None]
              + w[sl, None, None] * phi[None, :, :])
        D += np.einsum('i,iqp->qp', y[sl], np.exp(2j * np.pi * ph))
    return D


def predict(u, v, w, X, N, fov, phi, chunk=512):
    """V_i = sum_{q,p} X[q][p] exp(-2 pi i (u_i l_p + v_i m_q + w_i phi[q][p]))."""
    l = pixel_l(N, fov)
    V = np.zeros(len(u), dtype=np.complex128)
    for c0 in range(0, len(u), chunk):
        sl = slice(c0, c0 + chunk)
        ph = (u[sl, None, None] * l[None, None, :] + v[sl, None, None] * l[None, :, None]
              + w[sl, None, None] * phi[None, :, :])
        V[sl] = np.einsum('qp,iqp->i', X, np.exp(-2j * np.pi * ph))
    return V
