"""Separable phase-error factor epsilon (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3: replacing g_w by g~_w leaves an image-space phase error
Delta phi = 2 pi w eps(l, m) with
    eps = -(1/2 l^2 + gamma l^4 + 1/2 m^2 + gamma m^4) - (sqrt(1 - l^2 - m^2) - 1)
        = (1/8 - gamma)(l^4 + m^4) + 1/4 l^2 m^2 + O(l^6 + m^6).
gamma = 5/24 minimises the maximum of the quartic part over the image at
m_max^4 / 12; gamma = 1/8 is accurate on the axes.
"""
import numpy as np


def eps_exact(l, m, gamma):
    return -(0.5 * l ** 2 + gamma * l ** 4 + 0.5 * m ** 2 + gamma * m ** 4) - (np.sqrt(1.0 - l ** 2 - m ** 2) - 1.0)


def eps_quartic(l, m, gamma):
    return (0.125 - gamma) * (l ** 4 + m ** 4) + 0.25 * l ** 2 * m ** 2


def max_abs_eps(fov, gamma, n=801):
    """max |eps| over the square image |l|, |m| <= fov/2 (dense sampling; the
    maximum lies on the boundary, which is sampled exactly)."""
    x = np.linspace(-fov / 2, fov / 2, n)
    L, M = np.meshgrid(x, x)
    return np.abs(eps_exact(L, M, gamma)).max()
