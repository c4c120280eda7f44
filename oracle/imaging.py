"""Grid correction and the grid <-> image steps around the FFT (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2: with an anti-aliasing kernel C (inverse transform c) the dirty image
is  I_D/n = F^-1[sum_i V^W_i * G_{w_i} * C] / c.  With the separable taper of
Section 3, c(l_p, m_q) = c1(l_p) c1(m_q).  The factor n:

* dirty image (Section 2):   I_D = n * D,      D = F+[G] / (c1 c1)
* model for prediction:      X = I / n          (prediction equation)
* adjoint pair: grid with D/n and degrid with X = I/n are exact adjoints,
  because 1/(n c1 c1) is real and diagonal.  (Reading: the paper states only
  the dirty-image and prediction equations.)

``n_power`` is the exponent applied to n: +1, -1 or 0.
"""
import numpy as np

from .geometry import fplus, fminus, n_image


def image_from_grid(G, c1, fov, n_power=0):
    N = G.shape[0]
    D = fplus(G) / (c1[None, :] * c1[:, None])
    if n_power:
        D = D * n_image(N, fov) ** n_power
    return D


def grid_from_image(X, c1, fov, n_power=0):
    N = X.shape[0]
    Y = X / (c1[None, :] * c1[:, None])
    if n_power:
        Y = Y * n_image(N, fov) ** n_power
    return fminus(Y)
