"""Image-plane facet preprocessing (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4.1: for a facet centred at l0 = (l0, m0) with n0 = h(l0) and
h(x) = sqrt(1 - |x|^2), the w screen relative to the facet centre is
exp(2 pi i w [h(l0 + l) - n0]).  Its Taylor expansion about l0 has

* a linear term  -(l0 . l)/n0, absorbed by the coordinate change
  u' = u - w l0 / n0  (and v' = v - w m0 / n0);
* separable quadratic terms  -1/2 (1/n0 + l0^2/n0^3) l^2  and
  -1/2 (1/n0 + m0^2/n0^3) m^2, handled by the facet tables g^l_w and g^m_w;
* a cross term -(l0 m0 / n0^3) l m, which is not separable and is dropped,
  as are higher orders (no l^4 term: b = 0).

The paper prints only u'.  Reading for the visibility phase (derived by
evaluating the dirty-image equation at l0 + l): writing
w (n - 1) = w (n - n0) + w (n0 - 1) gives
    V' = W V exp(+2 pi i (u l0 + v m0 + w (n0 - 1))),
after which facet pixel p stands for direction l0 + l_p.
"""
import numpy as np


def facet_coefficients(l0, m0):
    """(n0, a_l, a_m) for the facet tables; b = 0 for both axes."""
    n0 = np.sqrt(1.0 - l0 * l0 - m0 * m0)
    a_l = 0.5 * (1.0 / n0 + l0 * l0 / n0 ** 3)
    a_m = 0.5 * (1.0 / n0 + m0 * m0 / n0 ** 3)
    return n0, a_l, a_m


def facet_rotate(u, v, w, y, l0, m0):
    """(u', v', w, y') for one facet."""
    n0 = np.sqrt(1.0 - l0 * l0 - m0 * m0)
    y2 = y * np.exp(2j * np.pi * (u * l0 + v * m0 + w * (n0 - 1.0)))
    return u - w * l0 / n0, v - w * m0 / n0, w, y2

