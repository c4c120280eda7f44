"""Chi-squared misfit of a predicted model and its image gradient (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 6: the separable approximation serves prediction as well as imaging,
which is what Cotton-Schwab major cycles need.  For a real model image x the
forward (prediction) operator is
    A x = degrid( F-[ x / (n c1 c1) ] )
and its adjoint is
    A^H r = (1 / (n c1 c1)) F+[ grid(r) ]          (gridding with weights 1).
The misfit and its gradient with respect to the real image x are
    chi2(x)   = sum_i W_i |(A x)_i - Vt_i|^2
    grad(x)   = 2 Re( A^H [ W (A x - Vt) ] ).
"""
import numpy as np

from . import gridder, imaging


class SeparableOperator:
    """A and A^H for fixed bins, tables and taper."""

    def __init__(self, q, T, c1, N, S, fov, Tv=None):
        self.q, self.T, self.Tv, self.c1, self.N, self.S, self.fov = q, T, Tv, c1, N, S, fov

    def forward(self, x):
        Gh = imaging.grid_from_image(x.astype(np.complex128), self.c1, self.fov, n_power=-1)
        return gridder.degrid_separable(self.q, Gh, self.T, self.N, self.S, Tv=self.Tv)

    def adjoint(self, r):
        G = gridder.grid_separable(self.q, r, self.T, self.N, self.S, Tv=self.Tv)
        return imaging.image_from_grid(G, self.c1, self.fov, n_power=-1)


def chi2(op, x, Vt, W):
    r = op.forward(x) - Vt
    keep = ~op.q['dropped']
    return float(np.sum(W[keep] * np.abs(r[keep]) ** 2))


def chi2_grad(op, x, Vt, W):
    r = (op.forward(x) - Vt) * W
    r = np.where(op.q['dropped'], 0, r)
    return 2.0 * np.real(op.adjoint(r))
