"""Shared helpers for the GPU parity tests: device transfer, oracle pipelines
for the same inputs, and error measures.  Inputs come from the seeded
generators; expected values come from the oracle only."""
import math

import numpy as np

import oracle


def dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype)


def rel_rms(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def inner(a):
    N = a.shape[0]
    s = slice(N // 4, 3 * N // 4)
    return a[s, s]


def coverage_max(q, N, S):
    """Largest number of kept footprints (S x S cells at cell - S//2 ..) that
    cover one cell of the N x N grid: the number of FP32 terms summed into the
    heaviest cell."""
    keep = ~q['dropped']
    if not keep.any():
        return 0
    h = S // 2
    cu, cv = q['cell_u'][keep], q['cell_v'][keep]
    d = np.zeros((N + 1, N + 1), np.int64)
    np.add.at(d, (cv - h, cu - h), 1)
    np.add.at(d, (cv - h, cu + h + 1), -1)
    np.add.at(d, (cv + h + 1, cu - h), -1)
    np.add.at(d, (cv + h + 1, cu + h + 1), 1)
    return int(d.cumsum(0).cumsum(1).max())


def grid_bound(kmax):
    """FP32 gridding bound, relative RMS: 1e-6, or sqrt(K) 2^-24 where the
    heaviest cell sums K terms and that is larger (the rounding of a K-term
    FP32 sum with random signs grows as sqrt(K) times the unit roundoff)."""
    return max(1e-6, math.sqrt(kmax) * 2.0 ** -24)


class OracleSetup:
    """Oracle tables, taper and bins for one parameter set."""

    def __init__(self, u, v, w, N, fov, S, O, P, w_lo, w_hi, tile_c, width=None, a=0.5,
                 b=5.0 / 24.0, facet=None, taper="pswf"):
        self.N, self.fov, self.S, self.O, self.P = N, fov, S, O, P
        if taper == "none":
            self.c1 = np.ones(N)
        else:
            self.c1 = oracle.pswf.taper_c1(N, fov, S if width is None else width)
        self.facet = facet
        wc = oracle.tables.w_plane_centres(P, w_lo, w_hi)
        if facet is not None:
            l0, m0 = facet
            n0, a_l, a_m = oracle.facet.facet_coefficients(l0, m0)
            u2, v2, w2, _ = oracle.facet.facet_rotate(u, v, w, np.ones(len(u), complex), l0, m0)
            self.q = oracle.quantise.quantise(u2, v2, w2, N, fov, O, S, P, w_lo, w_hi, tile_c)
            self.Tu = oracle.tables.separable_table(wc, N, fov, S, O, self.c1, a=a_l, b=0.0)
            self.Tv = oracle.tables.separable_table(wc, N, fov, S, O, self.c1, a=a_m, b=0.0)
            self.uvw = (u, v, w)
        else:
            self.q = oracle.quantise.quantise(u, v, w, N, fov, O, S, P, w_lo, w_hi, tile_c)
            self.Tu = oracle.tables.separable_table(wc, N, fov, S, O, self.c1, a=a, b=b)
            self.Tv = self.Tu

    def weighted(self, V, W):
        y = np.asarray(V, complex) * np.asarray(W, float)
        if self.facet is not None:
            u, v, w = self.uvw
            _, _, _, y = oracle.facet.facet_rotate(u, v, w, y, *self.facet)
        return y

    def grid(self, V, W):
        return oracle.gridder.grid_separable(self.q, self.weighted(V, W), self.Tu, self.N, self.S,
                                             Tv=self.Tv)

    def image(self, V, W, n_power=0):
        G = self.grid(V, W)
        D = oracle.geometry.fplus(G) / (self.c1[None, :] * self.c1[:, None])
        if n_power:
            l0, m0 = self.facet if self.facet is not None else (0.0, 0.0)
            l = oracle.geometry.pixel_l(self.N, self.fov)
            n = np.sqrt(1 - (l0 + l[None, :]) ** 2 - (m0 + l[:, None]) ** 2)
            D = D * n ** n_power
        return D

    def degrid_grid(self, G):
        V = oracle.gridder.degrid_separable(self.q, G, self.Tu, self.N, self.S, Tv=self.Tv)
        if self.facet is not None:
            u, v, w = self.uvw
            _, _, _, rot = oracle.facet.facet_rotate(u, v, w, np.ones(len(u), complex), *self.facet)
            V = V * np.conj(rot)
        return V

    def degrid_image(self, X, n_power=0):
        Y = np.asarray(X, complex) / (self.c1[None, :] * self.c1[:, None])
        if n_power:
            l0, m0 = self.facet if self.facet is not None else (0.0, 0.0)
            l = oracle.geometry.pixel_l(self.N, self.fov)
            n = np.sqrt(1 - (l0 + l[None, :]) ** 2 - (m0 + l[:, None]) ** 2)
            Y = Y * n ** n_power
        return self.degrid_grid(oracle.geometry.fminus(Y))

    def coverage_max(self):
        """Largest number of kept footprints that cover one grid cell."""
        return coverage_max(self.q, self.N, self.S)

    def grid_bound(self):
        return grid_bound(self.coverage_max())

    def bins_array(self):
        q = self.q
        out = np.stack([q['cell_u'], q['fi_u'], q['cell_v'], q['fi_v'], q['k'], q['tile'],
                        q['dropped'].astype(np.int64)], axis=1)
        out[q['dropped']] = [0, 0, 0, 0, 0, -1, 1]
        return out
