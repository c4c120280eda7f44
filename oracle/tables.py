"""Oversampled GCF lookup tables (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2: the GCF F_w is the Fourier transform of g_w * c, sampled on an
oversampled grid and stored as a lookup table.  Section 3: g_w is replaced by
the separable g~_w(l,m) = g1_w(l) g1_w(m) with
    g1_w(l) = exp(2 pi i w [-1/2 l^2 - gamma l^4]),
so one 1D table per w-plane replaces the 2D one.  Section 4.1 (facets) uses
g^l_w(l) = exp(2 pi i w [-a_l l^2]) and g^m_w(m) = exp(2 pi i w [-a_m m^2]);
both are covered by the general axis phase  -(a l^2 + b l^4).

Reading of how the GCF is sampled (the paper only says "sampled"): the table
entry for grid offset Delta (in cells) is the inverse of the centred F+ of the
image-domain function over the N image pixels,
    T(Delta) = (1/N) sum_{p<N} c1(l_p) exp(-2 pi i w (a l_p^2 + b l_p^4))
                         * exp(-2 pi i Delta (p - N/2) / N),
so that sum_s T(s - h - f/O) exp(+2 pi i (s - h - f/O)(p - N/2)/N) reproduces
c1(l_p) g1_w(l_p) exactly when s runs over N consecutive cells (full support)
and approximately (truncation) for support S < N.

Table layout: T[k][fi][s], k = w-plane, fi = f + O/2 with f in [-O/2, O/2) the
sub-cell offset of the visibility in 1/O cells, s in [0, S) the tap; the tap
sits at grid cell  cell - h + s  with h = floor(S/2), i.e. at offset
Delta = s - h - f/O from the visibility.

w-planes (reading; the paper gives only a count): P uniform planes on
[w_lo, w_hi], plane k represents w_k = w_lo + (k + 1/2)(w_hi - w_lo)/P.
"""
import numpy as np

from .geometry import pixel_l


def w_plane_centres(P, w_lo, w_hi):
    """w value represented by each of P uniform planes on [w_lo, w_hi]."""
    k = np.arange(P, dtype=np.float64)
    return w_lo + (k + 0.5) * (w_hi - w_lo) / P


def tap_offsets(S, O):
    """Delta[fi][s] = s - floor(S/2) - (fi - floor(O/2))/O, in grid cells."""
    h = S // 2
    fi = np.arange(O, dtype=np.float64)
    s = np.arange(S, dtype=np.float64)
    return (s[None, :] - h) - (fi[:, None] - O // 2) / O


def axis_screen(w, N, fov, c1, a, b):
    """c1(l_p) * exp(-2 pi i w (a l_p^2 + b l_p^4)) for every pixel p."""
    l = pixel_l(N, fov)
    return c1 * np.exp(-2j * np.pi * w * (a * l ** 2 + b * l ** 4))


def separable_table(w_centres, N, fov, S, O, c1, a=0.5, b=5.0 / 24.0):
    """T[k][fi][s] (complex128) for each plane centre w_k: the 1D GCF table.

    Direct sum over the N image pixels (no FFT), following the formula in the
    module docstring; a = 1/2, b = gamma = 5/24 by default (Section 3: the
    minimax choice of gamma).
    """
    p = np.arange(N, dtype=np.float64)
    D = tap_offsets(S, O)                                     # [O][S]
    E = np.exp(-2j * np.pi * D[..., None] * (p - N / 2) / N)  # [O][S][N]
    out = np.empty((len(w_centres), O, S), dtype=np.complex128)
    for k, w in enumerate(w_centres):
        A = axis_screen(w, N, fov, c1, a, b)                  # [N]
        out[k] = (E @ A) / N
    return out


def exact_table_2d(w_centres, N, fov, S, O, c1, l0=0.0, m0=0.0):
    """Non-separable reference table T2[k][fu][fv][su][sv] (tiny sizes only).

    Uses the exact phase screen g_w = exp(2 pi i w (n - 1)) of Section 2 with a
    separable taper c1(l) c1(m); with a facet centre (l0, m0) the screen is
    Section 4.1's exp(2 pi i w [h(l0+l, m0+m) - n0]) after removing the linear
    term that the facet coordinate shift absorbs:
        phase = w [h(l0+l, m0+m) - n0 + (l0 l + m0 m)/n0].
    """
    l = pixel_l(N, fov)
    L, M = l[None, :], l[:, None]                            # [q][p]
    n0 = np.sqrt(1.0 - l0 * l0 - m0 * m0)
    n = np.sqrt(1.0 - (l0 + L) ** 2 - (m0 + M) ** 2)
    base = n - n0 + (l0 * L + m0 * M) / n0
    p = np.arange(N, dtype=np.float64)
    D = tap_offsets(S, O)
    E = np.exp(-2j * np.pi * D[..., None] * (p - N / 2) / N)  # [O][S][N]
    taper = c1[None, :] * c1[:, None]                         # [q][p]
    out = np.empty((len(w_centres), O, O, S, S), dtype=np.complex128)
    for k, w in enumerate(w_centres):
        A = taper * np.exp(2j * np.pi * w * base)              # A[q][p]
        # T2[fu][fv][su][sv] = (1/N^2) sum_{q,p} E[fv][sv][q] A[q][p] E[fu][su][p]
        out[k] = np.einsum('xsp,qp,ytq->xyst', E, A, E, optimize=True) / (N * N)
    return out
