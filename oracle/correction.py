"""The correction F_w - F~_w, a small 2D table applied beside the separable
GCF (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 6 proposes storing the difference between the exact GCF F_w and its
separable approximation F~_w as a small full 2D table and applying it in
addition to the separable kernel.  In the image domain that difference is the
taper times the gap between the exact and the separable phase screens,

    c1(l) c1(m) [exp(2 pi i w (n - 1)) - g1_w(l) g1_w(m)],

which is small wherever the separable screen is accurate, so its transform
needs less support and/or a lower oversampling rate than the GCF itself.

Readings (the paper names the idea only):

* The table is sampled like the 1D tables (``tables``: a direct sum over the N
  image pixels) with its own odd support S_c and oversampling O_c (a power of
  two dividing O):

      C[k][fu][fv][su][sv] = (1/N^2) sum_{q,p} c1(l_p) c1(m_q)
          [exp(2 pi i w_k (n_pq - 1)) - exp(-2 pi i w_k (phi_u(l_p) + phi_v(m_q)))]
          exp(-2 pi i [Du (p - N/2) + Dv (q - N/2)] / N),

  Du = su - floor(S_c/2) - (fu - O_c/2)/O_c (Dv likewise), phi(l) = a l^2 +
  b l^4 the separable screen's exponent per axis.  With S_c = S and O_c = O
  this is exactly the exact 2D table minus the outer product of the 1D tables.
* A visibility's correction sample is the point of the 1/O_c lattice nearest to
  its quantised position cell + f/O, ties towards +; in integers, with t =
  cell O + f and r = O / O_c:  t_c = floor((t + floor(r/2)) / r),  cell_c =
  floor((t_c + O_c/2) / O_c),  f_c = t_c - cell_c O_c.  cell_c is cell or
  cell + 1 (always cell when O_c is O or 1), so the correction footprint, S_c
  cells about cell_c, stays inside the separable footprint when S_c <= S - 2
  (S_c <= S when cell_c = cell) and adds no off-grid cases.
* The correction uses the visibility's own w-plane k.
"""
import numpy as np

from . import gridder
from .geometry import pixel_l
from .tables import tap_offsets


def coarse_axis(cell, fi, O, Oc):
    """(cell_c, fi_c) of one axis: nearest point of the 1/O_c lattice."""
    r = O // Oc
    t = cell * O + (fi - O // 2)
    tc = (t + r // 2) // r                 # floor division (NumPy // on int64)
    cc = (tc + Oc // 2) // Oc
    return cc, tc - cc * Oc + Oc // 2


def coarse_bins(q, O, Oc):
    """Bins of the correction: the quantiser's dict with cell and fi moved to
    the coarse lattice (same plane, same dropped flags)."""
    cu, fu = coarse_axis(q['cell_u'], q['fi_u'], O, Oc)
    cv, fv = coarse_axis(q['cell_v'], q['fi_v'], O, Oc)
    return dict(cell_u=cu, fi_u=fu, cell_v=cv, fi_v=fv, k=q['k'], dropped=q['dropped'])


def correction_table(w_centres, N, fov, Sc, Oc, c1, a_u=0.5, b_u=5.0 / 24.0, a_v=None, b_v=None):
    """C[k][fu][fv][su][sv] (complex128) by the direct double sum above."""
    if a_v is None:
        a_v = a_u
    if b_v is None:
        b_v = b_u
    l = pixel_l(N, fov)
    L, M = l[None, :], l[:, None]                              # [q][p]
    n_minus_1 = np.sqrt(1.0 - L * L - M * M) - 1.0
    phi = (a_u * L ** 2 + b_u * L ** 4) + (a_v * M ** 2 + b_v * M ** 4)
    taper = c1[None, :] * c1[:, None]
    p = np.arange(N, dtype=np.float64)
    E = np.exp(-2j * np.pi * tap_offsets(Sc, Oc)[..., None] * (p - N / 2) / N)  # [Oc][Sc][N]
    out = np.empty((len(w_centres), Oc, Oc, Sc, Sc), dtype=np.complex128)
    for k, w in enumerate(w_centres):
        A = taper * (np.exp(2j * np.pi * w * n_minus_1) - np.exp(-2j * np.pi * w * phi))
        out[k] = np.einsum('xsp,qp,ytq->xyst', E, A, E, optimize=True) / (N * N)
    return out


def grid(q, y, T, C, N, S, O, Sc, Oc, wrap=False):
    """Separable gridding plus the correction's 2D footprint at the coarse bins."""
    G = gridder.grid_separable(q, y, T, N, S, wrap=wrap)
    return G + gridder.grid_exact(coarse_bins(q, O, Oc), y, C, N, Sc, wrap=wrap)


def degrid(q, G, T, C, N, S, O, Sc, Oc, wrap=False):
    """Adjoint of ``grid``: separable degridding plus the correction's."""
    V = gridder.degrid_separable(q, G, T, N, S, wrap=wrap)
    return V + gridder.degrid_exact(coarse_bins(q, O, Oc), G, C, N, Sc, wrap=wrap)


def grid_cells(q, y, T, C, N, S, O, Sc, Oc, cells):
    """Selected grid cells of ``grid``: each the separable sum plus the
    correction sum over every kept visibility whose footprint covers it (used
    to check full-size gridding at sampled outputs)."""
    out = gridder.grid_cells(q, y, T, N, S, cells)
    qc = coarse_bins(q, O, Oc)
    h = Sc // 2
    keep = ~qc['dropped']
    for n, (jv, ju) in enumerate(cells):
        su = ju - qc['cell_u'] + h
        sv = jv - qc['cell_v'] + h
        i = np.flatnonzero(keep & (su >= 0) & (su < Sc) & (sv >= 0) & (sv < Sc))
        out[n] += np.sum(y[i] * C[qc['k'][i], qc['fi_u'][i], qc['fi_v'][i], su[i], sv[i]])
    return out
