"""W-stacking hybrid: w-slices corrected in image space, residual w by
separable W projection (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4.3: visibilities are partitioned by w; within each partition the
partition's w is corrected in image space by a phase factor, and the residual
w by (here separable) W projection.  Splitting w_i = w_s + dw_i in the
dirty-image equation of Section 2,

    exp(2 pi i w_i (n - 1)) = exp(2 pi i w_s (n - 1)) exp(2 pi i dw_i (n - 1)),

so with D_s the separable W-projection image of slice s on its residual w
(gridding, F+, division by the taper, factor n as in ``imaging``),

    D = sum_s exp(2 pi i w_s (n - 1)) D_s .

Prediction is the adjoint: slice s degrids the model times
exp(-2 pi i w_s (n - 1)) on its residual w.

Readings (the paper fixes none of these):

* slices are uniform on [w_lo, w_hi]: slice s = clamp(floor((w - w_lo) n_s /
  (w_hi - w_lo)), 0, n_s - 1), centre w_s = w_lo + (s + 1/2)(w_hi - w_lo)/n_s
  (the same rule as the w-planes; Section 4.3 takes evenly spaced slices);
* the residual w - w_s of every slice is binned into P uniform planes on
  [-h, h], h = (w_hi - w_lo) / (2 n_s), one table set shared by all slices;
* n - 1 is evaluated as -(l^2 + m^2) / (1 + n), which equals it exactly and
  avoids the cancellation of n - 1 near the centre.

Non-uniform slices (Section 4.3 suggests many narrow slices near w = 0 and
wider ones at large |w|, slice widths adapted to the visibility density):

* with increasing edges e_0 < ... < e_ns, slice s holds e_s <= w < e_{s+1}
  (w below e_0 in slice 0, w at or above e_ns in the last slice, non-finite w
  in slice 0), centre w_s = (e_s + e_{s+1}) / 2, and its residual w goes to
  P uniform planes on its own range [-h_s, h_s], h_s = (e_{s+1} - e_s) / 2,
  with a table set per slice (a narrow slice gets finely spaced planes);
* density-adapted edges: the finite w are counted in nfine uniform bins of
  [w_lo, w_hi] (bin index as the plane index); edge k (0 < k < ns) is the
  first bin boundary j at which the count below reaches k n / ns (n finite
  visibilities), kept strictly increasing and leaving one bin for each later
  slice; e_k = w_lo + j d with d = (w_hi - w_lo) / nfine, e_0 = w_lo,
  e_ns = w_hi.  Slices then hold about n / ns visibilities each, so they are
  narrow where w is dense.
"""
import numpy as np

from . import geometry, gridder, imaging, quantise, tables


def slice_of(w, n_slices, w_lo, w_hi, edges=None):
    """Slice index, slice centres and residual w - w_s of each visibility
    (non-finite w goes to slice 0 with a non-finite residual, which the
    plane quantiser then drops).  edges: None for uniform slices on
    [w_lo, w_hi], else the n_slices + 1 increasing slice edges."""
    w = np.asarray(w, np.float64)
    if edges is None:
        s, _ = quantise.plane_index(w, n_slices, w_lo, w_hi)
        ws = tables.w_plane_centres(n_slices, w_lo, w_hi)
    else:
        e = np.asarray(edges, np.float64)
        s = np.clip(np.searchsorted(e, w, side='right') - 1, 0, n_slices - 1)
        s = np.where(np.isfinite(w), s, 0)
        ws = (e[:-1] + e[1:]) * 0.5
    return s, ws, w - ws[s]


def residual_range(n_slices, w_lo, w_hi, edges=None, k=0):
    """Residual range [-h, h] of slice k: h = (w_hi - w_lo) / (2 n_s) for
    uniform slices (all alike), h_k = (e_{k+1} - e_k) / 2 with edges."""
    if edges is None:
        h = (np.float64(w_hi) - np.float64(w_lo)) / (2 * n_slices)
    else:
        e = np.asarray(edges, np.float64)
        h = (e[k + 1] - e[k]) * 0.5
    return -h, h


def density_edges(w, n_slices, w_lo, w_hi, nfine=16384):
    """Slice edges with about equal visibility counts per slice (see the
    module docstring)."""
    w = np.asarray(w, np.float64)
    fin = np.isfinite(w)
    j, _ = quantise.plane_index(w[fin], nfine, w_lo, w_hi)
    counts = np.bincount(j, minlength=nfine)
    below = np.concatenate([[0], np.cumsum(counts)])    # below[j]: count in bins < j
    n = int(below[-1])
    d = (np.float64(w_hi) - np.float64(w_lo)) / nfine
    e = np.empty(n_slices + 1)
    e[0], e[n_slices] = w_lo, w_hi
    prev = 0
    for k in range(1, n_slices):
        # first j with below[j] * ns >= k n (integers)
        jk = int(np.searchsorted(below * n_slices, k * n, side='left'))
        jk = min(max(jk, prev + 1), nfine - (n_slices - k))
        e[k] = np.float64(w_lo) + np.float64(jk) * d
        prev = jk
    return e


def slice_phase(N, fov, w_s, sign):
    """exp(sign 2 pi i w_s (n - 1)) at the pixels, indexed [q][p]."""
    l = geometry.pixel_l(N, fov)
    r2 = l[None, :] ** 2 + l[:, None] ** 2
    n = np.sqrt(1.0 - r2)
    return np.exp(sign * 2j * np.pi * w_s * (-r2 / (1.0 + n)))


def _bins(u, v, w, N, fov, O, S, P, w_lo, w_hi):
    return quantise.quantise(u, v, w, N, fov, O, S, P, w_lo, w_hi, 1)


def residual_tables(N, fov, S, O, P, n_slices, w_lo, w_hi, c1, a=0.5, b=5.0 / 24.0, edges=None,
                    k=0):
    r_lo, r_hi = residual_range(n_slices, w_lo, w_hi, edges, k)
    return tables.separable_table(tables.w_plane_centres(P, r_lo, r_hi), N, fov, S, O, c1, a=a, b=b)


def _slice_tables(N, fov, S, O, P, n_slices, w_lo, w_hi, c1, a, b, edges):
    """Per slice: residual range and tables (computed once for uniform slices)."""
    out, cache = [], {}
    for k in range(n_slices):
        r = residual_range(n_slices, w_lo, w_hi, edges, k)
        if r not in cache:
            cache[r] = tables.separable_table(tables.w_plane_centres(P, r[0], r[1]), N, fov, S, O,
                                              c1, a=a, b=b)
        out.append((r, cache[r]))
    return out


def image(u, v, w, y, N, fov, S, O, P, n_slices, w_lo, w_hi, c1, n_power=0, a=0.5,
          b=5.0 / 24.0, bins=_bins, wrap=False, edges=None):
    """Sum over slices of exp(2 pi i w_s (n - 1)) times the slice's corrected image."""
    s, ws, dw = slice_of(w, n_slices, w_lo, w_hi, edges)
    st = _slice_tables(N, fov, S, O, P, n_slices, w_lo, w_hi, c1, a, b, edges)
    D = np.zeros((N, N), dtype=np.complex128)
    for k in range(n_slices):
        idx = np.flatnonzero(s == k)
        if len(idx) == 0:
            continue
        (r_lo, r_hi), T = st[k]
        q = bins(u[idx], v[idx], dw[idx], N, fov, O, S, P, r_lo, r_hi)
        G = gridder.grid_separable(q, y[idx], T, N, S, wrap=wrap)
        D += slice_phase(N, fov, ws[k], +1) * imaging.image_from_grid(G, c1, fov, n_power)
    return D


def predict(u, v, w, X, N, fov, S, O, P, n_slices, w_lo, w_hi, c1, n_power=0, a=0.5,
            b=5.0 / 24.0, bins=_bins, wrap=False, edges=None):
    """Visibilities of model X: slice s degrids X exp(-2 pi i w_s (n - 1))."""
    s, ws, dw = slice_of(w, n_slices, w_lo, w_hi, edges)
    st = _slice_tables(N, fov, S, O, P, n_slices, w_lo, w_hi, c1, a, b, edges)
    V = np.zeros(len(u), dtype=np.complex128)
    for k in range(n_slices):
        idx = np.flatnonzero(s == k)
        if len(idx) == 0:
            continue
        (r_lo, r_hi), T = st[k]
        q = bins(u[idx], v[idx], dw[idx], N, fov, O, S, P, r_lo, r_hi)
        G = imaging.grid_from_image(X * slice_phase(N, fov, ws[k], -1), c1, fov, n_power)
        V[idx] = gridder.degrid_separable(q, G, T, N, S, wrap=wrap)
    return V


def bins(u, v, w, N, fov, O, S, P, n_slices, w_lo, w_hi, edges=None):
    """Bins of every visibility in caller order (residual w, planes of its
    slice's residual range)."""
    s, _, dw = slice_of(w, n_slices, w_lo, w_hi, edges)
    if edges is None:
        r_lo, r_hi = residual_range(n_slices, w_lo, w_hi)
        return quantise.quantise(u, v, dw, N, fov, O, S, P, r_lo, r_hi, 1)
    out = None
    for k in range(n_slices):
        idx = np.flatnonzero(s == k)
        if len(idx) == 0:
            continue
        r_lo, r_hi = residual_range(n_slices, w_lo, w_hi, edges, k)
        q = quantise.quantise(u[idx], v[idx], dw[idx], N, fov, O, S, P, r_lo, r_hi, 1)
        if out is None:
            out = {key: np.zeros(len(u), dtype=val.dtype) for key, val in q.items()}
        for key, val in q.items():
            out[key][idx] = val
    return out
