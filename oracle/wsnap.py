"""W snapshots: per-snapshot plane fit, residual w by separable W projection,
and image reprojection (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4.2: for each snapshot a single d0 = (d_u, d_v) is found with
w ~ u . d0.  Writing w = u . d0 + w', the phase of the dirty-image equation
becomes

    u . l + w (n(l) - 1) = u . l^s + w' (n(l) - 1),   l^s = l + d0 (n(l) - 1),

so the snapshot is imaged with W projection on the residual w' (here the
separable path), which yields D_s on the regular pixel grid in the coordinate
l^s (its w' term uses n at l^s: the error the paper analyses), and the
reprojection maps l^s back to l: output pixel l takes D_s(l + d0 (n(l) - 1)).
Snapshot images are summed.  Prediction is the adjoint (the transposed
reprojection, then degridding).

Readings (the paper fixes none of these):

* d0 is the unweighted least-squares plane through the origin over the
  snapshot's visibilities with finite u, v, w: with the sums
  Suu, Suv, Svv, Suw, Svw and det = Suu Svv - Suv^2, by Cramer's rule
  d_u = (Suw Svv - Svw Suv) / det,  d_v = (Svw Suu - Suw Suv) / det,
  and d0 = 0 when det is not above 1e-12 Suu Svv (a degenerate snapshot).
* w' = w - (d_u u + d_v v), each operation one IEEE double operation in that
  order.  The residual w-planes: P uniform planes on [-h, h] with
  h = max |w'| over all snapshots times (1 + 2^-20) (h = 1 if every w' is 0),
  one table set for all snapshots.
* Reprojection samples D_s at the fractional pixel x = l^s N / fov + N/2 (y
  from m^s alike) by separable cubic convolution (Keys, a = -1/2) over the
  4 x 4 nearest pixels; pixels outside the image contribute 0.  n - 1 is
  evaluated as -(l^2 + m^2) / (1 + n).
"""
import numpy as np

from . import geometry, gridder, imaging, quantise, tables

KEYS_A = -0.5


def fit_plane(u, v, w):
    """d0 = (d_u, d_v) by the least-squares reading above."""
    u, v, w = (np.asarray(x, np.float64) for x in (u, v, w))
    ok = np.isfinite(u) & np.isfinite(v) & np.isfinite(w)
    u, v, w = u[ok], v[ok], w[ok]
    suu, suv, svv = np.sum(u * u), np.sum(u * v), np.sum(v * v)
    suw, svw = np.sum(u * w), np.sum(v * w)
    det = suu * svv - suv * suv
    if not det > 1e-12 * suu * svv:
        return 0.0, 0.0
    return (suw * svv - svw * suv) / det, (svw * suu - suw * suv) / det


def residuals(u, v, w, offsets):
    """Per-snapshot d0 [n_snap][2], residual w' per visibility and h."""
    d0 = np.zeros((len(offsets) - 1, 2))
    wr = np.empty(len(u))
    for s in range(len(offsets) - 1):
        sl = slice(offsets[s], offsets[s + 1])
        du, dv = fit_plane(u[sl], v[sl], w[sl])
        d0[s] = du, dv
        wr[sl] = w[sl] - (du * u[sl] + dv * v[sl])
    fin = wr[np.isfinite(wr)]
    m = float(np.max(np.abs(fin))) if len(fin) else 0.0
    h = m * (1.0 + 2.0 ** -20) if m > 0 else 1.0
    return d0, wr, h


def keys(t):
    """Keys' cubic convolution kernel with a = -1/2."""
    t = np.abs(np.asarray(t, np.float64))
    a = KEYS_A
    return np.where(t <= 1, (a + 2) * t ** 3 - (a + 3) * t ** 2 + 1,
                    np.where(t < 2, a * t ** 3 - 5 * a * t ** 2 + 8 * a * t - 4 * a, 0.0))


def sample_points(N, fov, d0):
    """Fractional pixel coordinates (x, y) [q][p] of l^s, m^s for every
    output pixel."""
    l = geometry.pixel_l(N, fov)
    L, M = l[None, :], l[:, None]
    r2 = L * L + M * M
    nm1 = -r2 / (1.0 + np.sqrt(1.0 - r2))
    ls = L + d0[0] * nm1
    ms = M + d0[1] * nm1
    return ls * N / fov + N / 2, ms * N / fov + N / 2


def _taps(x, N):
    """Indices [.., 4] and weights [.., 4] along one axis (weights 0 off the image)."""
    x0 = np.floor(x)
    f = x - x0
    idx = x0[..., None].astype(np.int64) + np.arange(-1, 3)
    wts = np.stack([keys(1 + f), keys(f), keys(1 - f), keys(2 - f)], axis=-1)
    inside = (idx >= 0) & (idx < N)
    return np.clip(idx, 0, N - 1), np.where(inside, wts, 0.0)


def reproject(D, N, fov, d0):
    """R[q][p] = D_s at (l_p + d_u (n - 1), m_q + d_v (n - 1))."""
    x, y = sample_points(N, fov, d0)
    ix, wx = _taps(x, N)                       # [q][p][4]
    iy, wy = _taps(y, N)
    out = np.zeros((N, N), dtype=np.complex128)
    for j in range(4):
        for i in range(4):
            out += wy[..., j] * wx[..., i] * D[iy[..., j], ix[..., i]]
    return out


def reproject_adjoint(X, N, fov, d0):
    """Transpose of ``reproject``: each output pixel's value goes back to the
    4 x 4 snapshot pixels it was sampled from, with the same weights."""
    x, y = sample_points(N, fov, d0)
    ix, wx = _taps(x, N)
    iy, wy = _taps(y, N)
    Y = np.zeros(N * N, dtype=np.complex128)
    for j in range(4):
        for i in range(4):
            val = wy[..., j] * wx[..., i] * X
            flat = (iy[..., j] * N + ix[..., i]).ravel()
            Y += np.bincount(flat, weights=val.real.ravel(), minlength=N * N)
            Y += 1j * np.bincount(flat, weights=val.imag.ravel(), minlength=N * N)
    return Y.reshape(N, N)


def residual_tables(N, fov, S, O, P, h, c1, a=0.5, b=5.0 / 24.0):
    return tables.separable_table(tables.w_plane_centres(P, -h, h), N, fov, S, O, c1, a=a, b=b)


def image(u, v, w, y, offsets, N, fov, S, O, P, c1, n_power=0, a=0.5, b=5.0 / 24.0):
    """Sum over snapshots of the reprojected residual-w snapshot images, times n^n_power."""
    d0, wr, h = residuals(u, v, w, offsets)
    T = residual_tables(N, fov, S, O, P, h, c1, a, b)
    out = np.zeros((N, N), dtype=np.complex128)
    for s in range(len(offsets) - 1):
        sl = slice(offsets[s], offsets[s + 1])
        if offsets[s + 1] == offsets[s]:
            continue
        q = quantise.quantise(u[sl], v[sl], wr[sl], N, fov, O, S, P, -h, h, 1)
        D = imaging.image_from_grid(gridder.grid_separable(q, y[sl], T, N, S), c1, fov)
        out += reproject(D, N, fov, d0[s])
    if n_power:
        out = out * geometry.n_image(N, fov) ** n_power
    return out


def predict(u, v, w, X, offsets, N, fov, S, O, P, c1, n_power=0, a=0.5, b=5.0 / 24.0):
    """Adjoint of ``image``: per snapshot, the transposed reprojection of
    X n^n_power, then the separable prediction on the residual w."""
    d0, wr, h = residuals(u, v, w, offsets)
    T = residual_tables(N, fov, S, O, P, h, c1, a, b)
    Xn = X * geometry.n_image(N, fov) ** n_power if n_power else X
    V = np.zeros(len(u), dtype=np.complex128)
    for s in range(len(offsets) - 1):
        sl = slice(offsets[s], offsets[s + 1])
        if offsets[s + 1] == offsets[s]:
            continue
        q = quantise.quantise(u[sl], v[sl], wr[sl], N, fov, O, S, P, -h, h, 1)
        G = imaging.grid_from_image(reproject_adjoint(Xn, N, fov, d0[s]), c1, fov)
        V[sl] = gridder.degrid_separable(q, G, T, N, S)
    return V
