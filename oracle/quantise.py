"""Coordinate quantisation, w-plane assignment and tile binning (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2: u, v, w are in wavelengths and the GCF is tabulated with an
oversampling factor (typically 8).  The paper does not fix the rounding rules;
the readings used here are:

* Continuous cell coordinate  x = u * fov + N/2  (cell j is centred at
  u_j = (j - N/2)/fov).  Oversampled position t = x * O, rounded half up:
  q = floor(t + 1/2).  Nearest cell  cell = floor((q + O/2) / O)  (integer
  floor division), sub-cell offset f = q - cell*O in [-O/2, O/2), table row
  fi = f + O/2.  Every floating-point operation is a single IEEE double
  operation in exactly this order (multiply, then add; no fused multiply-add),
  so any faithful implementation reproduces the integers bit for bit.
* w-plane  k = clamp(floor((w - w_lo) * inv_dw), 0, P-1)  with
  inv_dw = P / (w_hi - w_lo) computed once.
* A visibility whose S x S footprint (cells cell-h .. cell+h, h = floor(S/2))
  leaves [0, N) in either axis, or whose u, v or w is not finite, is dropped
  (skipped and counted), never wrapped.
* Tiles are c x c blocks of cells: tile = (cell_v // c) * ntx + (cell_u // c)
  with ntx = ceil(N / c).
"""
import numpy as np


SPEED_OF_LIGHT = 299792458.0   # m/s


def channel_coordinates(uvw_m, freq_hz):
    """u, v, w in wavelengths (Section 2's units) of every (row, channel) pair,
    row-major (visibility row * nchan + ch): u = u_m * (f / c), the division
    first and then the multiplication, each one IEEE double operation (the
    reading that makes a channel-shared layout reproduce the same bins)."""
    uvw_m = np.asarray(uvw_m, np.float64).reshape(-1, 3)
    scale = np.asarray(freq_hz, np.float64) / np.float64(SPEED_OF_LIGHT)   # [nchan]
    out = uvw_m[:, None, :] * scale[None, :, None]                          # [row][ch][3]
    return out[..., 0].ravel(), out[..., 1].ravel(), out[..., 2].ravel()


def plane_index(w, P, w_lo, w_hi):
    inv_dw = np.float64(P) / (np.float64(w_hi) - np.float64(w_lo))
    with np.errstate(invalid='ignore'):
        t = (np.asarray(w, np.float64) - np.float64(w_lo)) * inv_dw
        k = np.floor(t)
    ok = np.isfinite(k)
    k = np.where(ok, np.clip(k, 0, P - 1), 0).astype(np.int64)
    return k, ok


def axis_quantise(u, N, fov, O):
    """(cell, fi, ok) for one axis; see module docstring for the exact order."""
    u = np.asarray(u, np.float64)
    with np.errstate(invalid='ignore', over='ignore'):
        x = u * np.float64(fov)
        x = x + np.float64(N / 2)
        t = x * np.float64(O)
        q = np.floor(t + 0.5)
    # guard the float -> int conversion; anything this far out is off-grid anyway
    ok = np.isfinite(q) & (np.abs(q) < 2.0 ** 40)
    qi = np.where(ok, q, 0).astype(np.int64)
    cell = (qi + O // 2) // O          # Python/NumPy // is floor division
    f = qi - cell * O
    fi = f + O // 2
    return cell, fi, ok


def quantise(u, v, w, N, fov, O, S, P, w_lo, w_hi, tile_c):
    """Per-visibility bins: dict of int64 arrays cell_u, fi_u, cell_v, fi_v, k,
    tile and a bool array dropped."""
    h = S // 2
    cu, fu, oku = axis_quantise(u, N, fov, O)
    cv, fv, okv = axis_quantise(v, N, fov, O)
    k, okw = plane_index(w, P, w_lo, w_hi)
    on_grid = (cu - h >= 0) & (cu + h <= N - 1) & (cv - h >= 0) & (cv + h <= N - 1)
    dropped = ~(oku & okv & okw & on_grid)
    ntx = -(-N // tile_c)
    tile = (cv // tile_c) * ntx + (cu // tile_c)
    return dict(cell_u=cu, fi_u=fu, cell_v=cv, fi_v=fv, k=k,
                tile=np.where(dropped, -1, tile), dropped=dropped)


def dequantised(q, N, fov, O):
    """uv coordinates (wavelengths) the quantised bins stand for:
    u_hat = (cell + f/O - N/2) / fov."""
    def one(cell, fi):
        x = cell + (fi - O // 2) / O
        return (x - N / 2) / fov
    return one(q['cell_u'], q['fi_u']), one(q['cell_v'], q['fi_v'])
