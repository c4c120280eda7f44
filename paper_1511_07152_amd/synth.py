"""Seeded synthetic inputs for the separable W-projection workloads.

This module holds only input generation: array layouts, earth-rotation uvw
tracks and random visibilities/images.  It contains none of the gridding
method's arithmetic and imports nothing from the library or the oracle, so
both can be fed the same arrays.

The paper (arXiv:1511.07152) measures on no dataset; all inputs are synthetic.
Seeds are 15110715200 + workload number and every generator draws from one
``numpy.random.default_rng(seed)`` (PCG64) in a fixed order.

Visibility order is the usual measurement-set order: time (slowest), baseline,
channel (fastest).  u, v, w are in wavelengths (Section 2).
"""
import math

import numpy as np

C0 = 299_792_458.0          # speed of light, m/s
SEED0 = 15110715200


def deg(x):
    return x * math.pi / 180.0


# ---------------------------------------------------------------------------
# array geometry
# ---------------------------------------------------------------------------
def disc_antennas(rng, n_ant, radius_m):
    """Antennas uniform by area in a disc; coplanar local east/north/up (up=0)."""
    r = radius_m * np.sqrt(rng.uniform(0.0, 1.0, n_ant))
    phi = 2.0 * math.pi * rng.uniform(0.0, 1.0, n_ant)
    return np.stack([r * np.cos(phi), r * np.sin(phi), np.zeros(n_ant)], axis=1)


def baselines(enu):
    i, j = np.triu_indices(len(enu), k=1)
    return enu[j] - enu[i]                    # [nbl][3], no autocorrelations


def enu_to_xyz(b_enu, lat):
    e, n, u = b_enu[:, 0], b_enu[:, 1], b_enu[:, 2]
    x = -math.sin(lat) * n + math.cos(lat) * u
    y = e
    z = math.cos(lat) * n + math.sin(lat) * u
    return np.stack([x, y, z], axis=1)


def uvw_metres(b_xyz, ha, dec):
    """Textbook (u, v, w) of each baseline at each hour angle: [ntime][nbl][3]."""
    X, Y, Z = b_xyz[:, 0][None], b_xyz[:, 1][None], b_xyz[:, 2][None]
    sh, ch = np.sin(ha)[:, None], np.cos(ha)[:, None]
    sd, cd = math.sin(dec), math.cos(dec)
    u = sh * X + ch * Y
    v = -sd * ch * X + sd * sh * Y + cd * Z
    w = cd * ch * X - cd * sh * Y + sd * Z
    return np.stack([u, v, w], axis=-1)


def track(rng, n_ant, radius_m, lat, dec, ha_hours, dump_s, freqs_hz, time_slice=None,
          rows=False):
    """uvw in wavelengths, measurement-set order (time, baseline, channel);
    with rows=True also the per-row metres [ntime * nbl][3] they scale from."""
    enu = disc_antennas(rng, n_ant, radius_m)
    bxyz = enu_to_xyz(baselines(enu), lat)
    h0, h1 = ha_hours
    ndump = int(round((h1 - h0) * 3600.0 / dump_s))
    t = np.arange(ndump) if time_slice is None else np.arange(*time_slice)
    ha = deg(15.0) * (h0 + (t + 0.5) * dump_s / 3600.0)     # mid-dump hour angle
    uvw_m = uvw_metres(bxyz, ha, dec)                      # [nt][nbl][3]
    scale = np.asarray(freqs_hz, np.float64) / C0           # [nchan]
    uvw = uvw_m[:, :, None, :] * scale[None, None, :, None]  # [nt][nbl][nchan][3]
    uvw = uvw.reshape(-1, 3)
    out = (np.ascontiguousarray(uvw[:, 0]), np.ascontiguousarray(uvw[:, 1]),
           np.ascontiguousarray(uvw[:, 2]))
    if rows:
        return out + (np.ascontiguousarray(uvw_m.reshape(-1, 3)),)
    return out


def gaussian_vis(rng, n):
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return re + 1j * im


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def small_uniform(seed, nvis, N, fov, cells, wmax):
    """u, v uniform within +/- ``cells`` grid cells of the centre, w uniform in
    [-wmax, wmax], complex Gaussian V, unit weights."""
    rng = np.random.default_rng(seed)
    xu = rng.uniform(-cells, cells, nvis)
    xv = rng.uniform(-cells, cells, nvis)
    w = rng.uniform(-wmax, wmax, nvis)
    V = gaussian_vis(rng, nvis)
    return dict(u=xu / fov, v=xv / fov, w=w, V=V, W=np.ones(nvis))


def accuracy_64():
    """64 x 64 grid, 2 deg field, 2,000 visibilities within +/-28 cells,
    |w| <= 200, 8 w-planes, support 7, oversample 8."""
    fov = deg(2.0)
    d = small_uniform(SEED0 + 1, 2000, 64, fov, 28.0, 200.0)
    d.update(N=64, fov=fov, P=8, w_lo=-200.0, w_hi=200.0, S=7, O=8)
    return d


def _w_range(w):
    wm = float(np.max(np.abs(w))) * (1.0 + 1e-9) + 1e-9
    return -wm, wm


def array_4096(dump_s=10.0, channels=16):
    """4096^2 grid, 3 deg field, 64 antennas in an 8 km disc, dec -30 deg,
    latitude -30.7 deg, 8 h track in 10 s dumps, 16 channels at 600 + 8c MHz,
    128 w-planes over +/- max|w|, support 15, oversample 8 (92,897,280 vis)."""
    rng = np.random.default_rng(SEED0 + 2)
    freqs = 600e6 + 8e6 * np.arange(channels)
    u, v, w, uvw_m = track(rng, 64, 8000.0, deg(-30.7), deg(-30.0), (-4.0, 4.0), dump_s, freqs,
                           rows=True)
    V = gaussian_vis(rng, len(u)).astype(np.complex64)
    w_lo, w_hi = _w_range(w)
    return dict(u=u, v=v, w=w, V=V, W=np.ones(len(u), np.float32), N=4096, fov=deg(3.0),
                P=128, w_lo=w_lo, w_hi=w_hi, S=15, O=8, uvw_m=uvw_m, freqs=freqs)


def model_2048(N=2048, fov_deg=3.0, time_slice=None):
    """Differentiation workload: 2048^2 real model (500 point sources inside
    |l|,|m| <= 0.4 fov, flux log-uniform in [1e-3, 1], plus N(0, 1e-4^2) noise),
    3 deg field, 32 antennas in a 4 km disc, 6 h track in 20 s dumps, 8 channels
    at 600 + 8c MHz, 64 w-planes, support 15, oversample 8 (4,285,440 vis).
    A reduced model (smaller N, a narrower field so that the same baselines
    stay on the grid, a slice of the dumps) keeps the array, the kernels
    (S = 15, 64 planes, O = 8) and the recipe."""
    rng = np.random.default_rng(SEED0 + 4)
    fov = deg(fov_deg)
    lim = int(0.4 * N)                       # 0.4 fov in pixels from the centre
    x = np.zeros((N, N), np.float64)
    px = rng.integers(N // 2 - lim, N // 2 + lim + 1, 500)
    py = rng.integers(N // 2 - lim, N // 2 + lim + 1, 500)
    flux = 10.0 ** rng.uniform(-3.0, 0.0, 500)
    np.add.at(x, (py, px), flux)
    x += rng.normal(0.0, 1e-4, (N, N))
    freqs = 600e6 + 8e6 * np.arange(8)
    u, v, w = track(rng, 32, 4000.0, deg(-30.7), deg(-30.0), (-3.0, 3.0), 20.0, freqs,
                    time_slice=time_slice)
    noise = gaussian_vis(rng, len(u))
    w_lo, w_hi = _w_range(w)
    return dict(x=x, u=u, v=v, w=w, W=np.ones(len(u)), noise=noise, N=N, fov=fov,
                P=64, w_lo=w_lo, w_hi=w_hi, S=15, O=8)


def facets_36(scale=1.0):
    """Batching workload: 36 facets (6 x 6) over a 10 deg field, 1024^2 each,
    facet field 10/6 deg; per-facet visibility counts round(300,000 e^z),
    z ~ N(0,1) (times ``scale``), each a contiguous time slice of a 64-antenna
    3 km array (dec -30 deg, +/-4 h, 10 s, 16 channels at 600 + 8c MHz);
    64 w-planes, support 11, oversample 8."""
    rng = np.random.default_rng(SEED0 + 5)
    centres = deg(np.array([-25, -15, -5, 5, 15, 25]) / 6.0)
    z = rng.standard_normal(36)
    counts = np.maximum(1, np.round(300_000 * np.exp(z) * scale)).astype(np.int64)
    enu_rng_seed = int(rng.integers(0, 2 ** 31))
    freqs = 600e6 + 8e6 * np.arange(16)
    per_dump = 2016 * 16
    ndump = 2880
    jobs = []
    for f in range(36):
        l0 = float(centres[f % 6])
        m0 = float(centres[f // 6])
        nd = int(-(-counts[f] // per_dump))
        t0 = int(rng.integers(0, ndump - nd + 1))
        arr_rng = np.random.default_rng(enu_rng_seed)       # same antennas for every facet
        u, v, w = track(arr_rng, 64, 3000.0, deg(-30.7), deg(-30.0), (-4.0, 4.0), 10.0, freqs,
                        time_slice=(t0, t0 + nd))
        n = int(counts[f])
        V = gaussian_vis(rng, n)
        jobs.append(dict(u=u[:n], v=v[:n], w=w[:n], V=V, W=np.ones(n), l0=l0, m0=m0))
    return dict(jobs=jobs, N=1024, fov=deg(10.0 / 6.0), P=64, S=11, O=8)


def random_image(seed, N, real=False):
    rng = np.random.default_rng(seed)
    if real:
        return rng.standard_normal((N, N))
    return rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
