"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative RMS unless stated): tables 1e-6; grids 1e-6, or
sqrt(K) 2^-24 where the heaviest cell sums K > 2^8 footprints (the rounding of
a K-term FP32 sum with random signs; only the 3,000-visibility tile reaches
it here); images over the inner half (|l|,|m| <= fov/4, where 1/(c1 c1) does
not amplify FP32 rounding) and degridded visibilities 1e-5, the FP32 bound;
bins bit-exact.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import OracleSetup, dev, inner, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1511_07152_amd import _lib
    _lib.load()
    return _lib


def _acc():
    from paper_1511_07152_amd import synth
    return synth.accuracy_64()


def _make(lib, d, **kw):
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], d["w_lo"], d["w_hi"], **kw)
    plan = lib.Plan(K, dev(d["u"], torch.float64), dev(d["v"], torch.float64), dev(d["w"], torch.float64))
    return K, plan


def _oracle(d, plan, **kw):
    return OracleSetup(d["u"], d["v"], d["w"], d["N"], d["fov"], d["S"], d["O"], d["P"],
                       d["w_lo"], d["w_hi"], plan.tile_size, **kw)


# ------------------------------------------------------------------ tables
@pytest.mark.parametrize("N,S,W", [(64, 7, None), (4096, 15, None), (256, 11, 9.0)])
def test_taper_matches_oracle(lib, N, S, W):
    K = lib.Kernels(N, math.radians(3.0), S, 8, 2, -100.0, 100.0, taper_width=W or 0.0)
    got = K.taper().cpu().numpy()
    want = oracle.pswf.taper_c1(N, math.radians(3.0), W or S)
    assert np.max(np.abs(got - want)) < 1e-11


@pytest.mark.parametrize("case", ["acc64", "s15", "facet", "axes"])
def test_tables_match_oracle(lib, case):
    fov, N, S, O, P, wlo, whi = math.radians(2.0), 64, 7, 8, 8, -200.0, 200.0
    kw, okw = {}, {}
    if case == "s15":
        N, S, P, wlo, whi, fov = 512, 15, 5, -3000.0, 3000.0, math.radians(3.0)
    if case == "facet":
        kw = okw = dict(facet=(0.04, -0.07))
    K = lib.Kernels(N, fov, S, O, P, wlo, whi, **({"a": 0.4, "b": 0.1, "a_v": 0.6, "b_v": 0.3}
                                                    if case == "axes" else kw))
    wc = oracle.tables.w_plane_centres(P, wlo, whi)
    c1 = oracle.pswf.taper_c1(N, fov, S)
    if case == "facet":
        n0, a_l, a_m = oracle.facet.facet_coefficients(*okw["facet"])
        want_u = oracle.tables.separable_table(wc, N, fov, S, O, c1, a=a_l, b=0.0)
        want_v = oracle.tables.separable_table(wc, N, fov, S, O, c1, a=a_m, b=0.0)
    elif case == "axes":
        want_u = oracle.tables.separable_table(wc, N, fov, S, O, c1, a=0.4, b=0.1)
        want_v = oracle.tables.separable_table(wc, N, fov, S, O, c1, a=0.6, b=0.3)
    else:
        want_u = want_v = oracle.tables.separable_table(wc, N, fov, S, O, c1)
    for axis, want in ((0, want_u), (1, want_v)):
        got = K.table(axis).cpu().numpy()
        assert np.max(np.abs(got - want)) <= 1e-6 * np.max(np.abs(want))


# ------------------------------------------------------------------ bins
def _edge_uvw(N, fov, O):
    """Ties, cell centres, grid edges, off-grid, non-finite values."""
    xs = [0.0, 0.5, -0.5, 0.25, 1.0 / (2 * O), -1.0 / (2 * O), 3.5 / O, N / 2 - 4.0, N / 2 - 3.5,
          N / 2 - 3.49, -N / 2 + 3.0, -N / 2 + 2.5, -N / 2 + 2.51, 1e7, -1e7]
    u = np.array(xs) / fov
    uu, vv = np.meshgrid(u, u[::-1])
    u, v = uu.ravel(), vv.ravel()
    w = np.linspace(-250, 250, len(u))
    u = np.r_[u, np.nan, 0.0, np.inf, 0.0]
    v = np.r_[v, 0.0, -np.inf, 0.0, 0.0]
    w = np.r_[w, 0.0, 0.0, 0.0, np.nan]
    return u, v, w


@pytest.mark.parametrize("S", [7, 15])
def test_bins_bit_exact(lib, S):
    d = _acc()
    d["S"] = S
    rng = np.random.default_rng(99)
    eu, ev, ew = _edge_uvw(d["N"], d["fov"], d["O"])
    ru = rng.uniform(-40, 40, 3000) / d["fov"]
    rv = rng.uniform(-40, 40, 3000) / d["fov"]
    rw = rng.uniform(-300, 300, 3000)
    d["u"], d["v"], d["w"] = np.r_[d["u"], eu, ru], np.r_[d["v"], ev, rv], np.r_[d["w"], ew, rw]
    K, plan = _make(lib, d)
    o = _oracle(d, plan)
    got = plan.bins().cpu().numpy().astype(np.int64)
    want = o.bins_array()
    assert np.array_equal(got, want)
    assert plan.n_dropped == int(o.q["dropped"].sum())


# ------------------------------------------------------------------ gridding
@pytest.mark.parametrize("nvis", [1, 3, 17, 1000, 2000])
def test_grid_only_matches_oracle(lib, nvis):
    d = _acc()
    for k in ("u", "v", "w", "V", "W"):
        d[k] = d[k][:nvis]
    K, plan = _make(lib, d)
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    o = _oracle(d, plan)
    assert rel_rms(G, o.grid(d["V"], d["W"])) <= o.grid_bound() == 1e-6


def test_grid_heavy_tile_and_weights(lib):
    # 3,000 visibilities inside one tile (split into several work items) plus
    # non-unit weights
    d = _acc()
    rng = np.random.default_rng(5)
    n = 3000
    d["u"] = np.r_[d["u"], rng.uniform(0.0, 0.4, n) / d["fov"]]
    d["v"] = np.r_[d["v"], rng.uniform(0.0, 0.4, n) / d["fov"]]
    d["w"] = np.r_[d["w"], rng.uniform(-200, 200, n)]
    d["V"] = np.r_[d["V"], rng.standard_normal(n) + 1j * rng.standard_normal(n)]
    d["W"] = rng.uniform(0.1, 3.0, len(d["u"]))
    K, plan = _make(lib, d)
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    o = _oracle(d, plan)
    assert o.coverage_max() > 3000
    assert rel_rms(G, o.grid(d["V"], d["W"])) <= o.grid_bound()


@pytest.mark.parametrize("flags,npow", [(0, 0), ("MUL_N", 1), ("DIV_N", -1)])
def test_image_matches_oracle(lib, flags, npow):
    d = _acc()
    K, plan = _make(lib, d)
    f = getattr(lib, flags) if flags else 0
    img = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32), flags=f).cpu().numpy()
    want = _oracle(d, plan).image(d["V"], d["W"], n_power=npow)
    e_in = rel_rms(inner(img), inner(want))
    # the full image as well: at the edges 1 / (c1 c1) lifts the FP32
    # rounding of the grid far above the tapered signal, so only the inner
    # half carries the 1e-5 bound; the full-image figure is reported
    e_full = rel_rms(img, want)
    print("image (%s): inner half %.2e, full image %.2e" % (flags or "plain", e_in, e_full))
    assert e_in <= 1e-5 and np.isfinite(e_full)


def test_image_tracks_dft(lib):
    # end-to-end against the direct DFT of the dirty-image equation at the
    # quantised coordinates with the separable phase: bounded by truncation
    # of the GCF to S taps (no closed form; same bound the oracle meets)
    d = _acc()
    K, plan = _make(lib, d)
    img = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32)).cpu().numpy()
    o = _oracle(d, plan)
    uh, vh = oracle.quantise.dequantised(o.q, d["N"], d["fov"], d["O"])
    wc = oracle.tables.w_plane_centres(d["P"], d["w_lo"], d["w_hi"])
    ref = oracle.dft.dirty(uh, vh, wc[o.q["k"]], d["V"] * d["W"], d["N"], d["fov"],
                           oracle.dft.phase_screen(d["N"], d["fov"], "sep"))
    assert rel_rms(inner(img), inner(ref)) < 1e-2


# ------------------------------------------------------------------ degridding
def _inner_model(rng, N):
    """Random complex model supported on the inner half |l|, |m| < fov/4.

    The pre-correction divides by c1(l) c1(m), which reaches ~1e-7 in the
    corners for S = 7: content there would be amplified by 1e7 and FP32
    rounding in the FFT would dominate.  Model images in practice live inside
    the taper's well-conditioned region, and so do the parity inputs."""
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    mask = np.zeros((N, N), bool)
    mask[N // 4:3 * N // 4, N // 4:3 * N // 4] = True
    return np.where(mask, X, 0)


def test_degrid_grid_only_matches_oracle(lib):
    d = _acc()
    K, plan = _make(lib, d)
    rng = np.random.default_rng(11)
    G = rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))
    V = lib.degrid(plan, dev(G, torch.complex64), flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(V, _oracle(d, plan).degrid_grid(G)) <= 1e-5


@pytest.mark.parametrize("flags,npow", [(0, 0), ("DIV_N", -1)])
def test_degrid_image_matches_oracle(lib, flags, npow):
    d = _acc()
    K, plan = _make(lib, d)
    rng = np.random.default_rng(12)
    X = _inner_model(rng, 64)
    f = getattr(lib, flags) if flags else 0
    V = lib.degrid(plan, dev(X, torch.complex64), flags=f).cpu().numpy()
    assert rel_rms(V, _oracle(d, plan).degrid_image(X, n_power=npow)) <= 1e-5


def test_adjoint_identity(lib):
    d = _acc()
    K, plan = _make(lib, d)
    rng = np.random.default_rng(13)
    X = _inner_model(rng, 64)
    y = d["V"]
    Gy = lib.grid(plan, dev(y, torch.complex64), None, flags=lib.DIV_N).cpu().numpy().astype(complex)
    AX = lib.degrid(plan, dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy().astype(complex)
    lhs, rhs = np.vdot(X, Gy), np.vdot(AX, y)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(Gy) * np.linalg.norm(X)


# ------------------------------------------------------------------ edge cases
def test_empty_and_all_dropped(lib):
    d = _acc()
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], d["w_lo"], d["w_hi"])
    z = torch.zeros(0, dtype=torch.float64, device="cuda")
    plan = lib.Plan(K, z, z, z)
    assert plan.n_dropped == 0
    G = lib.grid(plan, torch.zeros(0, dtype=torch.complex64, device="cuda"), flags=lib.GRID_ONLY)
    assert float(G.abs().max()) == 0.0
    far = dev(np.full(10, 1e9), torch.float64)
    plan2 = lib.Plan(K, far, far, far)
    assert plan2.n_dropped == 10
    V = lib.degrid(plan2, torch.ones((64, 64), dtype=torch.complex64, device="cuda"))
    assert float(V.abs().max()) == 0.0


def test_repeat_runs_agree(lib):
    d = _acc()
    K, plan = _make(lib, d)
    V, W = dev(d["V"], torch.complex64), dev(d["W"], torch.float32)
    a = lib.grid(plan, V, W, flags=lib.GRID_ONLY).cpu().numpy()
    b = lib.grid(plan, V, W, flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(a, b) <= 1e-6


def test_odd_tile_layout(lib):
    # N = 70 with S = 11 (tile 6): ceil(70 / 6) = 12 tiles per row, last one ragged
    rng = np.random.default_rng(17)
    N, fov, S, O, P = 70, math.radians(2.5), 11, 4, 5
    n = 1500
    d = dict(u=rng.uniform(-30, 30, n) / fov, v=rng.uniform(-30, 30, n) / fov,
             w=rng.uniform(-100, 100, n), V=rng.standard_normal(n) + 1j * rng.standard_normal(n),
             W=np.ones(n), N=N, fov=fov, S=S, O=O, P=P, w_lo=-100.0, w_hi=100.0)
    K, plan = _make(lib, d)
    assert plan.tile_size == 6
    o = _oracle(d, plan)
    assert np.array_equal(plan.bins().cpu().numpy().astype(np.int64), o.bins_array())
    G = lib.grid(plan, dev(d["V"], torch.complex64), None, flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(G, o.grid(d["V"], d["W"])) <= o.grid_bound()
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    V = lib.degrid(plan, dev(X, torch.complex64), flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(V, o.degrid_grid(X)) <= 1e-5


# ------------------------------------------------------------------ facets
def test_facet_grid_and_degrid(lib):
    d = _acc()
    facet = (0.03, -0.02)
    K, plan = _make(lib, d, facet=facet)
    o = _oracle(d, plan, facet=facet)
    assert np.array_equal(plan.bins().cpu().numpy().astype(np.int64), o.bins_array())
    img = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                   flags=lib.MUL_N).cpu().numpy()
    assert rel_rms(inner(img), inner(o.image(d["V"], d["W"], n_power=1))) <= 1e-5
    rng = np.random.default_rng(19)
    X = _inner_model(rng, 64)
    V = lib.degrid(plan, dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy()
    assert rel_rms(V, o.degrid_image(X, n_power=-1)) <= 1e-5


# ------------------------------------------------------------------ table placement
def test_large_tables_cache_path(lib):
    # P = 256, O = 8, S = 15: one padded table is 256 * 8 * 17 * 8 B = 278 KB,
    # more than a workgroup's LDS, so degridding reads the taps through the
    # caches instead of staging them in LDS; both paths must agree with the oracle
    rng = np.random.default_rng(23)
    N, fov, S, O, P = 64, math.radians(2.0), 15, 8, 256
    n = 3000
    d = dict(u=rng.uniform(-24, 24, n) / fov, v=rng.uniform(-24, 24, n) / fov,
             w=rng.uniform(-200, 200, n), V=rng.standard_normal(n) + 1j * rng.standard_normal(n),
             W=rng.uniform(0.5, 2.0, n), N=N, fov=fov, S=S, O=O, P=P, w_lo=-200.0, w_hi=200.0)
    K, plan = _make(lib, d)
    o = _oracle(d, plan)
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(G, o.grid(d["V"], d["W"])) <= o.grid_bound()
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    V = lib.degrid(plan, dev(X, torch.complex64), flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(V, o.degrid_grid(X)) <= 1e-5


# ------------------------------------------------------------------ grid edges
@pytest.mark.parametrize("N,S", [(64, 15), (40, 7), (18, 3)])
def test_grid_and_degrid_at_grid_corners(lib, N, S):
    # Footprints at all four grid edges and corners: the 16-cell regions of the
    # edge tiles reach past the grid, and at the first and last cells of the
    # grid the degridding region loads are moved inside the grid and
    # re-indexed.  Cells j = h .. N-1-h are the extreme ones whose footprint
    # stays inside (h = S // 2); sub-cell offsets within +-0.4 keep the cell.
    rng = np.random.default_rng(29 + N)
    fov, O, P = math.radians(2.0), 8, 4
    h = S // 2
    lo, hi = h, N - 1 - h
    corners = np.array([(a, b) for a in (lo, hi) for b in (lo, hi)] * 30)
    edges = np.array([(a, b) for a in (lo, hi) for b in rng.integers(lo, hi + 1, 20)] +
                     [(b, a) for a in (lo, hi) for b in rng.integers(lo, hi + 1, 20)])
    inner_ = rng.integers(lo, hi + 1, (300, 2))
    cells = np.concatenate([corners, edges, inner_]).astype(float)
    n = len(cells)
    u = (cells[:, 0] - N // 2 + rng.uniform(-0.4, 0.4, n)) / fov
    v = (cells[:, 1] - N // 2 + rng.uniform(-0.4, 0.4, n)) / fov
    d = dict(u=u, v=v, w=rng.uniform(-100, 100, n),
             V=rng.standard_normal(n) + 1j * rng.standard_normal(n), W=rng.uniform(0.5, 2.0, n),
             N=N, fov=fov, S=S, O=O, P=P, w_lo=-100.0, w_hi=100.0)
    K, plan = _make(lib, d)
    o = _oracle(d, plan)
    assert np.array_equal(plan.bins().cpu().numpy().astype(np.int64), o.bins_array())
    assert not o.bins_array()[:, 6].any()   # every footprint inside the grid
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(G, o.grid(d["V"], d["W"])) <= o.grid_bound()
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    V = lib.degrid(plan, dev(X, torch.complex64), flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(V, o.degrid_grid(X)) <= 1e-5


@pytest.mark.parametrize("S", [7, 21])
def test_real_images(lib, S):
    # SEPW_REAL: a real model image goes into the prediction as float32, and
    # gridding can return the real part of the image; both must equal the
    # complex calls on the same data (the same arithmetic, so to rounding)
    d = _acc()
    # taper of width 11 at S = 21: the default width S makes 1/(c1 c1) lift the
    # rounding differences of two runs' FP32 atomics above 1e-6 over the inner half
    K = lib.Kernels(d["N"], d["fov"], S, d["O"], d["P"], d["w_lo"], d["w_hi"],
                    taper_width=min(S, 11))
    plan = lib.Plan(K, dev(d["u"], torch.float64), dev(d["v"], torch.float64),
                    dev(d["w"], torch.float64))
    rng = np.random.default_rng(5)
    N = d["N"]
    x = np.zeros((N, N), np.float32)
    x[N // 4:3 * N // 4, N // 4:3 * N // 4] = rng.standard_normal((N // 2, N // 2))
    vr = lib.degrid(plan, dev(x, torch.float32), flags=lib.DIV_N).cpu().numpy()
    vc = lib.degrid(plan, dev(x.astype(np.complex64), torch.complex64), flags=lib.DIV_N).cpu().numpy()
    assert rel_rms(vr, vc) <= 1e-6
    V, W = dev(d["V"], torch.complex64), dev(d["W"], torch.float32)
    ir = lib.grid(plan, V, W, flags=lib.DIV_N | lib.REAL)
    assert ir.dtype == torch.float32
    ic = lib.grid(plan, V, W, flags=lib.DIV_N).cpu().numpy()
    assert rel_rms(inner(ir.cpu().numpy()), inner(ic.real)) <= 1e-6
    with pytest.raises(lib.SepwError):
        lib.grid(plan, V, W, flags=lib.GRID_ONLY | lib.REAL)


def test_dropped_count_to_device_memory(lib):
    # n_dropped as a device pointer: written on the stream, equal to the
    # host count (which makes the call synchronise)
    d = _acc()
    rng = np.random.default_rng(9)
    d["u"] = d["u"].copy()
    d["u"][:37] = rng.uniform(31.0, 40.0, 37) / d["fov"]      # footprints off the grid
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], d["w_lo"], d["w_hi"])
    uvw = [dev(d[k], torch.float64) for k in ("u", "v", "w")]
    host = lib.Plan(K, *uvw)
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    plan = lib.Plan(K, *uvw, count_dropped=cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == host.n_dropped >= 37
    cnt2 = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    plan.rebin(uvw[0][:1000], uvw[1][:1000], uvw[2][:1000], count_dropped=cnt2)
    torch.cuda.synchronize()
    assert int(cnt2.item()) == int(_oracle(d, plan).q["dropped"][:1000].sum())
