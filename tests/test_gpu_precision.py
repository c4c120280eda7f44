"""Precision form: FP16 / BF16 MFMA operands with FP32 accumulation and
power-of-two operand scaling, against the FP64 oracle.

Tolerance 3e-3 relative RMS for grid, inner-half image and degridded
visibilities (a 16-bit operand rounds to 2^-11 (FP16) or 2^-8 (BF16)
relative; products of two rounded operands summed with random signs keep
roughly that relative RMS).  The measured errors are printed.
"""
import numpy as np
import pytest

from gpu_helpers import OracleSetup, dev, inner, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 3e-3


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


def _make(lib, d, precision, **kw):
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], d["w_lo"], d["w_hi"],
                    precision=precision, **kw)
    plan = lib.Plan(K, dev(d["u"], torch.float64), dev(d["v"], torch.float64), dev(d["w"], torch.float64))
    o = OracleSetup(d["u"], d["v"], d["w"], d["N"], d["fov"], d["S"], d["O"], d["P"], d["w_lo"],
                    d["w_hi"], plan.tile_size, **kw)
    return K, plan, o


def _inner_model(rng, N):
    X = np.zeros((N, N), complex)
    X[N // 4:3 * N // 4, N // 4:3 * N // 4] = (rng.standard_normal((N // 2, N // 2))
                                               + 1j * rng.standard_normal((N // 2, N // 2)))
    return X


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_grid_and_image(lib, precision):
    d = _acc()
    K, plan, o = _make(lib, d, precision)
    V, W = dev(d["V"], torch.complex64), dev(d["W"], torch.float32)
    G = lib.grid(plan, V, W, flags=lib.GRID_ONLY).cpu().numpy()
    e_grid = rel_rms(G, o.grid(d["V"], d["W"]))
    img = lib.grid(plan, V, W, flags=lib.MUL_N).cpu().numpy()
    e_img = rel_rms(inner(img), inner(o.image(d["V"], d["W"], n_power=1)))
    print("%s: grid %.2e image %.2e" % (precision, e_grid, e_img))
    assert e_grid <= TOL and e_img <= TOL


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_degrid(lib, precision):
    d = _acc()
    K, plan, o = _make(lib, d, precision)
    rng = np.random.default_rng(41)
    X = _inner_model(rng, d["N"])
    Vp = lib.degrid(plan, dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy()
    e = rel_rms(Vp, o.degrid_image(X, n_power=-1))
    G = rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))
    Vg = lib.degrid(plan, dev(G, torch.complex64), flags=lib.GRID_ONLY).cpu().numpy()
    e2 = rel_rms(Vg, o.degrid_grid(G))
    print("%s: degrid(image) %.2e degrid(grid) %.2e" % (precision, e, e2))
    assert e <= TOL and e2 <= TOL


@pytest.mark.parametrize("scale", [1e-5, 1e5])
def test_fp16_scaling_keeps_relative_error(lib, scale):
    # operand scaling: visibilities far outside FP16's comfortable range
    d = _acc()
    d["V"] = d["V"] * scale
    K, plan, o = _make(lib, d, "fp16")
    G = lib.grid(plan, dev(d["V"], torch.complex64), None, flags=lib.GRID_ONLY).cpu().numpy()
    e = rel_rms(G, o.grid(d["V"], d["W"]))
    X = _inner_model(np.random.default_rng(42), d["N"]) * scale
    Vp = lib.degrid(plan, dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy()
    e2 = rel_rms(Vp, o.degrid_image(X, n_power=-1))
    print("fp16 at scale %g: grid %.2e degrid %.2e" % (scale, e, e2))
    assert e <= TOL and e2 <= TOL


def test_facet_fp16(lib):
    d = _acc()
    facet = (0.03, -0.02)
    K, plan, o = _make(lib, d, "fp16", facet=facet)
    img = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                   flags=lib.MUL_N).cpu().numpy()
    assert rel_rms(inner(img), inner(o.image(d["V"], d["W"], n_power=1))) <= TOL


def test_heavy_tile_fp16(lib):
    d = _acc()
    rng = np.random.default_rng(43)
    n = 3000
    d["u"] = np.r_[d["u"], rng.uniform(0.0, 0.4, n) / d["fov"]]
    d["v"] = np.r_[d["v"], rng.uniform(0.0, 0.4, n) / d["fov"]]
    d["w"] = np.r_[d["w"], rng.uniform(-200, 200, n)]
    d["V"] = np.r_[d["V"], (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 50]
    d["W"] = rng.uniform(0.1, 3.0, len(d["u"]))
    K, plan, o = _make(lib, d, "bf16")
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(G, o.grid(d["V"], d["W"])) <= TOL


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_large_tables_cache_path(lib, precision):
    # P = 256, O = 8, S = 15: the FP32 v-table of the degridding epilogue is
    # 256 * 8 * 17 * 8 B = 278 KB, more than a workgroup's LDS, so the 16-bit
    # degridding kernel reads it through the caches (grid-stride items) instead
    # of staging it in LDS (per-XCD lists); both launches must match the oracle
    rng = np.random.default_rng(47)
    N, fov, S, O, P = 64, np.radians(2.0), 15, 8, 256
    n = 3000
    d = dict(u=rng.uniform(-24, 24, n) / fov, v=rng.uniform(-24, 24, n) / fov,
             w=rng.uniform(-200, 200, n), N=N, fov=fov, S=S, O=O, P=P, w_lo=-200.0, w_hi=200.0)
    V = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    W = rng.uniform(0.5, 2.0, n)
    K, plan, o = _make(lib, d, precision)
    G = lib.grid(plan, dev(V, torch.complex64), dev(W, torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    e_grid = rel_rms(G, o.grid(V, W))
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    Vg = lib.degrid(plan, dev(X, torch.complex64), flags=lib.GRID_ONLY).cpu().numpy()
    e_deg = rel_rms(Vg, o.degrid_grid(X))
    print("%s, P = 256: grid %.2e degrid %.2e" % (precision, e_grid, e_deg))
    assert e_grid <= TOL and e_deg <= TOL


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
@pytest.mark.parametrize("N,S", [(64, 15), (40, 7)])
def test_grid_corners(lib, precision, N, S):
    # Footprints at all four grid edges and corners with the 16-bit kernels:
    # the edge tiles' regions reach past the grid, so the ring flushes and the
    # region loads clip there (cells h .. N-1-h keep every footprint inside)
    rng = np.random.default_rng(53 + N)
    fov, O, P = np.radians(2.0), 8, 4
    h = S // 2
    lo, hi = h, N - 1 - h
    corners = np.array([(a, b) for a in (lo, hi) for b in (lo, hi)] * 30)
    edges = np.array([(a, b) for a in (lo, hi) for b in rng.integers(lo, hi + 1, 20)] +
                     [(b, a) for a in (lo, hi) for b in rng.integers(lo, hi + 1, 20)])
    cells = np.concatenate([corners, edges, rng.integers(lo, hi + 1, (300, 2))]).astype(float)
    n = len(cells)
    d = dict(u=(cells[:, 0] - N // 2 + rng.uniform(-0.4, 0.4, n)) / fov,
             v=(cells[:, 1] - N // 2 + rng.uniform(-0.4, 0.4, n)) / fov,
             w=rng.uniform(-100, 100, n), N=N, fov=fov, S=S, O=O, P=P, w_lo=-100.0, w_hi=100.0)
    V = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    W = rng.uniform(0.5, 2.0, n)
    K, plan, o = _make(lib, d, precision)
    G = lib.grid(plan, dev(V, torch.complex64), dev(W, torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    X = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    Vg = lib.degrid(plan, dev(X, torch.complex64), flags=lib.GRID_ONLY).cpu().numpy()
    e_grid, e_deg = rel_rms(G, o.grid(V, W)), rel_rms(Vg, o.degrid_grid(X))
    print("%s, N = %d, S = %d corners: grid %.2e degrid %.2e" % (precision, N, S, e_grid, e_deg))
    assert e_grid <= TOL and e_deg <= TOL
