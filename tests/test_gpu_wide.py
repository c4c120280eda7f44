"""GPU parity for supports above the 16-cell MFMA region (S = 17..31, the
per-visibility FP32 path) against the FP64 oracle, through the C ABI.

Bins are bit-exact; grids within the FP32 bound (1e-6, or sqrt(K) 2^-24
where the heaviest cell sums K footprints: at S = 31 a cell takes up to a
few thousand of them); images over the inner half and degridded
visibilities 1e-5; the adjoint identity 1e-5.  The batched calls take the
job-by-job route for these supports and must equal the per-plan calls to
1e-6 (the FP32 atomics add in no fixed order).
"""
import math

import numpy as np
import pytest

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


def _data(N, S, nvis, seed, fov_deg=2.0, wmax=300.0):
    from paper_1511_07152_amd import synth
    fov = math.radians(fov_deg)
    cells = N / 2 - S / 2 - 2          # footprints inside the grid (a few off it below)
    d = synth.small_uniform(seed, nvis, N, fov, cells, wmax)
    rng = np.random.default_rng(seed + 1)
    # a few visibilities whose footprint leaves the grid: dropped and counted
    d["u"][:5] = rng.uniform(N / 2 - S / 2 + 0.5, N / 2, 5) / fov
    d.update(N=N, fov=fov, S=S, O=8, P=8, w_lo=-wmax, w_hi=wmax)
    d["W"] = rng.uniform(0.5, 2.0, nvis)
    return d


def _make(lib, d, **kw):
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], d["w_lo"], d["w_hi"], **kw)
    plan = lib.Plan(K, dev(d["u"], torch.float64), dev(d["v"], torch.float64),
                    dev(d["w"], torch.float64))
    return K, plan


def _oracle(d, plan, **kw):
    return OracleSetup(d["u"], d["v"], d["w"], d["N"], d["fov"], d["S"], d["O"], d["P"],
                       d["w_lo"], d["w_hi"], plan.tile_size, **kw)


CASES = [(64, 21, 1500), (64, 17, 700), (128, 31, 1200)]


@pytest.mark.parametrize("N,S,nvis", CASES)
def test_bins_and_grid(lib, N, S, nvis):
    d = _data(N, S, nvis, seed=S)
    K, plan = _make(lib, d)
    o = _oracle(d, plan)
    assert plan.tile_size == 33 - S
    assert np.array_equal(plan.bins().cpu().numpy().astype(np.int64), o.bins_array())
    assert plan.n_dropped == int(o.q["dropped"].sum()) >= 5
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(G, o.grid(d["V"], d["W"])) <= o.grid_bound()


@pytest.mark.parametrize("N,S,nvis", CASES)
def test_degrid_from_grid(lib, N, S, nvis):
    d = _data(N, S, nvis, seed=100 + S)
    K, plan = _make(lib, d)
    o = _oracle(d, plan)
    rng = np.random.default_rng(7)
    G = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64)
    V = lib.degrid(plan, dev(G, torch.complex64), flags=lib.GRID_ONLY).cpu().numpy()
    want = o.degrid_grid(G.astype(complex))
    assert np.all(V[o.q["dropped"]] == 0)
    assert rel_rms(V, want) <= 1e-5


# Images and predictions use a taper of width 11 cells: with the default width
# (= S) the PSWF of a 21- or 31-cell support falls so steeply that 1/(c1 c1)
# amplifies FP32 rounding far more over the inner half than the 1e-5 bound
# allows (about 1/c1(fov/4)^2 ~ 1e4 at W = 21), a property of the taper, not
# of the gridding.
@pytest.mark.parametrize("flags,npow", [(0, 0), ("MUL_N", 1)])
def test_image(lib, flags, npow):
    d = _data(64, 21, 1500, seed=3)
    K, plan = _make(lib, d, taper_width=11.0)
    f = getattr(lib, flags) if flags else 0
    img = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                   flags=f).cpu().numpy()
    want = _oracle(d, plan, width=11.0).image(d["V"], d["W"], n_power=npow)
    assert rel_rms(inner(img), inner(want)) <= 1e-5


def test_degrid_from_image_and_adjoint(lib):
    d = _data(128, 31, 1200, seed=9)
    N = d["N"]
    K, plan = _make(lib, d, taper_width=11.0)
    o = _oracle(d, plan, width=11.0)
    rng = np.random.default_rng(11)
    X = np.zeros((N, N), complex)
    s = slice(N // 4, 3 * N // 4)
    X[s, s] = rng.standard_normal((N // 2, N // 2)) + 1j * rng.standard_normal((N // 2, N // 2))
    V = lib.degrid(plan, dev(X.astype(np.complex64), torch.complex64), flags=lib.DIV_N).cpu().numpy()
    assert rel_rms(V, o.degrid_image(X, n_power=-1)) <= 1e-5
    # <A y, X> = <y, A^H X> for the pair grid(DIV_N) / degrid(DIV_N), unit weights
    y = (rng.standard_normal(len(d["u"])) + 1j * rng.standard_normal(len(d["u"]))).astype(np.complex64)
    y[o.q["dropped"]] = 0
    Ay = lib.grid(plan, dev(y, torch.complex64), None, flags=lib.DIV_N).cpu().numpy().astype(complex)
    lhs, rhs = np.vdot(X, Ay), np.vdot(V.astype(complex), y.astype(complex))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(Ay) * np.linalg.norm(X)


def test_facet_grid(lib):
    d = _data(64, 21, 1000, seed=21)
    facet = (0.01, -0.015)
    K, plan = _make(lib, d, facet=facet)
    o = _oracle(d, plan, facet=facet)
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(G, o.grid(d["V"], d["W"])) <= o.grid_bound()


def test_batched_equals_per_plan(lib):
    ds = [_data(64, 21, n, seed=50 + i) for i, n in enumerate((900, 10, 400))]
    K = lib.Kernels(64, ds[0]["fov"], 21, 8, 8, -300.0, 300.0)
    plans = [lib.Plan(K, dev(d["u"], torch.float64), dev(d["v"], torch.float64),
                      dev(d["w"], torch.float64)) for d in ds]
    vis = [dev(d["V"], torch.complex64) for d in ds]
    wts = [dev(d["W"], torch.float32) for d in ds]
    got = lib.grid_batched(plans, vis, wts, flags=lib.GRID_ONLY)
    for p, v, w, g in zip(plans, vis, wts, got):
        want = lib.grid(p, v, w, flags=lib.GRID_ONLY)
        # FP32 atomics add in no fixed order: equal to rounding
        assert rel_rms(g.cpu().numpy(), want.cpu().numpy()) <= 1e-6


def test_wide_rejects_16bit_and_correction(lib):
    with pytest.raises(Exception):
        lib.Kernels(64, math.radians(2.0), 21, 8, 8, -300.0, 300.0, precision="fp16")
    K = lib.Kernels(64, math.radians(2.0), 21, 8, 8, -300.0, 300.0)
    with pytest.raises(Exception):
        K.set_correction(13, 8)
