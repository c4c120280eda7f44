"""GPU parity of the W-stacking hybrid (Section 4.3) against the oracle.

The library's slices, residual-w plans, per-slice imaging and image-space
phase are compared with oracle.wstack on the same seeded inputs: images over
the inner half and predicted visibilities within the FP32 bound 1e-5
(relative RMS), the adjoint identity within 1e-5, dropped counts exactly.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import dev, inner, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1511_07152_amd import _lib
    _lib.load()
    return _lib


def _case(seed, N=64, n=2500, ns=5, w_lo=-2000.0, w_hi=2000.0, cells=25):
    rng = np.random.default_rng(seed)
    fov = math.radians(3.0)
    d = dict(u=rng.uniform(-cells, cells, n) / fov, v=rng.uniform(-cells, cells, n) / fov,
             w=rng.uniform(w_lo, w_hi, n), V=rng.standard_normal(n) + 1j * rng.standard_normal(n),
             W=rng.uniform(0.5, 2.0, n), N=N, fov=fov, S=7, O=8, P=4, ns=ns, w_lo=w_lo, w_hi=w_hi)
    return rng, d


def _make(lib, d):
    h = (d["w_hi"] - d["w_lo"]) / (2 * d["ns"])
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], -h, h)
    ws = lib.WStack(K, d["ns"], d["w_lo"], d["w_hi"], dev(d["u"], torch.float64),
                    dev(d["v"], torch.float64), dev(d["w"], torch.float64))
    return K, ws


def _args(d):
    c1 = oracle.pswf.taper_c1(d["N"], d["fov"], d["S"])
    return (d["N"], d["fov"], d["S"], d["O"], d["P"], d["ns"], d["w_lo"], d["w_hi"], c1)


def test_wstack_image_matches_oracle(lib):
    rng, d = _case(61)
    K, ws = _make(lib, d)
    img = ws.grid(dev(d["V"], torch.complex64), dev(d["W"], torch.float32), flags=lib.MUL_N)
    want = oracle.wstack.image(d["u"], d["v"], d["w"], d["V"] * d["W"], *_args(d), n_power=1)
    assert rel_rms(inner(img.cpu().numpy()), inner(want)) <= 1e-5


def test_wstack_predict_matches_oracle(lib):
    rng, d = _case(62)
    K, ws = _make(lib, d)
    X = np.zeros((d["N"], d["N"]), complex)
    q = slice(d["N"] // 4, 3 * d["N"] // 4)
    X[q, q] = rng.standard_normal((d["N"] // 2, d["N"] // 2))
    V = ws.degrid(dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy()
    want = oracle.wstack.predict(d["u"], d["v"], d["w"], X, *_args(d), n_power=-1)
    assert rel_rms(V, want) <= 1e-5


def test_wstack_grid_and_degrid_are_adjoint(lib):
    rng, d = _case(63, ns=3)
    K, ws = _make(lib, d)
    y = d["V"]
    # model on the inner half only: towards the edges 1 / (c1 c1) amplifies the
    # FP32 rounding of the image far beyond the identity's scale (as in the
    # plain path's adjoint test)
    N = d["N"]
    X = np.zeros((N, N), complex)
    q = slice(N // 4, 3 * N // 4)
    X[q, q] = rng.standard_normal((N // 2, N // 2)) + 1j * rng.standard_normal((N // 2, N // 2))
    D = ws.grid(dev(y, torch.complex64), None, flags=lib.DIV_N).cpu().numpy().astype(complex)
    V = ws.degrid(dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy().astype(complex)
    lhs, rhs = np.vdot(X, D), np.vdot(V, y)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(D) * np.linalg.norm(X)


def test_wstack_dropped_count_and_empty_slices(lib):
    # w only in two of eight slices; some footprints leave the grid
    rng, d = _case(64, ns=8, cells=31)
    d["w"] = np.where(rng.random(len(d["w"])) < 0.5, -1900.0, 1100.0) + rng.uniform(-50, 50, len(d["w"]))
    K, ws = _make(lib, d)
    q = oracle.wstack.bins(d["u"], d["v"], d["w"], d["N"], d["fov"], d["O"], d["S"], d["P"],
                           d["ns"], d["w_lo"], d["w_hi"])
    assert ws.n_dropped == int(q["dropped"].sum()) and ws.n_dropped > 0
    img = ws.grid(dev(d["V"], torch.complex64), None).cpu().numpy()
    want = oracle.wstack.image(d["u"], d["v"], d["w"], d["V"], *_args(d))
    assert rel_rms(inner(img), inner(want)) <= 1e-5
    V = ws.degrid(dev(want, torch.complex64)).cpu().numpy()
    assert np.all(V[q["dropped"]] == 0)


def test_wstack_arguments_checked(lib):
    rng, d = _case(65, n=100)
    h = (d["w_hi"] - d["w_lo"]) / (2 * d["ns"])
    u, v, w = (dev(d[k], torch.float64) for k in ("u", "v", "w"))
    wrong = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], -2 * h, 2 * h)
    with pytest.raises(lib.SepwError):
        lib.WStack(wrong, d["ns"], d["w_lo"], d["w_hi"], u, v, w)
    K, ws = _make(lib, d)
    with pytest.raises(lib.SepwError):
        ws.grid(dev(d["V"], torch.complex64), None, flags=lib.GRID_ONLY)
    z = torch.zeros(0, dtype=torch.float64, device="cuda")
    empty = lib.WStack(K, d["ns"], d["w_lo"], d["w_hi"], z, z, z)
    img = empty.grid(torch.zeros(0, dtype=torch.complex64, device="cuda"), None)
    assert float(img.abs().max()) == 0.0


# ---- non-uniform slices (Section 4.3: narrow where w is dense)

EDGES = np.array([-2000.0, -700.0, -150.0, 0.0, 100.0, 900.0, 2000.0])


def _make_edges(lib, d, edges, **kw):
    # the kernels' own w range is not used: every slice gets tables on its range
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], -1.0, 1.0, **kw)
    ws = lib.WStack(K, len(edges) - 1, 0.0, 0.0, dev(d["u"], torch.float64),
                    dev(d["v"], torch.float64), dev(d["w"], torch.float64), edges=edges)
    return K, ws


def _args_edges(d, edges):
    c1 = oracle.pswf.taper_c1(d["N"], d["fov"], d["S"])
    return (d["N"], d["fov"], d["S"], d["O"], d["P"], len(edges) - 1, edges[0], edges[-1], c1)


def test_nonuniform_slices_match_oracle(lib):
    rng, d = _case(83, cells=31)
    d["w"][:50] = rng.uniform(-2500.0, 2500.0, 50)     # some beyond the outer edges
    K, ws = _make_edges(lib, d, EDGES)
    q = oracle.wstack.bins(d["u"], d["v"], d["w"], d["N"], d["fov"], d["O"], d["S"], d["P"],
                           len(EDGES) - 1, EDGES[0], EDGES[-1], edges=EDGES)
    assert ws.n_dropped == int(q["dropped"].sum()) and ws.n_dropped > 0
    img = ws.grid(dev(d["V"], torch.complex64), dev(d["W"], torch.float32), flags=lib.MUL_N)
    want = oracle.wstack.image(d["u"], d["v"], d["w"], d["V"] * d["W"], *_args_edges(d, EDGES),
                               n_power=1, edges=EDGES)
    assert rel_rms(inner(img.cpu().numpy()), inner(want)) <= 1e-5
    N = d["N"]
    X = np.zeros((N, N), complex)
    s = slice(N // 4, 3 * N // 4)
    X[s, s] = rng.standard_normal((N // 2, N // 2)) + 1j * rng.standard_normal((N // 2, N // 2))
    V = ws.degrid(dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy()
    wantv = oracle.wstack.predict(d["u"], d["v"], d["w"], X, *_args_edges(d, EDGES), n_power=-1,
                                  edges=EDGES)
    assert rel_rms(V, wantv) <= 1e-5
    assert np.all(V[q["dropped"]] == 0)


def test_uniform_edges_equal_uniform_slices(lib):
    rng, d = _case(84)
    K, ws = _make(lib, d)
    e = d["w_lo"] + np.arange(d["ns"] + 1) * (d["w_hi"] - d["w_lo"]) / d["ns"]
    K2, ws2 = _make_edges(lib, d, e)
    a = ws.grid(dev(d["V"], torch.complex64), None).cpu().numpy()
    b = ws2.grid(dev(d["V"], torch.complex64), None).cpu().numpy()
    assert rel_rms(inner(b), inner(a)) <= 1e-6


def test_density_edges_match_oracle(lib):
    rng = np.random.default_rng(85)
    w = np.r_[rng.laplace(0.0, 300.0, 300_000), rng.uniform(-6000, 6000, 1000), np.nan, np.inf,
              -np.inf, 4999.999, -5000.0]
    wd = dev(w, torch.float64)
    for ns in (1, 2, 7, 64, 1000):
        got = lib.density_edges(wd, ns, -5000.0, 5000.0)
        want = oracle.wstack.density_edges(w, ns, -5000.0, 5000.0, nfine=16384)
        assert np.array_equal(got, want), ns


def test_density_sliced_wstack_matches_oracle(lib):
    # core-heavy w: density-adapted slices are narrow near 0
    rng, d = _case(86)
    d["w"] = np.clip(rng.laplace(0.0, 150.0, len(d["w"])), -1999.0, 1999.0)
    e = lib.density_edges(dev(d["w"], torch.float64), 6, d["w_lo"], d["w_hi"])
    assert np.array_equal(e, oracle.wstack.density_edges(d["w"], 6, d["w_lo"], d["w_hi"],
                                                         nfine=16384))
    assert e[3] - e[2] < (e[1] - e[0]) / 4
    K, ws = _make_edges(lib, d, e)
    img = ws.grid(dev(d["V"], torch.complex64), dev(d["W"], torch.float32), flags=lib.MUL_N)
    want = oracle.wstack.image(d["u"], d["v"], d["w"], d["V"] * d["W"], *_args_edges(d, e),
                               n_power=1, edges=e)
    assert rel_rms(inner(img.cpu().numpy()), inner(want)) <= 1e-5


def test_nonuniform_slices_with_user_taper(lib):
    # a caller's taper samples reach every slice's tables and the corrections
    rng, d = _case(87)
    c1 = oracle.pswf.taper_c1(d["N"], d["fov"], 5)       # not the default width S = 7
    K, ws = _make_edges(lib, d, EDGES, taper="user", taper_samples=c1)
    img = ws.grid(dev(d["V"], torch.complex64), None)
    args = (d["N"], d["fov"], d["S"], d["O"], d["P"], len(EDGES) - 1, EDGES[0], EDGES[-1], c1)
    want = oracle.wstack.image(d["u"], d["v"], d["w"], d["V"], *args, edges=EDGES)
    assert rel_rms(inner(img.cpu().numpy()), inner(want)) <= 1e-5


def test_nonuniform_slices_reject_correction_tables(lib):
    rng, d = _case(88, n=100)
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], -1.0, 1.0)
    K.set_correction(5, 4)
    with pytest.raises(lib.SepwError) as e:
        lib.WStack(K, len(EDGES) - 1, 0.0, 0.0, dev(d["u"], torch.float64),
                   dev(d["v"], torch.float64), dev(d["w"], torch.float64), edges=EDGES)
    assert e.value.code == -5


def test_wstack_with_correction_equals_its_slices(lib):
    # the batched W-stacking launches with the correction (run as separable
    # terms) give what single-plan calls give slice by slice
    rng = np.random.default_rng(89)
    N, fov, S, O, P, ns, wmax, n = 64, 1.0, 7, 8, 4, 3, 600.0, 3000
    u = rng.uniform(-28, 28, n) / fov
    v = rng.uniform(-28, 28, n) / fov
    w = rng.uniform(-wmax, wmax, n)
    V = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    h = wmax / ns
    K = lib.Kernels(N, fov, S, O, P, -h, h)
    K.set_correction(5, 8)
    assert K.correction_rank() >= 1
    ws = lib.WStack(K, ns, -wmax, wmax, dev(u, torch.float64), dev(v, torch.float64),
                    dev(w, torch.float64))
    s, ws_c, dw = oracle.wstack.slice_of(w, ns, -wmax, wmax)
    X = np.zeros((N, N), complex)
    X[N // 4:3 * N // 4, N // 4:3 * N // 4] = rng.standard_normal((N // 2, N // 2))
    img = np.zeros((N, N), complex)
    Vs = np.zeros(n, complex)
    for k in range(ns):
        idx = np.flatnonzero(s == k)
        p = lib.Plan(K, dev(u[idx], torch.float64), dev(v[idx], torch.float64),
                     dev(dw[idx], torch.float64))
        g = lib.grid(p, dev(V[idx], torch.complex64), None, flags=lib.MUL_N).cpu().numpy()
        img += oracle.wstack.slice_phase(N, fov, ws_c[k], +1) * g
        Xk = X * oracle.wstack.slice_phase(N, fov, ws_c[k], -1)
        Vs[idx] = lib.degrid(p, dev(Xk, torch.complex64), flags=lib.DIV_N).cpu().numpy()
    got = ws.grid(dev(V, torch.complex64), None, flags=lib.MUL_N).cpu().numpy()
    assert rel_rms(inner(got), inner(img)) <= 1e-5
    gotv = ws.degrid(dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy()
    assert rel_rms(gotv, Vs) <= 1e-5
    # the correction is there: without it the prediction differs far more
    K.set_correction(0, 0)
    bare = lib.WStack(K, ns, -wmax, wmax, dev(u, torch.float64), dev(v, torch.float64),
                      dev(w, torch.float64)).degrid(dev(X, torch.complex64), flags=lib.DIV_N)
    assert rel_rms(bare.cpu().numpy(), Vs) > 1e-3


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_nonuniform_slices_in_16bit(lib, precision):
    # slice tables of the 16-bit forms (they use the caller kernels' operand
    # grid, FFT plan and work grid): within the 16-bit bound of the oracle
    rng, d = _case(90)
    K, ws = _make_edges(lib, d, EDGES, precision=precision)
    img = ws.grid(dev(d["V"], torch.complex64), dev(d["W"], torch.float32), flags=lib.MUL_N)
    want = oracle.wstack.image(d["u"], d["v"], d["w"], d["V"] * d["W"], *_args_edges(d, EDGES),
                               n_power=1, edges=EDGES)
    assert rel_rms(inner(img.cpu().numpy()), inner(want)) <= 3e-3
    N = d["N"]
    X = np.zeros((N, N), complex)
    s = slice(N // 4, 3 * N // 4)
    X[s, s] = rng.standard_normal((N // 2, N // 2)) + 1j * rng.standard_normal((N // 2, N // 2))
    V = ws.degrid(dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy()
    wantv = oracle.wstack.predict(d["u"], d["v"], d["w"], X, *_args_edges(d, EDGES), n_power=-1,
                                  edges=EDGES)
    assert rel_rms(V, wantv) <= 3e-3
