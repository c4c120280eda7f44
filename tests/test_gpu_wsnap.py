"""GPU parity of W snapshots (Section 4.2) against the oracle.

The library's per-snapshot planes (FP64, block-ordered sums) are compared with
oracle.wsnap.fit_plane within 1e-12 relative; images (inner half) and
predicted visibilities with oracle.wsnap.image / predict within the FP32
bound 1e-5 (relative RMS), on snapshots whose planes tilt enough that the
reprojection moves the image by several pixels at the edges (the scatter form
of the transposed reprojection) and on mildly tilted ones (its gather form);
the adjoint identity within 1e-5; empty and degenerate snapshots; argument
checks.
"""
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


# geometries: a strong tilt (the transposed reprojection scatters with
# atomics) and a mild one (warp within 0.1 of the identity: the gather form)
GEOMETRIES = {"scatter": dict(fov=0.4, dmax=2.5), "gather": dict(fov=0.05, dmax=1.5)}


def _case(seed, N=64, fov=0.4, sizes=(700, 0, 1, 900, 500), dmax=2.5):
    rng = np.random.default_rng(seed)
    cells = N / 2 - 6
    us, vs, ws = [], [], []
    for n in sizes:
        d = rng.uniform(-dmax, dmax, 2)               # each snapshot its own plane
        u = rng.uniform(-cells, cells, n) / fov
        v = rng.uniform(-cells, cells, n) / fov
        us.append(u)
        vs.append(v)
        ws.append(d[0] * u + d[1] * v + rng.normal(0, 2.0, n))
    offs = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    u, v, w = np.concatenate(us), np.concatenate(vs), np.concatenate(ws)
    n = len(u)
    return rng, dict(u=u, v=v, w=w, offs=offs, N=N, fov=fov, S=7, O=8, P=4,
                     V=rng.standard_normal(n) + 1j * rng.standard_normal(n),
                     W=rng.uniform(0.5, 2.0, n))


def _make(lib, d):
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], -1.0, 1.0)
    ws = lib.WSnap(K, d["offs"], dev(d["u"], torch.float64), dev(d["v"], torch.float64),
                   dev(d["w"], torch.float64))
    return K, ws


def _args(d):
    c1 = oracle.pswf.taper_c1(d["N"], d["fov"], d["S"])
    return (list(d["offs"]), d["N"], d["fov"], d["S"], d["O"], d["P"], c1)


def test_planes_match_oracle(lib):
    _, d = _case(71)
    K, ws = _make(lib, d)
    d0, _, h = oracle.wsnap.residuals(d["u"], d["v"], d["w"], list(d["offs"]))
    for s in range(len(d["offs"]) - 1):
        got, hg = ws.plane(s)
        assert np.allclose(got, d0[s], rtol=1e-12, atol=1e-15)
    assert abs(hg - h) <= 1e-12 * h
    assert ws.plane(1)[0] == (0.0, 0.0) and ws.plane(2)[0] == (0.0, 0.0)   # empty, single


@pytest.mark.parametrize("geom", ["scatter", "gather"])
@pytest.mark.parametrize("flags,npow", [(0, 0), ("MUL_N", 1), ("DIV_N", -1)])
def test_wsnap_image_matches_oracle(lib, flags, npow, geom):
    _, d = _case(72, **GEOMETRIES[geom])
    K, ws = _make(lib, d)
    f = getattr(lib, flags) if flags else 0
    img = ws.grid(dev(d["V"], torch.complex64), dev(d["W"], torch.float32), flags=f).cpu().numpy()
    want = oracle.wsnap.image(d["u"], d["v"], d["w"], d["V"] * d["W"], *_args(d), n_power=npow)
    assert rel_rms(inner(img), inner(want)) <= 1e-5


@pytest.mark.parametrize("geom", ["scatter", "gather"])
def test_wsnap_predict_matches_oracle(lib, geom):
    rng, d = _case(73, **GEOMETRIES[geom])
    K, ws = _make(lib, d)
    N = d["N"]
    X = np.zeros((N, N), complex)
    X[N // 4:3 * N // 4, N // 4:3 * N // 4] = rng.standard_normal((N // 2, N // 2))
    V = ws.degrid(dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy()
    want = oracle.wsnap.predict(d["u"], d["v"], d["w"], X, *_args(d), n_power=-1)
    assert rel_rms(V, want) <= 1e-5


@pytest.mark.parametrize("geom", ["scatter", "gather"])
def test_wsnap_grid_and_degrid_are_adjoint(lib, geom):
    rng, d = _case(74, **GEOMETRIES[geom])
    K, ws = _make(lib, d)
    N = d["N"]
    X = np.zeros((N, N), complex)
    X[N // 4:3 * N // 4, N // 4:3 * N // 4] = (rng.standard_normal((N // 2, N // 2))
                                               + 1j * rng.standard_normal((N // 2, N // 2)))
    y = d["V"]
    Gy = ws.grid(dev(y, torch.complex64), flags=lib.DIV_N).cpu().numpy().astype(complex)
    GX = ws.degrid(dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy().astype(complex)
    lhs, rhs = np.vdot(X, Gy), np.vdot(GX, y)
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(Gy) * np.linalg.norm(X)


def test_wsnap_argument_checks(lib):
    _, d = _case(75, sizes=(50, 60))
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], -1.0, 1.0)
    u, v, w = (dev(d[k], torch.float64) for k in ("u", "v", "w"))
    for offs in ([1, 110], [0, 60, 50], [0]):
        with pytest.raises((lib.SepwError, ValueError)) as e:
            lib.WSnap(K, offs, u, v, w)
        if isinstance(e.value, lib.SepwError):
            assert e.value.code == lib.ERR_ARG
    Kf = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], -1.0, 1.0, facet=(0.02, 0.01))
    with pytest.raises(lib.SepwError) as e:
        lib.WSnap(Kf, [0, 110], u, v, w)
    assert e.value.code == lib.ERR_UNSUPPORTED
    ws = lib.WSnap(K, [0, 50, 110], u, v, w)
    with pytest.raises(lib.SepwError):
        ws.grid(dev(d["V"], torch.complex64), flags=lib.GRID_ONLY)
    with pytest.raises(lib.SepwError):
        ws.degrid(torch.zeros((d["N"], d["N"]), dtype=torch.complex64, device="cuda"), flags=lib.MUL_N)


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_wsnap_in_16bit(lib, precision):
    # the 16-bit forms go snapshot by snapshot through the single-plan calls
    # (the transposed reprojection, then the 16-bit degridder's operand grid)
    rng, d = _case(77, **GEOMETRIES["gather"])
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], -1.0, 1.0, precision=precision)
    ws = lib.WSnap(K, d["offs"], dev(d["u"], torch.float64), dev(d["v"], torch.float64),
                   dev(d["w"], torch.float64))
    img = ws.grid(dev(d["V"], torch.complex64), dev(d["W"], torch.float32)).cpu().numpy()
    want = oracle.wsnap.image(d["u"], d["v"], d["w"], d["V"] * d["W"], *_args(d))
    assert rel_rms(inner(img), inner(want)) <= 3e-3
    N = d["N"]
    X = np.zeros((N, N), complex)
    X[N // 4:3 * N // 4, N // 4:3 * N // 4] = rng.standard_normal((N // 2, N // 2))
    V = ws.degrid(dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy()
    assert rel_rms(V, oracle.wsnap.predict(d["u"], d["v"], d["w"], X, *_args(d), n_power=-1)) <= 3e-3
