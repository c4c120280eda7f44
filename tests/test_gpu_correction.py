"""GPU parity of the correction table F_w - F~_w (Section 6) against the oracle.

The library's FP64 generation (folded about the image centre) is compared
entry by entry with oracle.correction.correction_table (direct double sum)
within 1e-6 of the table's largest entry (FP32 storage), including the full
4096 grid and the largest tap-offset range; gridding and degridding with the
correction attached are compared with oracle.correction.grid / degrid on the
same bins within the FP32 bound 1e-5 (relative RMS, as the separable path),
for every lane layout of the passes (S_c^2 in 1, 9..16, 25..32, 49..64, 81..128
and 169..256 lanes) and for coarse samples that move to the next cell.
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


def _case(seed, N, S, O, P, n=2500, wmax=200.0, fov=1.0, spread=None):
    # a wide field and large w make the correction about 1 % of the grid, far
    # above the FP32 bound, so a pass that added nothing could not pass
    rng = np.random.default_rng(seed)
    cells = spread or (N / 2 - 2)
    # half the visibilities in a small patch (heavy tiles), the rest spread to the edges
    k = n // 2
    u = np.r_[rng.normal(0, 3, k), rng.uniform(-cells, cells, n - k)] / fov
    v = np.r_[rng.normal(0, 3, k), rng.uniform(-cells, cells, n - k)] / fov
    d = dict(u=u, v=v, w=rng.uniform(-wmax, wmax, n),
             V=rng.standard_normal(n) + 1j * rng.standard_normal(n), W=rng.uniform(0.5, 2.0, n),
             N=N, fov=fov, S=S, O=O, P=P, w_lo=-wmax, w_hi=wmax)
    return rng, d


def _make(lib, d, Sc, Oc, form="terms", **kw):
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], d["w_lo"], d["w_hi"], **kw)
    K.set_correction(Sc, Oc)
    if form == "table":
        K.correction_terms(False)
        assert K.correction_rank() == -1
    elif kw.get("precision", "fp32") == "fp32":
        assert 1 <= K.correction_rank() <= 8
    plan = lib.Plan(K, dev(d["u"], torch.float64), dev(d["v"], torch.float64), dev(d["w"], torch.float64))
    return K, plan


def _oracle_table(d, Sc, Oc, c1, a=0.5, b=5.0 / 24.0, a_v=None, b_v=None):
    wc = oracle.tables.w_plane_centres(d["P"], d["w_lo"], d["w_hi"])
    C = oracle.correction.correction_table(wc, d["N"], d["fov"], Sc, Oc, c1, a, b, a_v, b_v)
    return C


def _to_device_layout(C):
    return np.transpose(C, (0, 1, 2, 4, 3))      # [k][fu][fv][sv][su]


TABLE_CASES = [
    # N, S, O, P, Sc, Oc, kwargs
    (64, 7, 8, 3, 5, 8, {}),
    (18, 5, 4, 2, 3, 2, {}),                                   # N/2 odd: ragged fold rows
    (64, 15, 8, 2, 15, 8, {}),                                 # largest offset range (61 |d|)
    (40, 9, 8, 3, 7, 4, dict(a=0.43, b=0.1, a_v=0.61, b_v=0.3)),   # axes differ
    (32, 7, 8, 2, 5, 8, dict(taper="none")),
    (48, 5, 2, 5, 1, 1, {}),
]


@pytest.mark.parametrize("N,S,O,P,Sc,Oc,kw", TABLE_CASES)
def test_correction_table_matches_oracle(lib, N, S, O, P, Sc, Oc, kw):
    _, d = _case(1, N, S, O, P, n=10, fov=0.3)
    K = lib.Kernels(N, d["fov"], S, O, P, d["w_lo"], d["w_hi"], **kw)
    K.set_correction(Sc, Oc)
    got = K.correction_table().cpu().numpy()
    c1 = np.ones(N) if kw.get("taper") == "none" else oracle.pswf.taper_c1(N, d["fov"], S)
    want = _to_device_layout(_oracle_table(d, Sc, Oc, c1, kw.get("a", 0.5), kw.get("b", 5.0 / 24.0),
                                           kw.get("a_v"), kw.get("b_v")))
    assert np.max(np.abs(got - want)) <= 1e-6 * np.max(np.abs(want))


def test_correction_table_full_grid(lib):
    # 4096 grid: 33 folded column blocks per plane, 2048 folded rows
    d = dict(N=4096, fov=math.radians(3.0), S=15, O=8, P=2, w_lo=-3000.0, w_hi=3000.0)
    K = lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], d["w_lo"], d["w_hi"])
    K.set_correction(9, 8)
    got = K.correction_table().cpu().numpy()
    want = _to_device_layout(_oracle_table(d, 9, 8, oracle.pswf.taper_c1(d["N"], d["fov"], 15)))
    assert np.max(np.abs(got - want)) <= 1e-6 * np.max(np.abs(want))


def test_correction_table_zero_at_w_zero(lib):
    K = lib.Kernels(32, 0.3, 7, 8, 1, -5.0, 5.0)
    K.set_correction(5, 4)
    assert np.all(K.correction_table().cpu().numpy() == 0)


APPLY_CASES = [
    # N, S, O, P, Sc, Oc: lanes per visibility 32, 32 (next-cell moves), 64, 16, 1, 256, 128
    (64, 7, 8, 4, 5, 8),
    (64, 7, 8, 4, 5, 4),
    (64, 7, 8, 4, 7, 8),
    (64, 7, 8, 4, 3, 1),
    (64, 7, 4, 3, 1, 2),
    (96, 15, 8, 4, 13, 8),
    (96, 15, 8, 4, 9, 2),
]


@pytest.mark.parametrize("form", ["terms", "table"])
@pytest.mark.parametrize("N,S,O,P,Sc,Oc", APPLY_CASES)
def test_corrected_grid_matches_oracle(lib, N, S, O, P, Sc, Oc, form):
    _, d = _case(10 + Sc * Oc, N, S, O, P)
    K, plan = _make(lib, d, Sc, Oc, form)
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    o = OracleSetup(d["u"], d["v"], d["w"], N, d["fov"], S, O, P, d["w_lo"], d["w_hi"], plan.tile_size)
    C = _oracle_table(d, Sc, Oc, o.c1)
    want = oracle.correction.grid(o.q, d["V"] * d["W"], o.Tu, C, N, S, O, Sc, Oc)
    assert rel_rms(G, want) <= 1e-5
    # the correction is really there: without it the result differs by more
    plain = o.grid(d["V"], d["W"])
    assert rel_rms(plain, want) > 1e3 * max(rel_rms(G, want), 1e-9)


@pytest.mark.parametrize("form", ["terms", "table"])
@pytest.mark.parametrize("N,S,O,P,Sc,Oc", APPLY_CASES)
def test_corrected_degrid_matches_oracle(lib, N, S, O, P, Sc, Oc, form):
    rng, d = _case(20 + Sc * Oc, N, S, O, P)
    K, plan = _make(lib, d, Sc, Oc, form)
    G = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    V = lib.degrid(plan, dev(G, torch.complex64), flags=lib.GRID_ONLY).cpu().numpy()
    o = OracleSetup(d["u"], d["v"], d["w"], N, d["fov"], S, O, P, d["w_lo"], d["w_hi"], plan.tile_size)
    C = _oracle_table(d, Sc, Oc, o.c1)
    assert rel_rms(V, oracle.correction.degrid(o.q, G, o.Tu, C, N, S, O, Sc, Oc)) <= 1e-5


@pytest.mark.parametrize("form", ["terms", "table"])
def test_corrected_image_and_prediction(lib, form):
    rng, d = _case(31, 64, 9, 8, 4)
    K, plan = _make(lib, d, 7, 8, form)
    o = OracleSetup(d["u"], d["v"], d["w"], 64, d["fov"], 9, 8, 4, d["w_lo"], d["w_hi"], plan.tile_size)
    C = _oracle_table(d, 7, 8, o.c1)
    img = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                   flags=lib.MUL_N).cpu().numpy()
    want = oracle.imaging.image_from_grid(
        oracle.correction.grid(o.q, d["V"] * d["W"], o.Tu, C, 64, 9, 8, 7, 8), o.c1, d["fov"], 1)
    assert rel_rms(inner(img), inner(want)) <= 1e-5
    X = np.zeros((64, 64), complex)
    X[16:48, 16:48] = rng.standard_normal((32, 32))
    V = lib.degrid(plan, dev(X, torch.complex64), flags=lib.DIV_N).cpu().numpy()
    Vw = oracle.correction.degrid(o.q, oracle.imaging.grid_from_image(X, o.c1, d["fov"], -1),
                                  o.Tu, C, 64, 9, 8, 7, 8)
    assert rel_rms(V, Vw) <= 1e-5


def test_corrected_batched_matches_job_by_job(lib):
    _, d = _case(41, 64, 7, 8, 4)
    K = lib.Kernels(d["N"], d["fov"], 7, 8, 4, d["w_lo"], d["w_hi"])
    K.set_correction(5, 8)
    plans, vis = [], []
    for j in range(3):
        sl = slice(j * 800, (j + 1) * 800 + 37 * j)
        plans.append(lib.Plan(K, dev(d["u"][sl], torch.float64), dev(d["v"][sl], torch.float64),
                              dev(d["w"][sl], torch.float64)))
        vis.append(dev(d["V"][sl], torch.complex64))
    outs = lib.grid_batched(plans, vis, flags=lib.GRID_ONLY)
    for p, x, g in zip(plans, vis, outs):
        one = lib.grid(p, x, flags=lib.GRID_ONLY)
        assert rel_rms(g.cpu().numpy(), one.cpu().numpy()) <= 1e-6


def test_correction_removed_and_regenerated(lib):
    _, d = _case(51, 64, 7, 8, 4)
    K, plan = _make(lib, d, 5, 8)
    K.set_correction(0, 0)
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    o = OracleSetup(d["u"], d["v"], d["w"], 64, d["fov"], 7, 8, 4, d["w_lo"], d["w_hi"], plan.tile_size)
    assert rel_rms(G, o.grid(d["V"], d["W"])) <= o.grid_bound()
    # re-attached, then a new w range: the table follows the range
    K.set_correction(5, 4)
    K.set_wrange(-900.0, 700.0)
    d2 = dict(d, w_lo=-900.0, w_hi=700.0)
    want = _to_device_layout(_oracle_table(d2, 5, 4, o.c1))
    got = K.correction_table().cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-6 * np.max(np.abs(want))


def test_corrected_fp16_form(lib):
    _, d = _case(61, 64, 7, 8, 4)
    K, plan = _make(lib, d, 5, 8, precision="fp16")
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    o = OracleSetup(d["u"], d["v"], d["w"], 64, d["fov"], 7, 8, 4, d["w_lo"], d["w_hi"], plan.tile_size)
    want = oracle.correction.grid(o.q, d["V"] * d["W"], o.Tu, _oracle_table(d, 5, 8, o.c1), 64, 7, 8, 5, 8)
    assert rel_rms(G, want) <= 3e-3


def test_correction_argument_checks(lib):
    K = lib.Kernels(64, 0.1, 7, 8, 2, -100.0, 100.0)
    for sc, oc in [(4, 8), (-1, 8), (9, 8), (5, 16), (5, 3), (7, 4), (7, 2)]:
        with pytest.raises(lib.SepwError) as e:
            K.set_correction(sc, oc)
        assert e.value.code == lib.ERR_ARG
    K.set_correction(7, 1)                    # O_c = 1 keeps the visibility's cell: S_c = S allowed
    K.set_correction(5, 4)
    K16 = lib.Kernels(64, 0.1, 15, 16, 2, -100.0, 100.0)
    with pytest.raises(lib.SepwError) as e:   # (15/2) 16 + 8 = 120 > 63
        K16.set_correction(15, 16)
    assert e.value.code == lib.ERR_UNSUPPORTED
    Kf = lib.Kernels(64, 0.1, 7, 8, 2, -100.0, 100.0, facet=(0.05, 0.02))
    with pytest.raises(lib.SepwError) as e:
        Kf.set_correction(5, 8)
    assert e.value.code == lib.ERR_UNSUPPORTED
    samples = np.linspace(0.5, 1.0, 64)       # not symmetric about the centre
    Ku = lib.Kernels(64, 0.1, 7, 8, 2, -100.0, 100.0, taper="user", taper_samples=samples)
    with pytest.raises(lib.SepwError) as e:
        Ku.set_correction(5, 8)
    assert e.value.code == lib.ERR_UNSUPPORTED
    with pytest.raises(ValueError):
        Ku.correction_table()


def test_correction_terms_at_three_degrees(lib):
    # at a 3 degree field the exponent gap is l^2 m^2 and the two fourth
    # powers: three separable terms per plane
    fov = math.radians(3.0)
    K = lib.Kernels(256, fov, 15, 8, 8, -28000.0, 28000.0)
    K.set_correction(13, 8)
    assert K.correction_rank() == 3
    K.correction_terms(False)
    assert K.correction_rank() == -1
    K.correction_terms(True)
    assert K.correction_rank() == 3
    # a plane at w = 0 has no correction: no terms
    Z = lib.Kernels(32, 0.3, 7, 8, 1, -5.0, 5.0)
    Z.set_correction(5, 4)
    assert Z.correction_rank() == 0
    # the 16-bit kernels walk the table
    H = lib.Kernels(64, 1.0, 7, 8, 4, -200.0, 200.0, precision="fp16")
    H.set_correction(5, 8)
    assert H.correction_rank() == -1


@pytest.mark.parametrize("form", ["terms", "table"])
def test_corrected_step_at_three_degrees(lib, form):
    # the terms reproduce the table's footprints where the correction is tiny
    # (about 1e-7 of the separable kernel): both forms equal the oracle
    rng = np.random.default_rng(71)
    N, fov, S, O, P = 256, math.radians(3.0), 15, 8, 8
    n = 4000
    d = dict(u=rng.uniform(-120, 120, n) / fov, v=rng.uniform(-120, 120, n) / fov,
             w=rng.uniform(-28000.0, 28000.0, n),
             V=rng.standard_normal(n) + 1j * rng.standard_normal(n), W=rng.uniform(0.5, 2.0, n),
             N=N, fov=fov, S=S, O=O, P=P, w_lo=-28000.0, w_hi=28000.0)
    K, plan = _make(lib, d, 13, 8, form)
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    o = OracleSetup(d["u"], d["v"], d["w"], N, fov, S, O, P, d["w_lo"], d["w_hi"], plan.tile_size)
    C = _oracle_table(d, 13, 8, o.c1)
    want = oracle.correction.grid(o.q, d["V"] * d["W"], o.Tu, C, N, S, O, 13, 8)
    assert rel_rms(G, want) <= 1e-5


@pytest.mark.parametrize("P", [4, 80])
def test_corrected_asymmetric_axes(lib, P):
    # screens that differ per axis: the terms take the general (two-table)
    # form; at 80 planes a term's two tables no longer fit LDS together
    ax = dict(a=0.43, b=0.1, a_v=0.61, b_v=0.3)
    rng, d = _case(81 + P, 64, 7, 8, P)
    K, plan = _make(lib, d, 5, 8, **ax)
    assert 1 <= K.correction_rank() <= 8
    o = OracleSetup(d["u"], d["v"], d["w"], 64, d["fov"], 7, 8, P, d["w_lo"], d["w_hi"],
                    plan.tile_size)
    wc = oracle.tables.w_plane_centres(P, d["w_lo"], d["w_hi"])
    Tu = oracle.tables.separable_table(wc, 64, d["fov"], 7, 8, o.c1, a=ax["a"], b=ax["b"])
    Tv = oracle.tables.separable_table(wc, 64, d["fov"], 7, 8, o.c1, a=ax["a_v"], b=ax["b_v"])
    C = _oracle_table(d, 5, 8, o.c1, **ax)
    qc = oracle.correction.coarse_bins(o.q, 8, 8)
    y = d["V"] * d["W"]
    want = (oracle.gridder.grid_separable(o.q, y, Tu, 64, 7, Tv=Tv)
            + oracle.gridder.grid_exact(qc, y, C, 64, 5))
    G = lib.grid(plan, dev(d["V"], torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(G, want) <= 1e-5
    X = rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))
    wantv = (oracle.gridder.degrid_separable(o.q, X, Tu, 64, 7, Tv=Tv)
             + oracle.gridder.degrid_exact(qc, X, C, 64, 5))
    V = lib.degrid(plan, dev(X, torch.complex64), flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(V, wantv) <= 1e-5
