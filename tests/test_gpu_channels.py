"""GPU parity of the channel-shared coordinate layout (uvw per row in metres,
scaled per channel in the quantiser) against the oracle.

Bins are compared bit for bit with oracle.quantise on the oracle's own
channel coordinates (u = u_m (f / c)), plain and in facet mode; gridding and
degridding through a channel-shared plan match those through a plain plan on
the same coordinates (the same bins, so the same sums up to FP32 summation
order).
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import OracleSetup, dev, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1511_07152_amd import _lib
    _lib.load()
    return _lib


def _rows(seed, nrows, nchan, N=96, fov=math.radians(4.0)):
    rng = np.random.default_rng(seed)
    f = 700e6 + 3.1e6 * np.arange(nchan)
    lam = 299792458.0 / f.max()
    cells = N / 2 - 1          # the top channel reaches (and some visibilities leave) the edge
    uvw = np.stack([rng.uniform(-cells, cells, nrows) / fov * lam,
                    rng.uniform(-cells, cells, nrows) / fov * lam,
                    rng.uniform(-300, 300, nrows) * lam], axis=1)
    n = nrows * nchan
    V = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return uvw, f, V, dict(N=N, fov=fov, S=7, O=8, P=6)


def _kernels(lib, d, w_lo, w_hi, **kw):
    return lib.Kernels(d["N"], d["fov"], d["S"], d["O"], d["P"], w_lo, w_hi, **kw)


@pytest.mark.parametrize("nrows,nchan", [(1, 1), (700, 1), (513, 16), (300, 7)])
def test_channel_bins_bit_exact(lib, nrows, nchan):
    uvw, f, _, d = _rows(11 + nchan, nrows, nchan)
    u, v, w = oracle.quantise.channel_coordinates(uvw, f)
    K = _kernels(lib, d, -300.0 * 1.1, 300.0 * 1.1)
    plan = lib.Plan.from_channels(K, dev(uvw, torch.float64), dev(f, torch.float64))
    o = OracleSetup(u, v, w, d["N"], d["fov"], d["S"], d["O"], d["P"], -330.0, 330.0, plan.tile_size)
    assert np.array_equal(plan.bins().cpu().numpy().astype(np.int64), o.bins_array())
    assert plan.n_dropped == int(o.q["dropped"].sum())


def test_channel_bins_bit_exact_facet(lib):
    uvw, f, _, d = _rows(21, 400, 8, fov=math.radians(2.0))
    u, v, w = oracle.quantise.channel_coordinates(uvw, f)
    facet = (math.radians(1.5), math.radians(-1.0))
    K = _kernels(lib, d, -400.0, 400.0, facet=facet)
    plan = lib.Plan.from_channels(K, dev(uvw, torch.float64), dev(f, torch.float64))
    o = OracleSetup(u, v, w, d["N"], d["fov"], d["S"], d["O"], d["P"], -400.0, 400.0,
                    plan.tile_size, facet=facet)
    assert np.array_equal(plan.bins().cpu().numpy().astype(np.int64), o.bins_array())


def test_channel_plan_grids_like_plain_plan(lib):
    uvw, f, V, d = _rows(31, 900, 12)
    u, v, w = oracle.quantise.channel_coordinates(uvw, f)
    K = _kernels(lib, d, -330.0, 330.0)
    pc = lib.Plan.from_channels(K, dev(uvw, torch.float64), dev(f, torch.float64))
    pp = lib.Plan(K, dev(u, torch.float64), dev(v, torch.float64), dev(w, torch.float64))
    Vd = dev(V, torch.complex64)
    a = lib.grid(pc, Vd, flags=lib.GRID_ONLY).cpu().numpy()
    b = lib.grid(pp, Vd, flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(a, b) <= 1e-6
    rng = np.random.default_rng(5)
    X = dev(rng.standard_normal((d["N"], d["N"])) + 1j * rng.standard_normal((d["N"], d["N"])),
            torch.complex64)
    va = lib.degrid(pc, X, flags=lib.GRID_ONLY).cpu().numpy()
    vb = lib.degrid(pp, X, flags=lib.GRID_ONLY).cpu().numpy()
    assert rel_rms(va, vb) <= 1e-6
    o = OracleSetup(u, v, w, d["N"], d["fov"], d["S"], d["O"], d["P"], -330.0, 330.0, pc.tile_size)
    assert rel_rms(a, o.grid(V, np.ones(len(V)))) <= o.grid_bound()


def test_channel_rebin_smaller_batch_and_errors(lib):
    uvw, f, _, d = _rows(41, 600, 10)
    K = _kernels(lib, d, -330.0, 330.0)
    plan = lib.Plan.from_channels(K, dev(uvw, torch.float64), dev(f, torch.float64))
    uvw2, f2 = uvw[:250], f[:6]
    plan.rebin_channels(dev(uvw2, torch.float64), dev(f2, torch.float64), count_dropped=True)
    u, v, w = oracle.quantise.channel_coordinates(uvw2, f2)
    o = OracleSetup(u, v, w, d["N"], d["fov"], d["S"], d["O"], d["P"], -330.0, 330.0, plan.tile_size)
    assert np.array_equal(plan.bins().cpu().numpy().astype(np.int64), o.bins_array())
    assert plan.n_dropped == int(o.q["dropped"].sum())
    with pytest.raises(lib.SepwError) as e:     # above the plan's capacity
        plan.rebin_channels(dev(uvw, torch.float64), dev(np.r_[f, f], torch.float64))
    assert e.value.code == lib.ERR_ARG
    empty = lib.Plan.from_channels(K, torch.zeros((0, 3), dtype=torch.float64, device="cuda"),
                                   dev(f, torch.float64))
    assert empty.nvis == 0 and empty.n_dropped == 0
