"""Where a NaN or Inf reaches, through the C ABI.

On the tiled MFMA path (S <= 15) a non-finite W V spreads over the 16 x 16
region of its tile (zero taps times NaN or Inf are NaN), never further: every
cell more than 16 cells from its own cell stays finite and equals the
oracle's grid of the same data with that visibility removed.  A non-finite
grid cell makes non-finite only visibilities within 16 cells of it, and the
others equal the oracle's prediction from the grid with that cell zeroed.
The footprint itself is always non-finite.  On the per-visibility path
(S = 17..31) the spread is exactly the footprint.  Tolerances: the FP32
grid bound, 1e-5 for FP32 predictions, 3e-3 for the 16-bit forms.
"""
import math

import numpy as np
import pytest

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


def _setup(lib, S, precision):
    from paper_1511_07152_amd import synth
    N, fov = 64, math.radians(2.0)
    d = synth.small_uniform(17 + S, 2000, N, fov, N / 2 - S / 2 - 2, 200.0)
    d["W"] = np.random.default_rng(5).uniform(0.5, 2.0, len(d["u"]))
    K = lib.Kernels(N, fov, S, 8, 8, -200.0, 200.0, precision=precision)
    plan = lib.Plan(K, dev(d["u"], torch.float64), dev(d["v"], torch.float64),
                    dev(d["w"], torch.float64))
    o = OracleSetup(d["u"], d["v"], d["w"], N, fov, S, 8, 8, -200.0, 200.0, plan.tile_size)
    return N, d, K, plan, o


def _near(xs, ys, x0, y0, r):
    return (np.abs(xs - x0) <= r) & (np.abs(ys - y0) <= r)


CASES = [(7, "fp32"), (7, "fp16"), (7, "bf16"), (21, "fp32")]


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("S,precision", CASES)
def test_grid_nonfinite_visibility(lib, S, precision, bad):
    N, d, K, plan, o = _setup(lib, S, precision)
    q, h = o.q, S // 2
    keep = ~q["dropped"]
    # a kept visibility near the centre
    j = int(np.flatnonzero(keep & _near(q["cell_u"], q["cell_v"], N // 2, N // 2, 4))[0])
    cu, cv = int(q["cell_u"][j]), int(q["cell_v"][j])
    V = d["V"].astype(np.complex64)
    V[j] = complex(bad, 0.0)
    G = lib.grid(plan, dev(V, torch.complex64), dev(d["W"], torch.float32),
                 flags=lib.GRID_ONLY).cpu().numpy()
    ys, xs = np.mgrid[0:N, 0:N]
    bad_cells = ~np.isfinite(G)
    assert bad_cells[_near(xs, ys, cu, cv, h)].all()
    reach = h if S > 15 else 16
    assert not bad_cells[~_near(xs, ys, cu, cv, reach)].any()
    V0 = d["V"].copy()
    V0[j] = 0
    want = o.grid(V0, d["W"])
    far = ~_near(xs, ys, cu, cv, reach)
    tol = o.grid_bound() if precision == "fp32" else 3e-3
    assert rel_rms(G[far], want[far]) <= tol


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("S,precision", CASES)
def test_degrid_nonfinite_cell(lib, S, precision, bad):
    N, d, K, plan, o = _setup(lib, S, precision)
    q, h = o.q, S // 2
    rng = np.random.default_rng(23)
    G = (rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))).astype(np.complex64)
    x0, y0 = N // 2 + 3, N // 2 - 2
    G[y0, x0] = complex(bad, bad)
    V = lib.degrid(plan, dev(G, torch.complex64), flags=lib.GRID_ONLY).cpu().numpy()
    keep = ~q["dropped"]
    cu, cv = q["cell_u"], q["cell_v"]
    bad_vis = ~np.isfinite(V)
    hit = keep & _near(cu, cv, x0, y0, h)
    assert hit.any() and bad_vis[hit].all()
    reach = h if S > 15 else 16
    assert not bad_vis[~(keep & _near(cu, cv, x0, y0, reach))].any()
    G0 = G.astype(complex)
    G0[y0, x0] = 0
    want = o.degrid_grid(G0)
    ok = ~bad_vis
    tol = 1e-5 if precision == "fp32" else 3e-3
    assert rel_rms(V[ok], want[ok]) <= tol
