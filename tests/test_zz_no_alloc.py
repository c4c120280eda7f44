"""sepw_grid_batched_noalloc (the batched gridding call that allocates
nothing) against sepw_grid_batched on the same jobs, through the C ABI: two
calls in a row, the second with fewer and smaller jobs, to the batched bound
1e-6 (the two calls run the same kernels; only the order of the FP32 atomic
additions may differ); and the size limit."""
import ctypes
import math

import numpy as np
import pytest

from gpu_helpers import dev, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1511_07152_amd import _lib
    _lib.load()
    return _lib


def _facet_jobs(lib, seed, N, fov, S, counts):
    rng = np.random.default_rng(seed)
    plans, Ks, vis, wts = [], [], [], []
    for n in counts:
        l0, m0 = math.radians(rng.uniform(-4, 4)), math.radians(rng.uniform(-4, 4))
        cells = N / 2 - 8
        u = rng.uniform(-cells, cells, n) / fov
        v = rng.uniform(-cells, cells, n) / fov
        w = rng.uniform(-300, 300, n)
        K = lib.Kernels(N, fov, S, 8, 8, -350.0, 350.0, facet=(l0, m0))
        Ks.append(K)
        plans.append(lib.Plan(K, dev(u, torch.float64), dev(v, torch.float64), dev(w, torch.float64)))
        vis.append(dev(rng.standard_normal(n) + 1j * rng.standard_normal(n), torch.complex64))
        wts.append(dev(rng.uniform(0.5, 1.5, n), torch.float32))
    return plans, Ks, vis, wts


@pytest.mark.parametrize("flags", ["MUL_N", "GRID_ONLY"])
def test_noalloc_matches_batched_twice(lib, flags):
    f = getattr(lib, flags)
    N, fov, S = 128, math.radians(1.5), 11
    for seed, counts in ((61, [5000, 17, 0, 2300, 800, 1, 12000]), (62, [900, 3, 40])):
        plans, Ks, vis, wts = _facet_jobs(lib, seed, N, fov, S, counts)
        want = [x.cpu().numpy() for x in lib.grid_batched(plans, vis, wts, flags=f)]
        got = [x.cpu().numpy() for x in lib.grid_batched(plans, vis, wts, flags=f, noalloc=True)]
        torch.cuda.synchronize()
        print("noalloc, %d jobs: %s" % (len(counts), flags), flush=True)
        for j, n in enumerate(counts):
            if n == 0:
                assert np.abs(got[j]).max() == 0.0
                continue
            g, w = (got[j], want[j]) if flags == "GRID_ONLY" else (got[j][32:96, 32:96], want[j][32:96, 32:96])
            assert rel_rms(g, w) <= 1e-6, (j, n)
        for p in plans:
            p.close()
        for K in Ks:
            K.close()


def test_noalloc_rejects_too_many_jobs(lib):
    N, fov, S = 64, math.radians(1.5), 7
    plans, Ks, vis, wts = _facet_jobs(lib, 63, N, fov, S, [50])
    n = 257
    out = torch.zeros((N, N), dtype=torch.complex64, device="cuda")
    arr = ctypes.c_void_p * n
    hp = arr(*([plans[0].handle] * n))
    vp = arr(*([vis[0].data_ptr()] * n))
    op = arr(*([out.data_ptr()] * n))
    rc = lib.load().sepw_grid_batched_noalloc(n, hp, vp, None, op, lib.GRID_ONLY, None)
    assert rc == -5   # SEPW_ERR_UNSUPPORTED, before any device work
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
    plans[0].close()
    Ks[0].close()
