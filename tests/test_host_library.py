"""Host-only checks of the C ABI: the library loads without a GPU, exports every
function include/sepw.h declares, and rejects invalid arguments before any
device work (or reports that no device is present)."""
import ctypes
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sepw.h")
LIB = os.path.join(ROOT, "paper_1511_07152_amd", "libsepw.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsepw.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sepw_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sepw_make_kernels", "sepw_plan_create", "sepw_grid", "sepw_degrid",
              "sepw_grid_batched", "sepw_free_kernels", "sepw_free_plan", "sepw_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def _params(lib, **kw):
    from paper_1511_07152_amd._lib import KernelParams
    p = KernelParams()
    lib.sepw_default_params(ctypes.byref(p))
    p.grid_size, p.support, p.oversample, p.n_planes = 64, 7, 8, 8
    p.fov, p.w_lo, p.w_hi = math.radians(2.0), -200.0, 200.0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.fixture(scope="module")
def lib():
    from paper_1511_07152_amd import _lib
    return _lib.load()


def test_defaults(lib):
    p = _params(lib)
    assert p.a_u == 0.5 and p.b_u == pytest.approx(5 / 24) and p.taper == 0 and p.precision == 0


BAD = [
    dict(grid_size=63), dict(grid_size=0), dict(support=8), dict(support=0), dict(support=65),
    dict(oversample=3), dict(oversample=0), dict(oversample=256), dict(n_planes=0),
    dict(fov=0.0), dict(fov=-1.0), dict(fov=float("nan")), dict(fov=2.0),
    dict(w_lo=1.0, w_hi=1.0), dict(w_lo=float("inf")), dict(taper=7), dict(precision=9),
    dict(taper=2),  # user taper without samples
    dict(facet=1, l0=0.8, m0=0.8),
]


@pytest.mark.parametrize("bad", BAD, ids=[str(b) for b in BAD])
def test_invalid_kernel_params_rejected(lib, bad):
    p = _params(lib, **bad)
    h = ctypes.c_void_p(1)
    rc = lib.sepw_make_kernels(ctypes.byref(p), None, ctypes.byref(h))
    assert rc == -1 and not h.value


def test_unsupported_support(lib):
    # above 31 cells, and above 15 for the 16-bit forms (the per-visibility
    # path of wide supports is FP32 only)
    for kw in (dict(support=33), dict(support=17, precision=1), dict(support=31, precision=2)):
        p = _params(lib, **kw)
        h = ctypes.c_void_p()
        assert lib.sepw_make_kernels(ctypes.byref(p), None, ctypes.byref(h)) == -5, kw
        assert not h.value


def test_wide_support_passes_validation(lib):
    # S = 17 .. 31 in FP32 is valid: without a device the call gets past the
    # argument checks to the device lookup
    if lib.sepw_device_count() > 0:
        pytest.skip("a device is present")
    for S in (17, 21, 31):
        p = _params(lib, support=S)
        h = ctypes.c_void_p()
        assert lib.sepw_make_kernels(ctypes.byref(p), None, ctypes.byref(h)) == -2


def test_no_device_reported_after_validation(lib):
    if lib.sepw_device_count() > 0:
        pytest.skip("a device is present")
    p = _params(lib)
    h = ctypes.c_void_p()
    assert lib.sepw_make_kernels(ctypes.byref(p), None, ctypes.byref(h)) == -2


def test_null_handles_rejected(lib):
    h = ctypes.c_void_p()
    assert lib.sepw_make_kernels(None, None, ctypes.byref(h)) == -1
    assert lib.sepw_plan_create(None, 10, None, None, None, None, None, ctypes.byref(h)) == -1
    assert lib.sepw_grid(None, None, None, None, 0, None) == -1
    assert lib.sepw_degrid(None, None, None, 0, None) == -1
    assert lib.sepw_grid_batched(0, None, None, None, None, 0, None) == -1
    assert lib.sepw_plan_set_item_slots(None, 256, None) == -1
    assert lib.sepw_plan_set_degrid_item_slots(None, 256, None) == -1
    assert lib.sepw_autotune_batched(0, None, None, None, None, None, None, None) == -1
    assert lib.sepw_wstack_create(None, 4, -1.0, 1.0, 10, None, None, None, None, None,
                                  ctypes.byref(h)) == -1
    assert lib.sepw_wstack_grid(None, None, None, None, 0, None) == -1
    assert lib.sepw_wstack_degrid(None, None, None, 0, None) == -1
    assert lib.sepw_free_wstack(None) == -1
    assert lib.sepw_kernels_set_correction(None, 5, 8, None) == -1
    assert lib.sepw_kernels_set_correction(None, 0, 0, None) == -1
    assert lib.sepw_kernels_correction_table(None, None, None) == -1
    assert lib.sepw_kernels_correction_terms(None, 1, None) == -1
    rank = ctypes.c_int32(0)
    assert lib.sepw_kernels_correction_rank(None, ctypes.byref(rank)) == -1
    assert lib.sepw_plan_create_channels(None, 10, 4, None, None, None, None, ctypes.byref(h)) == -1
    assert lib.sepw_plan_rebin_channels(None, 10, 4, None, None, None, None) == -1
    assert lib.sepw_wsnap_create(None, 2, None, None, None, None, None, None, ctypes.byref(h)) == -1
    assert lib.sepw_wsnap_grid(None, None, None, None, 0, None) == -1
    assert lib.sepw_wsnap_degrid(None, None, None, 0, None) == -1
    assert lib.sepw_wsnap_plane(None, 0, None, None) == -1
    assert lib.sepw_free_wsnap(None) == -1
    assert lib.sepw_free_kernels(None) == -1 and lib.sepw_free_plan(None) == -1
    assert lib.sepw_strerror(-1) == b"invalid argument"


def test_wstack_edges_arguments_rejected(lib):
    h = ctypes.c_void_p()
    E = ctypes.c_double * 4
    assert lib.sepw_wstack_create_edges(None, 3, E(-1.0, 0.0, 0.5, 1.0), 10, None, None, None,
                                        None, None, ctypes.byref(h)) == -1
    out = E()
    assert lib.sepw_wstack_density_edges(10, None, 3, -1.0, 1.0, out, None) == -1      # null w
    assert lib.sepw_wstack_density_edges(0, None, 0, -1.0, 1.0, out, None) == -1       # no slices
    assert lib.sepw_wstack_density_edges(0, None, 3, 1.0, -1.0, out, None) == -1       # range
    assert lib.sepw_wstack_density_edges(0, None, 3, -1.0, float("inf"), out, None) == -1
    assert lib.sepw_wstack_density_edges(0, None, 3, -1.0, 1.0, None, None) == -1      # null out
    if lib.sepw_device_count() == 0:
        assert lib.sepw_wstack_density_edges(0, None, 3, -1.0, 1.0, out, None) == -2
