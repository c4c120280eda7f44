"""ctypes binding of libsepw.so (include/sepw.h).

Argument marshalling only: torch tensors supply device memory and the current
HIP stream; every step of the computation runs in the library's kernels.  The
library is loaded from this package directory and must have been built
(``python -m paper_1511_07152_amd.build``); a missing library raises.
"""
import ctypes
import os

import torch  # noqa: F401  (load torch's HIP runtime before the library binds to it)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsepw.so")

OK, ERR_ARG, ERR_NO_DEVICE, ERR_HIP, ERR_OOM, ERR_UNSUPPORTED, ERR_FFT = 0, -1, -2, -3, -4, -5, -6
TAPER_PSWF, TAPER_NONE, TAPER_USER = 0, 1, 2
FP32, FP16, BF16 = 0, 1, 2
GRID_ONLY, MUL_N, DIV_N, REAL = 0x1, 0x2, 0x4, 0x8

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class KernelParams(ctypes.Structure):
    _fields_ = [
        ("grid_size", c_int32), ("support", c_int32), ("oversample", c_int32), ("n_planes", c_int32),
        ("fov", c_double), ("w_lo", c_double), ("w_hi", c_double),
        ("taper", c_int32), ("precision", c_int32), ("taper_width", c_double),
        ("taper_samples", ctypes.POINTER(c_double)),
        ("a_u", c_double), ("b_u", c_double), ("a_v", c_double), ("b_v", c_double),
        ("facet", c_int32), ("reserved", c_int32), ("l0", c_double), ("m0", c_double),
    ]


class SepwError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (what, _strerror(code), code))


_lib = None


def load():
    """Load libsepw.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsepw.so is not built (%s); run python -m paper_1511_07152_amd.build"
                           % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.sepw_default_params.argtypes = [P(KernelParams)]
    lib.sepw_default_params.restype = None
    lib.sepw_make_kernels.argtypes = [P(KernelParams), c_void_p, P(c_void_p)]
    lib.sepw_kernels_table.argtypes = [c_void_p, c_int32, c_void_p, c_void_p]
    lib.sepw_kernels_taper.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.sepw_kernels_set_correction.argtypes = [c_void_p, c_int32, c_int32, c_void_p]
    lib.sepw_kernels_correction_table.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.sepw_kernels_correction_rank.argtypes = [c_void_p, P(c_int32)]
    lib.sepw_kernels_correction_terms.argtypes = [c_void_p, c_int32, c_void_p]
    lib.sepw_plan_create.argtypes = [c_void_p, c_int64, c_void_p, c_void_p, c_void_p,
                                     P(c_int64), c_void_p, P(c_void_p)]
    lib.sepw_plan_bins.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.sepw_plan_create_channels.argtypes = [c_void_p, c_int64, c_int32, c_void_p, c_void_p,
                                              P(c_int64), c_void_p, P(c_void_p)]
    lib.sepw_plan_rebin_channels.argtypes = [c_void_p, c_int64, c_int32, c_void_p, c_void_p,
                                             P(c_int64), c_void_p]
    lib.sepw_plan_rebin.argtypes = [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, P(c_int64),
                                    c_void_p]
    lib.sepw_kernels_set_wrange.argtypes = [c_void_p, c_double, c_double, c_void_p]
    lib.sepw_timing_enable.argtypes = [c_int32]
    lib.sepw_timing_collect.argtypes = [P(c_double), P(c_int64)]
    lib.sepw_plan_tile_size.argtypes = [c_void_p]
    lib.sepw_grid.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_uint32, c_void_p]
    lib.sepw_degrid.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.c_uint32, c_void_p]
    lib.sepw_grid_batched.argtypes = [c_int32, P(c_void_p), P(c_void_p), P(c_void_p), P(c_void_p),
                                      ctypes.c_uint32, c_void_p]
    lib.sepw_grid_batched_noalloc.argtypes = lib.sepw_grid_batched.argtypes
    lib.sepw_plan_set_item_slots.argtypes = [c_void_p, c_int32, c_void_p]
    lib.sepw_plan_set_degrid_item_slots.argtypes = [c_void_p, c_int32, c_void_p]
    lib.sepw_autotune_batched.argtypes = [c_int32, P(c_void_p), P(c_void_p), P(c_void_p),
                                          P(c_void_p), c_void_p, P(c_int32), P(c_int32)]
    lib.sepw_wstack_create.argtypes = [c_void_p, c_int32, c_double, c_double, c_int64, c_void_p,
                                       c_void_p, c_void_p, P(c_int64), c_void_p, P(c_void_p)]
    lib.sepw_wstack_create_edges.argtypes = [c_void_p, c_int32, P(c_double), c_int64, c_void_p,
                                             c_void_p, c_void_p, P(c_int64), c_void_p, P(c_void_p)]
    lib.sepw_wstack_density_edges.argtypes = [c_int64, c_void_p, c_int32, c_double, c_double,
                                              P(c_double), c_void_p]
    lib.sepw_wstack_grid.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_uint32,
                                     c_void_p]
    lib.sepw_wstack_degrid.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.c_uint32, c_void_p]
    lib.sepw_free_wstack.argtypes = [c_void_p]
    lib.sepw_wsnap_create.argtypes = [c_void_p, c_int32, P(c_int64), c_void_p, c_void_p, c_void_p,
                                      P(c_int64), c_void_p, P(c_void_p)]
    lib.sepw_wsnap_grid.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_uint32, c_void_p]
    lib.sepw_wsnap_degrid.argtypes = [c_void_p, c_void_p, c_void_p, ctypes.c_uint32, c_void_p]
    lib.sepw_wsnap_plane.argtypes = [c_void_p, c_int32, P(c_double), P(c_double)]
    lib.sepw_free_wsnap.argtypes = [c_void_p]
    lib.sepw_free_kernels.argtypes = [c_void_p]
    lib.sepw_free_plan.argtypes = [c_void_p]
    lib.sepw_strerror.argtypes = [ctypes.c_int]
    lib.sepw_strerror.restype = ctypes.c_char_p
    lib.sepw_device_count.argtypes = []
    for name in ("sepw_make_kernels", "sepw_kernels_table", "sepw_kernels_taper", "sepw_plan_create",
                 "sepw_plan_bins", "sepw_plan_tile_size", "sepw_grid", "sepw_degrid",
                 "sepw_grid_batched", "sepw_grid_batched_noalloc", "sepw_free_kernels",
                 "sepw_free_plan", "sepw_device_count",
                 "sepw_plan_rebin", "sepw_kernels_set_wrange", "sepw_timing_enable",
                 "sepw_timing_collect", "sepw_plan_set_item_slots", "sepw_plan_set_degrid_item_slots",
                 "sepw_autotune_batched", "sepw_wstack_create", "sepw_wstack_grid",
                 "sepw_wstack_degrid", "sepw_free_wstack", "sepw_kernels_set_correction",
                 "sepw_kernels_correction_table", "sepw_kernels_correction_rank",
                 "sepw_kernels_correction_terms",
                 "sepw_plan_create_channels",
                 "sepw_plan_rebin_channels", "sepw_wsnap_create", "sepw_wsnap_grid",
                 "sepw_wsnap_degrid", "sepw_wsnap_plane", "sepw_free_wsnap"):
        getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


def _strerror(code):
    try:
        return load().sepw_strerror(code).decode()
    except Exception:  # pragma: no cover
        return "error"


def _check(rc, what):
    if rc != OK:
        raise SepwError(rc, what)


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return c_void_p(t.data_ptr()) if t is not None else c_void_p(0)


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) torch tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    return t.contiguous()


class Kernels:
    """GCF tables, taper and FFT plan on the current device (sepw_make_kernels)."""

    def __init__(self, N, fov, S, O, P, w_lo, w_hi, taper="pswf", taper_width=0.0,
                 taper_samples=None, a=0.5, b=5.0 / 24.0, a_v=None, b_v=None, facet=None,
                 precision="fp32"):
        lib = load()
        prm = KernelParams()
        lib.sepw_default_params(ctypes.byref(prm))
        prm.grid_size, prm.support, prm.oversample, prm.n_planes = int(N), int(S), int(O), int(P)
        prm.fov, prm.w_lo, prm.w_hi = float(fov), float(w_lo), float(w_hi)
        prm.taper = {"pswf": TAPER_PSWF, "none": TAPER_NONE, "user": TAPER_USER}[taper]
        prm.taper_width = float(taper_width)
        self._samples = None
        if taper == "user":
            import numpy as np
            self._samples = np.ascontiguousarray(taper_samples, dtype=np.float64)
            prm.taper_samples = self._samples.ctypes.data_as(ctypes.POINTER(c_double))
        prm.a_u, prm.b_u = float(a), float(b)
        prm.a_v = float(a if a_v is None else a_v)
        prm.b_v = float(b if b_v is None else b_v)
        if facet is not None:
            prm.facet, prm.l0, prm.m0 = 1, float(facet[0]), float(facet[1])
        prm.precision = {"fp32": FP32, "fp16": FP16, "bf16": BF16}[precision]
        self.N, self.S, self.O, self.P, self.fov = int(N), int(S), int(O), int(P), float(fov)
        self.precision = precision
        h = c_void_p()
        _check(lib.sepw_make_kernels(ctypes.byref(prm), _stream(), ctypes.byref(h)), "sepw_make_kernels")
        self._h = h

    @property
    def handle(self):
        return self._h

    def table(self, axis=0):
        out = torch.empty((self.P, self.O, self.S), dtype=torch.complex64, device="cuda")
        _check(load().sepw_kernels_table(self._h, axis, _ptr(out), _stream()), "sepw_kernels_table")
        return out

    def set_wrange(self, w_lo, w_hi):
        """sepw_kernels_set_wrange: regenerate the tables for a new w range."""
        _check(load().sepw_kernels_set_wrange(self._h, float(w_lo), float(w_hi), _stream()),
               "sepw_kernels_set_wrange")

    def set_correction(self, support, oversample):
        """sepw_kernels_set_correction: attach the 2D correction table F_w - F~_w
        (support 0 removes it)."""
        _check(load().sepw_kernels_set_correction(self._h, int(support), int(oversample), _stream()),
               "sepw_kernels_set_correction")
        self.corr = (int(support), int(oversample)) if support else None

    def correction_terms(self, enable):
        """sepw_kernels_correction_terms: run corrections as separable terms
        (True, the default) or by walking the table (False)."""
        _check(load().sepw_kernels_correction_terms(self._h, 1 if enable else 0, _stream()),
               "sepw_kernels_correction_terms")

    def correction_rank(self):
        """sepw_kernels_correction_rank: separable terms the correction runs as
        (-1: the correction passes walk the table)."""
        r = ctypes.c_int32(0)
        _check(load().sepw_kernels_correction_rank(self._h, ctypes.byref(r)),
               "sepw_kernels_correction_rank")
        return r.value

    def correction_table(self):
        """The attached correction table, [P][Oc][Oc][Sc(v)][Sc(u)] complex64."""
        if not getattr(self, "corr", None):
            raise ValueError("no correction table attached")
        Sc, Oc = self.corr
        out = torch.empty((self.P, Oc, Oc, Sc, Sc), dtype=torch.complex64, device="cuda")
        _check(load().sepw_kernels_correction_table(self._h, _ptr(out), _stream()),
               "sepw_kernels_correction_table")
        return out

    def taper(self):
        out = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(load().sepw_kernels_taper(self._h, _ptr(out), _stream()), "sepw_kernels_taper")
        return out

    def close(self):
        if self._h is not None and self._h.value:
            load().sepw_free_kernels(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dropped_arg(count, host):
    """n_dropped argument: a one-element int64 device tensor (written on the
    stream, no synchronisation), True (host value, the call synchronises) or
    False / None (not counted)."""
    if isinstance(count, torch.Tensor):
        if not count.is_cuda or count.dtype != torch.int64 or count.numel() < 1:
            raise TypeError("count_dropped must be a CUDA int64 tensor")
        return ctypes.cast(c_void_p(count.data_ptr()), ctypes.POINTER(c_int64))
    return ctypes.byref(host) if count else None


def _dropped_value(count, host):
    if isinstance(count, torch.Tensor):
        return count
    return host.value if count else None


class Plan:
    """Binned visibilities for one Kernels object (sepw_plan_create)."""

    def __init__(self, kernels, u, v, w, count_dropped=True):
        lib = load()
        u = _dev(u, torch.float64, "u")
        v = _dev(v, torch.float64, "v")
        w = _dev(w, torch.float64, "w")
        if not (u.numel() == v.numel() == w.numel()):
            raise ValueError("u, v, w must have the same length")
        self.kernels = kernels
        self.nvis = u.numel()
        nd = c_int64(-1)
        h = c_void_p()
        _check(lib.sepw_plan_create(kernels.handle, self.nvis, _ptr(u), _ptr(v), _ptr(w),
                                    _dropped_arg(count_dropped, nd), _stream(),
                                    ctypes.byref(h)), "sepw_plan_create")
        self._h = h
        self.n_dropped = _dropped_value(count_dropped, nd)

    @property
    def handle(self):
        return self._h

    @classmethod
    def from_channels(cls, kernels, uvw, freq, count_dropped=True):
        """sepw_plan_create_channels: uvw [nrows][3] in metres (float64), freq
        [nchan] in Hz (float64); visibility i = row * nchan + ch."""
        lib = load()
        uvw = _dev(uvw, torch.float64, "uvw")
        freq = _dev(freq, torch.float64, "freq")
        if uvw.dim() != 2 or uvw.shape[1] != 3:
            raise ValueError("uvw must be [nrows][3]")
        self = cls.__new__(cls)
        self.kernels = kernels
        self.nvis = uvw.shape[0] * freq.numel()
        nd = c_int64(-1)
        h = c_void_p()
        _check(lib.sepw_plan_create_channels(kernels.handle, uvw.shape[0], freq.numel(), _ptr(uvw),
                                             _ptr(freq), ctypes.byref(nd) if count_dropped else None,
                                             _stream(), ctypes.byref(h)), "sepw_plan_create_channels")
        self._h = h
        self.n_dropped = nd.value if count_dropped else None
        return self

    def rebin_channels(self, uvw, freq, count_dropped=False):
        """sepw_plan_rebin_channels: bin a new batch of channel-shared rows."""
        uvw = _dev(uvw, torch.float64, "uvw")
        freq = _dev(freq, torch.float64, "freq")
        nd = c_int64(-1)
        _check(load().sepw_plan_rebin_channels(self._h, uvw.shape[0], freq.numel(), _ptr(uvw),
                                               _ptr(freq), ctypes.byref(nd) if count_dropped else None,
                                               _stream()), "sepw_plan_rebin_channels")
        self.nvis = uvw.shape[0] * freq.numel()
        if count_dropped:
            self.n_dropped = nd.value
        return self

    @property
    def tile_size(self):
        return load().sepw_plan_tile_size(self._h)

    def rebin(self, u, v, w, count_dropped=False):
        """sepw_plan_rebin: bin a new batch (no allocation)."""
        u = _dev(u, torch.float64, "u")
        v = _dev(v, torch.float64, "v")
        w = _dev(w, torch.float64, "w")
        nd = c_int64(-1)
        _check(load().sepw_plan_rebin(self._h, u.numel(), _ptr(u), _ptr(v), _ptr(w),
                                      _dropped_arg(count_dropped, nd), _stream()),
               "sepw_plan_rebin")
        self.nvis = u.numel()
        if count_dropped is not False and count_dropped is not None:
            self.n_dropped = _dropped_value(count_dropped, nd)
        return self

    def set_item_slots(self, slots):
        """sepw_plan_set_item_slots: work-item length (multiple of 4 in [64, 8192])."""
        _check(load().sepw_plan_set_item_slots(self._h, int(slots), _stream()),
               "sepw_plan_set_item_slots")
        return self

    def set_degrid_item_slots(self, slots):
        """sepw_plan_set_degrid_item_slots: degridding work-item length."""
        _check(load().sepw_plan_set_degrid_item_slots(self._h, int(slots), _stream()),
               "sepw_plan_set_degrid_item_slots")
        return self

    def bins(self):
        out = torch.empty((self.nvis, 7), dtype=torch.int32, device="cuda")
        _check(load().sepw_plan_bins(self._h, _ptr(out), _stream()), "sepw_plan_bins")
        return out

    def close(self):
        if self._h is not None and self._h.value:
            load().sepw_free_plan(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def density_edges(w, n_slices, w_lo, w_hi):
    """sepw_wstack_density_edges: n_slices + 1 slice edges (numpy float64)
    with about equal visibility counts per slice."""
    lib = load()
    w = _dev(w, torch.float64, "w")
    out = (c_double * (int(n_slices) + 1))()
    _check(lib.sepw_wstack_density_edges(w.numel(), _ptr(w), int(n_slices), float(w_lo),
                                         float(w_hi), out, _stream()), "sepw_wstack_density_edges")
    import numpy as np
    return np.array(out[:], dtype=np.float64)


class WStack:
    """sepw_wstack_create: W-stacking hybrid over n_slices uniform w-slices on
    [w_lo, w_hi]; ``kernels`` hold the residual tables (planes on [-h, h],
    h = (w_hi - w_lo) / (2 n_slices)).  With ``edges`` (n_slices + 1
    increasing values; w_lo, w_hi ignored) sepw_wstack_create_edges: slices
    [e_s, e_{s+1}), each with tables of its own on [-h_s, h_s],
    h_s = (e_{s+1} - e_s) / 2 (the kernels' own w range is not used)."""

    def __init__(self, kernels, n_slices, w_lo, w_hi, u, v, w, count_dropped=True, edges=None):
        lib = load()
        u = _dev(u, torch.float64, "u")
        v = _dev(v, torch.float64, "v")
        w = _dev(w, torch.float64, "w")
        if not (u.numel() == v.numel() == w.numel()):
            raise ValueError("u, v, w must have the same length")
        self.kernels = kernels
        self.nvis = u.numel()
        nd = c_int64(-1)
        h = c_void_p()
        pnd = ctypes.byref(nd) if count_dropped else None
        if edges is None:
            _check(lib.sepw_wstack_create(kernels.handle, int(n_slices), float(w_lo), float(w_hi),
                                          self.nvis, _ptr(u), _ptr(v), _ptr(w), pnd, _stream(),
                                          ctypes.byref(h)), "sepw_wstack_create")
        else:
            if len(edges) != int(n_slices) + 1:
                raise ValueError("edges must hold n_slices + 1 values")
            e = (c_double * len(edges))(*[float(x) for x in edges])
            _check(lib.sepw_wstack_create_edges(kernels.handle, int(n_slices), e, self.nvis,
                                                _ptr(u), _ptr(v), _ptr(w), pnd, _stream(),
                                                ctypes.byref(h)), "sepw_wstack_create_edges")
        self._h = h
        self.n_dropped = nd.value if count_dropped else None

    @property
    def handle(self):
        return self._h

    def grid(self, vis, weight=None, flags=0, out=None):
        """sepw_wstack_grid: complex64 N x N image."""
        vis = _dev(vis, torch.complex64, "vis")
        if weight is not None:
            weight = _dev(weight, torch.float32, "weight")
        N = self.kernels.N
        if out is None:
            out = torch.empty((N, N), dtype=torch.complex64, device="cuda")
        _check(load().sepw_wstack_grid(self._h, _ptr(vis), _ptr(weight), _ptr(out), flags,
                                       _stream()), "sepw_wstack_grid")
        return out

    def degrid(self, image, flags=0, out=None):
        """sepw_wstack_degrid: complex64 visibilities in the caller's order."""
        image = _dev(image, torch.complex64, "image")
        if out is None:
            out = torch.empty(self.nvis, dtype=torch.complex64, device="cuda")
        _check(load().sepw_wstack_degrid(self._h, _ptr(image), _ptr(out), flags, _stream()),
               "sepw_wstack_degrid")
        return out

    def close(self):
        if self._h is not None and self._h.value:
            load().sepw_free_wstack(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STAGES = ("tables", "quantise", "sort", "gather", "grid", "fft", "correct", "degrid", "fill",
          "corr_table", "corr_apply")


def timing_enable(on=True):
    _check(load().sepw_timing_enable(1 if on else 0), "sepw_timing_enable")


def timing_collect():
    """{stage: (total ms, launches)} for everything recorded since the last collect."""
    ms = (c_double * len(STAGES))()
    n = (c_int64 * len(STAGES))()
    _check(load().sepw_timing_collect(ms, n), "sepw_timing_collect")
    return {name: (ms[i], n[i]) for i, name in enumerate(STAGES)}


def make_kernels(*args, **kwargs):
    return Kernels(*args, **kwargs)


def plan_create(kernels, u, v, w):
    return Plan(kernels, u, v, w)


class WSnap:
    """sepw_wsnap_create: W snapshots over contiguous snapshots of the caller's
    visibilities (offsets: n_snap + 1 host integers); ``kernels`` get the
    residual w range."""

    def __init__(self, kernels, offsets, u, v, w, count_dropped=True):
        lib = load()
        u = _dev(u, torch.float64, "u")
        v = _dev(v, torch.float64, "v")
        w = _dev(w, torch.float64, "w")
        offs = (c_int64 * len(offsets))(*[int(x) for x in offsets])
        self.kernels = kernels
        self.n_snap = len(offsets) - 1
        self.offsets = [int(x) for x in offsets]
        self.nvis = self.offsets[-1]
        nd = c_int64(-1)
        h = c_void_p()
        _check(lib.sepw_wsnap_create(kernels.handle, self.n_snap, offs, _ptr(u), _ptr(v), _ptr(w),
                                     ctypes.byref(nd) if count_dropped else None, _stream(),
                                     ctypes.byref(h)), "sepw_wsnap_create")
        self._h = h
        self.n_dropped = nd.value if count_dropped else None

    def plane(self, s):
        """(d_u, d_v) of snapshot s and the residual range h."""
        d = (c_double * 2)()
        h = c_double()
        _check(load().sepw_wsnap_plane(self._h, int(s), d, ctypes.byref(h)), "sepw_wsnap_plane")
        return (d[0], d[1]), h.value

    def grid(self, vis, weight=None, flags=0, out=None):
        vis = _dev(vis, torch.complex64, "vis")
        if weight is not None:
            weight = _dev(weight, torch.float32, "weight")
        N = self.kernels.N
        if out is None:
            out = torch.empty((N, N), dtype=torch.complex64, device="cuda")
        _check(load().sepw_wsnap_grid(self._h, _ptr(vis), _ptr(weight), _ptr(out), flags, _stream()),
               "sepw_wsnap_grid")
        return out

    def degrid(self, image, flags=0, out=None):
        image = _dev(image, torch.complex64, "image")
        if out is None:
            out = torch.empty(self.nvis, dtype=torch.complex64, device="cuda")
        _check(load().sepw_wsnap_degrid(self._h, _ptr(image), _ptr(out), flags, _stream()),
               "sepw_wsnap_degrid")
        return out

    def close(self):
        if self._h is not None and self._h.value:
            load().sepw_free_wsnap(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def grid(plan, vis, weight=None, flags=0, out=None):
    """sepw_grid: complex64 N x N uv grid (GRID_ONLY) or image; with REAL in
    flags the real part of the image as float32 N x N."""
    vis = _dev(vis, torch.complex64, "vis")
    if weight is not None:
        weight = _dev(weight, torch.float32, "weight")
    N = plan.kernels.N
    if out is None:
        dt = torch.float32 if flags & REAL else torch.complex64
        out = torch.empty((N, N), dtype=dt, device="cuda")
    else:
        out = _dev(out, torch.float32 if flags & REAL else torch.complex64, "out")
    _check(load().sepw_grid(plan.handle, _ptr(vis), _ptr(weight), _ptr(out), flags, _stream()),
           "sepw_grid")
    return out


def degrid(plan, image, flags=0, out=None):
    """sepw_degrid: complex64 visibilities in the caller's order; a real
    float32 image goes in as such (REAL)."""
    if isinstance(image, torch.Tensor) and image.dtype == torch.float32 and not flags & GRID_ONLY:
        flags |= REAL
    image = _dev(image, torch.float32 if flags & REAL else torch.complex64, "image")
    if out is None:
        out = torch.empty(plan.nvis, dtype=torch.complex64, device="cuda")
    _check(load().sepw_degrid(plan.handle, _ptr(image), _ptr(out), flags, _stream()), "sepw_degrid")
    return out


def _batch_args(plans, vis, weights, outs):
    n = len(plans)
    vis = [_dev(x, torch.complex64, "vis") for x in vis]
    if weights is None:
        weights = [None] * n
    weights = [None if x is None else _dev(x, torch.float32, "weight") for x in weights]
    if outs is None:
        outs = [torch.empty((p.kernels.N, p.kernels.N), dtype=torch.complex64, device="cuda")
                for p in plans]
    arr = c_void_p * n
    return (n, arr(*[p.handle for p in plans]), arr(*[x.data_ptr() for x in vis]),
            arr(*[0 if x is None else x.data_ptr() for x in weights]),
            arr(*[x.data_ptr() for x in outs]), (vis, weights, outs))


def autotune_batched(plans, vis, weights=None, outs=None):
    """sepw_autotune_batched: returns (item_slots, blocks_per_cu) it settled on."""
    n, hp, vp, wp, op, keep = _batch_args(plans, vis, weights, outs)
    slots, width = c_int32(0), c_int32(0)
    _check(load().sepw_autotune_batched(n, hp, vp, wp, op, _stream(), ctypes.byref(slots),
                                        ctypes.byref(width)), "sepw_autotune_batched")
    return slots.value, width.value


def grid_batched(plans, vis, weights=None, flags=0, outs=None, noalloc=False):
    """sepw_grid_batched over several (facet / snapshot) plans
    (sepw_grid_batched_noalloc with noalloc=True)."""
    n = len(plans)
    vis = [_dev(x, torch.complex64, "vis") for x in vis]
    if weights is None:
        weights = [None] * n
    weights = [None if x is None else _dev(x, torch.float32, "weight") for x in weights]
    if outs is None:
        outs = [torch.empty((p.kernels.N, p.kernels.N), dtype=torch.complex64, device="cuda")
                for p in plans]
    arr = c_void_p * n
    hp = arr(*[p.handle for p in plans])
    vp = arr(*[x.data_ptr() for x in vis])
    wp = arr(*[0 if x is None else x.data_ptr() for x in weights])
    op = arr(*[x.data_ptr() for x in outs])
    fn = "sepw_grid_batched_noalloc" if noalloc else "sepw_grid_batched"
    _check(getattr(load(), fn)(n, hp, vp, wp, op, flags, _stream()), fn)
    return outs
