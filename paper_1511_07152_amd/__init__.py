"""Separable W-projection gridding and degridding for MI355X (gfx950).

Hot path of Merry (2015), arXiv:1511.07152, as hand-written HIP kernels behind
the C ABI in include/sepw.h (libsepw.so).  This package holds the ctypes
binding (``_lib``), the autograd prediction operator (``autograd``), the
seeded input generators (``synth``) and the build script (``build``).

Attributes of the binding are imported lazily so that ``synth`` can be used
without loading torch or the HIP library.
"""

_BINDING = ("Kernels", "Plan", "make_kernels", "plan_create", "grid", "degrid", "grid_batched",
            "GRID_ONLY", "MUL_N", "DIV_N", "SepwError", "load")


def __getattr__(name):
    if name in _BINDING:
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
