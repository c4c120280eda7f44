"""FP64 CPU oracle for separable W-projection gridding (Merry 2015, arXiv:1511.07152).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or runs
anything in this package; only the test suite, the smoke check and the CPU
baseline leg of the benchmark call it.  It shares no code, headers, tables or
constants with the HIP path.  Random inputs are produced elsewhere (a seeded
generator module that holds none of the method's arithmetic) and are passed in.

Everything here is plain NumPy in float64 / complex128, written to be checked
by eye against the paper:

* ``geometry``   pixel and cell coordinates, centred transforms F+ and F-
                 (Section 2, the dirty-image equation and its inverse FFT form)
* ``pswf``       prolate spheroidal taper c(l) (Section 2, anti-aliasing kernel C
                 and its inverse transform c; assumed separable in Section 3)
* ``tables``     oversampled 1D GCF tables per w-plane (Section 3, separable
                 phase screen g^1_w; Section 2, oversampled lookup tables) and the
                 exact non-separable 2D tables used as the reference
* ``quantise``   uv to grid cell / oversample index, w to plane, tile binning
* ``gridder``    convolutional gridding and degridding (Section 2, W projection
                 equation; Section 5, separable inner loop)
* ``dft``        direct evaluation of the dirty-image and prediction equations
                 (Section 2)
* ``phase_error`` the separable phase-error factor epsilon (Section 3)
* ``facet``      image-plane facet preprocessing and facet tables (Section 4.1)
* ``imaging``    grid correction by the taper and the factor n around F+ / F-
* ``chi2``       chi-squared data misfit of a predicted model and its image
                 gradient through the gridding adjoint (Section 6, major cycles)
* ``wstack``     W-stacking hybrid: w-slices corrected in image space, residual
                 w by separable W projection (Section 4.3)
* ``correction`` the 2D correction table F_w - F~_w applied beside the
                 separable GCF (Section 6)
* ``wsnap``      W snapshots: per-snapshot plane fit, residual w by separable
                 W projection, image reprojection (Section 4.2)

Readings of points the paper leaves open are documented at each function.
"""

from . import geometry, pswf, tables, quantise, gridder, dft, phase_error, facet, imaging, chi2, wstack, correction, wsnap  # noqa: F401,E501
