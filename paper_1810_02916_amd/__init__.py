"""MI355X-native near-field force of the compact near/far force split
(Garrison, Eisenstein & Pinto, arXiv:1810.02916, Sec. 2.1 and 4.3).

The compute lives in libnf.so (hand-written HIP for gfx950, C ABI in
include/nf.h); this package only marshals arguments to it.
"""
from .nearfield import (  # noqa: F401
    SPLINE_PER_PLUMMER,
    Binned,
    CapturedForce,
    NearFieldAccel,
    accel,
    accel_vjp,
    bin_particles,
    bin_particles_batched,
    eps_spline_from_plummer,
    nearfield_accel,
    rebin,
)
