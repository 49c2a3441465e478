"""MI355X-native iPEPS real-time evolution of the disorder-dilated 2D XXZ model.

The compute path is the gfx950 library ``libipeps.so`` (HIP kernels behind the
C ABI in include/ipeps.h); this package only marshals arguments to it.
"""
from .native import (FLAG_AUTOTUNE, FLAG_FACTORED_CUTS, FLAG_FORMED_CUTS, Config,  # noqa: F401
                     Batch, IpepsError, Obs, Server, Slab, State, footprint_bytes, load, ff_bessel_j, ff_neel_dynamics,
                     ff_neel_dynamics_device, ff_spectrum_ipr, ff_spectrum_ipr_device, make_config)
