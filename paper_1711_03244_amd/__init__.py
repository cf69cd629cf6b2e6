"""MI355X-native voxel Monte Carlo photon transport (MCX-CL hot path).

The GPU library is ``libmcx.so`` (HIP for gfx950) behind the C ABI declared
in ``include/mcx.h``; :mod:`paper_1711_03244_amd.mcx` is its thin ctypes
binding and :mod:`paper_1711_03244_amd.workloads` builds seeded inputs.
Importing the package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
