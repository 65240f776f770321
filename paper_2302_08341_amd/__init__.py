"""MI355X-native ensemble local-inertial flood model with a particle filter.

The compute path is libflood.so (HIP kernels for gfx950 behind the C ABI in
include/flood.h); :mod:`paper_2302_08341_amd.flood` is its ctypes binding.
"""
from .flood import (FIELD_H, FIELD_QX, FIELD_QY, FIELD_PEAK, EDGE_OPEN, EDGE_WALL, FloodEnsemble, FloodError,  # noqa: F401
                    load_library)
