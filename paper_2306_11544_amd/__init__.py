"""MI355X-native agent-mechanics step (binning, 27-voxel forces, Adams-Bashforth).

The compute path is libmech.so (hand-written gfx950 HIP kernels behind a C ABI, see
include/mech.h); `binding` marshals arguments to it.
"""
from .binding import *  # noqa: F401,F403
from .binding import EXPORTS, MechError, MechParams, Population, lib  # noqa: F401
