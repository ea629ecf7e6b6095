"""MI355X-native DMAS-CF beamforming (n-th order Delay-Multiply-and-Sum with
Coherence-Factor weighting, Newton-Girard power sums, fused envelope).

The compute path is libdmas.so (hand-written HIP for gfx950, C ABI in
include/dmas.h); this package is its Python binding.
"""

from .dmas import (DTYPES, DmasError, Plan, Server, design_lowpass, load_library,  # noqa: F401
                   plan_for_frame, server_clock, version)
