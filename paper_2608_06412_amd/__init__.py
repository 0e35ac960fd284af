"""MI355X-native accessibility-field hot path (HIP for gfx950).

``Context`` wraps one device-resident map: ``integrate_frame`` (scan-centric
TSDF integration of a LiDAR frame), ``set_tool_kernels`` (rotated tool
kernels), ``score_points`` (label every confident surface point) and
``read_labels``.  The work runs in libaf.so; this package only marshals
arguments.
"""
from .af import (ACCESSIBLE, BLOCKED, NO_CANDIDATE, NOT_EVALUATED, UNSCORED,  # noqa: F401
                 AFError, Context, Server, default_config, lib, load_library, window_blocks)
