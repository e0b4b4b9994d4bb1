"""Seeded synthetic inputs for the sparse TSDF fusion path.

This package generates inputs only: analytic scenes, camera paths and depth
maps with sensor noise.  It contains none of the fusion or raycasting
arithmetic, so the CPU oracle and the HIP path can both draw their inputs
from it without sharing any of the method's code.
"""

from .scenes import (  # noqa: F401
    Intrinsics,
    Scene,
    look_at,
    render_depth,
    scene_sdf,
    sphere_scene,
    plane_scene,
    procedural_scene,
    hand_scene,
    add_sensor_noise,
    edge_dropout,
)
from .configs import (  # noqa: F401
    GridSpec,
    SequenceSpec,
    config_c1,
    config_c2,
    config_c3,
    config_c5,
    sequence_frame,
)
