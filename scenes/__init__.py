"""Seeded synthetic scenes shared by the tests, the benchmark and the smoke check.

This module only *synthesises inputs*: analytic geometry, a pinhole ray caster
that plays the role of the paper's renderer (the depth tuple of the
preliminaries in the method section), soft target masks, and surface point
samples that stand in for Gaussian centres.  It holds none of the fusion
arithmetic: no projection of voxels, no gates, no weights, no thresholds.
Both the CPU oracle and the HIP library consume what it produces.

Conventions of the produced data (also stated in the design doc):
  * camera: OpenCV pinhole, x right, y down, z forward; ``c2w`` is a 3x4
    row-major ``[R | o]`` with world = R @ cam + o (columns of R are the camera
    axes in world coordinates, the last column is the camera centre).
  * depth maps are planar (camera-Z) float32, 0 where the pixel ray hits
    nothing.  They follow the shell model: along the ray through the pixel
    centre, t_min = t_hit - h/2, t_med = t_hit, t_max = t_hit + h/2, converted
    to planar depth by the ray's obliquity.
  * soft masks are sigmoid(k * signed pixel distance to the visible-target
    silhouette) plus Gaussian noise, clipped to [0, 1].

Every function takes an explicit seed; numpy ``Generator(PCG64(seed))``.
"""

from .geometry import (  # noqa: F401
    Sphere, Box, Quad, InnerBox, look_at_camera, cast_rays, pixel_rays,
)
from .configs import (  # noqa: F401
    Scene, View, make_tiny_sphere, make_forward_facing, make_unbounded,
    make_diff_scene, make_grid_scene, make_click_view, CONFIG_NAMES, make_config, cached, config_scene,
    make_serving_workload,
)
