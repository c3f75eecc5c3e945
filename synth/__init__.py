"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds input generation only: reference images, template cuts
(exact, quarter-turn, bilinear rotate + scale), probe radius grids and
request streams.  It contains none of the screening arithmetic (no star
geometry, no feature sums, no comparison), so that the oracle and the HIP
path can both draw inputs from it without sharing any method code.
"""
from .images import (  # noqa: F401
    make_rng,
    blob_image,
    cut_patch,
    rotate_scale_patch,
    pick_centre,
    patch_std,
)
from .workloads import (  # noqa: F401
    WORKLOADS,
    Workload,
    PlantedTemplate,
    make_workload,
    radius_grid_cfg5,
    serving_requests,
)
