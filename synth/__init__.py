"""Seeded synthetic inputs for the gradient-guided Monte Carlo SLAM filter.

This package is the one module that both the FP64 CPU oracle (``oracle/``) and
the HIP library (``paper_2504_18056_amd``) are fed from.  It builds scenes,
ray-cast scans, likelihood grids, particle sets, trajectories and the random
numbers the filter consumes (prediction noise, the systematic-resampling
offset).  It holds none of the filter's own arithmetic: no point transform,
no trilinear interpolation, no gradient, no pose step, no weighting and no
resampling.

The paper's datasets (a forest-like Livox MID-360 sequence, an indoor elevator
sequence and a survey map; Sec. IV) are not available; these generators stand
in for them with the shapes given in the workload descriptions in
``synth.configs``.
"""

from .rng import splitmix64_uniforms  # noqa: F401
from . import geometry, scene, configs  # noqa: F401
