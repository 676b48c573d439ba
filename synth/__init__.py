"""Seeded synthetic TPC events (FP64 physics, FP32 cluster SoA).

This package only simulates detector input: charged helices in a uniform
solenoid crossing the pad-row planes of a 36-sector, 159-row drift chamber,
Gaussian smearing, noise, merged-cluster doubling and (optionally) an
injected miscalibration.  It contains none of the tracker's arithmetic and is
shared by the oracle tests and the GPU path as the one source of inputs.
"""
from .events import (  # noqa: F401
    Geometry, Event, CalibTheta, default_geometry, make_event, make_config, make_configs,
    bspline_basis, draw_theta, CONFIGS,
)
from .timeframe import TimeFrame, make_timeframe, make_tf_config, TF_CONFIGS, TF_SLICE  # noqa: F401
from .its import ItsGeometry, ItsEvent, default_its_geometry, make_its_event, make_its_config, ITS_CONFIGS  # noqa: F401
