"""Seeded synthetic ptychography scans (objects, probes, scan positions, start
values, photon noise).

This package draws random numbers and builds the test objects and probes; it
holds none of the solver's arithmetic (no propagation of frames, no
projections). Both the GPU path and the FP64 oracle consume what it makes.
"""
from .gen import (  # noqa: F401
    STREAMS,
    Scan,
    apply_poisson,
    config_scan,
    fig3_scan,
    gradient_point,
    batch_scans,
    raster_positions,
    streams_for,
)
