"""Seeded synthetic inputs for the two-step minor-cycle reconstruction.

This module only *makes inputs*: a sky, an antenna array, earth-rotation uv
tracks, natural-weight grids split by baseline length, the normalised PSF of
each split and the dirty images.  It holds none of the solver's arithmetic
(no FISTA, no prox, no filters, no step sizes) and is imported both by the
FP64 oracle tests and by the GPU path's tests and benchmark, which is why it
lives apart from both.

The data the paper uses (MeerKAT Galactic-Centre cut-outs, Sect. 4.1) is not
available, so these skies stand in for it: compact sources plus extended
elliptical emission, a 64-antenna 4 h configuration for the small case, and
SKA-Mid-sized arrays for the large ones.
"""
from .generator import (
    SkyConfig,
    ArrayConfig,
    ProblemConfig,
    Problem,
    make_sky,
    make_antennas,
    uv_tracks,
    grid_weights,
    partition_counts,
    make_problem,
    make_problems,
    preset,
    PRESETS,
    tiny,
    channel_set,
    sky_set,
    coarse_low,
    late_state,
)

__all__ = [
    "SkyConfig",
    "ArrayConfig",
    "ProblemConfig",
    "Problem",
    "make_sky",
    "make_antennas",
    "uv_tracks",
    "grid_weights",
    "partition_counts",
    "make_problem",
    "make_problems",
    "preset",
    "PRESETS",
    "tiny",
    "channel_set",
    "sky_set",
    "coarse_low",
    "late_state",
]
