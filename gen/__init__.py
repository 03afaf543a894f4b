"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package holds only random-number draws and image painting. It holds none of
the segmentation method's arithmetic (no gradient, no watershed, no waterfall):
both the HIP path and the CPU oracle consume the float images it produces.
"""
from .synth import (  # noqa: F401
    blobs2d,
    blobs3d,
    ellipses2d,
    config_image,
    batch_sizes,
    paper_row,
    serpentine,
    CONFIGS,
)
