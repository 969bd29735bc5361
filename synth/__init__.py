"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package draws images and centre tracks only.  It contains none of the
segmentation method's arithmetic (no thresholding, smoothing, edge detector,
initial condition, assembly, solve or rescaling), so that the oracle and the
GPU path can both consume its output without sharing any of the method.
"""
from synth.gen import (  # noqa: F401
    CENTRE_DTYPE,
    Image4D,
    spheres_cfg1,
    nuclei_cfg2,
    window_job,
    windows_cfg4,
    serving_stream,
    serving_windows,
)
