"""Seeded synthetic inputs for the fast-SVT matrix completion path.

This package produces the *inputs* of a completion problem (the sampled set
Phi, the observed values M_Phi, and the ground truth where one exists).  It
holds none of the method's arithmetic: no SVD, no thresholding, no iteration.
Both the CPU oracle and the HIP library consume what it returns, and neither
of them is imported here.

The paper's workloads (a colour photograph and the MovieLens rating sets) are
not available; the generators below build stand-ins with the same shapes,
sampling ratios and value ranges.
"""

from .sampler import splitmix64_output, sample_cells, cells_to_coo
from .problems import (Problem, planted, image_like, ratings, serving_trace,
                       request_problem, zipf_degrees, sparse_square)
from .image import landscape_rgb, inpainting, mae_all_pixels
from .configs import CONFIGS, get_config, make_problem, serving_params

__all__ = [
    "splitmix64_output", "sample_cells", "cells_to_coo",
    "Problem", "planted", "image_like", "ratings", "serving_trace",
    "request_problem", "zipf_degrees", "sparse_square",
    "landscape_rgb", "inpainting", "mae_all_pixels",
    "CONFIGS", "get_config", "make_problem", "serving_params",
]
