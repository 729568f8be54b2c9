"""MI355X-native fast SVT matrix completion.

Singular value thresholding (Cai et al.) accelerated with the block-Krylov
randomized SVD rSVD-BKI, eigSVD and subspace recycling of Feng, Yu & Li,
"Faster Matrix Completion Using Randomized SVD" (arXiv 1810.06860), with every
step of a solve running as HIP kernels on one gfx950 GPU behind the C ABI in
include/mcsvt.h.
"""

from ._ffi import (LIB_PATH, MC_EDONE, MC_ENOTCONV, MC_OK, MCError, STATUS_NAMES,
                   lib)
from .svt import (RSVD, SVT, default_params, footprint, rsvd_bki, rsvd_pi, step_group,
                  step_many)

__all__ = ["SVT", "RSVD", "rsvd_bki", "rsvd_pi", "step_many", "step_group", "footprint", "default_params",
           "MCError", "lib", "LIB_PATH", "MC_OK", "MC_EDONE", "MC_ENOTCONV",
           "STATUS_NAMES"]
