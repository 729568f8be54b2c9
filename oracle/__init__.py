"""CPU oracle for fast-SVT matrix completion — TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 implementations of what the hot path computes, written from
Feng, Yu & Li, "Faster Matrix Completion Using Randomized SVD" (arXiv
1810.06860).  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the product library never does, and it
shares no code with it (the seeded input generators in ``synth`` are the only
common dependency, and they hold none of the method's arithmetic).

Modules
-------
philox    counter-based Gaussian test matrices (Philox4x32-10 + Box-Muller),
          the one random stream both sides must draw identically.
csr       canonical CSR / CSC layout of the sampled set Phi.
eigsvd    eigSVD (Alg. 3).
rsvd      basic rSVD (Alg. 1), rSVD-PI (Alg. 4), rSVD-BKI (Alg. 5).
svt       plain SVT with an exact dense SVD (Eq. (6), Alg. 2) -- the
          definition the fast method approximates.
fast_svt  fast SVT (Alg. 6): rSVD-BKI, subspace recycling (Sec. IV.B),
          adaptive power parameter.

Parity status
-------------
Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
lemmas of the paper, library routines on special cases, brute force on tiny
inputs or published known-answer vectors.  The full fast-SVT solve versus
the exact SVT is pinned only to a tolerance (the paper claims equal accuracy,
not equal iterates): "parity unpinned" beyond the 1e-3 relative Frobenius
agreement of the recovered matrix.
"""

from .philox import philox4x32_10, gaussian_block
from .csr import canonical_csr
from .eigsvd import eigsvd, eigsvd_top
from .rsvd import lu_factor, basic_rsvd, rsvd_pi, rsvd_bki
from .svt import (SVTParams, shrink, shrink_factors, spectral_norm, initial_c, svt_exact,
                  SVTResult)
from .fast_svt import FastSVT, fast_svt, adapt_p

__all__ = [
    "philox4x32_10", "gaussian_block", "canonical_csr", "eigsvd",
    "eigsvd_top", "lu_factor", "basic_rsvd", "rsvd_pi", "rsvd_bki",
    "SVTParams", "shrink", "shrink_factors", "spectral_norm", "initial_c", "svt_exact",
    "SVTResult", "FastSVT", "fast_svt", "adapt_p",
]
