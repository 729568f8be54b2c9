"""Named workloads and the solver settings each one is run with.

The settings are plain numbers handed to both the oracle and the HIP
library: tau = 5n (Sec. II.C), l = 5, s = 10, and the step size
delta = 1.2 * m*n/|Phi| ("1.2/ratio") for the uniformly sampled workloads.
Under the power-law sampling of the rating workloads that step diverges at
the first step (the heavy rows are observed almost completely, so the update
overshoots there by a factor close to delta); they use delta = 1.9, inside the
0 < delta < 2 range for which SVT is known to converge.  Also
the recycling settings the paper uses for images (strategy 2,
i_reuse = 100, q_reuse = 10, Sec. V.B) and ratings (strategy 1, i_reuse = 50,
q_reuse = 10, Sec. V.C).

The image-inpainting workloads (Sec. V.B: three colour channels stacked
into a 6144 x 2048 matrix, 10 % or 20 % of the pixels observed) take the
paper's epsilon (0.052 / 0.047), step budgets (400 / 700), strategy-2
recycling and delta = 1.2/ratio, with the Ritz guard: on the stand-in image
the paper's rule alone lets inaccurate recycled results through and the
residual climbs back (0.41 after 400 steps at 10 %, against convergence at
step 231 with the guard, on the 1/4-scaled instance).

The image1024 workload recycles by the paper's rule alone (ritz_tol = 0): its
recycled results have Ritz residuals of 0.07-1.6 % and the solve follows the
guarded one to four digits of the residual.  The rating workloads keep the
Ritz guard (ritz_tol = 1e-4): on them strategy-1 results have Ritz residuals
of 1-10 %, and taking them unchecked stalls the residual (0.82 against 0.17
after 400 steps of ratings70k).
"""

from .problems import planted, image_like, ratings
from .image import inpainting


RATINGS_DELTA = 1.9


def _base(m, n, nnz, **kw):
    p = dict(tau=5.0 * n, delta=1.2 * m * n / nnz, eps=1e-4, i_max=200,
             l=5, s=10, p_init=3, p_min=1, p_max=8, adaptive_p=1,
             i_reuse=0, q_reuse=10, recycle=0, ritz_tol=1e-4, k_max=0,
             seed=12345)
    p.update(kw)
    return p


CONFIGS = {
    # 500 x 500 planted rank 10, 20 % observed, plain fast SVT in FP64.
    "planted500": dict(
        make=lambda: planted(500, 500, 10, 0.2, seed_data=1, seed_phi=101,
                             name="planted500"),
        shape=(500, 500, 50000),
        params=lambda m, n, nnz: _base(m, n, nnz, eps=1e-4, i_max=200)),
    # 1024 x 1024 image-like, 50 % observed, p = 2 fixed ("3 Krylov blocks"),
    # strategy-2 recycling.
    "image1024": dict(
        make=lambda: image_like(1024, 0.5, seed_data=2, seed_phi=102,
                                name="image1024"),
        shape=(1024, 1024, 524288),
        params=lambda m, n, nnz: _base(m, n, nnz, eps=0.05, i_max=300,
                                       p_init=2, adaptive_p=0, recycle=2,
                                       i_reuse=100, q_reuse=10, ritz_tol=0.0)),
    # 70,000 x 10,700, 1e7 integer ratings, strategy-1 recycling.
    "ratings70k": dict(
        make=lambda: ratings(70000, 10700, 10_000_000, 20, seed_data=3,
                             name="ratings70k"),
        shape=(70000, 10700, 10_000_000),
        params=lambda m, n, nnz: _base(m, n, nnz, eps=0.16, i_max=400, delta=RATINGS_DELTA,
                                       recycle=1, i_reuse=50, q_reuse=10)),
    # 1/10-scaled instance of the same generator (m, n / 10, nnz / 100).
    "ratings70k_s10": dict(
        make=lambda: ratings(7000, 1070, 100_000, 20, seed_data=3,
                             name="ratings70k_s10"),
        shape=(7000, 1070, 100_000),
        params=lambda m, n, nnz: _base(m, n, nnz, eps=0.16, i_max=400, delta=RATINGS_DELTA,
                                       recycle=1, i_reuse=50, q_reuse=10)),
    # 140,000 x 27,000, 2e7 ratings, rank cap 100.
    "ratings140k": dict(
        make=lambda: ratings(140000, 27000, 20_000_000, 30, seed_data=5,
                             name="ratings140k"),
        shape=(140000, 27000, 20_000_000),
        params=lambda m, n, nnz: _base(m, n, nnz, eps=0.16, i_max=400, delta=RATINGS_DELTA,
                                       recycle=1, i_reuse=50, q_reuse=10,
                                       k_max=100)),
    "ratings140k_s10": dict(
        make=lambda: ratings(14000, 2700, 200_000, 30, seed_data=5,
                             name="ratings140k_s10"),
        shape=(14000, 2700, 200_000),
        params=lambda m, n, nnz: _base(m, n, nnz, eps=0.16, i_max=400, delta=RATINGS_DELTA,
                                       recycle=1, i_reuse=50, q_reuse=10,
                                       k_max=100)),
    # Image inpainting (Sec. V.B): 2048 x 2048 colour stand-in, channels
    # stacked into 6144 x 2048, 10 % / 20 % of the pixels in all channels.
    "inpaint10": dict(
        make=lambda: inpainting(2048, 0.1, seed_img=8, seed_phi=108, name="inpaint10"),
        shape=(6144, 2048, 3 * 419430),
        params=lambda m, n, nnz: _base(m, n, nnz, eps=0.052, i_max=400, recycle=2,
                                       i_reuse=100, q_reuse=10)),
    "inpaint20": dict(
        make=lambda: inpainting(2048, 0.2, seed_img=8, seed_phi=108, name="inpaint20"),
        shape=(6144, 2048, 3 * 838861),
        params=lambda m, n, nnz: _base(m, n, nnz, eps=0.047, i_max=700, recycle=2,
                                       i_reuse=100, q_reuse=10)),
    # 1/4-scaled instances (512 x 512 image, 1536 x 512 stacked): oracle-sized
    "inpaint10_s4": dict(
        make=lambda: inpainting(512, 0.1, seed_img=8, seed_phi=108, name="inpaint10_s4"),
        shape=(1536, 512, 3 * 26214),
        params=lambda m, n, nnz: _base(m, n, nnz, eps=0.052, i_max=400, recycle=2,
                                       i_reuse=100, q_reuse=10)),
    "inpaint20_s4": dict(
        make=lambda: inpainting(512, 0.2, seed_img=8, seed_phi=108, name="inpaint20_s4"),
        shape=(1536, 512, 3 * 52429),
        params=lambda m, n, nnz: _base(m, n, nnz, eps=0.047, i_max=700, recycle=2,
                                       i_reuse=100, q_reuse=10)),
}


def get_config(name):
    return CONFIGS[name]


def make_problem(name):
    """Return (problem, params) for a named workload."""
    cfg = CONFIGS[name]
    prob = cfg["make"]()
    return prob, cfg["params"](prob.m, prob.n, prob.nnz)


SERVING_RANK_CAP = 256


def serving_params(m, n, nnz):
    """Per-request settings of the serving workload (no recycling).  Each
    request carries a rank cap (the planted ranks are at most 50), so the
    device footprint that admission prices bounds what the solve holds."""
    return _base(m, n, nnz, eps=1e-4, i_max=200,
                 k_max=min(SERVING_RANK_CAP, m, n))
