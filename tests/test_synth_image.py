"""The image-inpainting workload (Sec. V.B) on the CPU: the stand-in image,
its pixel sampling across the three stacked channels, the MAE of Eq. (10),
and the oracle's fast SVT on the 1/4-scaled instance."""

import numpy as np
import pytest

import synth
from oracle import FastSVT


def test_stacked_image_and_pixel_sampling():
    prob = synth.inpainting(64, 0.2, seed_img=3, seed_phi=4)
    assert (prob.m, prob.n) == (192, 64)
    K = prob.meta["pixels"]
    assert K == int(np.floor(0.2 * 64 * 64 + 0.5)) and prob.nnz == 3 * K
    assert prob.dense.min() >= 0.0 and prob.dense.max() <= 1.0
    # row-major COO, no duplicate cell, values are the image's
    key = prob.rows * prob.n + prob.cols
    assert np.all(np.diff(key) > 0)
    np.testing.assert_array_equal(prob.vals, prob.dense[prob.rows, prob.cols])
    # a pixel is observed in all three channels (rows i, H + i, 2H + i)
    per_ch = [set(zip(prob.rows[prob.rows // 64 == c] % 64,
                      prob.cols[prob.rows // 64 == c])) for c in range(3)]
    assert per_ch[0] == per_ch[1] == per_ch[2] and len(per_ch[0]) == K
    # the pixel set is the uniform sampler's on the 64 x 64 grid
    cells = synth.sample_cells(64, 64, K, 4)
    assert per_ch[0] == set(zip(cells // 64, cells % 64))
    # channels differ (a colour image, not three copies)
    rgb = synth.landscape_rgb(64, 3)
    assert rgb.shape == (3, 64, 64)
    assert np.abs(rgb[0] - rgb[2]).mean() > 1.0


def test_mae_is_eq10_over_all_pixels():
    prob = synth.inpainting(32, 0.1, seed_img=5, seed_phi=6)
    X = prob.dense + 0.01 * np.cos(np.arange(prob.m * prob.n)).reshape(prob.m, prob.n)
    want = sum(abs(X[i, j] - prob.dense[i, j]) for i in range(prob.m)
               for j in range(prob.n)) / (prob.m * prob.n) * 255.0
    assert synth.mae_all_pixels(X, prob) == pytest.approx(want, rel=1e-12)
    assert synth.mae_all_pixels(prob.dense, prob) == 0.0


def test_oracle_inpaints_the_scaled_instance():
    # 1536 x 512, 10 % of the pixels: the guarded fast SVT reaches the
    # paper's epsilon within its step budget
    from threadpoolctl import threadpool_limits
    prob, prm = synth.make_problem("inpaint10_s4")
    with threadpool_limits(limits=2):        # small products: threads only add overhead
        orc = FastSVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
        for _ in range(prm["i_max"]):
            info = orc.step()
            if info.converged:
                break
    assert info.converged and info.res < 0.052
    X = (orc.U * orc.sig) @ orc.V.T
    mae = synth.mae_all_pixels(X, prob)
    assert mae < 15.0
