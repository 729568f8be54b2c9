"""Colour-image stand-in for the image-inpainting experiment (Sec. V.B).

The paper completes a 2048 x 2048 landscape photograph whose three colour
channels are stacked into one 6144 x 2048 matrix, from 10 % or 20 % of its
pixels.  The photograph is not available; this module builds a seeded
stand-in with the same shape and statistics that matter to a low-rank
completion: a luminance field with a power-law spectrum (amplitude ~ f^-1.4,
the decay of natural images), a vertical sky-to-ground gradient, and two
smoother chroma fields that tint the channels differently (bluish at the
top), clipped to the 8-bit range [0, 255].

Sampling: a pixel (i, j) drawn by the uniform sampler of ``sampler`` is
observed in all three channels, i.e. the stacked rows i, H + i and 2H + i of
column j.  Values are handed to the solver as intensities in [0, 1] (the
paper's tau = 5n presumes entries of order one); the MAE of Eq. (10) is
reported back on the 0-255 scale.
"""

import numpy as np

from .problems import Problem
from .sampler import sample_cells, cells_to_coo


def _field(h, w, beta, rng):
    """Zero-mean, unit-variance random field with amplitude spectrum f^-beta."""
    fy = np.fft.fftfreq(h)[:, None]
    fx = np.fft.rfftfreq(w)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    f[0, 0] = 1.0
    amp = f ** -beta
    amp[0, 0] = 0.0
    z = rng.standard_normal(amp.shape) + 1j * rng.standard_normal(amp.shape)
    a = np.fft.irfft2(z * amp, s=(h, w))
    return (a - a.mean()) / a.std()


def landscape_rgb(size=2048, seed=8):
    """Three channels (3, size, size) of the stand-in image, values in [0, 255]."""
    rng = np.random.default_rng(seed)
    lum = _field(size, size, 1.4, rng)
    c1 = _field(size, size, 1.8, rng)
    c2 = _field(size, size, 1.8, rng)
    sky = (0.5 - (np.arange(size, dtype=np.float64) + 0.5) / size)[:, None]
    L = 125.0 + 45.0 * lum + 40.0 * sky
    rgb = np.stack([L + 18.0 * c1 - 15.0 * sky,
                    L - 6.0 * c1 + 10.0 * c2,
                    L - 12.0 * c2 + 30.0 * sky])
    return np.clip(rgb, 0.0, 255.0)


def inpainting(size=2048, ratio=0.1, seed_img=8, seed_phi=108, name="inpaint"):
    """The stacked (3 size) x size matrix scaled to [0, 1], observed at a
    uniform sample of round(ratio size^2) pixels in all three channels."""
    rgb = landscape_rgb(size, seed_img) / 255.0
    dense = rgb.reshape(3 * size, size)
    K = int(np.floor(ratio * size * size + 0.5))
    pr, pc = cells_to_coo(sample_cells(size, size, K, seed_phi), size)
    rows = np.concatenate([pr + c * size for c in range(3)])
    cols = np.concatenate([pc] * 3)
    vals = dense[rows, cols].copy()
    return Problem(3 * size, size, rows, cols, vals, name=name, dense=dense,
                   meta=dict(ratio=ratio, seed_img=seed_img, seed_phi=seed_phi,
                             pixels=K, channels=3, value_scale=255.0))


def mae_all_pixels(X, prob):
    """Eq. (10) over every entry of the stacked matrix, on the 0-255 scale."""
    return float(np.mean(np.abs(X - prob.dense)) * prob.meta["value_scale"])
