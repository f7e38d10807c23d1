"""Gaussian-blob images: the synthetic stand-in for the paper's CIFAR-10 / CelebA inputs.

The paper measures on similar real images (Section 3: images of one category share structure;
Section 5, Experiment 2).  Those datasets are not available here, so every input is a seeded sum of
isotropic Gaussian blobs, and a "target" is its seed with the blob centres jittered (and, optionally,
the amplitudes scaled), which keeps the "similar images" structure the method relies on.

Layout: an image of width W and height H is a float64 array of shape (C, W, H); pixel (i, j) with
i along the width (x) and j along the height (y).  Flattening one channel in C order gives the
unknown ordering p = i*H + j used by the linear systems (Section 2.3, vector definition: the
y index runs fastest).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_BASE = 251117634


def rng_for(*key: int) -> np.random.Generator:
    """Counter-style generator keyed by a tuple of small integers (config, role, index, ...)."""
    return np.random.default_rng([SEED_BASE, *[int(k) for k in key]])


@dataclass
class BlobSet:
    """Blob parameters of one image: centres (pixel units), widths and per-channel amplitudes."""
    ci: np.ndarray      # (B,) centre along the width, in [0, W)
    cj: np.ndarray      # (B,) centre along the height, in [0, H)
    sigma: np.ndarray   # (B,) standard deviation in pixels
    amp: np.ndarray     # (C, B) amplitude per channel


def draw_seed(rng: np.random.Generator, H: int, W: int, n_blobs: int, channels: int = 1,
              sigma_range=(2.0, 5.0), amp_range=(0.2, 1.0)) -> BlobSet:
    """Seed blobs: centres uniform over the image, sigma ~ U[2,5] px, amplitude ~ U[0.2,1].

    Centres and widths are shared by all channels; amplitudes are drawn per channel.
    """
    ci = rng.uniform(0.0, W, n_blobs)
    cj = rng.uniform(0.0, H, n_blobs)
    sigma = rng.uniform(sigma_range[0], sigma_range[1], n_blobs)
    amp = rng.uniform(amp_range[0], amp_range[1], (channels, n_blobs))
    return BlobSet(ci, cj, sigma, amp)


def jitter_target(rng: np.random.Generator, seed: BlobSet, jitter_px: float,
                  amp_scale: tuple[float, float] | None) -> BlobSet:
    """A target: the seed's blobs with each centre coordinate moved by N(0, jitter_px^2) and,
    when amp_scale is given, each amplitude multiplied by U[amp_scale]."""
    B = seed.ci.shape[0]
    ci = seed.ci + rng.normal(0.0, jitter_px, B)
    cj = seed.cj + rng.normal(0.0, jitter_px, B)
    amp = seed.amp.copy()
    if amp_scale is not None:
        amp = amp * rng.uniform(amp_scale[0], amp_scale[1], amp.shape)
    return BlobSet(ci, cj, seed.sigma.copy(), amp)


def render(blobs: BlobSet, H: int, W: int) -> np.ndarray:
    """Render to a (C, W, H) float64 image clipped to [0, 1]."""
    i = np.arange(W, dtype=np.float64)[:, None]
    j = np.arange(H, dtype=np.float64)[None, :]
    C = blobs.amp.shape[0]
    out = np.zeros((C, W, H), dtype=np.float64)
    for b in range(blobs.ci.shape[0]):
        g = np.exp(-((i - blobs.ci[b]) ** 2 + (j - blobs.cj[b]) ** 2) / (2.0 * blobs.sigma[b] ** 2))
        out += blobs.amp[:, b][:, None, None] * g[None]
    return np.clip(out, 0.0, 1.0)
