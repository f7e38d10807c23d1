"""Seeded synthetic inputs (Gaussian-blob images) shared by the oracle tests and the GPU path.

This package holds input generation only: no part of the linear-system method lives here.
"""
from .blobs import BlobSet, draw_seed, jitter_target, render
from .configs import (CONFIGS, Config, config_images, cycle_blocks, initial_state,
                      interleaved_images)

__all__ = ["BlobSet", "draw_seed", "jitter_target", "render", "CONFIGS", "Config",
           "config_images", "cycle_blocks", "initial_state", "interleaved_images"]
