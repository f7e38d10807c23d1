"""The five measured workloads and their seeded image sets.

Each workload is a set of groups; a group is one grid size with one seed image and N targets.
The constants g = 0.5, f = 0 and T = 100 follow the paper's experimental setup (Section 5);
grid sizes follow Experiment 2 (32x32, 64x64, 128x128).  Workload names state their sizes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .blobs import draw_seed, jitter_target, render, rng_for

ROLE_SEED, ROLE_TARGET, ROLE_EVAL = 0, 1, 2


@dataclass(frozen=True)
class Group:
    H: int                     # square grid H x H (W == H)
    n_targets: int
    n_blobs: int
    jitter: float | tuple      # px; a (lo, hi) tuple draws one jitter scale per target, U[lo, hi]
    amp_scale: tuple | None    # amplitude multiplier range for targets, or None


@dataclass(frozen=True)
class Config:
    key: int                   # RNG key of the workload
    name: str
    T: int                     # timesteps, dt = 1/T
    m: int                     # seed basis dimension = GMRES restart length
    channels: int
    groups: tuple = field(default_factory=tuple)
    precision: str = "fp64"
    g: float = 0.5
    tol: float = 1e-8

    @property
    def n_targets(self) -> int:
        return sum(gr.n_targets for gr in self.groups) * self.channels


CONFIGS = {
    "c1": Config(1, "grid28_1seed_1target_T50_m30_fp64", T=50, m=30, channels=1,
                 groups=(Group(28, 1, 8, 1.0, None),)),
    "c2": Config(2, "grid64_1seed_63targets_T100_m40_fp64", T=100, m=40, channels=1,
                 groups=(Group(64, 63, 8, 2.0, (0.9, 1.1)),)),
    "c3": Config(3, "grid128_1seed_255targets_T100_m60_mixed", T=100, m=60, channels=1,
                 groups=(Group(128, 255, 24, 2.0, (0.9, 1.1)),), precision="mixed"),
    "c4": Config(4, "uneven_32_64_128_1024targets_rgb_T100", T=100, m=40, channels=3,
                 groups=(Group(32, 342, 8, (0.5, 4.0), (0.9, 1.1)),
                         Group(64, 341, 8, (0.5, 4.0), (0.9, 1.1)),
                         Group(128, 341, 24, (0.5, 4.0), (0.9, 1.1)))),
    "c5": Config(5, "grid64_learned_guess_4096train_1024eval_T100_m40", T=100, m=40, channels=1,
                 groups=(Group(64, 4096, 8, 2.0, (0.9, 1.1)),)),
    # diverse set: 4 prototypes x 50 images, interleaved (clustered seed selection)
    "c7": Config(7, "grid64_200images_4prototypes_T100_m40", T=100, m=40, channels=1,
                 groups=tuple(Group(64, 50, 8, 2.0, (0.9, 1.1)) for _ in range(4))),
    # image cycle (Experiment 2's protocol): 100 similar images, a new seed every 50
    "c6": Config(6, "grid64_100images_cycle50_a20_T100_m40", T=100, m=40, channels=1,
                 groups=(Group(64, 100, 8, (0.5, 4.0), (0.9, 1.1)),)),
}


def config_images(cfg: Config, group: int = 0, first: int = 0, count: int | None = None,
                  role: int = ROLE_TARGET):
    """Seed image (C, H, H) and target images (count, C, H, H) of one group, all in [0, 1].

    Target k is generated from its own key (cfg.key, role, group, k), so any sub-range is
    reproducible without generating the ones before it.
    """
    gr = cfg.groups[group]
    H = gr.H
    seed_blobs = draw_seed(rng_for(cfg.key, ROLE_SEED, group), H, H, gr.n_blobs, cfg.channels)
    seed = render(seed_blobs, H, H)
    if count is None:
        count = gr.n_targets - first
    targets = np.empty((count, cfg.channels, H, H), dtype=np.float64)
    for t in range(count):
        rng = rng_for(cfg.key, role, group, first + t)
        if isinstance(gr.jitter, tuple):
            s = rng.uniform(gr.jitter[0], gr.jitter[1])
        else:
            s = gr.jitter
        targets[t] = render(jitter_target(rng, seed_blobs, s, gr.amp_scale), H, H)
    return seed, targets


def initial_state(image: np.ndarray) -> np.ndarray:
    """Initial log-density m^0 of one channel: the clipped pixel intensities themselves,
    flattened in the unknown ordering p = i*H + j (float64, contiguous)."""
    return np.ascontiguousarray(image, dtype=np.float64).reshape(-1)


def cycle_blocks(cfg: Config, cycle: int, count: int | None = None):
    """Images 0..count-1 of group 0 in blocks of `cycle`: block g is (seed (1, n), targets
    (cycle - 1, 1, n)) with image g*cycle as its seed and the rest of the block as targets
    (initial states m^0, flattened)."""
    _, imgs = config_images(cfg, 0, 0, count)
    blocks = []
    for g0 in range(0, imgs.shape[0], cycle):
        blk = imgs[g0:g0 + cycle, 0].reshape(-1, 1, imgs.shape[-2] * imgs.shape[-1])
        blocks.append((np.ascontiguousarray(blk[0]), np.ascontiguousarray(blk[1:])))
    return blocks


def interleaved_images(cfg: Config):
    """The targets of all groups interleaved (image k from group k mod G, index k // G), as
    (count, H*H) initial states of one channel: a set whose similar images are not adjacent."""
    per = [config_images(cfg, g)[1][:, 0] for g in range(len(cfg.groups))]
    G, n = len(per), min(len(p) for p in per)
    H = cfg.groups[0].H
    out = np.empty((G * n, H * H))
    for k in range(G * n):
        out[k] = per[k % G][k // G].reshape(-1)
    return out
