"""Helpers for the GPU parity tests: device tensors and descriptor packing."""
import numpy as np


def dev():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    return torch.device("cuda:0")


def t64(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev())


def cpu(t):
    return t.detach().cpu().numpy()


def blob_pair(H, seed=0, jitter=1.0):
    """A seed/target pair of blob images on an H x H grid, flattened (p = i*H + j)."""
    from synth.blobs import draw_seed, jitter_target, render, rng_for
    rng = rng_for(900, H, seed)
    sb = draw_seed(rng, H, H, 8)
    tb = jitter_target(rng, sb, jitter, (0.9, 1.1))
    return render(sb, H, H)[0].reshape(-1), render(tb, H, H)[0].reshape(-1)
