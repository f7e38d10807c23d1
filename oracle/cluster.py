"""Clustered seed selection (test infrastructure only; shares nothing with the HIP library).

The paper suggests clustering the images so that every group of similar images gets its own
seed (its closing discussion of diverse datasets).  Definition used here:
  features  each image (H x H, p = i*H + j) averaged over pool x pool blocks, flattened in the
            same order (feature f = fi * (H/pool) + fj)
  init      farthest-first traversal: centroid 0 = image 0; centroid k = the image whose squared
            distance to the nearest of centroids 0..k-1 is largest (lowest index on ties; an
            image already chosen has distance 0)
  Lloyd     assignment: nearest centroid by squared Euclidean distance (lowest cluster on ties);
            stop when no assignment changes (after at least one) or after max_iters
            assignments; update: each centroid the mean of its members (an empty cluster keeps
            its centroid); after the last update the images are assigned once more
  seeds     seed of cluster c = its member nearest to centroid c (lowest index on ties), -1 if
            the cluster is empty
"""
from __future__ import annotations

import numpy as np


def features(images, H: int, pool: int) -> np.ndarray:
    """(N, (H/pool)^2) block means."""
    X = np.asarray(images, dtype=np.float64).reshape(-1, H // pool, pool, H // pool, pool)
    return X.mean(axis=(2, 4)).reshape(X.shape[0], -1)


def sqdist(F, C) -> np.ndarray:
    """(N, K) squared distances, summed over features in order."""
    return np.array([[np.sum((f - c) ** 2) for c in C] for f in F])


def cluster_seeds(images, H: int, pool: int, K: int, max_iters: int = 50):
    """Returns (assign (N,), seeds (K,), iterations)."""
    F = features(images, H, pool)
    N = F.shape[0]
    chosen = [0]
    C = [F[0].copy()]
    for _ in range(1, K):
        d = sqdist(F, C).min(axis=1)
        chosen.append(int(np.argmax(d)))           # first index of the largest
        C.append(F[chosen[-1]].copy())
    C = np.array(C)
    assign = None
    it = 0
    while it < max_iters:
        new = np.argmin(sqdist(F, C), axis=1)      # first index of the smallest
        it += 1
        if assign is not None and np.array_equal(new, assign):
            break
        assign = new
        for c in range(K):
            members = np.nonzero(assign == c)[0]
            if len(members):
                C[c] = F[members].sum(axis=0) / len(members)
    D = sqdist(F, C)
    assign = np.argmin(D, axis=1)
    seeds = np.full(K, -1)
    for c in range(K):
        members = np.nonzero(assign == c)[0]
        if len(members):
            seeds[c] = members[np.argmin(D[members, c])]
    return assign, seeds, it
