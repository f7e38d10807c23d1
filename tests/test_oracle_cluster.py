"""Pins of the oracle's clustered seed selection: block means by hand, recovery of well
separated groups, the k-means objective never rising, the K = 1 and K = N extremes, and the
farthest-first start on points whose order is known."""
import numpy as np

from oracle import cluster as CL


def test_block_means_by_hand():
    H = 4
    img = np.arange(16, dtype=np.float64)           # p = i*4 + j
    F = CL.features(img[None], H, 2)
    # block (0,0): p 0,1,4,5; (0,1): 2,3,6,7; (1,0): 8,9,12,13; (1,1): 10,11,14,15
    assert np.array_equal(F[0], [2.5, 4.5, 10.5, 12.5])


def groups(K=4, per=12, H=16, seed=0):
    rng = np.random.default_rng(seed)
    protos = rng.uniform(0, 1, (K, H * H))
    labels = np.arange(K * per) % K                 # interleaved
    imgs = protos[labels] + 0.01 * rng.normal(size=(K * per, H * H))
    return imgs, labels


def test_recovers_well_separated_groups():
    imgs, labels = groups()
    assign, seeds, it = CL.cluster_seeds(imgs, 16, 4, 4)
    # the partition equals the true one up to cluster names
    for c in range(4):
        members = np.nonzero(assign == c)[0]
        assert len(set(labels[members])) == 1 and len(members) == 12
        assert assign[seeds[c]] == c
    assert it <= 3


def test_objective_never_rises():
    rng = np.random.default_rng(3)
    imgs = rng.uniform(0, 1, (40, 64))
    F = CL.features(imgs, 8, 2)
    prev = np.inf
    for iters in range(1, 8):
        assign, _, _ = CL.cluster_seeds(imgs, 8, 2, 5, max_iters=iters)
        C = np.array([F[assign == c].mean(axis=0) if np.any(assign == c) else np.zeros(16)
                      for c in range(5)])
        obj = sum(np.sum((F[i] - C[assign[i]]) ** 2) for i in range(40))
        assert obj <= prev + 1e-12
        prev = obj


def test_extremes():
    rng = np.random.default_rng(4)
    imgs = rng.uniform(0, 1, (9, 16))
    F = CL.features(imgs, 4, 1)
    a, s, _ = CL.cluster_seeds(imgs, 4, 1, 1)
    assert np.all(a == 0)
    d = np.sum((F - F.mean(axis=0)) ** 2, axis=1)
    assert s[0] == int(np.argmin(d))
    a, s, _ = CL.cluster_seeds(imgs, 4, 1, 9)
    assert sorted(a.tolist()) == list(range(9)) and np.array_equal(a[s], np.arange(9))


def test_farthest_first_start_on_a_line():
    """Points 0, 1, 2, 10 (as 1-pixel images): the start picks 0, then 10 (index 3), then 2
    (nearest chosen 0 or 10 at distance 4 from 2 vs 1 from 1); the clusters are {0,1,2} split
    as {0,1} / {2} / {10} after Lloyd."""
    imgs = np.array([[0.0], [1.0], [2.0], [10.0]])
    a, s, _ = CL.cluster_seeds(imgs, 1, 1, 3)
    assert a[3] != a[0] and a[2] != a[0] and a[0] == a[1]
    assert s[a[3]] == 3 and s[a[2]] == 2
