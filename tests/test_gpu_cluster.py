"""GPU parity of the clustered seed selection (xkp_cluster_seeds) against the oracle, the Lloyd
fixed-point property on unstructured data, and a clustered chain whose projected guesses beat
one seed for all on a diverse image set.  Every call goes through the C ABI."""
import numpy as np
import pytest

from gpu_util import cpu, t64
from oracle import cluster as CL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    from paper_2511_17634_amd import xkp
    xkp.load()
    return xkp


def test_cluster_matches_oracle_on_the_diverse_set(X):
    from synth import CONFIGS, interleaved_images
    imgs = interleaved_images(CONFIGS["c7"])
    ctx = X.Context(64 * 64, 8, 1)
    for K, pool in ((4, 8), (6, 4), (1, 16)):
        a, s, it = ctx.cluster_seeds(t64(imgs), 64, pool, K)
        ao, so, ito = CL.cluster_seeds(imgs, 64, pool, K)
        assert np.array_equal(cpu(a), ao) and np.array_equal(cpu(s), so) and it == ito, K


def test_lloyd_fixed_point_on_unstructured_data(X):
    """Uniform random images: each image ends at its nearest centroid (centroids recomputed
    from the returned assignment), and each seed is its cluster's member nearest the centroid."""
    rng = np.random.default_rng(9)
    H, pool, K = 16, 2, 7
    imgs = rng.uniform(0, 1, (90, H * H))
    ctx = X.Context(H * H, 8, 1)
    a, s, it = ctx.cluster_seeds(t64(imgs), H, pool, K, max_iters=200)
    a, s = cpu(a), cpu(s)
    F = CL.features(imgs, H, pool)
    C = np.array([F[a == c].mean(axis=0) for c in range(K)])
    D = CL.sqdist(F, C)
    assert np.all(D[np.arange(90), a] <= D.min(axis=1) * (1 + 1e-12))
    for c in range(K):
        members = np.nonzero(a == c)[0]
        assert s[c] in members and D[s[c], c] <= D[members, c].min() * (1 + 1e-12)
    # the oracle reaches the same partition
    ao, so, _ = CL.cluster_seeds(imgs, H, pool, K, max_iters=200)
    assert np.array_equal(a, ao) and np.array_equal(s, so)
    # host-side argument errors
    with pytest.raises(X.XkpError):
        ctx.cluster_seeds(t64(imgs), H, 3, K)        # pool does not divide H
    with pytest.raises(X.XkpError):
        ctx.cluster_seeds(t64(imgs), H, pool, 65)


def test_clustered_chain_beats_one_seed_on_a_diverse_set(X):
    """Two prototypes, 8 images each, interleaved at 32x32: one seed per cluster gives better
    projected guesses than one seed for all, and every solve converges."""
    import torch
    from paper_2511_17634_amd.driver import Batch, Group, cluster_groups
    from synth.blobs import draw_seed, jitter_target, render, rng_for
    H, T, m = 32, 5, 20
    protos = [draw_seed(rng_for(77, p), H, H, 8) for p in range(2)]
    imgs = np.stack([render(jitter_target(rng_for(78, k), protos[k % 2], 1.0, (0.9, 1.1)),
                            H, H)[0].reshape(-1) for k in range(16)])
    ctx = X.Context(H * H, 8, 1)
    a, s, _ = ctx.cluster_seeds(t64(imgs), H, 4, 2)
    a = cpu(a)
    assert len(set(a[0::2])) == 1 and len(set(a[1::2])) == 1 and a[0] != a[1]
    groups = cluster_groups(imgs, H, a, cpu(s))
    assert len(groups) == 2 and sum(g.N for g in groups) == 14
    res = {}
    for name, gr in (("clustered", groups),
                     ("one_seed", [Group(H, imgs[0][None], imgs[1:][:, None])])):
        b = Batch(gr, T, m)
        b.run()
        torch.cuda.synchronize()
        s_inf, t_inf = b.all_infos()
        assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
        assert np.all(t_inf["res_true"] <= 1e-8)
        res[name] = float(np.mean(t_inf["guess_res"]))
    assert res["clustered"] < res["one_seed"], res
