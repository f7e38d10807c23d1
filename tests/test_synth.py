"""The seeded blob generator: reproducible, in range, targets near their seed."""
import numpy as np

from synth import CONFIGS, config_images, initial_state


def test_reproducible_and_in_range():
    cfg = CONFIGS["c2"]
    s1, t1 = config_images(cfg, 0, 5, 3)
    s2, t2 = config_images(cfg, 0, 0, 8)
    assert np.array_equal(s1, s2) and np.array_equal(t1, t2[5:8])
    assert t1.shape == (3, 1, 64, 64) and 0 <= t1.min() and t1.max() <= 1
    assert np.abs(t1[0] - s1).mean() < np.abs(s1).mean()


def test_uneven_workload_shapes():
    cfg = CONFIGS["c4"]
    assert [g.n_targets for g in cfg.groups] == [342, 341, 341]
    assert cfg.n_targets == 3072
    s, t = config_images(cfg, 2, 0, 2)
    assert s.shape == (3, 128, 128) and t.shape == (2, 3, 128, 128)
    assert initial_state(t[0, 1]).shape == (128 * 128,)
