"""Parity at the measured workloads' full sizes, in the launch configuration the benchmark
times (autotuned launch, chain replayed from a captured graph): every solve is verified by the
library's FP64 residual, and sampled targets follow the oracle's chain within the accumulated
tolerance bound.  Every call goes through the C ABI."""
import numpy as np
import pytest

from gpu_util import cpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    from paper_2511_17634_amd import xkp
    xkp.load()
    return xkp


def test_benchmark_workload_full_size_sampled(X):
    """64x64, 1 seed + 63 targets, T = 100, m = 40: the benchmark's chain (autotuned, graph
    replay); targets 0, 31 and 62 and the seed against the oracle chain."""
    import torch
    from oracle.chain import run_chain
    from paper_2511_17634_amd.driver import Chain
    from synth import CONFIGS, config_images, initial_state
    cfg = CONFIGS["c2"]
    H = cfg.groups[0].H
    seed, tg = config_images(cfg, 0)
    s0 = initial_state(seed[0])
    t0 = np.stack([initial_state(t[0]) for t in tg])
    ch = Chain(H, cfg.T, cfg.m, s0, t0)
    ch.autotune()
    ch.run()
    ch.capture()
    ch.replay()
    torch.cuda.synchronize()
    s_inf, t_inf = ch.all_infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.all(t_inf["res_true"] <= cfg.tol)
    assert np.all(ch.verify_last() <= cfg.tol * (1 + 1e-6))
    pick = [0, 31, 62]
    ms_o, mt_o, st = run_chain(s0, t0[pick], H, cfg.T, cfg.m)
    bound = cfg.T * cfg.tol * max(np.linalg.norm(s0), np.linalg.norm(t0, axis=1).max())
    assert np.abs(cpu(ch.target_state)[pick] - mt_o).max() <= bound
    assert np.abs(cpu(ch.seed_state) - ms_o).max() <= bound
    # the projected guesses the oracle forms on its own seed basis agree in quality
    g_gpu = t_inf["guess_res"][:, pick]
    g_o = np.array(st.guess_res)
    assert np.abs(g_gpu - g_o).max() <= 1e-6 + 1e-3 * g_o.max()


def test_uneven_workload_full_size_sampled(X):
    """32/64/128 x RGB, 3072 targets + 9 seeds in one launch per timestep (autotuned): ten
    timesteps; one target of each size (channel 0) and its seed against the oracle chain."""
    import torch
    from oracle.chain import run_chain
    from paper_2511_17634_amd.driver import Batch, Group
    from synth import CONFIGS, config_images
    cfg = CONFIGS["c4"]
    groups = []
    for gi, gr in enumerate(cfg.groups):
        seed, tg = config_images(cfg, gi)
        groups.append(Group(gr.H, seed.reshape(cfg.channels, -1),
                            tg.reshape(tg.shape[0], cfg.channels, -1)))
    b = Batch(groups, cfg.T, cfg.m)
    b.autotune()
    b.reset()
    steps = 10
    for _ in range(steps):
        b.step()
    torch.cuda.synchronize()
    s_inf, t_inf = b.infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.all(t_inf["res_true"] <= cfg.tol)
    for gi, gr in enumerate(b.groups):
        ms_g, mt_g = b.group_states(gi)
        t = gr.N // 2
        ms_o, mt_o, _ = run_chain(gr.seed_m0[0], gr.target_m0[t, 0][None], gr.H, cfg.T, cfg.m,
                                  steps=steps)
        bound = steps * cfg.tol * max(np.linalg.norm(gr.seed_m0[0]),
                                      np.linalg.norm(gr.target_m0[t, 0]))
        assert np.abs(cpu(mt_g[t, 0]) - mt_o[0]).max() <= bound, gr.H
        assert np.abs(cpu(ms_g[0]) - ms_o).max() <= bound, gr.H


def test_mixed_workload_full_batch_sampled(X):
    """128x128, 1 seed + 255 targets, m = 60, mixed precision, autotuned: three timesteps;
    targets 0, 127 and 254 and the seed against the FP64 oracle chain (mixed precision must
    still meet the FP64 tolerance, so the states agree within the accumulated bound)."""
    import torch
    from oracle.chain import run_chain
    from paper_2511_17634_amd.driver import Chain
    from synth import CONFIGS, config_images, initial_state
    cfg = CONFIGS["c3"]
    H = cfg.groups[0].H
    seed, tg = config_images(cfg, 0)
    s0 = initial_state(seed[0])
    t0 = np.stack([initial_state(t[0]) for t in tg])
    ch = Chain(H, cfg.T, cfg.m, s0, t0, precision=X.MIXED)
    ch.autotune()
    ch.reset()
    steps = 3
    for _ in range(steps):
        ch.step()
    torch.cuda.synchronize()
    s_inf, t_inf = ch.infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.all(t_inf["res_true"] <= cfg.tol)
    pick = [0, 127, 254]
    ms_o, mt_o, _ = run_chain(s0, t0[pick], H, cfg.T, cfg.m, steps=steps)
    bound = steps * cfg.tol * max(np.linalg.norm(s0), np.linalg.norm(t0, axis=1).max())
    assert np.abs(cpu(ch.target_state)[pick] - mt_o).max() <= bound
    assert np.abs(cpu(ch.seed_state) - ms_o).max() <= bound
