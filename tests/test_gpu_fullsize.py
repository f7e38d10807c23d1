"""Parity at the measured workloads' full sizes, in the launch configuration the benchmark
times (autotuned launch, chain replayed from a captured graph): every solve is verified by the
library's FP64 residual, and sampled targets follow the oracle's chain within the accumulated
tolerance bound.  Every call goes through the C ABI."""
import numpy as np
import pytest

import oracle
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


def _oracle_chains(jobs, T, m, workers=16):
    """Oracle chains in threads: jobs = [(H, seed m0, [target m0...])]; returns per job
    (target states [T, N, n], guess residuals [T, N]), seed chain first, then its targets."""
    from concurrent.futures import ThreadPoolExecutor

    def seed_chain(job):
        H, s0, _ = job
        dt, ms, out = 1.0 / T, np.array(s0), []
        for _ in range(T):
            A = oracle.Operator(H, dt, 0.5, ms)
            r = oracle.gmres(A, oracle.rhs(A, ms), m=m, keep_basis=True)
            out.append((r.V, r.Hbar))
            ms = r.x
        return out

    def target_chain(args):
        H, t0, bases = args
        dt, mt = 1.0 / T, np.array(t0)
        rec, gr = np.empty((T, H * H)), np.empty(T)
        for n in range(T):
            A = oracle.Operator(H, dt, 0.5, mt)
            b = oracle.rhs(A, mt)
            x0, _, _ = oracle.project(A, b, *bases[n])
            gr[n] = oracle.residual(A, b, x0)
            mt = oracle.gmres(A, b, x0=x0, m=m, passes=1).x
            rec[n] = mt
        return rec, gr
    with ThreadPoolExecutor(workers) as ex:
        bases = list(ex.map(seed_chain, jobs))
        tj = [(H, t, bases[k]) for k, (H, _, ts) in enumerate(jobs) for t in ts]
        res = list(ex.map(target_chain, tj))
    out, i = [], 0
    for H, _, ts in jobs:
        r = res[i:i + len(ts)]
        i += len(ts)
        out.append((np.stack([a for a, _ in r], axis=1), np.stack([g for _, g in r], axis=1)))
    return out


def test_uneven_workload_all_timesteps_sampled(X):
    """32/64/128 x RGB, 3072 targets + 9 seeds in one launch per timestep (autotuned): all 100
    timesteps; one target of each size in every channel against the oracle chain of its own
    seed: the state after every timestep within the accumulated tolerance bound, and every
    projected guess's residual (within 5 %, median within 1 %)."""
    import torch
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
    picks, jobs = [], []
    off = 0
    for gr in b.groups:                       # largest grid first, as the batch lays them out
        t = gr.N // 2
        for c in range(gr.C):
            picks.append(off + t * gr.C + c)
            jobs.append((gr.H, gr.seed_m0[c], [gr.target_m0[t, c]]))
        off += gr.N * gr.C
    rec = cpu(b.record_chain(picks))
    s_inf, t_inf = b.all_infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.all(t_inf["res_true"] <= cfg.tol)
    ref = _oracle_chains(jobs, cfg.T, cfg.m)
    steps = np.arange(1, cfg.T + 1)[:, None]
    for j, (H, s0, ts) in enumerate(jobs):
        ro, go = ref[j]
        n = H * H
        bound = steps * cfg.tol * max(np.linalg.norm(s0), np.linalg.norm(ts[0]))
        err = np.abs(rec[:, j, :n] - ro[:, 0]).max(axis=1, keepdims=True)
        assert np.all(err <= bound), (H, j, float((err / bound).max()))
        # the guesses: the seed states of the two chains differ within the tolerance, and the
        # later Krylov columns amplify that (at 128x128 the kept cycle runs all 40 steps), so a
        # guess residual can move by a few per cent (a wrong basis, source or transposed
        # projection moves it by tens of per cent)
        g = t_inf["guess_res"][:, picks[j]]
        rel = np.abs(g - go[:, 0]) / go[:, 0]
        assert rel.max() <= 0.05 and np.median(rel) <= 1e-2, (H, j, rel.max(), np.median(rel))


def test_mixed_workload_all_timesteps_sampled(X):
    """128x128, 1 seed + 255 targets, m = 60, mixed precision, autotuned: all 100 timesteps;
    targets 0, 127 and 254 against the FP64 oracle chain: the state after every timestep within
    the accumulated tolerance bound (mixed precision still meets the FP64 tolerance), and the
    projected guesses' residuals (within 5 % plus the BF16 contraction's 2e-3, median within 1 %)."""
    import torch
    from paper_2511_17634_amd.driver import Chain
    from synth import CONFIGS, config_images, initial_state
    cfg = CONFIGS["c3"]
    H = cfg.groups[0].H
    seed, tg = config_images(cfg, 0)
    s0 = initial_state(seed[0])
    t0 = np.stack([initial_state(t[0]) for t in tg])
    ch = Chain(H, cfg.T, cfg.m, s0, t0, precision=X.MIXED)
    ch.autotune()
    pick = [0, 127, 254]
    rec = cpu(ch.record_chain(pick))
    s_inf, t_inf = ch.all_infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.all(t_inf["res_true"] <= cfg.tol)
    (ro, go), = _oracle_chains([(H, s0, list(t0[pick]))], cfg.T, cfg.m)
    steps = np.arange(1, cfg.T + 1)[:, None]
    bound = steps * cfg.tol * max(np.linalg.norm(s0), np.linalg.norm(t0[pick], axis=1).max())
    err = np.abs(rec - ro).max(axis=2)
    assert np.all(err <= bound), float((err / bound).max())
    # the BF16 contraction perturbs each guess's residual by up to about 1e-3 absolute on top
    # of the seed chains' own difference (a few per cent)
    g = t_inf["guess_res"][:, pick]
    rel = np.abs(g - go) / go
    assert np.all(np.abs(g - go) <= 0.05 * go + 2e-3), float(np.abs(g - go).max())
    assert np.median(rel) <= 1e-2, np.median(rel)
