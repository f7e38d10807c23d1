"""GPU Picard passes per timestep (K linearisations around the previous iterate) against the
oracle chain: states, iteration counts of every pass, the final solve's FP64 residual and the
contraction of the nonlinear residual.  Every call goes through the C ABI."""
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


@pytest.mark.parametrize("K", [2, 3])
def test_picard_chain_matches_oracle(X, K):
    import torch
    from oracle.chain import run_chain
    from paper_2511_17634_amd.driver import Chain
    from synth import CONFIGS, config_images, initial_state
    cfg = CONFIGS["c1"]
    H = cfg.groups[0].H
    seed, tg = config_images(cfg, 0, 0, 2)
    s0 = initial_state(seed[0])
    t0 = np.stack([initial_state(t[0]) for t in tg])
    ch = Chain(H, cfg.T, cfg.m, s0, t0, picard=K)
    ch.run()
    torch.cuda.synchronize()
    s_inf, t_inf = ch.all_infos()
    ps, pt = ch.picard_infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.all(ps["status"] == X.OK) and np.all(pt["status"] == X.OK)
    assert np.all(pt["res_true"] <= cfg.tol)
    assert np.all(ch.verify_last() <= cfg.tol * (1 + 1e-6))
    ms_o, mt_o, st = run_chain(s0, t0, H, cfg.T, cfg.m, picard=K)
    bound = cfg.T * cfg.tol * max(np.linalg.norm(s0), np.linalg.norm(t0, axis=1).max())
    assert np.abs(cpu(ch.target_state) - mt_o).max() <= bound
    assert np.abs(cpu(ch.seed_state) - ms_o).max() <= bound
    assert np.abs(t_inf["iters"].astype(int) - np.array(st.iters)).max() <= 2
    assert np.abs(pt["iters"].astype(int) - np.array(st.picard_iters)).max() <= 2
    # later passes start from the previous iterate: fewer iterations than the first
    assert pt["iters"][:, -1].mean() < t_inf["iters"].mean()
    # the last state nearly solves the nonlinear step: ||A(m) m - b|| / ||b|| small
    m_prev = run_chain(s0, t0, H, cfg.T, cfg.m, picard=K, steps=cfg.T - 1)[1]
    for i in range(len(t0)):
        mK = cpu(ch.target_state)[i]
        A = oracle.Operator(H, 1.0 / cfg.T, cfg.g, mK)
        b = oracle.rhs(A, m_prev[i])
        r = np.linalg.norm(oracle.apply(A, mK) - b) / np.linalg.norm(b)
        A1 = oracle.Operator(H, 1.0 / cfg.T, cfg.g, m_prev[i])
        x1, _ = oracle.banded_solve(A1, b)                 # one pass only
        A1x = oracle.Operator(H, 1.0 / cfg.T, cfg.g, x1)
        r1 = np.linalg.norm(oracle.apply(A1x, x1) - b) / np.linalg.norm(b)
        assert r < r1, (r, r1)
    # the same chain replayed from a captured graph, twice, equals the eager chain bitwise
    eager = cpu(ch.target_state).copy(), cpu(ch.seed_state).copy()
    ch.capture()
    for _ in range(2):
        ch.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cpu(ch.target_state), eager[0])
        assert np.array_equal(cpu(ch.seed_state), eager[1])
        ch.run()                      # eager work between the replays
        torch.cuda.synchronize()
