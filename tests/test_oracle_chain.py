"""Pins of the timestep chain: the Cole-Hopf exact solution of the log-density equation, the
discrete maximum principle, and agreement of the three solution routes."""
import numpy as np
import pytest

import oracle
from oracle.chain import run_chain
from synth import CONFIGS, config_images, initial_state


def cole_hopf_error(H, T, g=0.5, eps=0.9, t_end=0.5):
    """With f = 0, p = exp(m) solves p_t = (g^2/2) lap p (eq. log_fp), and zero padding of m is
    p = 1 on the ghost ring at distance h outside the grid.  On the box of side L = 1 + h between
    the ghost rows, p = 1 + eps exp(-g^2 pi^2 t / L^2) sin(pi xi/L) sin(pi eta/L) is exact."""
    h = 1.0 / H
    L = 1.0 + h
    i, j = np.meshgrid(np.arange(H), np.arange(H), indexing="ij")
    S = (np.sin(np.pi * (i * h + h) / L) * np.sin(np.pi * (j * h + h) / L)).reshape(-1)
    m = np.log1p(eps * S)
    dt = t_end / T
    for _ in range(T):
        A = oracle.Operator(H, dt, g, m)            # one linearisation pass: m~ = m^{n-1}
        m, st = oracle.banded_solve(A, oracle.rhs(A, m))
        assert st == oracle.OK
    exact = np.log1p(eps * np.exp(-g * g * np.pi**2 * t_end / L**2) * S)
    return np.abs(m - exact).max()


def test_cole_hopf_first_order_convergence(olib):
    e = [cole_hopf_error(32, T) for T in (10, 20, 40)]
    assert 1.8 <= e[0] / e[1] <= 2.2 and 1.8 <= e[1] / e[2] <= 2.2
    assert e[2] < 4e-3


def test_maximum_principle_and_zero_image(olib):
    cfg = CONFIGS["c1"]
    seed, tg = config_images(cfg, 0, 0, 1)
    H = cfg.groups[0].H
    m = initial_state(tg[0, 0])
    for _ in range(5):
        A = oracle.Operator(H, 1.0 / cfg.T, cfg.g, m)
        new, _ = oracle.banded_solve(A, oracle.rhs(A, m))
        assert new.min() >= -1e-14 and new.max() <= m.max() + 1e-14
        m = new
    A = oracle.Operator(H, 1.0 / cfg.T, cfg.g, np.zeros(H * H))
    z = oracle.gmres(A, oracle.rhs(A, np.zeros(H * H)), m=cfg.m)
    assert np.all(z.x == 0)


@pytest.mark.parametrize("mode", [oracle.TARGET_GALERKIN, oracle.SEED_GALERKIN])
def test_chain_routes_agree_with_direct(olib, mode):
    """Projection+polish, plain GMRES and banded LU give the same chain within the accumulated
    Varah bound (each step's error <= dt * residual, amplified by at most 1 per step since the
    solution operator has infinity norm <= 1)."""
    cfg = CONFIGS["c1"]
    seed, tg = config_images(cfg, 0, 0, 1)
    H = cfg.groups[0].H
    s0 = initial_state(seed[0])
    t0 = initial_state(tg[0, 0])[None]
    steps = 6
    _, m_proj, st = run_chain(s0, t0, H, cfg.T, cfg.m, method="project", mode=mode, steps=steps)
    _, m_plain, _ = run_chain(s0, t0, H, cfg.T, cfg.m, method="plain", steps=steps)
    _, m_dir, _ = run_chain(s0, t0, H, cfg.T, cfg.m, method="direct", steps=steps)
    assert max(max(r) for r in st.res_true) <= cfg.tol
    # per step: ||x - x*||_inf <= dt ||r||_inf <= dt tol ||b||_2 = tol ||m^{n-1}||_2
    bound = steps * cfg.tol * max(np.linalg.norm(s0), np.linalg.norm(t0))
    assert np.abs(m_proj - m_dir).max() <= bound + 1e-13
    assert np.abs(m_plain - m_dir).max() <= bound + 1e-13


def test_picard_one_is_the_plain_chain_and_iterates_contract(olib):
    """K = 1 is the one-pass chain bitwise; more Picard passes contract to the fixed point of
    m -> A(m)^{-1} b, so the nonlinear residual ||A(m) m - b|| / ||b|| falls geometrically."""
    cfg = CONFIGS["c1"]
    seed, tg = config_images(cfg, 0, 0, 1)
    H = cfg.groups[0].H
    s0, t0 = initial_state(seed[0]), initial_state(tg[0, 0])[None]
    a = run_chain(s0, t0, H, cfg.T, cfg.m, method="direct", steps=2)
    b = run_chain(s0, t0, H, cfg.T, cfg.m, method="direct", steps=2, picard=1)
    assert np.array_equal(a[1], b[1])
    m_prev = run_chain(s0, t0, H, cfg.T, cfg.m, method="direct", steps=1)[1][0]
    A0 = oracle.Operator(H, 1.0 / cfg.T, cfg.g, m_prev)
    rhs = oracle.rhs(A0, m_prev)
    res = []
    for K in range(1, 8):
        mK = run_chain(m_prev, m_prev[None], H, cfg.T, cfg.m, method="direct", steps=1,
                       picard=K)[1][0]
        AK = oracle.Operator(H, 1.0 / cfg.T, cfg.g, mK)
        res.append(np.linalg.norm(oracle.apply(AK, mK) - rhs) / np.linalg.norm(rhs))
    assert all(r2 < 0.5 * r1 for r1, r2 in zip(res[:4], res[1:5])), res
    assert res[-1] < 1e-9, res


def test_picard_limit_keeps_first_order_cole_hopf(olib):
    """The chain with K = 4 Picard passes (close to the fully implicit nonlinear scheme) also
    converges at first order to the Cole-Hopf solution (dt = t_end / steps through T = 2 steps)."""
    def err(steps, K, H=32, g=0.5, eps=0.9):
        h = 1.0 / H
        L = 1.0 + h
        i, j = np.meshgrid(np.arange(H), np.arange(H), indexing="ij")
        S = (np.sin(np.pi * (i * h + h) / L) * np.sin(np.pi * (j * h + h) / L)).reshape(-1)
        m0 = np.log1p(eps * S)
        _, mt, _ = run_chain(m0, m0[None], H, 2 * steps, 30, g=g, method="direct",
                             steps=steps, picard=K)
        exact = np.log1p(eps * np.exp(-g * g * np.pi**2 * 0.5 / L**2) * S)
        return np.abs(mt[0] - exact).max()
    e = [err(T, 4) for T in (10, 20, 40)]
    assert 1.7 <= e[0] / e[1] <= 2.3 and 1.7 <= e[1] / e[2] <= 2.3, e
