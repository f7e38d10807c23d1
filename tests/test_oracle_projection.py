"""Pins of the oracle's seed basis and target projection (Section 3, Phases 1 and 2)."""
import numpy as np
import pytest

import oracle
from synth import CONFIGS, config_images, initial_state


def seed_and_target(H=16, T=100, m=20, seed=0):
    rng = np.random.default_rng(seed)
    ms = rng.uniform(0, 1, H * H)
    mt = np.clip(ms + 0.1 * rng.normal(size=H * H), 0, 1)
    As = oracle.Operator(H, 1.0 / T, 0.5, ms)
    At = oracle.Operator(H, 1.0 / T, 0.5, mt)
    bs, bt = oracle.rhs(As, ms), oracle.rhs(At, mt)
    sr = oracle.gmres(As, bs, m=m, keep_basis=True)
    return As, At, bs, bt, sr


@pytest.mark.parametrize("mode", [oracle.TARGET_GALERKIN, oracle.SEED_GALERKIN])
@pytest.mark.parametrize("warm", [False, True])
def test_galerkin_orthogonality(olib, mode, warm):
    As, At, bs, bt, sr = seed_and_target()
    k = sr.basis_dim
    V = sr.V[:, :k]
    xb = At.mt if warm else None
    x0, alpha, st = oracle.project(At, bt, sr.V, sr.Hbar, mode=mode, x_base=xb)
    assert st == oracle.OK
    rb = bt - (oracle.apply(At, xb) if warm else 0)
    Aop = At if mode == oracle.TARGET_GALERKIN else As
    AVa = oracle.apply(Aop, V @ alpha)
    assert np.abs(V.T @ (rb - AVa)).max() <= 1e-11 * np.linalg.norm(rb)
    assert np.allclose(x0, (xb if warm else 0) + V @ alpha, rtol=0, atol=1e-14 * np.abs(x0).max())


def test_least_squares_mode_minimises_projected_residual(olib):
    As, At, bs, bt, sr = seed_and_target(m=12)
    k = sr.basis_dim
    x0, alpha, st = oracle.project(At, bt, sr.V, sr.Hbar, mode=oracle.SEED_LSQ)
    assert st == oracle.OK
    z = sr.V.T @ bt
    ref, *_ = np.linalg.lstsq(sr.Hbar, z, rcond=None)
    assert np.allclose(alpha, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_mode_consistency_when_target_is_seed(olib):
    As, At, bs, bt, sr = seed_and_target()
    x_t, a_t, _ = oracle.project(As, bs, sr.V, sr.Hbar, mode=oracle.TARGET_GALERKIN)
    x_s, a_s, _ = oracle.project(As, bs, sr.V, sr.Hbar, mode=oracle.SEED_GALERKIN)
    assert np.abs(a_t - a_s).max() <= 1e-10 * np.abs(a_s).max()


def test_seed_self_projection_reproduces_seed_solution(olib):
    """Target = seed, x_base = 0: least-squares mode gives back the seed's own first-cycle GMRES
    iterate; on a grid where the first cycle converges that is the seed solution, and the
    Galerkin mode (the FOM iterate) lies within the Varah bound of it."""
    H, T = 6, 100
    rng = np.random.default_rng(1)
    ms = rng.uniform(0, 1, H * H)
    As = oracle.Operator(H, 1.0 / T, 0.5, ms)
    bs = oracle.rhs(As, ms)
    sr = oracle.gmres(As, bs, m=36, tol=1e-12, keep_basis=True)
    assert sr.restarts == 0
    x_l, _, _ = oracle.project(As, bs, sr.V, sr.Hbar, mode=oracle.SEED_LSQ)
    assert np.abs(x_l - sr.x).max() <= 1e-12 * np.abs(sr.x).max()
    x_g, _, _ = oracle.project(As, bs, sr.V, sr.Hbar, mode=oracle.SEED_GALERKIN)
    rinf = np.abs(bs - oracle.apply(As, x_g)).max()
    assert np.abs(x_g - sr.x).max() <= rinf / T + 1e-11 * np.abs(sr.x).max()
    polish = oracle.gmres(As, bs, x0=x_l, m=36, tol=1e-10)
    assert polish.iters == 0


def test_singular_projection_falls_back_to_base(olib):
    As, At, bs, bt, sr = seed_and_target(m=8)
    V = sr.V.copy()
    V[:, 2] = V[:, 1]                      # duplicated basis column: V^T A V is singular
    xb = At.mt
    x0, alpha, st = oracle.project(At, bt, V, sr.Hbar, mode=oracle.TARGET_GALERKIN, x_base=xb)
    assert st == oracle.ESINGULAR
    assert np.array_equal(x0, xb) and np.all(alpha == 0)


def test_projection_reduces_initial_residual_on_blob_images(olib):
    """On the 28x28 blob workload the projected guess has a smaller residual than x = 0."""
    cfg = CONFIGS["c1"]
    seed, tg = config_images(cfg, 0, 0, 1)
    H = cfg.groups[0].H
    ms, mt = initial_state(seed[0]), initial_state(tg[0, 0])
    As = oracle.Operator(H, 1.0 / cfg.T, cfg.g, ms)
    At = oracle.Operator(H, 1.0 / cfg.T, cfg.g, mt)
    sr = oracle.gmres(As, oracle.rhs(As, ms), m=cfg.m, keep_basis=True)
    bt = oracle.rhs(At, mt)
    for mode in (oracle.TARGET_GALERKIN, oracle.SEED_GALERKIN, oracle.SEED_LSQ):
        x0, _, st = oracle.project(At, bt, sr.V, sr.Hbar, mode=mode)
        assert st == oracle.OK
        assert oracle.residual(At, bt, x0) < 0.5
