"""Pins of the oracle's verification residual and of its image-cycle chain.

Residual (the "FP64-verified" check of every solve): ||b - A x||_2 / ||b||_2, and ||A x||_2 when
b = 0.  Pinned by the closed-form eigenpairs of the m~ = 0 operator (A u = lambda u for products
of sines, so b = lambda u + e and x = u leave exactly e), by the explicit matrix, by a planted
residual of known norm, and by its invariances.

Image-cycle chain (Experiment 2's protocol, a new seed every block of images with the Krylov
subspace expanded): a one-block cycle whose per-seed cap keeps every kept column is the plain
projected chain; two identical blocks gather, for the second block, the first seed's columns
followed by its next ones (the repeated copy is dependent), which is a one-block cycle with twice
the per-seed cap; two different blocks project the second block's targets on the basis gathered
from both seeds, in cycle order.
"""
import numpy as np
import pytest

import oracle
from oracle.chain import run_chain, run_cycle_chain
from synth import CONFIGS, cycle_blocks


def sine_mode(H, k, l):
    i, j = np.meshgrid(np.arange(H), np.arange(H), indexing="ij")   # p = i*H + j
    u = np.sin(k * np.pi * (i + 1) / (H + 1)) * np.sin(l * np.pi * (j + 1) / (H + 1))
    return u.reshape(-1)


def sine_eig(H, T, g, k, l):
    h2 = (1.0 / H) ** 2
    return T + (2 * g * g / h2) * (np.sin(k * np.pi / (2 * (H + 1))) ** 2
                                   + np.sin(l * np.pi / (2 * (H + 1))) ** 2)


@pytest.mark.parametrize("H", [4, 9, 16])
def test_residual_on_eigenpairs(olib, H):
    """m~ = 0: A u_kl = lambda_kl u_kl.  With b = lambda u_11 + c u_23 and x = u_11 the residual
    is exactly ||c u_23|| / ||b||; the modes are orthogonal, so ||b||^2 splits."""
    T, g, c = 50, 0.5, 3e-3
    A = oracle.Operator(H, 1.0 / T, g, np.zeros(H * H))
    u, e = sine_mode(H, 1, 1), sine_mode(H, 2, 3)
    lam = sine_eig(H, T, g, 1, 1)
    b = lam * u + c * e
    want = c * np.linalg.norm(e) / np.hypot(lam * np.linalg.norm(u), c * np.linalg.norm(e))
    assert abs(oracle.residual(A, b, u) - want) <= 1e-12 * want
    # b = 0: the norm of A x itself
    assert abs(oracle.residual(A, np.zeros(H * H), u) - lam * np.linalg.norm(u)) \
        <= 1e-13 * lam * np.linalg.norm(u)


@pytest.mark.parametrize("H,drift", [(3, False), (7, True), (12, False)])
def test_residual_matches_explicit_matrix(olib, H, drift):
    rng = np.random.default_rng(H)
    n = H * H
    mt = rng.uniform(0, 1, n)
    fx, fy = (rng.normal(size=n), rng.normal(size=n)) if drift else (None, None)
    A = oracle.Operator(H, 0.02, 0.5, mt, fx, fy)
    D = oracle.dense(A)
    b, x = rng.normal(size=n), rng.normal(size=n)
    want = np.linalg.norm(b - D @ x) / np.linalg.norm(b)
    assert abs(oracle.residual(A, b, x) - want) <= 1e-13 * want
    want0 = np.linalg.norm(D @ x)
    assert abs(oracle.residual(A, np.zeros(n), x) - want0) <= 1e-13 * want0
    assert oracle.residual(A, b, np.zeros(n)) == 1.0
    # a planted residual of known size: x = A^{-1} (b - r)
    r = 1e-7 * rng.normal(size=n)
    xr = np.linalg.solve(D, b - r)
    assert abs(oracle.residual(A, b, xr) - np.linalg.norm(r) / np.linalg.norm(b)) \
        <= 1e-6 * np.linalg.norm(r) / np.linalg.norm(b)
    # homogeneous of degree zero in (b, x); the transposed operator is not accepted as A
    assert abs(oracle.residual(A, 7.5 * b, 7.5 * x) - want) <= 1e-13 * want
    xt = np.linalg.solve(D.T, b)
    assert oracle.residual(A, b, xt) > 1e-6


def _blocks(count, cycle):
    """The first `count` images of the 64x64 cycle workload in blocks of `cycle`."""
    cfg = CONFIGS["c6"]
    return cfg, cycle_blocks(cfg, cycle, count)


def test_cycle_one_block_is_the_projected_chain(olib):
    """One block, per-seed cap >= m: the gathered basis is the seed's own kept basis, so guesses,
    iteration counts and states equal the projected chain's."""
    cfg, blocks = _blocks(4, 4)
    H, T, m, steps = cfg.groups[0].H, cfg.T, cfg.m, 3
    s0, t0 = blocks[0][0][0], blocks[0][1][:, 0]
    _, mt_c, st_c = run_cycle_chain([(s0, t0)], H, T, m, per_source=m, steps=steps)
    _, mt_p, st_p = run_chain(s0, t0, H, T, m, method="project", steps=steps)
    assert np.abs(np.array(st_c.guess_res) - np.array(st_p.guess_res)).max() <= 1e-10
    assert np.array_equal(np.array(st_c.iters), np.array(st_p.iters))
    bound = steps * cfg.tol * np.linalg.norm(t0, axis=1).max()
    assert np.abs(mt_c[0] - mt_p).max() <= bound


def test_cycle_identical_blocks_gather_the_next_columns(olib):
    """Two copies of one block: block 0 sees the seed's first a columns, block 1 the first 2a
    (the second copy's first a columns are dependent and dropped, its next a appended): the
    guesses of a one-block cycle with cap a and with cap 2a."""
    cfg, blocks = _blocks(3, 3)
    H, T, m, a, steps = cfg.groups[0].H, cfg.T, cfg.m, 6, 2
    s0, t0 = blocks[0][0][0], blocks[0][1][:, 0]
    N = len(t0)
    _, _, st2 = run_cycle_chain([(s0, t0), (s0, t0)], H, T, m, per_source=a, steps=steps)
    _, _, sa = run_cycle_chain([(s0, t0)], H, T, m, per_source=a, steps=steps)
    _, _, s2a = run_cycle_chain([(s0, t0)], H, T, m, per_source=2 * a, steps=steps)
    g = np.array(st2.guess_res)
    assert np.abs(g[:, :N] - np.array(sa.guess_res)).max() <= 1e-10
    assert np.abs(g[:, N:] - np.array(s2a.guess_res)).max() <= 1e-10
    # the larger basis changes the guess: the comparison above can tell the two apart
    assert np.abs(np.array(sa.guess_res) - np.array(s2a.guess_res)).max() > 1e-6


def test_cycle_second_block_projects_on_both_seeds(olib):
    """Two different blocks, one timestep: block 1's guesses are the target-Galerkin projections
    on accumulate([V_0, V_1]) (seed 0's columns first), not on either seed's basis alone."""
    cfg, blocks = _blocks(6, 3)
    H, T, m, a = cfg.groups[0].H, cfg.T, cfg.m, 6
    dt = 1.0 / T
    _, _, st = run_cycle_chain(blocks, H, T, m, per_source=a, steps=1)
    got = np.array(st.guess_res[0])
    Vs = []
    for s, _ in blocks:
        As = oracle.Operator(H, dt, cfg.g, s[0])
        r = oracle.gmres(As, oracle.rhs(As, s[0]), m=m, keep_basis=True)
        Vs.append(r.V[:, :r.basis_dim])

    def guesses(V, targets):
        k = V.shape[1]
        Vp = np.concatenate([V, np.zeros((V.shape[0], 1))], axis=1)
        out = []
        for t in targets:
            At = oracle.Operator(H, dt, cfg.g, t)
            bt = oracle.rhs(At, t)
            x0, _, _ = oracle.project(At, bt, Vp, np.zeros((k + 1, k)))
            out.append(oracle.residual(At, bt, x0))
        return np.array(out)
    t1 = blocks[1][1][:, 0]
    both = guesses(oracle.accumulate(Vs, a, m), t1)
    N0 = len(blocks[0][1])
    assert np.abs(got[N0:] - both).max() <= 1e-12
    assert np.abs(got[:N0] - guesses(oracle.accumulate(Vs[:1], a, m), blocks[0][1][:, 0])).max() \
        <= 1e-12
    for single in (Vs[0][:, :a], Vs[1][:, :a]):
        assert np.abs(guesses(single, t1) - both).max() > 1e-6


def test_cycle_pins_catch_a_wrong_source_set(olib, monkeypatch):
    """A cycle chain that gathers block g's basis from the seeds before it (leaving its own seed
    out) fails the hand computation above: the guesses of block 1 then equal seed 0's alone."""
    import oracle.chain as ch
    cfg, blocks = _blocks(6, 3)
    H, T, m, a = cfg.groups[0].H, cfg.T, cfg.m, 6
    _, _, good = run_cycle_chain(blocks, H, T, m, per_source=a, steps=1)
    real = ch.accumulate
    monkeypatch.setattr(ch, "accumulate", lambda srcs, ps, cap: real(srcs[:-1] or srcs, ps, cap))
    _, _, bad = run_cycle_chain(blocks, H, T, m, per_source=a, steps=1)
    N0 = len(blocks[0][1])
    assert np.abs(np.array(bad.guess_res[0][N0:]) - np.array(good.guess_res[0][N0:])).max() > 1e-6
