"""Pins of the oracle's direct and Krylov solvers against library routines, brute force and the
textbook invariants of restarted GMRES (Saad, Alg. 6.9 / 6.11)."""
import numpy as np
import pytest

import oracle


def rand_op(H, seed, T=100, g=0.5):
    rng = np.random.default_rng(seed)
    return oracle.Operator(H, 1.0 / T, g, rng.uniform(0, 1, H * H))


def test_dense_lu_matches_numpy(olib):
    rng = np.random.default_rng(0)
    for n in [1, 3, 17, 40]:
        D = rng.normal(size=(n, n)) + 0.1 * np.eye(n)
        b = rng.normal(size=n)
        x, st = oracle.lu_solve(D, b)
        assert st == oracle.OK
        assert np.allclose(x, np.linalg.solve(D, b), rtol=1e-10, atol=1e-10)


def test_dense_lu_flags_singular(olib):
    D = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [0.0, 1.0, 1.0]])
    _, st = oracle.lu_solve(D, np.ones(3))
    assert st == oracle.ESINGULAR


@pytest.mark.parametrize("H", [3, 6, 12])
def test_banded_matches_dense_solve(olib, H):
    A = rand_op(H, H)
    rng = np.random.default_rng(H)
    b = rng.normal(size=H * H)
    x, st = oracle.banded_solve(A, b)
    assert st == oracle.OK
    xd = np.linalg.solve(oracle.dense(A), b)
    assert np.abs(x - xd).max() <= 1e-12 * np.abs(xd).max()


def test_banded_residual_large(olib):
    A = rand_op(64, 1)
    b = oracle.rhs(A, A.mt)
    x, st = oracle.banded_solve(A, b)
    assert st == oracle.OK and oracle.residual(A, b, x) <= 1e-13


def brute_force_gmres(D, b, x0, j):
    """argmin over x0 + K_j(D, r0) of ||b - D x||_2 from the explicit Krylov matrix."""
    r0 = b - D @ x0
    K = np.empty((D.shape[0], j))
    v = r0.copy()
    for c in range(j):
        K[:, c] = v
        v = D @ v
    Q, _ = np.linalg.qr(K)           # same span, better conditioned
    c, *_ = np.linalg.lstsq(D @ Q, r0, rcond=None)
    return x0 + Q @ c


@pytest.mark.parametrize("passes", [1, 2])
@pytest.mark.parametrize("j", [1, 3, 8])
def test_gmres_minimal_residual_property(olib, j, passes):
    rng = np.random.default_rng(10 + j)
    n = 40
    D = 3 * np.eye(n) + rng.normal(size=(n, n)) / np.sqrt(n)     # nonsymmetric
    b = rng.normal(size=n)
    x0 = rng.normal(size=n)
    r = oracle.gmres_dense(D, b, x0=x0, m=j, max_iters=j, tol=0.0, passes=passes)
    assert r.iters == j
    xb = brute_force_gmres(D, b, x0, j)
    assert np.linalg.norm(r.x - xb) <= 1e-10 * np.linalg.norm(xb)


@pytest.mark.parametrize("passes", [1, 2])
def test_gmres_stencil_minimal_residual(olib, passes):
    A = rand_op(6, 7)
    D = oracle.dense(A)
    b = oracle.rhs(A, A.mt)
    for j in [2, 5]:
        r = oracle.gmres(A, b, m=j, max_iters=j, tol=0.0, passes=passes)
        xb = brute_force_gmres(D, b, np.zeros_like(b), j)
        assert np.linalg.norm(r.x - xb) <= 1e-10 * np.linalg.norm(xb)


def test_one_pass_basis_loses_orthogonality_that_the_second_pass_restores(olib):
    """With one modified Gram-Schmidt pass the Arnoldi basis loses orthogonality as the residual
    falls (in inverse proportion to it), here completely; the second pass keeps V^T V = I to the
    unit roundoff (the reason a kept basis gets two passes).  The GMRES residual still reaches
    the roundoff level with one pass: GMRES with modified Gram-Schmidt is backward stable."""
    rng = np.random.default_rng(5)
    n, j = 60, 30
    D = np.eye(n) + 0.3 * rng.normal(size=(n, n)) / np.sqrt(n)   # clustered spectrum
    b = rng.normal(size=n)
    r1 = oracle.gmres_dense(D, b, m=j, max_iters=j, tol=0.0, keep_basis=True, passes=1)
    r2 = oracle.gmres_dense(D, b, m=j, max_iters=j, tol=0.0, keep_basis=True, passes=2)
    o1 = np.abs(r1.V.T @ r1.V - np.eye(j + 1)).max()
    o2 = np.abs(r2.V.T @ r2.V - np.eye(j + 1)).max()
    assert o2 <= 1e-14 and o1 >= 1e-2, (o1, o2)
    for r in (r1, r2):
        assert np.abs(D @ r.V[:, :j] - r.V @ r.Hbar).max() <= 1e-13 * np.abs(D).max()
        assert np.linalg.norm(b - D @ r.x) <= 1e-14 * np.linalg.norm(b)
    # early in the cycle (residual 1e-5) one pass is still orthogonal to about u / residual
    r1 = oracle.gmres_dense(D, b, m=10, max_iters=10, tol=0.0, keep_basis=True, passes=1)
    assert np.abs(r1.V.T @ r1.V - np.eye(11)).max() <= 1e-9


def test_one_pass_gmres_matches_two_on_the_stencil(olib):
    """On the Fokker-Planck operator both variants take the same number of steps to 1e-8."""
    for H, m, seed in [(16, 20, 1), (24, 30, 2), (32, 40, 3)]:
        A = rand_op(H, seed, T=100)
        b = oracle.rhs(A, A.mt)
        r1 = oracle.gmres(A, b, m=m, tol=1e-8, passes=1)
        r2 = oracle.gmres(A, b, m=m, tol=1e-8, passes=2)
        assert r1.status == r2.status == oracle.OK
        assert r1.iters == r2.iters and r1.res_true <= 1e-8 and r2.res_true <= 1e-8


@pytest.mark.parametrize("H,m", [(8, 10), (16, 30)])
def test_arnoldi_relation_and_orthonormality(olib, H, m):
    A = rand_op(H, 2 * H)
    b = oracle.rhs(A, A.mt)
    r = oracle.gmres(A, b, m=m, tol=1e-30, keep_basis=True, max_restarts=0)
    k = r.basis_dim
    assert k == m
    V, Hb = r.V, r.Hbar
    assert np.abs(V.T @ V - np.eye(k + 1)).max() <= 1e-12
    AV = np.stack([oracle.apply(A, V[:, c]) for c in range(k)], axis=1)
    normA = np.abs(oracle.dense(A)).sum(axis=1).max()
    assert np.abs(AV - V @ Hb).max() <= 1e-12 * normA
    # Hessenberg structure and V_k^T A V_k = H_k
    assert np.all(np.tril(Hb, -2) == 0)
    assert np.abs(V[:, :k].T @ AV - Hb[:k]).max() <= 1e-10 * normA


def test_residual_history_monotone_within_cycle(olib):
    A = rand_op(16, 3)
    b = oracle.rhs(A, A.mt)
    r = oracle.gmres(A, b, m=20, tol=1e-10, hist_cap=400)
    h = r.hist
    for c0 in range(0, len(h), 20):
        seg = h[c0:c0 + 20]
        assert np.all(np.diff(seg) <= 1e-14)
    assert r.status == oracle.OK and r.res_true <= 1e-10


@pytest.mark.parametrize("H,m", [(28, 30), (32, 40)])
def test_gmres_solution_within_varah_bound(olib, H, m):
    T = 100
    A = rand_op(H, H, T=T)
    b = oracle.rhs(A, A.mt)
    r = oracle.gmres(A, b, m=m, tol=1e-8)
    xs, _ = oracle.banded_solve(A, b)
    assert r.status == oracle.OK and r.res_true <= 1e-8
    rinf = np.abs(b - oracle.apply(A, r.x)).max()
    assert np.abs(r.x - xs).max() <= (1.0 / T) * rinf * (1 + 1e-6) + 1e-13 * np.abs(xs).max()


def test_gmres_zero_rhs_and_exact_start(olib):
    A = rand_op(8, 1)
    r = oracle.gmres(A, np.zeros(64), x0=np.ones(64), m=5)
    assert r.status == oracle.OK and r.iters == 0 and np.all(r.x == 0)
    b = oracle.rhs(A, A.mt)
    xs, _ = oracle.banded_solve(A, b)
    r = oracle.gmres(A, b, x0=xs, m=5)
    assert r.iters == 0 and r.status == oracle.OK


def test_gmres_noconvergence_keeps_best_iterate(olib):
    A = rand_op(16, 4)
    b = oracle.rhs(A, A.mt)
    r = oracle.gmres(A, b, m=5, tol=1e-14, max_restarts=1)
    assert r.status == oracle.ENOCONV and r.restarts == 1 and r.iters == 10
    assert 0 < r.res_true < 1.0
    assert abs(oracle.residual(A, b, r.x) - r.res_true) <= 1e-12


def test_gmres_lucky_breakdown(olib):
    """b in a 3-dimensional invariant subspace: GMRES ends in 3 steps with the exact answer."""
    n = 30
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    D = Q @ np.diag(np.r_[[2.0, 3.0, 5.0], rng.uniform(1, 4, n - 3)]) @ Q.T
    b = Q[:, :3] @ np.array([1.0, -2.0, 0.5])
    r = oracle.gmres_dense(D, b, m=10, tol=1e-13, keep_basis=True)
    assert r.iters == 3 and r.basis_dim == 3 and r.status == oracle.OK
    assert np.allclose(r.x, np.linalg.solve(D, b), atol=1e-12)
    assert np.all(r.V[:, 3] == 0)
