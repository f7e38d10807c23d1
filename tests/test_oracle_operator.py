"""Pins of the oracle's operator and right-hand side (Section 2.3) against facts that do not come
from the coefficient formulas themselves:

* The linearised log-density equation (eq. log_fp with <grad m, grad m> replaced by
  <grad m~, grad m>, backward Euler in time) is, for the unknown u,
      L[u] = u/dt + f.grad u - (g^2/2) lap u - (g^2/2) grad m~ . grad u = b.
  Central differences are exact on quadratics, so on interior rows (A u)_p must equal L[u] at the
  grid point for every quadratic u, any m~ and any f (grad m~ taken by the central difference of
  Section 2.3).  This fixes every coefficient, every sign and the east/west/north/south layout.
* With m~ = 0 and f = 0 the matrix is dt^-1 I plus a scaled 2-D Dirichlet Laplacian whose
  eigenpairs are products of sines: this fixes h, g, dt, the zero-padding boundary and the
  ordering p = i*H + j.
* Interior row sums equal 1/dt for any m~ and f.
* b = m^{n-1}/dt - div f is exact for linear f.
"""
import numpy as np
import pytest

import oracle


def grid(H):
    h = 1.0 / H
    i, j = np.meshgrid(np.arange(H), np.arange(H), indexing="ij")   # p = i*H + j
    return h, i * h, j * h


def central_grad(a, H, h):
    """Central differences of a grid function with zero outside (Section 2.3 stencils)."""
    A = np.pad(a.reshape(H, H), 1)
    gx = (A[2:, 1:-1] - A[:-2, 1:-1]) / (2 * h)
    gy = (A[1:-1, 2:] - A[1:-1, :-2]) / (2 * h)
    return gx, gy


@pytest.mark.parametrize("H", [5, 9, 16])
@pytest.mark.parametrize("seed", [0, 1])
def test_operator_matches_pde_on_quadratics(olib, H, seed):
    rng = np.random.default_rng(seed)
    T, g = 37, 0.7
    dt = 1.0 / T
    h, X, Y = grid(H)
    mt = rng.uniform(-1, 1, H * H)
    fx = rng.uniform(-2, 2, H * H)
    fy = rng.uniform(-2, 2, H * H)
    A = oracle.Operator(H, dt, g, mt, fx, fy)
    gmx, gmy = central_grad(mt, H, h)
    c = rng.normal(size=6)
    u = c[0] + c[1] * X + c[2] * Y + c[3] * X**2 + c[4] * X * Y + c[5] * Y**2
    ux = c[1] + 2 * c[3] * X + c[4] * Y
    uy = c[2] + c[4] * X + 2 * c[5] * Y
    lap = 2 * c[3] + 2 * c[5]
    L = (u / dt + fx.reshape(H, H) * ux + fy.reshape(H, H) * uy - 0.5 * g * g * lap
         - 0.5 * g * g * (gmx * ux + gmy * uy))
    Au = oracle.apply(A, u).reshape(H, H)
    inner = (slice(1, H - 1), slice(1, H - 1))
    scale = np.abs(u).max() / dt + 8 * g * g / h**2 * np.abs(u).max()
    assert np.abs(Au[inner] - L[inner]).max() <= 1e-12 * scale


@pytest.mark.parametrize("H", [4, 7, 12])
def test_eigenpairs_zero_mtilde(olib, H):
    T, g = 50, 0.5
    dt, h = 1.0 / T, 1.0 / H
    A = oracle.Operator(H, dt, g, np.zeros(H * H))
    i, j = np.meshgrid(np.arange(H), np.arange(H), indexing="ij")
    for k, l in [(1, 1), (1, 2), (2, 1), (H, H), (H // 2 + 1, 1)]:
        u = np.sin(k * np.pi * (i + 1) / (H + 1)) * np.sin(l * np.pi * (j + 1) / (H + 1))
        lam = 1 / dt + 2 * g * g / h**2 * (np.sin(k * np.pi / (2 * (H + 1)))**2
                                           + np.sin(l * np.pi / (2 * (H + 1)))**2)
        Au = oracle.apply(A, u.reshape(-1))
        assert np.abs(Au - lam * u.reshape(-1)).max() <= 1e-13 * lam


def test_dense_matches_apply_and_structure(olib):
    H = 6
    rng = np.random.default_rng(3)
    A = oracle.Operator(H, 0.01, 0.5, rng.uniform(0, 1, H * H))
    D = oracle.dense(A)
    u = rng.normal(size=H * H)
    assert np.allclose(D @ u, oracle.apply(A, u), rtol=0, atol=1e-12 * np.abs(D).max())
    # block tridiagonal: only offsets 0, +-1, +-H; +-1 never crosses a grid column
    p, q = np.nonzero(D)
    assert set(np.unique(q - p)) <= {0, 1, -1, H, -H}
    assert not np.any((q - p == 1) & (p % H == H - 1))
    assert not np.any((q - p == -1) & (p % H == 0))


@pytest.mark.parametrize("seed", [0, 5])
def test_interior_row_sums(olib, seed):
    H = 10
    rng = np.random.default_rng(seed)
    A = oracle.Operator(H, 0.02, 0.9, rng.uniform(-3, 3, H * H), rng.normal(size=H * H),
                        rng.normal(size=H * H))
    s = oracle.apply(A, np.ones(H * H)).reshape(H, H)
    assert np.abs(s[1:-1, 1:-1] - 50.0).max() <= 1e-11 * 50 * H * H


def test_rhs_linear_drift(olib):
    H, T = 9, 20
    h, X, Y = grid(H)
    a, b_, c, d = 0.3, -1.2, 2.0, 0.7
    fx = a * X + b_ * Y
    fy = c * X + d * Y
    rng = np.random.default_rng(2)
    mprev = rng.uniform(0, 1, H * H)
    A = oracle.Operator(H, 1.0 / T, 0.5, mprev, fx, fy)
    b = oracle.rhs(A, mprev).reshape(H, H)
    expect = mprev.reshape(H, H) * T - (a + d)
    assert np.abs(b[1:-1, 1:-1] - expect[1:-1, 1:-1]).max() <= 1e-12 * T
    # f = 0: b is m^{n-1}/dt everywhere
    A0 = oracle.Operator(H, 1.0 / T, 0.5, mprev)
    assert np.allclose(oracle.rhs(A0, mprev), mprev * T, rtol=1e-15, atol=0)


def test_diagonal_dominance_and_varah_bound(olib):
    """With |m~| <= 1 (images in [0, 1]) the matrix is strictly row diagonally dominant with
    margin 1/dt, hence ||A^-1||_inf <= dt (Varah)."""
    H, T = 8, 100
    rng = np.random.default_rng(4)
    A = oracle.Operator(H, 1.0 / T, 0.5, rng.uniform(0, 1, H * H))
    D = oracle.dense(A)
    off = np.abs(D).sum(axis=1) - np.abs(np.diag(D))
    assert np.all(np.diag(D) - off >= T - 1e-9)
    assert np.abs(np.linalg.inv(D)).sum(axis=1).max() <= 1.0 / T * (1 + 1e-12)
