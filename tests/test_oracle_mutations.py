"""The pins bite: each planted mistake in the oracle (operator sign, east/west exchange, grid
spacing, column wrap, transposed projection) makes at least one pin fail."""
import numpy as np
import pytest

import oracle
from test_oracle_chain import cole_hopf_error


def eig_error():
    H, T, g = 7, 50, 0.5
    dt, h = 1.0 / T, 1.0 / H
    A = oracle.Operator(H, dt, g, np.zeros(H * H))
    i, j = np.meshgrid(np.arange(H), np.arange(H), indexing="ij")
    u = (np.sin(np.pi * (i + 1) / (H + 1)) * np.sin(2 * np.pi * (j + 1) / (H + 1))).reshape(-1)
    lam = 1 / dt + 2 * g * g / h**2 * (np.sin(np.pi / (2 * (H + 1)))**2
                                       + np.sin(2 * np.pi / (2 * (H + 1)))**2)
    return np.abs(oracle.apply(A, u) - lam * u).max() / lam


def cole_hopf_ratio_ok():
    e = [cole_hopf_error(32, T) for T in (10, 20, 40)]
    return 1.8 <= e[0] / e[1] <= 2.2 and e[2] < 4e-3


def galerkin_error():
    H, T = 12, 100
    rng = np.random.default_rng(0)
    ms = rng.uniform(0, 1, H * H)
    mt = np.clip(ms + 0.1 * rng.normal(size=H * H), 0, 1)
    As, At = oracle.Operator(H, 1 / T, 0.5, ms), oracle.Operator(H, 1 / T, 0.5, mt)
    sr = oracle.gmres(As, oracle.rhs(As, ms), m=10, keep_basis=True)
    bt = oracle.rhs(At, mt)
    x0, alpha, _ = oracle.project(At, bt, sr.V, sr.Hbar, mode=oracle.TARGET_GALERKIN)
    V = sr.V[:, :sr.basis_dim]
    return np.abs(V.T @ (bt - oracle.apply(At, V @ alpha))).max() / np.linalg.norm(bt)


@pytest.mark.parametrize("code", [1, 2, 3, 4, 5])
def test_planted_mistake_is_caught(olib, code):
    try:
        oracle.set_mutation(code)
        caught = (eig_error() > 1e-12) or (not cole_hopf_ratio_ok()) or (galerkin_error() > 1e-11)
    finally:
        oracle.set_mutation(0)
    assert caught


def test_unmutated_oracle_passes_the_same_checks(olib):
    assert eig_error() <= 1e-12 and cole_hopf_ratio_ok() and galerkin_error() <= 1e-11
