"""GPU parity of the operator kernels against the FP64 oracle: stencil apply, right-hand side,
residual.  Run through the C ABI (libxkp.so)."""
import numpy as np
import pytest

import oracle
from gpu_util import cpu, dev, t64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    from paper_2511_17634_amd import xkp
    xkp.load()
    return xkp


def row_abs(A):
    return sum(np.abs(c) for c in oracle.coeffs(A))


@pytest.mark.parametrize("H", [3, 5, 28, 37, 64, 90, 128])
def test_apply_matches_oracle(X, H):
    import torch
    rng = np.random.default_rng(H)
    T, g = 100, 0.5
    mt = rng.uniform(0, 1, H * H)
    fx, fy = (rng.normal(size=H * H), rng.normal(size=H * H)) if H % 2 else (None, None)
    u = rng.normal(size=H * H)
    A = oracle.Operator(H, 1.0 / T, g, mt, fx, fy)
    yo = oracle.apply(A, u)
    ctx = X.Context(H * H, 8, 2)
    tm, tu, y = t64(mt), t64(u), torch.full((H * H,), np.nan, dtype=torch.float64, device=dev())
    spec = X.SystemSpec(H, 1.0 / T, g, tm, b=tm, x=y, x0=tu,
                        fx=None if fx is None else t64(fx), fy=None if fy is None else t64(fy))
    d = X.pack_systems([spec], dev())
    ctx.apply(d, 1)
    torch.cuda.synchronize()
    err = np.abs(cpu(y) - yo)
    assert np.all(np.isfinite(cpu(y)))
    assert np.all(err <= 1e-14 * row_abs(A) * np.abs(u).max())


def test_apply_uneven_batch(X):
    """One call over systems of different sizes, each checked against the oracle."""
    import torch
    Hs = [4, 16, 28, 33, 64]
    rng = np.random.default_rng(7)
    specs, refs, outs = [], [], []
    for H in Hs:
        mt, u = rng.uniform(0, 1, H * H), rng.normal(size=H * H)
        A = oracle.Operator(H, 0.02, 0.5, mt)
        refs.append((oracle.apply(A, u), row_abs(A) * np.abs(u).max()))
        y = torch.zeros(H * H, dtype=torch.float64, device=dev())
        outs.append(y)
        specs.append(X.SystemSpec(H, 0.02, 0.5, t64(mt), b=t64(mt), x=y, x0=t64(u)))
    ctx = X.Context(64 * 64, 8, 8)
    ctx.apply(X.pack_systems(specs, dev()), len(specs))
    torch.cuda.synchronize()
    for y, (ref, sc) in zip(outs, refs):
        assert np.all(np.abs(cpu(y) - ref) <= 1e-14 * sc)


@pytest.mark.parametrize("with_f", [False, True])
def test_rhs_matches_oracle(X, with_f):
    import torch
    H, T = 29, 50
    rng = np.random.default_rng(3)
    mt = rng.uniform(0, 1, H * H)
    fx, fy = (rng.normal(size=H * H), rng.normal(size=H * H)) if with_f else (None, None)
    A = oracle.Operator(H, 1.0 / T, 0.5, mt, fx, fy)
    bo = oracle.rhs(A, mt)
    b = torch.zeros(H * H, dtype=torch.float64, device=dev())
    spec = X.SystemSpec(H, 1.0 / T, 0.5, t64(mt), b=b, x=b,
                        fx=None if fx is None else t64(fx), fy=None if fy is None else t64(fy))
    ctx = X.Context(H * H, 8, 1)
    ctx.build_rhs(X.pack_systems([spec], dev()), 1)
    torch.cuda.synchronize()
    assert np.allclose(cpu(b), bo, rtol=1e-15, atol=1e-13)


def test_residual_matches_oracle(X):
    import torch
    rng = np.random.default_rng(11)
    specs, ref = [], []
    for H in (8, 28, 64):
        mt = rng.uniform(0, 1, H * H)
        A = oracle.Operator(H, 0.01, 0.5, mt)
        b = oracle.rhs(A, mt)
        xs, _ = oracle.banded_solve(A, b)
        x = xs + 1e-9 * rng.normal(size=H * H)          # nearly converged: cancellation case
        ref.append(oracle.residual(A, b, x))
        specs.append(X.SystemSpec(H, 0.01, 0.5, t64(mt), b=t64(b), x=t64(x)))
    zero = torch.zeros(16, dtype=torch.float64, device=dev())
    specs.append(X.SystemSpec(4, 0.01, 0.5, zero, b=zero, x=zero))   # b = 0, x = 0
    ref.append(0.0)
    out = torch.full((len(specs),), np.nan, dtype=torch.float64, device=dev())
    ctx = X.Context(64 * 64, 8, 4)
    ctx.residual(X.pack_systems(specs, dev()), len(specs), out)
    torch.cuda.synchronize()
    got = cpu(out)
    # relative residuals of nearly converged iterates: the rounding of b - A x (summation
    # order differs) is a few ulps of |b| + |A||x|, far below the 1e-8 tolerance being checked
    assert np.all(np.abs(got - np.array(ref)) <= 1e-14 + 1e-9 * np.array(ref))
