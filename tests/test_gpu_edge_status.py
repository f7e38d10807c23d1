"""Per-system outcomes forced from the host, through the C ABI: a projected system made singular
by a duplicated seed-basis column (XKP_ESINGULAR, the guess falls back to x_base and the polish
still converges, as the oracle's projection does), and data that are not finite (NaN or Inf in
m~, b or x0) rejected with XKP_EINVAL instead of a solve."""
import numpy as np
import pytest

import oracle
from gpu_util import blob_pair, cpu, dev, t64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def X():
    from paper_2511_17634_amd import xkp
    xkp.load()
    return xkp


def _seed_basis(X, H, T, m, precision):
    import torch
    n = H * H
    s0, t0 = blob_pair(H, seed=77, jitter=1.5)
    ctx = X.Context(n, m, 4)
    ms = t64(s0)[None]
    b = torch.zeros_like(ms)
    x = torch.zeros_like(ms)
    d = X.pack_batch(H, 1.0 / T, 0.5, ms, b, x)
    ctx.build_rhs(d, 1)
    bases = X.Bases(1, n, m)
    inf = ctx.new_infos(1)
    ctx.seed_build(d, 1, bases.ptrs, X.Context.params(m, precision=precision), inf)
    torch.cuda.synchronize()
    assert X.infos_to_numpy(inf)[0]["status"] == X.OK
    return ctx, bases, t0


@pytest.mark.parametrize("split", [-1, 0])
@pytest.mark.parametrize("precision,polish_m", [("fp64", 0), ("fp64", 6), ("mixed", 0)])
def test_duplicated_basis_column_is_singular(X, precision, polish_m, split):
    """split >= 0: the projection runs in launches of its own."""
    import torch
    H, T, m = 48, 100, 20
    prec = X.MIXED if precision == "mixed" else X.FP64
    ctx, bases, t0 = _seed_basis(X, H, T, m, prec)
    if split >= 0:
        ctx.set_projection_split(split)
    k = bases.header(0)["k"]
    assert k >= 2
    # column 1 := column 0 (the FP64 columns and the BF16 copy): V^T A' V has two equal rows
    Vp = bases.V_padded(0)
    Vp[:, 1] = Vp[:, 0]
    Vb = bases.Vb_bits(0)
    Vb[:, 1] = Vb[:, 0]
    torch.cuda.synchronize()
    dt = 1.0 / T
    A = oracle.Operator(H, dt, 0.5, t0)
    bo = oracle.rhs(A, t0)
    xs, _ = oracle.banded_solve(A, bo)
    for warm in (True, False):
        mt = t64(t0)[None]
        bt = torch.zeros_like(mt)
        xt = torch.zeros_like(mt)
        d = X.pack_batch(H, dt, 0.5, mt, bt, xt, x0=mt if warm else None)
        ctx.build_rhs(d, 1)
        inf = ctx.new_infos(1)
        ctx.target_project_solve(d, 1, 1, bases.ptrs,
                                 X.Context.params(m, precision=prec, polish_m=polish_m), inf)
        torch.cuda.synchronize()
        i = X.infos_to_numpy(inf)[0]
        x = cpu(xt)[0]
        assert i["status"] == X.ESINGULAR, i["status"]
        # the guess fell back to x_base (m^{n-1}, or zero)
        want = oracle.residual(A, bo, t0) if warm else 1.0
        assert abs(i["guess_res"] - want) <= 1e-12 * max(want, 1.0), (i["guess_res"], want)
        assert i["res_true"] <= 1e-8 and oracle.residual(A, bo, x) <= 1e-8
        rinf = np.abs(bo - oracle.apply(A, x)).max()
        assert np.abs(x - xs).max() <= dt * rinf * (1 + 1e-6) + 1e-13 * np.abs(xs).max()
    # the oracle's projection on the same basis is singular too and returns x_base
    Vo = cpu(bases.V(0))[:, :k + 1]
    x0, _, st = oracle.project(A, bo, Vo, np.zeros((k + 1, k)), x_base=t0)
    assert st == oracle.ESINGULAR and np.array_equal(x0, t0)


@pytest.mark.parametrize("where,split", [("mt_seed", -1), ("mt_target", -1), ("mt_plain", -1),
                                         ("b_plain", -1), ("x0_target", -1), ("mt_target", 0),
                                         ("x0_target", 0)])
def test_non_finite_data_is_rejected(X, where, split):
    """One NaN (or Inf in x0) in a system's data: the system's status is XKP_EINVAL (no
    iterations spent on it), while a finite system solved in the same launch converges (split
    >= 0: targets projected in launches of their own)."""
    import torch
    H, T, m = 32, 100, 16
    n = H * H
    dt = 1.0 / T
    ctx, bases, t0 = _seed_basis(X, H, T, m, X.FP64)
    if split >= 0:
        ctx.set_projection_split(split)
    bad = t64(t0).clone()
    good = t64(t0)
    mts = torch.stack([bad, good])
    bs = torch.zeros_like(mts)
    xs = torch.zeros_like(mts)
    x0 = None
    if where.startswith("mt"):
        mts[0, n // 2 + 3] = float("nan")
    d = X.pack_batch(H, dt, 0.5, mts, bs, xs)
    ctx.build_rhs(d, 2)
    if where == "b_plain":
        bs[0, 17] = float("nan")
    if where == "x0_target":
        x0 = mts.clone()
        x0[0, 5] = float("inf")
        d = X.pack_batch(H, dt, 0.5, mts, bs, xs, x0=x0)
    inf = ctx.new_infos(2)
    if where == "mt_seed":
        kb = X.Bases(2, n, m)
        ctx.seed_build(d, 2, kb.ptrs, X.Context.params(m), inf)
    else:
        mode = "none" if where.endswith("plain") else "target_galerkin"
        ctx.target_project_solve(d, 2, 1, bases.ptrs, X.Context.params(m, mode=mode), inf)
    torch.cuda.synchronize()
    i = X.infos_to_numpy(inf)
    assert i["status"][0] == X.EINVAL, (where, i["status"])
    assert i["iters"][0] == 0
    assert i["status"][1] == X.OK and i["res_true"][1] <= 1e-8
