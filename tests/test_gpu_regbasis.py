"""GPU parity of the GMRES cycles that keep their Krylov basis in registers (discarded cycles of
grids up to 4096 unknowns whose restart length fits: two classical Gram-Schmidt passes, one
workgroup reduction each) against the FP64 oracle's GMRES with two modified passes: a single
cycle equals the minimal-residual iterate; restarted solves converge with the oracle's iteration
counts; projected targets in FP64 and mixed precision meet the tolerance.  Every call goes
through the C ABI."""
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


def _target(X, H, T, jitter=1.5, seed=9, waves=8, m=40):
    import torch
    ms, mt = blob_pair(H, seed=seed, jitter=jitter)
    ctx = X.Context(H * H, m, 1)
    ctx.set_launch(waves, 1)
    tm = t64(mt)
    bt = torch.zeros(H * H, dtype=torch.float64, device=dev())
    xt = torch.zeros(H * H, dtype=torch.float64, device=dev())
    d = X.pack_systems([X.SystemSpec(H, 1.0 / T, 0.5, tm, b=bt, x=xt)], dev())
    ctx.build_rhs(d, 1)
    return ctx, d, xt, ms, mt


@pytest.mark.parametrize("H,m,waves", [(48, 6, 8), (64, 6, 8), (32, 8, 8), (20, 8, 8),
                                       (64, 9, 4), (30, 15, 4)])
def test_register_cycle_is_the_minimal_residual_iterate(X, H, m, waves):
    """One cycle of m Arnoldi steps from 0 (tolerance unreachable, no restart): the iterate is
    GMRES's minimal-residual iterate over K_m, the oracle's with two Gram-Schmidt passes."""
    import torch
    T = 100
    ctx, d, xt, _, mt = _target(X, H, T, waves=waves)
    inf = ctx.new_infos(1)
    P = X.Context.params(m, tol=1e-300, max_restarts=0, mode="none")
    ctx.target_project_solve(d, 1, 0, None, P, inf)
    torch.cuda.synchronize()
    i = X.infos_to_numpy(inf)[0]
    assert i["status"] == X.ENOCONV and i["iters"] == m and i["restarts"] == 0
    A = oracle.Operator(H, 1.0 / T, 0.5, mt)
    b = oracle.rhs(A, mt)
    ro = oracle.gmres(A, b, m=m, max_iters=m, tol=0.0, passes=2)
    x = cpu(xt)
    assert np.abs(x - ro.x).max() <= 1e-11 * np.abs(ro.x).max()
    assert abs(i["res_true"] - ro.res_true) <= 1e-12
    assert abs(i["res_est"] - ro.res_est) <= 1e-10 * ro.res_est + 1e-14


@pytest.mark.parametrize("H,pm,waves", [(64, 6, 8), (64, 9, 4), (32, 8, 8)])
def test_register_restarts_match_oracle(X, H, pm, waves):
    """Plain GMRES(pm) to 1e-8 with restarts: converged (residual recomputed by the oracle),
    within the Varah bound of the direct solution, iteration count within max(2, 5 %) of the
    oracle's GMRES(pm)."""
    import torch
    T = 100
    ctx, d, xt, _, mt = _target(X, H, T, waves=waves)
    inf = ctx.new_infos(1)
    ctx.target_project_solve(d, 1, 0, None,
                             X.Context.params(40, polish_m=pm, mode="none"), inf)
    torch.cuda.synchronize()
    i = X.infos_to_numpy(inf)[0]
    A = oracle.Operator(H, 1.0 / T, 0.5, mt)
    b = oracle.rhs(A, mt)
    x = cpu(xt)
    assert i["status"] == X.OK and i["restarts"] >= 1
    assert oracle.residual(A, b, x) <= 1e-8 and abs(oracle.residual(A, b, x) - i["res_true"]) <= 1e-12
    xs, _ = oracle.banded_solve(A, b)
    rinf = np.abs(b - oracle.apply(A, x)).max()
    assert np.abs(x - xs).max() <= A.dt * rinf * (1 + 1e-6) + 1e-13 * np.abs(xs).max()
    ro = oracle.gmres(A, b, m=pm, tol=1e-8, passes=2)
    assert abs(int(i["iters"]) - ro.iters) <= max(2, 0.05 * ro.iters), (i["iters"], ro.iters)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_register_polish_of_projected_targets(X, precision):
    """Twelve 64x64 targets projected on a seed basis (m = 40) and polished by GMRES(6) with
    the basis in registers: every target meets the FP64 tolerance (oracle residual) within the
    Varah bound; in FP64 the guesses equal the memory path's and the iteration counts are
    within two of the oracle's GMRES(6) with two passes from the same guess."""
    import torch
    H, T, m, N, pm = 64, 100, 40, 12, 6
    prec = X.MIXED if precision == "mixed" else X.FP64
    n = H * H
    dt = 1.0 / T
    s0, _ = blob_pair(H, seed=31, jitter=2.0)
    tg = [blob_pair(H, seed=31, jitter=0.5 + 0.3 * i)[1] for i in range(N)]
    ctx = X.Context(n, m, N)
    ms = t64(s0)[None]
    bs = torch.zeros_like(ms)
    xs_ = torch.zeros_like(ms)
    sd = X.pack_batch(H, dt, 0.5, ms, bs, xs_)
    ctx.build_rhs(sd, 1)
    bases = X.Bases(1, n, m)
    si = ctx.new_infos(1)
    ctx.seed_build(sd, 1, bases.ptrs, X.Context.params(m, precision=prec), si)
    mt = t64(np.stack(tg))
    bt = torch.zeros_like(mt)
    res = {}
    for path, kw in (("reg", dict(polish_m=pm)), ("mem", dict(polish_m=pm, reorth="always"))):
        xt = torch.zeros_like(mt)
        d = X.pack_batch(H, dt, 0.5, mt, bt, xt)
        ctx.build_rhs(d, N)
        inf = ctx.new_infos(N)
        ctx.target_project_solve(d, N, 1, bases.ptrs, X.Context.params(m, precision=prec, **kw),
                                 inf)
        torch.cuda.synchronize()
        res[path] = (cpu(xt), X.infos_to_numpy(inf))
    x, i = res["reg"]
    assert np.all(i["status"] == X.OK)
    V = cpu(bases.V(0))
    k = bases.header(0)["k"]
    for t in range(N):
        A = oracle.Operator(H, dt, 0.5, tg[t])
        b = oracle.rhs(A, tg[t])
        r = oracle.residual(A, b, x[t])
        assert r <= 1e-8, (t, r)
        xs, _ = oracle.banded_solve(A, b)
        rinf = np.abs(b - oracle.apply(A, x[t])).max()
        assert np.abs(x[t] - xs).max() <= A.dt * rinf * (1 + 1e-6) + 1e-13 * np.abs(xs).max()
        if precision == "fp64":
            x0, _, _ = oracle.project(A, b, V[:, :k + 1], np.zeros((k + 1, k)))
            ro = oracle.gmres(A, b, x0=x0, m=pm, tol=1e-8, passes=2)
            assert abs(int(i["iters"][t]) - ro.iters) <= max(2, 0.05 * ro.iters), t
    # the guess is formed before the cycles: the same on both paths
    assert np.array_equal(i["guess_res"], res["mem"][1]["guess_res"])
    assert np.abs(i["iters"].astype(int) - res["mem"][1]["iters"].astype(int)).max() <= 2
