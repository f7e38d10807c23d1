"""The allocation-free target solve (xkp_target_project_solve_noalloc) against the context-based
xkp_target_project_solve on the same inputs, through the C ABI: two calls in a row, the second
on a smaller batch (smaller grid, other restart length and precision), so the fixed workspace
is reused with another layout.  The same kernels run in the same launch shape, so solutions and
per-system outcomes must agree bit for bit; every solution also meets the FP64 tolerance as
recomputed by the oracle."""
import numpy as np
import pytest

from gpu_util import blob_pair, cpu, dev, t64

pytestmark = pytest.mark.gpu


def _case(X, H, m, N, precision, seed0):
    """A seed basis and N targets on an H x H grid: (target descriptors, basis pointers,
    target arrays for the oracle check, solution tensor)."""
    import torch
    n, T, g = H * H, 100, 0.5
    dt = 1.0 / T
    s0, _ = blob_pair(H, seed=seed0, jitter=2.0)
    targets = [blob_pair(H, seed=seed0, jitter=0.5 + 0.25 * i)[1] for i in range(N)]
    ctx = X.Context(n, m, 1)
    ms, xs, bs = t64(s0)[None], torch.zeros((1, n), dtype=torch.float64, device=dev()), \
        torch.empty((1, n), dtype=torch.float64, device=dev())
    sd = X.pack_batch(H, dt, g, ms, bs, xs)
    ctx.build_rhs(sd, 1)
    bases = X.Bases(1, n, m)
    info = ctx.new_infos(1)
    ctx.seed_build(sd, 1, bases.ptrs, X.Context.params(m, precision=precision), info)
    mt = t64(np.stack(targets))
    bt = torch.empty_like(mt)
    td = X.pack_batch(H, dt, g, mt, bt, torch.zeros_like(mt))
    ctx.build_rhs(td, N)
    torch.cuda.synchronize()
    assert X.infos_to_numpy(info)[0]["status"] == X.OK
    return dict(H=H, n=n, dt=dt, g=g, m=m, N=N, mt=mt, bt=bt, bases=bases, ctx=ctx,
                precision=precision)


def _solve_both(X, c, params):
    """The same batch through both entry points: (x_ctx, infos_ctx, x_noalloc, infos_noalloc)."""
    import torch
    out = []
    for which in ("ctx", "noalloc"):
        x = torch.full_like(c["mt"], float("nan"))
        d = X.pack_batch(c["H"], c["dt"], c["g"], c["mt"], c["bt"], x)
        ctx = X.Context(c["n"], c["m"], c["N"])
        info = ctx.new_infos(c["N"])
        torch.cuda.synchronize()
        if which == "ctx":
            ctx.target_project_solve(d, c["N"], 1, c["bases"].ptrs, params, info)
        else:
            X.target_project_solve_noalloc(d, c["N"], 1, c["bases"].ptrs, params, info)
        torch.cuda.synchronize()
        out += [cpu(x), X.infos_to_numpy(info)]
    return out


def test_noalloc_matches_context_entry_point_twice():
    import oracle
    from paper_2511_17634_amd import xkp as X
    X.load()
    calls = [
        # 64x64, m = 40, FP64 target Galerkin, 12 targets
        (_case(X, 64, 40, 12, X.FP64, 21), dict(polish_m=10)),
        # then a smaller batch: 32x32, m = 16, mixed precision, 5 targets
        (_case(X, 32, 16, 5, X.MIXED, 22), dict(polish_m=8)),
    ]
    for c, kw in calls:
        P = X.Context.params(c["m"], precision=c["precision"], batch_max_n=c["n"], **kw)
        print(f"noalloc call: {c['N']} targets of {c['H']}x{c['H']}, m={c['m']}", flush=True)
        x_c, i_c, x_s, i_s = _solve_both(X, c, P)
        assert np.all(i_c["status"] == X.OK), i_c["status"]
        assert np.array_equal(x_c, x_s)
        for f in ("status", "iters", "restarts", "basis_dim", "res_true", "guess_res"):
            assert np.array_equal(i_c[f], i_s[f]), f
        mt, bt = cpu(c["mt"]), cpu(c["bt"])
        for t in range(c["N"]):
            A = oracle.Operator(c["H"], c["dt"], c["g"], mt[t])
            assert oracle.residual(A, bt[t], x_s[t]) <= 1e-8
