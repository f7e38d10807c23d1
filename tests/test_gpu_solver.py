"""GPU parity of the solver path against the FP64 oracle: seed build (restarted GMRES with the
kept first-cycle basis), target projection in every mode, polish, plain GMRES, the timestep chain
and the edge cases.  Every call goes through the C ABI."""
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


def varah_ok(A, b, x, xs):
    """||x - x*||_inf <= dt ||b - A x||_inf (+ rounding): the bound for |m~| <= 1 grids."""
    rinf = np.abs(b - oracle.apply(A, x)).max()
    return np.abs(x - xs).max() <= A.dt * rinf * (1 + 1e-6) + 1e-13 * np.abs(xs).max()


def seed_on_gpu(X, H, T, m, ms, x0=None, tol=1e-8):
    import torch
    n = H * H
    ctx = X.Context(n, m, 4)
    b = torch.zeros(n, dtype=torch.float64, device=dev())
    x = torch.zeros(n, dtype=torch.float64, device=dev())
    spec = X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=b, x=x, x0=None if x0 is None else t64(x0))
    d = X.pack_systems([spec], dev())
    ctx.build_rhs(d, 1)
    bases = X.Bases(1, n, m)
    info = ctx.new_infos(1)
    ctx.seed_build(d, 1, bases.ptrs, X.Context.params(m, tol=tol), info)
    torch.cuda.synchronize()
    return ctx, bases, cpu(x), cpu(b), X.infos_to_numpy(info)[0]


@pytest.mark.parametrize("H,m", [(28, 30), (37, 20), (64, 40), (100, 50), (128, 60)])
def test_seed_build_matches_oracle(X, H, m):
    T = 100 if H != 28 else 50
    ms, _ = blob_pair(H, seed=H)
    ctx, bases, x, b, info = seed_on_gpu(X, H, T, m, ms)
    A = oracle.Operator(H, 1.0 / T, 0.5, ms)
    bo = oracle.rhs(A, ms)
    assert np.allclose(b, bo, rtol=1e-15, atol=0)
    ro = oracle.gmres(A, bo, m=m, tol=1e-8, keep_basis=True)
    xs, _ = oracle.banded_solve(A, bo)
    assert info["status"] == X.OK
    assert info["res_true"] <= 1e-8 and oracle.residual(A, bo, x) <= 1e-8
    assert abs(info["res_true"] - oracle.residual(A, bo, x)) <= 1e-12
    assert varah_ok(A, bo, x, xs)
    assert abs(int(info["iters"]) - ro.iters) <= max(2, 0.05 * ro.iters)
    hdr = bases.header(0)
    assert hdr["n"] == H * H and hdr["m"] == m and hdr["k"] == ro.basis_dim == info["basis_dim"]
    k = hdr["k"]
    V = cpu(bases.V(0))
    Hb = cpu(bases.Hbar(0))
    for c in range(min(6, k + 1)):
        assert np.abs(V[:, c] - ro.V[:, c]).max() <= 1e-10
    assert np.abs(Hb[:6, :5] - ro.Hbar[:6, :5]).max() <= 1e-10 * np.abs(ro.Hbar).max()
    # the GPU basis is orthonormal and satisfies the Arnoldi relation on its own
    assert np.abs(V[:, :k + 1].T @ V[:, :k + 1] - np.eye(k + 1)).max() <= 1e-12
    AV = np.stack([oracle.apply(A, V[:, c]) for c in range(k)], axis=1)
    assert np.abs(AV - V[:, :k + 1] @ Hb[:k + 1, :k]).max() <= 1e-12 * row_norm(A)
    assert np.all(Hb[k + 1:, :] == 0) and np.all(Hb[:, k:] == 0)


def row_norm(A):
    return sum(np.abs(c) for c in oracle.coeffs(A)).max()


def target_setup(X, H, T, m, warm, jitter=1.0):
    import torch
    ms, mt = blob_pair(H, seed=3 * H + 1, jitter=jitter)
    ctx, bases, xs_gpu, bs, info_s = seed_on_gpu(X, H, T, m, ms)
    n = H * H
    bt = torch.zeros(n, dtype=torch.float64, device=dev())
    xt = torch.zeros(n, dtype=torch.float64, device=dev())
    tm = t64(mt)
    spec = X.SystemSpec(H, 1.0 / T, 0.5, tm, b=bt, x=xt, x0=tm if warm else None)
    d = X.pack_systems([spec], dev())
    ctx.build_rhs(d, 1)
    return ctx, bases, d, xt, ms, mt


@pytest.mark.parametrize("mode", ["target_galerkin", "seed_galerkin", "seed_lsq"])
@pytest.mark.parametrize("warm", [False, True])
@pytest.mark.parametrize("H,m", [(28, 30), (64, 40), (128, 60)])
def test_projection_guess_matches_oracle(X, mode, warm, H, m):
    """A huge tolerance stops the polish before its first step, so x is the projected guess x0
    (tol = 1 would not: a warm guess can have relative residual above 1)."""
    import torch
    T = 100
    ctx, bases, d, xt, ms, mt = target_setup(X, H, T, m, warm)
    info = ctx.new_infos(1)
    ctx.target_project_solve(d, 1, 1, bases.ptrs, X.Context.params(m, tol=1e300, mode=mode), info)
    torch.cuda.synchronize()
    inf = X.infos_to_numpy(info)[0]
    As = oracle.Operator(H, 1.0 / T, 0.5, ms)
    At = oracle.Operator(H, 1.0 / T, 0.5, mt)
    sr = oracle.gmres(As, oracle.rhs(As, ms), m=m, tol=1e-8, keep_basis=True)
    bt = oracle.rhs(At, mt)
    # the oracle projection on the GPU's own basis isolates the projection step
    k = bases.header(0)["k"]
    Vg = cpu(bases.V(0))[:, :k + 1]
    Hg = cpu(bases.Hbar(0))[:k + 1, :k]
    mid = {"target_galerkin": oracle.TARGET_GALERKIN, "seed_galerkin": oracle.SEED_GALERKIN,
           "seed_lsq": oracle.SEED_LSQ}[mode]
    x0o, _, st = oracle.project(At, bt, Vg, Hg, mode=mid, x_base=mt if warm else None)
    assert st == oracle.OK and inf["status"] == X.OK and inf["basis_dim"] == k
    x0 = cpu(xt)
    assert np.abs(x0 - x0o).max() <= 1e-9 * np.abs(x0o).max()
    assert inf["iters"] == 0
    assert abs(inf["guess_res"] - oracle.residual(At, bt, x0o)) <= 1e-9 * inf["guess_res"]
    # and against the oracle's own seed basis, end to end
    x0e, _, _ = oracle.project(At, bt, sr.V, sr.Hbar, mode=mid, x_base=mt if warm else None)
    assert np.abs(x0 - x0e).max() <= 1e-7 * np.abs(x0e).max()


@pytest.mark.parametrize("mode", ["target_galerkin", "seed_galerkin", "seed_lsq", "none"])
def test_project_and_polish_converges(X, mode):
    import torch
    H, T, m = 64, 100, 40
    ctx, bases, d, xt, ms, mt = target_setup(X, H, T, m, warm=False, jitter=2.0)
    info = ctx.new_infos(1)
    ctx.target_project_solve(d, 1, 1, bases.ptrs, X.Context.params(m, tol=1e-8, mode=mode), info)
    torch.cuda.synchronize()
    inf = X.infos_to_numpy(info)[0]
    At = oracle.Operator(H, 1.0 / T, 0.5, mt)
    bt = oracle.rhs(At, mt)
    x = cpu(xt)
    xs, _ = oracle.banded_solve(At, bt)
    assert inf["status"] == X.OK and inf["res_true"] <= 1e-8
    assert oracle.residual(At, bt, x) <= 1e-8
    assert varah_ok(At, bt, x, xs)
    if mode == "none":
        ro = oracle.gmres(At, bt, m=m, tol=1e-8)
        assert abs(int(inf["iters"]) - ro.iters) <= max(2, 0.05 * ro.iters)


def test_batched_targets_match_oracle(X):
    """Eight targets of one seed in one call; each compared with the oracle's projection+polish."""
    import torch
    H, T, m, N = 28, 50, 30, 8
    rng = np.random.default_rng(5)
    ms, _ = blob_pair(H, seed=77)
    tg = [np.clip(blob_pair(H, seed=77, jitter=1.0 + 0.2 * i)[1], 0, 1) for i in range(N)]
    ctx, bases, _, _, _ = seed_on_gpu(X, H, T, m, ms)
    n = H * H
    tmt = t64(np.stack(tg))
    bt = torch.zeros((N, n), dtype=torch.float64, device=dev())
    xt = torch.zeros((N, n), dtype=torch.float64, device=dev())
    d = X.pack_batch(H, 1.0 / T, 0.5, tmt, bt, xt, basis_id=0)
    ctx2 = X.Context(n, m, N)
    ctx2.build_rhs(d, N)
    info = ctx2.new_infos(N)
    ctx2.target_project_solve(d, N, 1, bases.ptrs, X.Context.params(m), info)
    torch.cuda.synchronize()
    infs = X.infos_to_numpy(info)
    As = oracle.Operator(H, 1.0 / T, 0.5, ms)
    sr = oracle.gmres(As, oracle.rhs(As, ms), m=m, keep_basis=True)
    for i in range(N):
        At = oracle.Operator(H, 1.0 / T, 0.5, tg[i])
        b = oracle.rhs(At, tg[i])
        x0, _, _ = oracle.project(At, b, sr.V, sr.Hbar)
        ro = oracle.gmres(At, b, x0=x0, m=m)
        xs, _ = oracle.banded_solve(At, b)
        x = cpu(xt[i])
        assert infs[i]["status"] == X.OK and infs[i]["res_true"] <= 1e-8
        assert varah_ok(At, b, x, xs)
        assert abs(int(infs[i]["iters"]) - ro.iters) <= max(2, 0.05 * ro.iters)


def test_chain_grid28_full_matches_oracle(X):
    """The whole 28x28 workload (1 seed + 1 target, T = 50, m = 30) on the GPU vs the oracle."""
    import torch
    from paper_2511_17634_amd.driver import Chain
    from oracle.chain import run_chain
    from synth import CONFIGS, config_images, initial_state
    cfg = CONFIGS["c1"]
    H = cfg.groups[0].H
    seed, tg = config_images(cfg, 0, 0, 1)
    s0, t0 = initial_state(seed[0]), initial_state(tg[0, 0])[None]
    ch = Chain(H, cfg.T, cfg.m, s0, t0)
    its = []
    for _ in range(cfg.T):
        ch.step()
        _, it = ch.infos()
        its.append(int(it[0]["iters"]))
        assert it[0]["status"] == X.OK and it[0]["res_true"] <= cfg.tol
    torch.cuda.synchronize()
    ms_o, mt_o, st = run_chain(s0, t0, H, cfg.T, cfg.m)
    bound = cfg.T * cfg.tol * max(np.linalg.norm(s0), np.linalg.norm(t0))
    assert np.abs(cpu(ch.target_state)[0] - mt_o[0]).max() <= bound
    assert np.abs(cpu(ch.seed_state) - ms_o).max() <= bound
    it_o = np.array(st.iters)[:, 0]
    assert np.abs(np.array(its) - it_o).max() <= 2


@pytest.mark.parametrize("split", [-1, 0])
def test_zero_rhs_and_exact_start(X, split):
    """split >= 0: the target is projected in launches of its own."""
    import torch
    H, m = 16, 10
    ctx, bases, x, b, info = seed_on_gpu(X, H, 100, m, np.zeros(H * H))
    if split >= 0:
        ctx.set_projection_split(split)
    assert info["status"] == X.OK and info["iters"] == 0 and np.all(x == 0)
    assert bases.header(0)["k"] == 0
    # a target projected on an empty basis keeps x_base and still converges
    ms, mt = blob_pair(H, seed=1)
    tm = t64(mt)
    bt = torch.zeros(H * H, dtype=torch.float64, device=dev())
    xt = torch.zeros(H * H, dtype=torch.float64, device=dev())
    d = X.pack_systems([X.SystemSpec(H, 0.01, 0.5, tm, b=bt, x=xt)], dev())
    ctx.build_rhs(d, 1)
    inf = ctx.new_infos(1)
    ctx.target_project_solve(d, 1, 1, bases.ptrs, X.Context.params(m), inf)
    torch.cuda.synchronize()
    i = X.infos_to_numpy(inf)[0]
    assert i["status"] == X.OK and i["basis_dim"] == 0 and i["res_true"] <= 1e-8
    # a seed started from its exact solution: zero iterations, empty basis
    A = oracle.Operator(H, 0.01, 0.5, ms)
    xs, _ = oracle.banded_solve(A, oracle.rhs(A, ms))
    _, bases2, x2, _, info2 = seed_on_gpu(X, H, 100, m, ms, x0=xs, tol=1e-8)
    assert info2["iters"] == 0 and bases2.header(0)["k"] == 0


def test_noconvergence_and_bad_descriptors(X):
    import torch
    H, m = 32, 5
    ms, mt = blob_pair(H, seed=2)
    ctx = X.Context(H * H, m, 4)
    tm = t64(mt)
    bt = torch.zeros(H * H, dtype=torch.float64, device=dev())
    xt = torch.zeros(H * H, dtype=torch.float64, device=dev())
    big = torch.zeros(64 * 64, dtype=torch.float64, device=dev())
    specs = [X.SystemSpec(H, 0.01, 0.5, tm, b=bt, x=xt),
             X.SystemSpec(64, 0.01, 0.5, big, b=big, x=big)]        # n above the context limit
    d = X.pack_systems(specs, dev())
    ctx.build_rhs(d, 1)
    inf = ctx.new_infos(2)
    ctx.target_project_solve(d, 2, 0, None, X.Context.params(m, tol=1e-15, max_restarts=1,
                                                             mode="none"), inf)
    torch.cuda.synchronize()
    i = X.infos_to_numpy(inf)
    assert i[0]["status"] == X.ENOCONV and i[0]["restarts"] == 1 and i[0]["iters"] == 2 * m
    assert 0 < i[0]["res_true"] < 1
    A = oracle.Operator(H, 0.01, 0.5, mt)
    assert abs(oracle.residual(A, oracle.rhs(A, mt), cpu(xt)) - i[0]["res_true"]) <= 1e-12
    assert i[1]["status"] == X.EINVAL
    # host-side argument errors come back synchronously
    with pytest.raises(X.XkpError):
        ctx.target_project_solve(d, 2, 0, None, X.Context.params(m + 10, mode="none"), inf)
    with pytest.raises(X.XkpError):
        ctx.target_project_solve(d, 2, 0, None, X.Context.params(m, mode="target_galerkin"), inf)


@pytest.mark.parametrize("H,m,tol", [(64, 40, 1e-300), (3, 20, 1e-300), (28, 30, 1e-8),
                                     (80, 30, 1e-300)])
def test_kept_cycle_basis(X, H, m, tol):
    """The kept first cycle (delayed re-orthogonalisation with one reduction per step up to 4096
    unknowns, two modified Gram-Schmidt passes above) against the oracle's two-pass MGS: the
    whole cycle (tolerance unreachable), a 3x3 grid whose Krylov space is exhausted (breakdown
    at k <= 9), and a cycle that converges.  Same Hessenberg matrix and basis to rounding,
    orthonormal, Arnoldi relation, zeros past column k."""
    import torch
    T = 100
    n = H * H
    ms, _ = blob_pair(H, seed=5 * H + 2) if H > 3 else (np.linspace(0.1, 0.9, n), None)
    ctx = X.Context(n, m, 1)
    b = torch.zeros(n, dtype=torch.float64, device=dev())
    x = torch.zeros(n, dtype=torch.float64, device=dev())
    d = X.pack_systems([X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=b, x=x)], dev())
    ctx.build_rhs(d, 1)
    bases = X.Bases(1, n, m)
    info = ctx.new_infos(1)
    ctx.seed_build(d, 1, bases.ptrs, X.Context.params(m, tol=tol, max_restarts=0), info)
    torch.cuda.synchronize()
    i = X.infos_to_numpy(info)[0]
    A = oracle.Operator(H, 1.0 / T, 0.5, ms)
    bo = oracle.rhs(A, ms)
    ro = oracle.gmres(A, bo, m=m, max_restarts=0, tol=tol, keep_basis=True)
    k = int(bases.header(0)["k"])
    assert k == ro.basis_dim == int(i["basis_dim"]) == int(i["iters"])
    if H == 3:
        assert k <= n < m
    elif tol < 1e-100:
        assert k == m and i["status"] == X.ENOCONV
    else:
        assert k < m and i["status"] == X.OK
    V = cpu(bases.V(0))
    Hb = cpu(bases.Hbar(0))
    scale = np.abs(ro.Hbar).max()
    assert np.abs(Hb[:k + 1, :k] - ro.Hbar[:k + 1, :k]).max() <= 1e-9 * scale
    for c in range(min(8, k + 1)):
        assert np.abs(V[:, c] - ro.V[:, c]).max() <= 1e-10
    if H != 3:   # past a breakdown the last column is zero on both sides
        assert np.abs(V[:, :k + 1].T @ V[:, :k + 1] - np.eye(k + 1)).max() <= 1e-12
    AV = np.stack([oracle.apply(A, V[:, c]) for c in range(k)], axis=1)
    assert np.abs(AV - V[:, :k + 1] @ Hb[:k + 1, :k]).max() <= 1e-12 * row_norm(A)
    assert np.all(Hb[k + 1:, :] == 0) and np.all(Hb[:, k:] == 0)
    assert abs(i["res_true"] - ro.res_true) <= 1e-12


def test_kept_cycle_paths_agree(X):
    """The same 64x64 seed in a launch for systems of at most 4096 unknowns (the kept cycle by
    delayed re-orthogonalisation) and in one sized for 128x128 (two modified Gram-Schmidt
    passes): same basis dimension and steps, basis, Hessenberg matrix and solution equal to
    rounding."""
    import torch
    H, T, m = 64, 100, 40
    n = H * H
    ms, _ = blob_pair(H, seed=11)
    ctx = X.Context(128 * 128, m, 1)
    out = []
    for batch_max_n in (n, 0):
        b = torch.zeros(n, dtype=torch.float64, device=dev())
        x = torch.zeros(n, dtype=torch.float64, device=dev())
        d = X.pack_systems([X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=b, x=x)], dev())
        ctx.build_rhs(d, 1)
        bases = X.Bases(1, n, m)
        info = ctx.new_infos(1)
        ctx.seed_build(d, 1, bases.ptrs, X.Context.params(m, batch_max_n=batch_max_n), info)
        torch.cuda.synchronize()
        out.append((X.infos_to_numpy(info)[0], bases.header(0)["k"], cpu(bases.V(0)),
                    cpu(bases.Hbar(0)), cpu(x)))
    (i1, k1, V1, H1, x1), (i2, k2, V2, H2, x2) = out
    assert i1["status"] == i2["status"] == X.OK
    assert k1 == k2 and i1["iters"] == i2["iters"]
    assert np.abs(H1 - H2).max() <= 1e-9 * np.abs(H2).max()
    assert np.abs(V1[:, :8] - V2[:, :8]).max() <= 1e-10
    assert np.abs(x1 - x2).max() <= 1e-9 * np.abs(x2).max()


@pytest.mark.parametrize("reorth,passes", [("auto", 1), ("always", 2)])
def test_gram_schmidt_passes_match_oracle(X, reorth, passes):
    """One cycle of eight Arnoldi steps from x_base = 0 (tolerance unreachable, no restart): the
    iterate is GMRES's minimal-residual iterate, with one modified Gram-Schmidt pass (the
    default for a discarded basis) as with two."""
    import torch
    H, T, m = 48, 100, 8
    ms, mt = blob_pair(H, seed=9, jitter=1.5)
    ctx = X.Context(H * H, m, 1)
    tm = t64(mt)
    bt = torch.zeros(H * H, dtype=torch.float64, device=dev())
    xt = torch.zeros(H * H, dtype=torch.float64, device=dev())
    d = X.pack_systems([X.SystemSpec(H, 1.0 / T, 0.5, tm, b=bt, x=xt)], dev())
    ctx.build_rhs(d, 1)
    inf = ctx.new_infos(1)
    P = X.Context.params(m, tol=1e-300, max_restarts=0, mode="none", reorth=reorth)
    ctx.target_project_solve(d, 1, 0, None, P, inf)
    torch.cuda.synchronize()
    i = X.infos_to_numpy(inf)[0]
    assert i["status"] == X.ENOCONV and i["iters"] == m and i["restarts"] == 0
    A = oracle.Operator(H, 1.0 / T, 0.5, mt)
    b = oracle.rhs(A, mt)
    ro = oracle.gmres(A, b, m=m, max_iters=m, tol=0.0, passes=passes)
    x = cpu(xt)
    assert np.abs(x - ro.x).max() <= 1e-11 * np.abs(ro.x).max()
    assert abs(i["res_true"] - ro.res_true) <= 1e-12


@pytest.mark.parametrize("H,m", [(64, 40), (128, 60)])
def test_reorth_modes_agree(X, H, m):
    """Projected and plain targets with one and with two Gram-Schmidt passes: both converge to
    the tolerance within one iteration of each other and within two of the oracle's count."""
    import torch
    T = 100
    ctx, bases, d, xt, ms, mt = target_setup(X, H, T, m, warm=True)
    At = oracle.Operator(H, 1.0 / T, 0.5, mt)
    bt = oracle.rhs(At, mt)
    xs, _ = oracle.banded_solve(At, bt)
    for mode in ("target_galerkin", "none"):
        its = {}
        for reorth in ("auto", "always"):
            info = ctx.new_infos(1)
            ctx.target_project_solve(d, 1, 1, bases.ptrs,
                                     X.Context.params(m, mode=mode, reorth=reorth), info)
            torch.cuda.synchronize()
            inf = X.infos_to_numpy(info)[0]
            x = cpu(xt)
            assert inf["status"] == X.OK and inf["res_true"] <= 1e-8, (mode, reorth)
            assert oracle.residual(At, bt, x) <= 1e-8 and varah_ok(At, bt, x, xs)
            its[reorth] = int(inf["iters"])
        assert abs(its["auto"] - its["always"]) <= 1, (mode, its)
        if mode == "none":
            for passes in (1, 2):
                ro = oracle.gmres(At, bt, x0=mt, m=m, tol=1e-8, passes=passes)
                assert abs(its["auto"] - ro.iters) <= 2, (passes, its, ro.iters)
    with pytest.raises(X.XkpError):
        P = X.Context.params(m, mode="none")
        P.reorth = 2
        ctx.target_project_solve(d, 1, 1, bases.ptrs, P, ctx.new_infos(1))


def test_seed_later_cycles_use_the_polish_restart(X):
    """A seed whose first cycle does not converge: with polish_m set, its kept basis is bitwise
    the one of the default run (the kept cycle has m steps either way) and the later cycles,
    restarted every polish_m steps, still reach the tolerance."""
    import torch
    H, T, m = 48, 100, 12
    ms, _ = blob_pair(H, seed=21)
    out = {}
    for pm in (0, 6):
        n = H * H
        ctx = X.Context(n, m, 1)
        b = torch.zeros(n, dtype=torch.float64, device=dev())
        x = torch.zeros(n, dtype=torch.float64, device=dev())
        d = X.pack_systems([X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=b, x=x)], dev())
        ctx.build_rhs(d, 1)
        bases = X.Bases(1, n, m)
        info = ctx.new_infos(1)
        ctx.seed_build(d, 1, bases.ptrs, X.Context.params(m, polish_m=pm), info)
        torch.cuda.synchronize()
        out[pm] = (X.infos_to_numpy(info)[0], bases.V_padded(0).clone(), bases.Hbar(0).clone())
    i0, i6 = out[0][0], out[6][0]
    assert i0["status"] == i6["status"] == X.OK and i6["res_true"] <= 1e-8
    assert i0["restarts"] >= 1 and i6["restarts"] > i0["restarts"]
    assert i0["basis_dim"] == i6["basis_dim"] == m
    assert torch.equal(out[0][1], out[6][1]) and torch.equal(out[0][2], out[6][2])
