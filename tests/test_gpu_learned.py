"""GPU parity of the learned-guess solve path: subspace coordinates V^T x, the guess
x0_L = x_base + V (scale alpha), the residual gate, and the fallback to the projection path (which
must reproduce xkp_target_project_solve exactly); the learned correction of the projection (a
zero correction is the projection bit for bit, the exact correction gives V V^T x*, a
correction is kept only where it lowers the guess's residual); the smallest residual the seed
subspace allows; and the trained pipeline against the projection."""
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


def zeros(n):
    import torch
    return torch.zeros(n, dtype=torch.float64, device=dev())


def setup(X, H=64, T=100, m=40, N=3):
    import torch
    ms, _ = blob_pair(H, seed=321)
    n = H * H
    ctx = X.Context(n, m, max(N, 1))
    sd = X.pack_systems([X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=zeros(n), x=zeros(n))], dev())
    ctx.build_rhs(sd, 1)
    bases = X.Bases(1, n, m)
    inf = ctx.new_infos(1)
    ctx.seed_build(sd, 1, bases.ptrs, X.Context.params(m), inf)
    mts = [blob_pair(H, seed=321, jitter=1.0 + 0.5 * i)[1] for i in range(N)]
    specs = [X.SystemSpec(H, 1.0 / T, 0.5, t64(mt), b=zeros(n), x=zeros(n)) for mt in mts]
    d = X.pack_systems(specs, dev())
    ctx.build_rhs(d, N)
    torch.cuda.synchronize()
    return ctx, bases, d, specs, mts


def test_basis_coeffs_are_subspace_coordinates(X):
    import torch
    ctx, bases, d, specs, mts = setup(X)
    rng = np.random.default_rng(0)
    xs = [rng.standard_normal(64 * 64) for _ in specs]
    for s, x in zip(specs, xs):
        s.x.copy_(torch.from_numpy(x))
    out = torch.empty((len(specs), 48), dtype=torch.float64, device=dev())
    ctx.basis_coeffs(d, len(specs), 1, bases.ptrs, 48, out)
    torch.cuda.synchronize()
    k = bases.header(0)["k"]
    V = cpu(bases.V(0))[:, :k]
    a = cpu(out)
    for i, x in enumerate(xs):
        ref = V.T @ x
        assert np.abs(a[i, :k] - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.all(a[i, k:] == 0)
    # kind 1: residual coordinates Hbar (V^T x) / beta
    ctx.basis_coeffs(d, len(specs), 1, bases.ptrs, 48, out, kind=1)
    torch.cuda.synchronize()
    z = cpu(out)
    Hb = cpu(bases.Hbar(0))[:k + 1, :k]
    beta = float(bases.buf[16:24].cpu().numpy().view(np.float64)[0])
    assert np.isfinite(beta) and beta > 0
    for i, x in enumerate(xs):
        ref = Hb @ (V.T @ x) / beta
        assert np.abs(z[i, :k + 1] - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.all(z[i, k + 1:] == 0)


def test_learned_guess_gate_and_fallback(X):
    import torch
    H, T, m, N = 64, 100, 40, 3
    ctx, bases, d, specs, mts = setup(X, H, T, m, N)
    k = bases.header(0)["k"]
    V = cpu(bases.V(0))[:, :k]
    Hb = cpu(bases.Hbar(0))[:k + 1, :k]
    beta = float(bases.buf[16:24].cpu().numpy().view(np.float64)[0])
    assert np.isfinite(beta) and beta > 0
    # the best guesses inside span V, alpha* = V^T x*, given as residual coordinates
    # zeta = Hbar alpha* / beta (stored divided by 8, scaled back by 8)
    xstar = []
    for mt in mts:
        At = oracle.Operator(H, 1.0 / T, 0.5, mt)
        xstar.append(oracle.banded_solve(At, oracle.rhs(At, mt))[0])
    alpha = np.zeros((N, 48), dtype=np.float32)
    for i, xs in enumerate(xstar):
        alpha[i, :k + 1] = (Hb @ (V.T @ xs)) / beta / 8.0
    al = torch.tensor(alpha, device=dev())
    info = ctx.new_infos(N)
    # gate infinite, no polish: x = V a with a the least-squares solution for the given zeta
    ctx.learned_solve(d, N, 1, bases.ptrs, X.Context.params(m, tol=1e300), al, 48, 8.0, 1e300,
                      info)
    torch.cuda.synchronize()
    inf = X.infos_to_numpy(info)
    for i in range(N):
        zeta = beta * 8.0 * alpha[i, :k + 1].astype(np.float64)
        a_ls = np.linalg.lstsq(Hb, zeta, rcond=None)[0]
        assert np.linalg.norm(a_ls - V.T @ xstar[i]) <= 1e-5 * np.linalg.norm(V.T @ xstar[i])
        x0 = V @ a_ls
        At = oracle.Operator(H, 1.0 / T, 0.5, mts[i])
        bt = oracle.rhs(At, mts[i])
        assert np.abs(cpu(specs[i].x) - x0).max() <= 1e-12 * np.abs(x0).max()
        assert inf[i]["guess_source"] == 2 and inf[i]["iters"] == 0
        assert abs(inf[i]["guess_res"] - oracle.residual(At, bt, x0)) <= 1e-9 * inf[i]["guess_res"]
    # gate infinite, polished: converges from the learned guess
    ctx.learned_solve(d, N, 1, bases.ptrs, X.Context.params(m), al, 48, 8.0, 1e300, info)
    torch.cuda.synchronize()
    inf = X.infos_to_numpy(info)
    for i in range(N):
        At = oracle.Operator(H, 1.0 / T, 0.5, mts[i])
        bt = oracle.rhs(At, mts[i])
        assert inf[i]["status"] == X.OK and inf[i]["guess_source"] == 2
        assert oracle.residual(At, bt, cpu(specs[i].x)) <= 1e-8
    # gate 0: every target falls back, identical to the projection path
    for mode, src in (("target_galerkin", 1), ("seed_galerkin", 1), ("none", 0)):
        P = X.Context.params(m, mode=mode)
        ctx.learned_solve(d, N, 1, bases.ptrs, P, al, 48, 8.0, 0.0, info)
        torch.cuda.synchronize()
        xl = [cpu(s.x).copy() for s in specs]
        il = X.infos_to_numpy(info).copy()
        info2 = ctx.new_infos(N)
        ctx.target_project_solve(d, N, 1, bases.ptrs, P, info2)
        torch.cuda.synchronize()
        i2 = X.infos_to_numpy(info2)
        for i in range(N):
            assert np.array_equal(xl[i], cpu(specs[i].x)), mode
            assert il[i]["iters"] == i2[i]["iters"] and il[i]["guess_source"] == src, mode
            assert i2[i]["guess_source"] == src


def test_learned_correction_zero_exact_and_kept_only_when_better(X):
    """xkp_learned_correction_solve: with a zero correction the guess is the projection's (not
    kept: guess_source 1) and the call equals xkp_target_project_solve bit for bit; with the
    exact correction (coordinates of x* minus those of the projected guess) the corrected guess
    is V V^T x*, kept (guess_source 3) exactly where its FP64 residual is below the projected
    guess's, and a gate of 0 keeps none."""
    import torch
    H, T, m, N = 64, 100, 40, 4
    ctx, bases, d, specs, mts = setup(X, H, T, m, N)
    k = bases.header(0)["k"]
    V = cpu(bases.V(0))[:, :k]
    P0 = X.Context.params(m, tol=1e300)
    # the projected guesses and their coordinates
    info_p = ctx.new_infos(N)
    ctx.target_project_solve(d, N, 1, bases.ptrs, P0, info_p)
    torch.cuda.synchronize()
    ip = X.infos_to_numpy(info_p).copy()
    xp = [cpu(s_.x).copy() for s_ in specs]
    zp = torch.empty((N, 48), dtype=torch.float64, device=dev())
    ctx.basis_coeffs(d, N, 1, bases.ptrs, 48, zp, kind=1)
    # zero correction
    zero = torch.zeros((N, 48), dtype=torch.float32, device=dev())
    info = ctx.new_infos(N)
    ctx.learned_correction_solve(d, N, 1, bases.ptrs, P0, zero, 48, 1.0, 1e300, info)
    torch.cuda.synchronize()
    i0 = X.infos_to_numpy(info)
    assert np.all(i0["guess_source"] == 1)
    for i in range(N):
        assert np.array_equal(cpu(specs[i].x), xp[i])
    assert np.array_equal(i0["guess_res"], ip["guess_res"])
    # the exact correction: coordinates of x* minus those of x0_P (kind 1, FP64 on the GPU)
    xstar = []
    for i, mt in enumerate(mts):
        At = oracle.Operator(H, 1.0 / T, 0.5, mt)
        xstar.append(oracle.banded_solve(At, oracle.rhs(At, mt))[0])
        specs[i].x.copy_(torch.from_numpy(xstar[-1]))
    zs = torch.empty((N, 48), dtype=torch.float64, device=dev())
    ctx.basis_coeffs(d, N, 1, bases.ptrs, 48, zs, kind=1)
    corr = (zs - zp).to(torch.float32)
    for gate, keep_any in ((1e300, True), (0.0, False)):
        info = ctx.new_infos(N)
        ctx.learned_correction_solve(d, N, 1, bases.ptrs, P0, corr, 48, 1.0, gate, info)
        torch.cuda.synchronize()
        ic = X.infos_to_numpy(info)
        for i in range(N):
            At = oracle.Operator(H, 1.0 / T, 0.5, mts[i])
            bt = oracle.rhs(At, mts[i])
            best = V @ (V.T @ xstar[i])
            # kept exactly where it beats the projected guess (FP32 correction: rounding only)
            better = oracle.residual(At, bt, best) < ip[i]["guess_res"] * (1 - 1e-6)
            x0 = cpu(specs[i].x)
            if keep_any and better:
                assert ic[i]["guess_source"] == 3, i
                assert np.abs(x0 - best).max() <= 1e-6 * np.abs(best).max(), i
                assert ic[i]["guess_res"] < ip[i]["guess_res"]
                assert abs(ic[i]["guess_res"] - oracle.residual(At, bt, x0)) <= \
                    1e-9 * ic[i]["guess_res"]
            elif not keep_any:
                assert ic[i]["guess_source"] == 1 and np.array_equal(x0, xp[i]), i
            else:
                assert ic[i]["guess_res"] <= ip[i]["guess_res"], i
    # the projection modes only: plain GMRES has nothing to correct
    with pytest.raises(X.XkpError):
        ctx.learned_correction_solve(d, N, 1, bases.ptrs, X.Context.params(m, mode="none"),
                                     corr, 48, 1.0, 1e300, ctx.new_infos(N))


def test_learned_pipeline_trains_and_falls_back(X):
    """The whole learned-guess pipeline at a small size (64x64, m = 40, T = 10): training data
    from the method's own chain, training on the GPU, then held-out targets solved with the
    learned guess behind the gate, and with the learned correction of the projection.  What
    training gains is asserted against the untrained network (held-out guess residual); what
    the learned guess and the correction gain or lose against the projection (the method
    without the network) is asserted and printed: guess residuals timestep by timestep, polish
    iterations; the seed subspace's residual floor lies below every guess built from it.  A
    gate of 1e-6 rejects every learned guess here, and the chain then equals the projection
    chain bit for bit."""
    import torch
    from oracle import cnn
    from paper_2511_17634_amd import learned
    from paper_2511_17634_amd.driver import Batch, Group
    from synth import CONFIGS, config_images, initial_state
    from synth.configs import ROLE_EVAL
    cfg = CONFIGS["c5"]
    T, m = 10, cfg.m
    seed, tg = config_images(cfg, 0, 0, 256)
    s0 = initial_state(seed[0])
    t0 = np.stack([initial_state(t[0]) for t in tg])
    _, ev = config_images(cfg, 0, 0, 32, role=ROLE_EVAL)
    e0 = np.stack([initial_state(t[0]) for t in ev])
    alpha, ok = learned.generate(s0, t0, T, m)
    assert ok
    ctx = X.Context(4096, m, 1)
    theta0 = cnn.init_params(m + 1, np.random.default_rng(0))
    net = X.Net(ctx, m + 1, 128, theta0)
    imgs = torch.tensor(t0, dtype=torch.float64, device=dev())
    hist = learned.train(net, imgs, alpha, 6, 128, 2e-3)
    assert hist[-1] < 0.1 * hist[0]

    def chain(**kw):
        b = Batch([Group(64, s0[None], e0[:, None])], T, m, **kw)
        b.run()
        si, ti = b.all_infos()
        assert np.all(ti["status"] == X.OK) and np.all(ti["res_true"] <= 1e-8)
        assert np.all(b.verify_last() <= 1e-8 * (1 + 1e-6))
        return b, ti

    bp, tp = chain(method="project")
    res = {}
    for name, params in (("trained", net.params), ("untrained", theta0)):
        for gate in (1e300, 1e-2, 1e-6):
            b, ti = chain(method="learned", learned=dict(params=params, scale=1.0, gate=gate))
            res[(name, gate)] = ti
            if gate == 1e-6:
                assert np.all(ti["guess_source"] == 1)
                assert torch.equal(b.state()[1], bp.state()[1])
                assert np.array_equal(ti["iters"], tp["iters"])
            if gate == 1e300:
                assert np.all(ti["guess_source"] == 2)
    tr, un = res[("trained", 1e300)], res[("untrained", 1e300)]
    assert np.median(tr["guess_res"]) < 0.5 * np.median(un["guess_res"])
    # the correction network: trained on the projected guess's coordinate error
    alpha2, alpha_p, ok2 = learned.generate(s0, t0, T, m, with_projection=True)
    assert ok2 and torch.equal(alpha2, alpha)
    netc = X.Net(ctx, m + 1, 128, theta0)
    histc = learned.train(netc, imgs, alpha - alpha_p, 6, 128, 2e-3)
    assert histc[-1] < histc[0]
    bc, tc = chain(method="learned",
                   learned=dict(params=netc.params, scale=1.0, gate=1e300, correction=True))
    assert np.all(np.isin(tc["guess_source"], (1, 3)))
    # against the projection, the method without the network: both chains solve every step to
    # 1e-8, so the guesses compare timestep by timestep.  The correction is kept only where it
    # lowers the residual: never worse than the projection beyond the chains' 1e-8 differences
    assert np.all(tc["guess_res"] <= tp["guess_res"] * (1 + 1e-6) + 1e-12)
    assert tc["iters"].mean() <= tp["iters"].mean() + 0.2
    # the seed subspace's floor on a sample: below every guess built from it
    floor = learned.span_floor(bp, [0, 16], (0, 4, 9))
    for (t, i), f in floor.items():
        assert f <= tp["guess_res"][t, i] * (1 + 1e-9)
        assert f <= tr["guess_res"][t, i] * (1 + 1e-9)
        assert f <= tc["guess_res"][t, i] * (1 + 1e-9)
    print(f"\nheld-out guess residual (median): trained {np.median(tr['guess_res']):.3g}, "
          f"untrained {np.median(un['guess_res']):.3g}, correction "
          f"{np.median(tc['guess_res']):.3g}, projection {np.median(tp['guess_res']):.3g}, "
          f"subspace floor {np.median(list(floor.values())):.3g}; mean polish iterations: "
          f"learned {tr['iters'].mean():.2f}, correction {tc['iters'].mean():.2f} (kept "
          f"{(tc['guess_source'] == 3).mean():.2f}), projection {tp['iters'].mean():.2f}; "
          f"accepted at gate 1e-2: {(res[('trained', 1e-2)]['guess_source'] == 2).mean():.2f}")


def test_learned_chain_graph_replays_match_eager(X):
    """A chain with the learned guess (network inference inside every timestep) captured once
    and replayed twice with eager work between: bitwise the eager chain."""
    import torch
    from oracle import cnn
    from paper_2511_17634_amd.driver import Batch, Group
    T, m = 6, 40
    s0, _ = blob_pair(64, seed=55)
    tg = np.stack([blob_pair(64, seed=55, jitter=1.0 + 0.3 * i)[1] for i in range(5)])
    theta = cnn.init_params(m + 1, np.random.default_rng(1)) * 0.01
    b = Batch([Group(64, s0[None], tg[:, None])], T, m, method="learned",
              learned=dict(params=theta, scale=1.0, gate=1e300))
    b.run()
    ref = cpu(b.state()[1]).copy()
    ref_i = b.all_infos()[1].copy()
    assert np.all(ref_i["status"] == X.OK) and np.all(ref_i["guess_source"] == 2)
    b.capture()
    for _ in range(2):
        b.replay()
        torch.cuda.synchronize()
        assert np.array_equal(cpu(b.state()[1]), ref)
        assert np.array_equal(b.all_infos()[1], ref_i)
        b.run()
        torch.cuda.synchronize()
