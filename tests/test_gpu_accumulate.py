"""GPU parity of the image-cycle subspace accumulation (xkp_basis_accumulate) against the
oracle, projection on an accumulated basis, the modes that must reject it, and a short cycle
chain against the oracle's cycle chain.  Every call goes through the C ABI."""
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


def seeds_on_gpu(X, H, T, m, images):
    """Seed bases of several images (one launch)."""
    import torch
    n = H * H
    S = len(images)
    ctx = X.Context(n, m, S)
    ms = t64(np.stack(images))
    b = torch.zeros((S, n), dtype=torch.float64, device=dev())
    x = torch.zeros((S, n), dtype=torch.float64, device=dev())
    d = X.pack_batch(H, 1.0 / T, 0.5, ms, b, x, basis_id=0)
    ctx.build_rhs(d, S)
    bases = X.Bases(S, n, m)
    info = ctx.new_infos(S)
    ctx.seed_build(d, S, bases.ptrs, X.Context.params(m), info)
    torch.cuda.synchronize()
    assert np.all(X.infos_to_numpy(info)["status"] == X.OK)
    return ctx, bases


@pytest.mark.parametrize("H,per_source,cap", [(40, 8, 20), (64, 20, 40), (24, 30, 50)])
def test_accumulate_matches_oracle(X, H, per_source, cap):
    import torch
    T, m = 100, 30
    imgs = [blob_pair(H, seed=200 + H, jitter=2.0 + 1.5 * i)[1] for i in range(3)]
    ctx, bases = seeds_on_gpu(X, H, T, max(m, cap), imgs)
    n = H * H
    acc = X.Bases(3, n, cap)
    ctx2 = X.Context(n, cap, 3)
    out_k = torch.full((3,), -7, dtype=torch.int32, device=dev())
    ctx2.basis_accumulate(n, 3, bases.ptrs, acc.ptrs, per_source, cap, out_k)
    torch.cuda.synchronize()
    ks = cpu(out_k)
    srcs = []
    for s in range(3):
        k = bases.header(s)["k"]
        srcs.append(cpu(bases.V(s))[:, :k])
    for j in range(3):
        Vo = oracle.accumulate(srcs[:j + 1], per_source, cap)
        h = acc.header(j)
        assert ks[j] == Vo.shape[1] == h["k"], (j, ks[j], Vo.shape)
        assert h["m"] == cap and h["kind"] == 1 and h["bf16"] == 1 and h["n"] == n
        kd = h["k"]
        Vg = cpu(acc.V(j))[:, :kd]
        assert np.abs(Vg - Vo).max() <= 1e-10, j
        assert np.abs(Vg.T @ Vg - np.eye(kd)).max() <= 1e-12
        # zero padding kept and the BF16 copy is torch's rounding of the columns
        assert torch.all(acc.V_padded(j)[n:, :kd] == 0)
        ref = acc.V_padded(j)[:, :kd].float().bfloat16().view(torch.int16)
        assert torch.equal(acc.Vb_bits(j)[:, :kd], ref)


def test_projection_on_accumulated_basis(X):
    import torch
    H, T, m, cap = 48, 100, 24, 24
    ims = [blob_pair(H, seed=300, jitter=j)[1] for j in (1.0, 3.0)]
    ctx, bases = seeds_on_gpu(X, H, T, m, ims)
    n = H * H
    acc = X.Bases(2, n, cap)
    ctx.basis_accumulate(n, 2, bases.ptrs, acc.ptrs, 12, cap)
    _, mt = blob_pair(H, seed=300, jitter=2.0)
    tm = t64(mt)
    bt = torch.zeros(n, dtype=torch.float64, device=dev())
    xt = torch.zeros(n, dtype=torch.float64, device=dev())
    d = X.pack_systems([X.SystemSpec(H, 1.0 / T, 0.5, tm, b=bt, x=xt, basis_id=1)], dev())
    ctx.build_rhs(d, 1)
    info = ctx.new_infos(1)
    # a huge tolerance stops the polish before its first step: x is the projected guess
    ctx.target_project_solve(d, 1, 2, acc.ptrs, X.Context.params(cap, tol=1e300), info)
    torch.cuda.synchronize()
    i = X.infos_to_numpy(info)[0]
    kd = acc.header(1)["k"]
    assert i["status"] == X.OK and i["basis_dim"] == kd == cap
    At = oracle.Operator(H, 1.0 / T, 0.5, mt)
    b = oracle.rhs(At, mt)
    Vp = np.concatenate([cpu(acc.V(1))[:, :kd], np.zeros((n, 1))], axis=1)
    x0o, _, st = oracle.project(At, b, Vp, np.zeros((kd + 1, kd)))
    assert st == oracle.OK
    assert np.abs(cpu(xt) - x0o).max() <= 1e-9 * np.abs(x0o).max()
    # polish to the tolerance in FP64 and in mixed precision
    for prec in (X.FP64, X.MIXED):
        info = ctx.new_infos(1)
        ctx.target_project_solve(d, 1, 2, acc.ptrs, X.Context.params(cap, precision=prec), info)
        torch.cuda.synchronize()
        i = X.infos_to_numpy(info)[0]
        assert i["status"] == X.OK and i["res_true"] <= 1e-8, prec
        assert oracle.residual(At, b, cpu(xt)) <= 1e-8
    # the Hessenberg-based modes and the learned coordinates refuse an accumulated basis
    for mode in ("seed_galerkin", "seed_lsq"):
        info = ctx.new_infos(1)
        ctx.target_project_solve(d, 1, 2, acc.ptrs, X.Context.params(cap, mode=mode), info)
        torch.cuda.synchronize()
        assert X.infos_to_numpy(info)[0]["status"] == X.EINVAL, mode
    alpha = torch.zeros((1, cap + 1), dtype=torch.float64, device=dev())
    ctx.basis_coeffs(d, 1, 2, acc.ptrs, cap + 1, alpha, kind=1)
    torch.cuda.synchronize()
    assert torch.all(torch.isnan(alpha))
    # a source of another size gives -1 and the host checks reject bad arguments
    out_k = torch.zeros(2, dtype=torch.int32, device=dev())
    ctx2 = X.Context(64 * 64, cap, 2)
    ctx2.basis_accumulate(64 * 64, 2, bases.ptrs, X.Bases(2, 64 * 64, cap).ptrs, 12, cap, out_k)
    torch.cuda.synchronize()
    assert np.all(cpu(out_k) == -1)
    with pytest.raises(X.XkpError):
        ctx.basis_accumulate(n, 2, bases.ptrs, acc.ptrs, 0, cap)
    with pytest.raises(X.XkpError):
        ctx.basis_accumulate(n, 2, bases.ptrs, acc.ptrs, 12, 65)


def test_cycle_chain_matches_oracle(X):
    """Three blocks of four 32x32 images (seeds 0, 4, 8), a = 6 columns per seed, m = 16,
    T = 6: every solve converges and the states match the oracle's cycle chain."""
    from paper_2511_17634_amd.driver import Batch, Group
    from oracle.chain import run_cycle_chain
    H, T, m, a = 32, 6, 16, 6
    imgs = [blob_pair(H, seed=400, jitter=0.5 + 0.4 * i)[1] for i in range(12)]
    blocks = [(imgs[4 * g][None], np.stack(imgs[4 * g + 1:4 * g + 4])[:, None])
              for g in range(3)]
    b = Batch([Group(H, s, t) for s, t in blocks], T, m, accumulate=a)
    b.run()
    s_inf, t_inf = b.all_infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.all(t_inf["res_true"] <= 1e-8)
    ms_o, mt_o, st = run_cycle_chain([(s[0], t[:, 0]) for s, t in blocks], H, T, m, a)
    _, mt_g = b.state()
    mt_g = cpu(mt_g).reshape(3, 3, -1)
    bound = T * 1e-8 * max(np.linalg.norm(t) for t in imgs)
    for g in range(3):
        assert np.abs(mt_g[g] - mt_o[g]).max() <= bound, g
    it_g = t_inf["iters"].reshape(T, 9).astype(int)
    assert np.abs(it_g - np.array(st.iters)).max() <= 2
    # the guess of every target, the one quantity that sees which columns were gathered and in
    # which order, against the oracle's guess on its own gathered basis
    g_gpu = t_inf["guess_res"].reshape(T, 9)
    g_o = np.array(st.guess_res)
    # (the states they are formed from agree to the chain's tolerance; a wrong source set or
    # column order moves a guess residual by 1e-1 on these images)
    assert np.all(np.abs(g_gpu - g_o) <= 1e-6 + 1e-5 * g_o), np.abs(g_gpu - g_o).max()
    # the blocks after the first see the larger gathered bases
    assert np.all(t_inf["basis_dim"].reshape(T, 3, 3)[:, 1:] > a)
