"""GPU parity of the mixed-precision path (FP32 operator inside the GMRES cycles, BF16 matrix-core
projection with FP32 accumulation, FP64 orthogonalisation / rotations / residuals) against the
FP64 oracle.  Tolerances follow from the number formats: FP32 and BF16 unit roundoffs 2^-24 and
2^-9 (round to nearest), and the final answers must still meet the FP64 tolerance.  Each test
prints every target's error against the oracle solution."""
import numpy as np
import pytest

import oracle
from gpu_util import blob_pair, cpu, dev, t64

pytestmark = pytest.mark.gpu
U32, UBF = 2.0 ** -24, 2.0 ** -9


@pytest.fixture(scope="module")
def X():
    from paper_2511_17634_amd import xkp
    xkp.load()
    return xkp


def zeros(n):
    import torch
    return torch.zeros(n, dtype=torch.float64, device=dev())


def seed(X, H, T, m, ms, precision):
    import torch
    n = H * H
    ctx = X.Context(n, m, 1)
    spec = X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=zeros(n), x=zeros(n))
    d = X.pack_systems([spec], dev())
    ctx.build_rhs(d, 1)
    bases = X.Bases(1, n, m)
    info = ctx.new_infos(1)
    ctx.seed_build(d, 1, bases.ptrs, X.Context.params(m, precision=precision), info)
    torch.cuda.synchronize()
    return bases, cpu(spec.x), X.infos_to_numpy(info)[0]


def varah_ok(A, b, x, xs):
    rinf = np.abs(b - oracle.apply(A, x)).max()
    return np.abs(x - xs).max() <= A.dt * rinf * (1 + 1e-6) + 1e-13 * np.abs(xs).max()


def masked_coeffs(A):
    """(diag, E, W, N, S) per row with the neighbours outside the grid dropped."""
    C = [c.copy() for c in oracle.coeffs(A)]
    H = A.H
    i, j = np.divmod(np.arange(H * H), H)
    C[1][i == H - 1] = 0
    C[2][i == 0] = 0
    C[3][j == H - 1] = 0
    C[4][j == 0] = 0
    return C


def neighbours(v, H):
    """v at (i+1, j), (i-1, j), (i, j+1), (i, j-1) (zero outside; masked coefficients drop the
    wrapped j-neighbours)."""
    out = []
    for d in (H, -H, 1, -1):
        nb = np.zeros_like(v)
        if d > 0:
            nb[:-d] = v[d:]
        else:
            nb[-d:] = v[:d]
        out.append(nb)
    return out


def op_fp32(A, v):
    """The operator in FP32 arithmetic (coefficients and operands rounded to FP32, the row's
    five products summed left to right in FP32)."""
    C = [c.astype(np.float32) for c in masked_coeffs(A)]
    v32 = v.astype(np.float32)
    nb = neighbours(v32, A.H)
    y = C[0] * v32
    for c, u in zip(C[1:], nb):
        y = y + c * u
    return y


def bf16(a):
    """Values of a rounded to FP32 then to the nearest BF16 (torch's conversion), as float64."""
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).double().numpy()


@pytest.mark.parametrize("H,m", [(64, 40), (128, 60)])
def test_mixed_seed_basis_and_solution(X, H, m):
    import torch
    T = 100
    ms, _ = blob_pair(H, seed=500 + H)
    bases, x, info = seed(X, H, T, m, ms, X.MIXED)
    A = oracle.Operator(H, 1.0 / T, 0.5, ms)
    b = oracle.rhs(A, ms)
    xs, _ = oracle.banded_solve(A, b)
    assert info["status"] == X.OK
    assert oracle.residual(A, b, x) <= 1e-8            # FP64-verified
    assert varah_ok(A, b, x, xs)
    err = np.abs(x - xs).max() / np.abs(xs).max()
    print(f"\nmixed seed {H}x{H}: iters {info['iters']}, restarts {info['restarts']}, "
          f"max rel error vs oracle {err:.2e}")
    hdr = bases.header(0)
    k = hdr["k"]
    assert hdr["bf16"] == 1 and k >= 1
    V = cpu(bases.V(0))[:, :k + 1]
    Hb = cpu(bases.Hbar(0))[:k + 1, :k]
    # FP64 orthogonalisation: orthonormal to FP64 rounding
    assert np.abs(V.T @ V - np.eye(k + 1)).max() <= 1e-12
    # seeds keep the FP64 operator in mixed mode: the Arnoldi relation holds to FP64 rounding
    AV = np.stack([oracle.apply(A, V[:, c]) for c in range(k)], axis=1)
    assert np.abs(AV - V[:, :k + 1] @ Hb).max() <= 1e-12 * np.abs(oracle.coeffs(A)[0]).max()
    # the BF16 copy is V rounded to FP32 then to the nearest BF16 (torch's conversion)
    vb = cpu(bases.Vb_bits(0))[:H * H, :k + 1]
    ref = torch.from_numpy(V.astype(np.float32)).to(torch.bfloat16).view(torch.int16).numpy()
    assert np.array_equal(vb, ref)


def mixed_target_setup(X, H, T, m, jitter, n_t=3, seed_precision=None):
    import torch
    ms, _ = blob_pair(H, seed=700 + H)
    bases, _, _ = seed(X, H, T, m, ms, seed_precision if seed_precision is not None else X.MIXED)
    mts = [blob_pair(H, seed=700 + H, jitter=jitter + 0.5 * i)[1] for i in range(n_t)]
    specs = [X.SystemSpec(H, 1.0 / T, 0.5, t64(mt), b=zeros(H * H), x=zeros(H * H))
             for mt in mts]
    ctx = X.Context(H * H, m, n_t)
    d = X.pack_systems(specs, dev())
    ctx.build_rhs(d, n_t)
    return ctx, bases, d, specs, mts


@pytest.mark.parametrize("split", [-1, 0])
@pytest.mark.parametrize("H,m", [(64, 40), (128, 60)])
def test_mixed_projection_guess_matches_bf16_emulation(X, H, m, split):
    """x0 of the mixed target-Galerkin projection vs the same projection emulated on the CPU:
    A'V_k with the FP32 operator, both factors rounded to BF16, their products summed exactly
    (FP64), V_k^T r_base and the solve in FP64.  What remains between the two is the FP32
    accumulation on the matrix cores (a random walk of about sqrt(n) u32 relative to the entries)
    and the FP32 evaluation order of the operator (flipping a few BF16 roundings); amplified by
    the condition number of the projected matrix this gives the tolerance
    64 cond(A_p) sqrt(n) u32.  The FP64 projection is printed beside it: its distance to the
    emulation is the BF16 rounding itself."""
    import torch
    T = 100
    ctx, bases, d, specs, mts = mixed_target_setup(X, H, T, m, jitter=1.0)
    if split >= 0:   # the projection in launches of its own
        ctx.set_projection_split(split)
    info = ctx.new_infos(len(specs))
    ctx.target_project_solve(d, len(specs), 1, bases.ptrs,
                             X.Context.params(m, tol=1e300, precision=X.MIXED), info)
    torch.cuda.synchronize()
    inf = X.infos_to_numpy(info)
    k = bases.header(0)["k"]
    V = cpu(bases.V(0))[:, :k]
    n = H * H
    Vb = bf16(V)
    for i, mt in enumerate(mts):
        At = oracle.Operator(H, 1.0 / T, 0.5, mt)
        bt = oracle.rhs(At, mt)
        Wb = bf16(np.stack([op_fp32(At, V[:, c]) for c in range(k)], axis=1))
        Ae = Vb.T @ Wb
        beta = V.T @ bt
        xe = V @ np.linalg.solve(Ae, beta)
        W64 = np.stack([oracle.apply(At, V[:, c]) for c in range(k)], axis=1)
        A64 = V.T @ W64
        x64 = V @ np.linalg.solve(A64, beta)
        tol = 64 * np.linalg.cond(Ae) * np.sqrt(n) * U32
        x0 = cpu(specs[i].x)
        rel = np.linalg.norm(x0 - xe) / np.linalg.norm(xe)
        rel64 = np.linalg.norm(x64 - xe) / np.linalg.norm(xe)
        print(f"\nmixed guess {H}x{H} target {i}: |x0 - x0_emul|/|x0_emul| = {rel:.2e} "
              f"(tol {tol:.2e}); BF16 effect |x0_fp64 - x0_emul|/|x0_emul| = {rel64:.2e}; "
              f"guess residual {inf[i]['guess_res']:.3e} (FP64 projection "
              f"{oracle.residual(At, bt, x64):.3e})")
        assert inf[i]["status"] == X.OK and inf[i]["basis_dim"] == k
        assert rel <= tol
        assert abs(inf[i]["guess_res"] - oracle.residual(At, bt, x0)) <= 1e-9 * inf[i]["guess_res"]


@pytest.mark.parametrize("H,m", [(64, 40), (128, 60)])
def test_mixed_project_and_polish_meets_fp64_tolerance(X, H, m):
    import torch
    T = 100
    ctx, bases, d, specs, mts = mixed_target_setup(X, H, T, m, jitter=2.0)
    info = ctx.new_infos(len(specs))
    ctx.target_project_solve(d, len(specs), 1, bases.ptrs,
                             X.Context.params(m, precision=X.MIXED), info)
    torch.cuda.synchronize()
    inf = X.infos_to_numpy(info)
    for i, mt in enumerate(mts):
        At = oracle.Operator(H, 1.0 / T, 0.5, mt)
        bt = oracle.rhs(At, mt)
        xs, _ = oracle.banded_solve(At, bt)
        x = cpu(specs[i].x)
        res = oracle.residual(At, bt, x)
        err = np.abs(x - xs).max() / np.abs(xs).max()
        ro = oracle.gmres(At, bt, m=m)
        print(f"\nmixed target {H}x{H} #{i}: iters {inf[i]['iters']} (FP64 plain oracle "
              f"{ro.iters}), restarts {inf[i]['restarts']}, residual {res:.2e}, "
              f"max rel error vs oracle {err:.2e}")
        assert inf[i]["status"] == X.OK and inf[i]["res_true"] <= 1e-8
        assert res <= 1e-8 and abs(res - inf[i]["res_true"]) <= 1e-12
        assert varah_ok(At, bt, x, xs)


def test_mixed_plain_gmres_and_seed_modes(X):
    """Plain GMRES and the seed-Galerkin / least-squares projections in mixed precision also
    meet the FP64 tolerance; a mixed target-Galerkin projection on a basis built in FP64 (no
    BF16 copy) is rejected per target."""
    import torch
    H, T, m = 64, 100, 40
    for mode in ("none", "seed_galerkin", "seed_lsq"):
        ctx, bases, d, specs, mts = mixed_target_setup(X, H, T, m, jitter=1.5, n_t=2)
        info = ctx.new_infos(2)
        ctx.target_project_solve(d, 2, 1, bases.ptrs,
                                 X.Context.params(m, precision=X.MIXED, mode=mode), info)
        torch.cuda.synchronize()
        inf = X.infos_to_numpy(info)
        for i, mt in enumerate(mts):
            At = oracle.Operator(H, 1.0 / T, 0.5, mt)
            bt = oracle.rhs(At, mt)
            assert inf[i]["status"] == X.OK, mode
            assert oracle.residual(At, bt, cpu(specs[i].x)) <= 1e-8, mode
    ctx, bases, d, specs, mts = mixed_target_setup(X, H, T, m, jitter=1.5, n_t=2,
                                                   seed_precision=X.FP64)
    assert bases.header(0)["bf16"] == 0
    info = ctx.new_infos(2)
    ctx.target_project_solve(d, 2, 1, bases.ptrs, X.Context.params(m, precision=X.MIXED), info)
    torch.cuda.synchronize()
    assert list(X.infos_to_numpy(info)["status"]) == [X.EINVAL, X.EINVAL]


def test_mixed_chain_grid128_matches_oracle(X):
    """Three timesteps of a 128x128 chain (1 seed + 2 targets, m = 60) in mixed precision vs
    the FP64 oracle chain."""
    from paper_2511_17634_amd.driver import Chain
    from oracle.chain import run_chain
    H, T, m, steps = 128, 100, 60, 3
    s0, _ = blob_pair(H, seed=901)
    t0 = np.stack([blob_pair(H, seed=901, jitter=1.0 + i)[1] for i in range(2)])
    ch = Chain(H, T, m, s0, t0, precision=X.MIXED)
    ch.reset()
    for _ in range(steps):
        ch.step()
        si, ti = ch.infos()
        assert si[0]["status"] == X.OK and np.all(ti["status"] == X.OK)
        assert np.all(ti["res_true"] <= 1e-8)
    ms_o, mt_o, st = run_chain(s0, t0, H, T, m, steps=steps)
    bound = steps * 1e-8 * max(np.linalg.norm(s0), np.linalg.norm(t0, axis=1).max())
    tg = cpu(ch.target_state)
    for i in range(2):
        e = np.abs(tg[i] - mt_o[i]).max()
        print(f"\nmixed chain target {i}: max error vs oracle chain {e:.2e} (bound {bound:.2e})")
        assert e <= bound
    assert np.abs(cpu(ch.seed_state) - ms_o).max() <= bound
