"""The 16-wave (1024-thread workgroups, 4 or 16 rows per thread, n <= 16384) and 4-wave
(256-thread, 4 or 16 rows per thread, n <= 4096) kernel variants against the 8-wave variant and
the oracle: seeds of several sizes in one launch, projections in every mode, project + polish,
mixed precision.  The variants sum in different orders, so they agree to rounding, not
bitwise."""
import numpy as np
import pytest

import oracle
from gpu_util import blob_pair, cpu, dev, t64

pytestmark = pytest.mark.gpu
SIZES_BY_WAVES = {16: [128, 100, 64, 45, 32, 20], 4: [64, 45, 32, 20]}


@pytest.fixture(scope="module")
def X():
    from paper_2511_17634_amd import xkp
    xkp.load()
    return xkp


def zeros(n):
    import torch
    return torch.zeros(n, dtype=torch.float64, device=dev())


def seeds(X, waves, m=30, T=100, precision=0, sizes=None):
    import torch
    sizes = sizes or SIZES_BY_WAVES[waves]
    specs, mss = [], []
    for H in sizes:
        ms, _ = blob_pair(H, seed=1000 + H)
        mss.append(ms)
        specs.append(X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=zeros(H * H), x=zeros(H * H)))
    ctx = X.Context(max(sizes) ** 2, m, len(specs))
    ctx.set_launch(waves)
    d = X.pack_systems(specs, dev())
    ctx.build_rhs(d, len(specs))
    bases = X.Bases(len(specs), [H * H for H in sizes], m)
    info = ctx.new_infos(len(specs))
    ctx.seed_build(d, len(specs), bases.ptrs, X.Context.params(m, precision=precision), info)
    torch.cuda.synchronize()
    return ctx, bases, [cpu(s.x) for s in specs], X.infos_to_numpy(info), mss


# (launches sized for 4096 unknowns at most run the seeds' kept cycle by delayed
# re-orthogonalisation, larger ones by two modified Gram-Schmidt passes: both for 16 waves)
@pytest.mark.parametrize("waves,sizes", [(16, None), (16, [64, 45, 32, 20]), (4, None)])
@pytest.mark.parametrize("precision", [0, 1])
def test_seeds_match_8_waves_and_oracle(X, waves, sizes, precision):
    sizes = sizes or SIZES_BY_WAVES[waves]
    _, b16, x16, i16, mss = seeds(X, waves, precision=precision, sizes=sizes)
    _, b8, x8, i8, _ = seeds(X, 8, precision=precision, sizes=sizes)
    for i, H in enumerate(sizes):
        A = oracle.Operator(H, 0.01, 0.5, mss[i])
        bo = oracle.rhs(A, mss[i])
        assert i16[i]["status"] == X.OK and oracle.residual(A, bo, x16[i]) <= 1e-8
        assert abs(int(i16[i]["iters"]) - int(i8[i]["iters"])) <= 1
        assert np.abs(x16[i] - x8[i]).max() <= 1e-8 * np.abs(x8[i]).max()
        k = min(b16.header(i)["k"], b8.header(i)["k"])
        assert np.abs(cpu(b16.V(i))[:, :6] - cpu(b8.V(i))[:, :6]).max() <= 1e-10
        assert k >= 1


@pytest.mark.parametrize("waves", [16, 4])
@pytest.mark.parametrize("mode", ["target_galerkin", "seed_galerkin", "seed_lsq"])
def test_projection_matches_oracle(X, waves, mode):
    """Targets of every size projected on the seeds' bases (guess only) vs the oracle's
    projection on the same bases, then polished."""
    import torch
    sizes = SIZES_BY_WAVES[waves]
    ctx, bases, _, _, mss = seeds(X, waves)
    specs, mts = [], []
    for i, H in enumerate(sizes):
        _, mt = blob_pair(H, seed=1000 + H, jitter=1.5)
        mts.append(mt)
        specs.append(X.SystemSpec(H, 0.01, 0.5, t64(mt), b=zeros(H * H), x=zeros(H * H),
                                  basis_id=i))
    d = X.pack_systems(specs, dev())
    ctx.build_rhs(d, len(specs))
    info = ctx.new_infos(len(specs))
    ctx.target_project_solve(d, len(specs), len(sizes), bases.ptrs,
                             X.Context.params(30, tol=1e300, mode=mode), info)
    torch.cuda.synchronize()
    mid = {"target_galerkin": oracle.TARGET_GALERKIN, "seed_galerkin": oracle.SEED_GALERKIN,
           "seed_lsq": oracle.SEED_LSQ}[mode]
    for i, H in enumerate(sizes):
        At = oracle.Operator(H, 0.01, 0.5, mts[i])
        bt = oracle.rhs(At, mts[i])
        k = bases.header(i)["k"]
        x0o, _, _ = oracle.project(At, bt, cpu(bases.V(i))[:, :k + 1],
                                   cpu(bases.Hbar(i))[:k + 1, :k], mode=mid)
        assert np.abs(cpu(specs[i].x) - x0o).max() <= 1e-9 * np.abs(x0o).max(), H
    ctx.target_project_solve(d, len(specs), len(sizes), bases.ptrs,
                             X.Context.params(30, mode=mode), info)
    torch.cuda.synchronize()
    inf = X.infos_to_numpy(info)
    for i, H in enumerate(sizes):
        At = oracle.Operator(H, 0.01, 0.5, mts[i])
        assert inf[i]["status"] == X.OK
        assert oracle.residual(At, oracle.rhs(At, mts[i]), cpu(specs[i].x)) <= 1e-8
