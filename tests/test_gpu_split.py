"""GPU parity of the target projection in launches of its own (xkp_ctx_set_projection_split:
row tiles across the chip, shares summed in tile order by each target's last tile, the small
solve on one wavefront, x0 by tiles, then the polish) against the FP64 oracle and against the
projection inside the solve launch, through the C ABI: every mode, cold and warm starts, sizes
with ragged last tiles, every tile count from one tile per target up, an uneven batch of
several bases, more targets than partial slots, the timestep chain and its HIP-graph replays."""
import numpy as np
import pytest

import oracle
from gpu_util import blob_pair, cpu, dev, t64

pytestmark = pytest.mark.gpu

MODES = {"target_galerkin": "TARGET_GALERKIN", "seed_galerkin": "SEED_GALERKIN",
         "seed_lsq": "SEED_LSQ"}


@pytest.fixture(scope="module")
def X():
    from paper_2511_17634_amd import xkp
    xkp.load()
    return xkp


def zeros(n):
    import torch
    return torch.zeros(n, dtype=torch.float64, device=dev())


def seed_basis(X, H, T, m, ms, precision=None):
    import torch
    n = H * H
    ctx = X.Context(n, m, 1)
    spec = X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=zeros(n), x=zeros(n))
    d = X.pack_systems([spec], dev())
    ctx.build_rhs(d, 1)
    bases = X.Bases(1, n, m)
    info = ctx.new_infos(1)
    ctx.seed_build(d, 1, bases.ptrs,
                   X.Context.params(m, precision=X.FP64 if precision is None else precision),
                   info)
    torch.cuda.synchronize()
    assert X.infos_to_numpy(info)[0]["status"] == X.OK
    return bases


def project(X, H, T, m, bases, mts, warm, split, mode="target_galerkin", tol=1e300,
            precision=None, polish_m=0, basis_ids=None, Hs=None):
    """Targets (all of side H, or of sides Hs) projected, and polished to tol (1e300: the guess
    itself), with the projection split into at most `split` tiles (-1: inside the solve
    launch).  Returns the iterates and the infos."""
    import torch
    Hs = [H] * len(mts) if Hs is None else Hs
    nmax = max(h * h for h in Hs)
    ctx = X.Context(nmax, m, len(mts))
    if split >= 0:
        ctx.set_projection_split(split)
    specs = [X.SystemSpec(h, 1.0 / T, 0.5, t64(mt), b=zeros(h * h), x=zeros(h * h),
                          x0=t64(mt) if warm else None,
                          basis_id=0 if basis_ids is None else basis_ids[i])
             for i, (h, mt) in enumerate(zip(Hs, mts))]
    d = X.pack_systems(specs, dev())
    ctx.build_rhs(d, len(mts))
    info = ctx.new_infos(len(mts))
    ctx.target_project_solve(d, len(mts), bases.count, bases.ptrs,
                             X.Context.params(m, tol=tol, mode=mode, polish_m=polish_m,
                                              precision=X.FP64 if precision is None
                                              else precision,
                                              batch_max_n=nmax), info)
    torch.cuda.synchronize()
    return [cpu(s.x) for s in specs], X.infos_to_numpy(info)


def oracle_guess(X, H, T, mt, bases, i, mode, warm):
    """The oracle's projection of target mt on the GPU's own basis i (isolates the projection)."""
    k = bases.header(i)["k"]
    V = cpu(bases.V(i))[:, :k + 1]
    Hb = cpu(bases.Hbar(i))[:k + 1, :k]
    A = oracle.Operator(H, 1.0 / T, 0.5, mt)
    b = oracle.rhs(A, mt)
    x0, _, st = oracle.project(A, b, V, Hb, mode=getattr(oracle, MODES[mode]),
                               x_base=mt if warm else None)
    return A, b, x0, st


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("warm", [False, True])
@pytest.mark.parametrize("H,m", [(28, 30), (37, 20), (64, 40), (100, 50), (128, 60)])
def test_split_guess_matches_oracle_and_in_launch(X, mode, warm, H, m):
    """x0 of the split projection equals the oracle's projection on the GPU basis to 1e-9 and the
    in-launch projection's to 1e-10 (only the order of the row sums differs); status, basis_dim
    and guess residual agree."""
    T = 100
    ms, _ = blob_pair(H, seed=11 * H)
    mts = [blob_pair(H, seed=11 * H, jitter=0.6 + 0.5 * i)[1] for i in range(3)]
    bases = seed_basis(X, H, T, m, ms)
    xs, inf = project(X, H, T, m, bases, mts, warm, 0, mode)
    xf, inff = project(X, H, T, m, bases, mts, warm, -1, mode)
    k = bases.header(0)["k"]
    for i, mt in enumerate(mts):
        A, b, x0o, st = oracle_guess(X, H, T, mt, bases, 0, mode, warm)
        assert st == oracle.OK and inf[i]["status"] == X.OK and inf[i]["basis_dim"] == k
        assert inf[i]["iters"] == 0
        assert np.abs(xs[i] - x0o).max() <= 1e-9 * np.abs(x0o).max(), i
        assert np.abs(xs[i] - xf[i]).max() <= 1e-10 * np.abs(xf[i]).max(), i
        assert abs(inf[i]["guess_res"] - oracle.residual(A, b, x0o)) <= 1e-9 * inf[i]["guess_res"]
        assert abs(inf[i]["guess_res"] - inff[i]["guess_res"]) <= 1e-9 * inff[i]["guess_res"]


@pytest.mark.parametrize("H,tiles", [(100, 1), (100, 2), (100, 3), (100, 5), (100, 0),
                                     (37, 4), (128, 7)])
def test_split_ragged_tiles(X, H, tiles):
    """Tile counts that leave a short last tile (n = 10000 over 3 tiles of 3584 rows, n = 1369
    over 3 tiles of 512, n = 16384 over 7 tiles of 2560): the guess is the oracle's, and the
    polished solve converges with the in-launch path's iteration counts (within one)."""
    T, m = 100, 40
    ms, _ = blob_pair(H, seed=5 + H)
    mts = [blob_pair(H, seed=5 + H, jitter=0.8 + 0.4 * i)[1] for i in range(2)]
    bases = seed_basis(X, H, T, m, ms)
    xs, inf = project(X, H, T, m, bases, mts, True, tiles)
    for i, mt in enumerate(mts):
        _, _, x0o, _ = oracle_guess(X, H, T, mt, bases, 0, "target_galerkin", True)
        assert np.abs(xs[i] - x0o).max() <= 1e-9 * np.abs(x0o).max(), i
    xp, infp = project(X, H, T, m, bases, mts, True, tiles, tol=1e-8, polish_m=10)
    xf, inff = project(X, H, T, m, bases, mts, True, -1, tol=1e-8, polish_m=10)
    for i, mt in enumerate(mts):
        A = oracle.Operator(H, 1.0 / T, 0.5, mt)
        b = oracle.rhs(A, mt)
        assert infp[i]["status"] == X.OK and oracle.residual(A, b, xp[i]) <= 1e-8
        assert abs(int(infp[i]["iters"]) - int(inff[i]["iters"])) <= 1


def test_split_uneven_batch_of_several_bases(X):
    """Three seeds (sides 100, 64, 32) and three targets of each in one call, largest first: every
    target's guess residual is the oracle's projection on its own GPU basis, and the polish meets
    the tolerance (oracle residual) within the Varah bound of the direct solution."""
    import torch
    T, m = 100, 30
    sides = [100, 64, 32]
    nmax = sides[0] ** 2
    ctx = X.Context(nmax, m, 3)
    seeds, mss = [], []
    for H in sides:
        ms, _ = blob_pair(H, seed=300 + H)
        mss.append(ms)
        seeds.append(X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=zeros(H * H), x=zeros(H * H)))
    d = X.pack_systems(seeds, dev())
    ctx.build_rhs(d, 3)
    bases = X.Bases(3, [H * H for H in sides], m)
    si = ctx.new_infos(3)
    ctx.seed_build(d, 3, bases.ptrs, X.Context.params(m, batch_max_n=nmax), si)
    torch.cuda.synchronize()
    Hs, mts, ids = [], [], []
    for bi, H in enumerate(sides):
        for t in range(3):
            Hs.append(H)
            mts.append(blob_pair(H, seed=300 + H, jitter=0.7 + 0.5 * t)[1])
            ids.append(bi)
    xs, inf = project(X, None, T, m, bases, mts, False, 0, tol=1e-8, Hs=Hs, basis_ids=ids)
    for i, (H, mt, bi) in enumerate(zip(Hs, mts, ids)):
        A, b, x0o, st = oracle_guess(X, H, T, mt, bases, bi, "target_galerkin", False)
        assert inf[i]["status"] == X.OK and inf[i]["basis_dim"] == bases.header(bi)["k"]
        assert abs(inf[i]["guess_res"] - oracle.residual(A, b, x0o)) <= 1e-9 * inf[i]["guess_res"]
        assert oracle.residual(A, b, xs[i]) <= 1e-8
        xd, _ = oracle.banded_solve(A, b)
        rinf = np.abs(b - oracle.apply(A, xs[i])).max()
        assert np.abs(xs[i] - xd).max() <= A.dt * rinf * (1 + 1e-6) + 1e-13 * np.abs(xd).max()


def test_split_more_targets_than_slots(X):
    """3000 targets of 16 x 16 (one tile each, 2048 partial slots): workgroups take several
    targets each, reusing their slot; every guess equals the in-launch projection's."""
    T, m, H, N = 100, 20, 16, 3000
    ms, _ = blob_pair(H, seed=9)
    bases = seed_basis(X, H, T, m, ms)
    rng = np.random.default_rng(4)
    base_t = blob_pair(H, seed=9, jitter=1.0)[1]
    mts = [np.clip(base_t + 0.05 * rng.normal(size=H * H), 0.0, None) for _ in range(N)]
    xs, inf = project(X, H, T, m, bases, mts, False, 0)
    xf, inff = project(X, H, T, m, bases, mts, False, -1)
    assert np.all(inf["status"] == X.OK) and np.all(inf["basis_dim"] == bases.header(0)["k"])
    scale = max(np.abs(x).max() for x in xf)
    assert max(np.abs(a - b).max() for a, b in zip(xs, xf)) <= 1e-10 * scale
    assert np.abs(inf["guess_res"] - inff["guess_res"]).max() <= 1e-9 * inff["guess_res"].max()


def test_split_chain_matches_oracle_and_graph_replays(X):
    """A chain of two sizes (sides 32 and 20, targets projected in launches of their own) against
    the oracle chain; then captured as a HIP graph and replayed three times with eager chains
    in between: every replay reproduces the eager states and infos."""
    import torch
    from oracle.chain import run_chain
    from paper_2511_17634_amd.driver import Batch, Group
    T, m = 8, 20
    groups = []
    for H, C, N in ((32, 2, 2), (20, 1, 3)):
        seed = np.stack([blob_pair(H, seed=80 + H + c)[0] for c in range(C)])
        tg = np.stack([np.stack([blob_pair(H, seed=80 + H + c, jitter=0.5 + t)[1]
                                 for c in range(C)]) for t in range(N)])
        groups.append(Group(H, seed, tg))
    b = Batch(groups, T, m)
    b.ctx.set_projection_split(0)
    b.run()
    s_inf, t_inf = b.all_infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.all(b.verify_last() <= 1e-8 * (1 + 1e-6))
    for gi, gr in enumerate(b.groups):
        ms_g, mt_g = (cpu(v) for v in b.group_states(gi))
        for c in range(gr.C):
            ms_o, mt_o, _ = run_chain(gr.seed_m0[c], gr.target_m0[:, c], gr.H, T, m)
            bound = T * 1e-8 * max(np.linalg.norm(gr.seed_m0[c]),
                                   np.linalg.norm(gr.target_m0[:, c], axis=1).max())
            assert np.abs(ms_g[c] - ms_o).max() <= bound
            assert np.abs(mt_g[:, c] - mt_o).max() <= bound
    ref_s, ref_t = (cpu(v).copy() for v in b.state())
    ref_si, ref_ti = s_inf.copy(), t_inf.copy()
    b.capture()
    for rep in range(3):
        b.replay()
        torch.cuda.synchronize()
        s, t = (cpu(v) for v in b.state())
        si, ti = b.all_infos()
        assert np.array_equal(s, ref_s) and np.array_equal(t, ref_t), rep
        assert np.array_equal(si, ref_si) and np.array_equal(ti, ref_ti), rep
        b.run()
        torch.cuda.synchronize()
        assert np.array_equal(cpu(b.state()[1]), ref_t)


def test_split_repeated_calls_are_bitwise_equal(X):
    """One context, two sets of 64 targets of 64 x 64 projected alternately six times over 8 tiles
    per target (a target's tiles run on different XCDs, and every call reuses the same partial
    slots): each call reproduces its set's first guesses bit for bit."""
    import torch
    T, m, H, N = 100, 40, 64, 64
    n = H * H
    ms, _ = blob_pair(H, seed=21)
    bases = seed_basis(X, H, T, m, ms)
    ctx = X.Context(n, m, N)
    ctx.set_projection_split(8)
    sets = []
    for s in range(2):
        specs = [X.SystemSpec(H, 1.0 / T, 0.5,
                              t64(blob_pair(H, seed=21, jitter=0.5 + 0.02 * i + 0.3 * s)[1]),
                              b=zeros(n), x=zeros(n)) for i in range(N)]
        d = X.pack_systems(specs, dev())
        ctx.build_rhs(d, N)
        sets.append((specs, d))
    P = X.Context.params(m, tol=1e300, batch_max_n=n)
    first = [None, None]
    for call in range(6):
        specs, d = sets[call % 2]
        info = ctx.new_infos(N)
        ctx.target_project_solve(d, N, bases.count, bases.ptrs, P, info)
        torch.cuda.synchronize()
        xs = np.stack([cpu(s.x) for s in specs])
        inf = X.infos_to_numpy(info)
        assert np.all(inf["status"] == X.OK) and np.all(inf["basis_dim"] == bases.header(0)["k"])
        if first[call % 2] is None:
            first[call % 2] = xs
        else:
            assert np.array_equal(xs, first[call % 2]), call
