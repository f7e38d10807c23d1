"""GPU parity of batching: systems of uneven sizes in one launch (each on the code path of its
own size class), the work queue with fewer workgroups than systems and across consecutive
launches, per-target basis selection, the polish restart length, the multi-size timestep chain
against the oracle, HIP-graph replays against the eager chain, and the launch autotuner.  Every
call goes through the C ABI."""
import numpy as np
import pytest

import oracle
from gpu_util import blob_pair, cpu, dev, t64

pytestmark = pytest.mark.gpu

# grid sides spanning the three size classes (<= 1024, <= 4096, <= 16384 unknowns) and both
# class boundaries, largest first
SIZES = [128, 100, 64, 45, 32, 20]


@pytest.fixture(scope="module")
def X():
    from paper_2511_17634_amd import xkp
    xkp.load()
    return xkp


def zeros(n):
    import torch
    return torch.zeros(n, dtype=torch.float64, device=dev())


def seeds_batch(X, sizes, T, m, key=0):
    """Seed systems of the given sizes, right-hand sides built on the GPU."""
    specs, mss = [], []
    for H in sizes:
        ms, _ = blob_pair(H, seed=key + H)
        mss.append(ms)
        specs.append(X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=zeros(H * H), x=zeros(H * H)))
    return specs, mss


def run_seeds(X, specs, m, max_n, tol=1e-8):
    import torch
    ctx = X.Context(max_n, m, len(specs))
    d = X.pack_systems(specs, dev())
    ctx.build_rhs(d, len(specs))
    bases = X.Bases(len(specs), [s.H * s.H for s in specs], m)
    info = ctx.new_infos(len(specs))
    ctx.seed_build(d, len(specs), bases.ptrs, X.Context.params(m, tol=tol), info)
    torch.cuda.synchronize()
    return bases, X.infos_to_numpy(info)


def test_uneven_seed_batch_matches_single_calls_and_oracle(X):
    T, m = 100, 30
    specs, mss = seeds_batch(X, SIZES, T, m)
    bases, infos = run_seeds(X, specs, m, max(H * H for H in SIZES))
    for i, H in enumerate(SIZES):
        n = H * H
        # the same seed alone, in a context sized for it (a leaner kernel)
        one, _ = seeds_batch(X, [H], T, m)
        b1, inf1 = run_seeds(X, one, m, n)
        x, x1 = cpu(specs[i].x), cpu(one[0].x)
        assert np.abs(x - x1).max() <= 1e-13 * np.abs(x1).max(), H
        assert infos[i]["iters"] == inf1[0]["iters"] and infos[i]["status"] == X.OK
        k = bases.header(i)["k"]
        assert k == b1.header(0)["k"] and bases.header(i)["n"] == n
        assert np.abs(cpu(bases.V(i))[:, :k + 1] - cpu(b1.V(0))[:, :k + 1]).max() <= 1e-12
        # and the oracle
        A = oracle.Operator(H, 1.0 / T, 0.5, mss[i])
        bo = oracle.rhs(A, mss[i])
        ro = oracle.gmres(A, bo, m=m, tol=1e-8)
        assert oracle.residual(A, bo, x) <= 1e-8
        assert abs(int(infos[i]["iters"]) - ro.iters) <= max(2, 0.05 * ro.iters), H


def test_uneven_targets_per_basis_projection_and_polish(X):
    """Twelve targets of four sizes, two channels each, interleaved, each projected on the basis
    of its own size and channel."""
    import torch
    T, m = 100, 30
    sizes = [100, 64, 32, 20]
    seed_specs, seed_ms = [], []
    for H in sizes:
        for ch in range(2):
            ms, _ = blob_pair(H, seed=10 * H + ch)
            seed_ms.append(ms)
            seed_specs.append(X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=zeros(H * H),
                                           x=zeros(H * H)))
    nmax = max(sizes) ** 2
    bases, sinf = run_seeds(X, seed_specs, m, nmax)
    assert np.all(sinf["status"] == X.OK)
    tg, specs = [], []
    for rep in range(2):
        for bi, H in enumerate([h for h in sizes for _ in range(2)]):
            _, mt = blob_pair(H, seed=10 * H + bi % 2, jitter=1.0 + rep)
            tg.append((H, bi, mt))
    order = np.random.default_rng(3).permutation(len(tg))
    tg = [tg[i] for i in order]
    for H, bi, mt in tg:
        specs.append(X.SystemSpec(H, 1.0 / T, 0.5, t64(mt), b=zeros(H * H), x=zeros(H * H),
                                  basis_id=bi))
    ctx = X.Context(nmax, m, len(specs))
    d = X.pack_systems(specs, dev())
    ctx.build_rhs(d, len(specs))
    info = ctx.new_infos(len(specs))
    # guess only: the projection of every target
    ctx.target_project_solve(d, len(specs), len(seed_specs), bases.ptrs,
                             X.Context.params(m, tol=1e300), info)
    torch.cuda.synchronize()
    inf = X.infos_to_numpy(info)
    x0s = []
    for i, (H, bi, mt) in enumerate(tg):
        At = oracle.Operator(H, 1.0 / T, 0.5, mt)
        bt = oracle.rhs(At, mt)
        k = bases.header(bi)["k"]
        x0o, _, st = oracle.project(At, bt, cpu(bases.V(bi))[:, :k + 1],
                                    cpu(bases.Hbar(bi))[:k + 1, :k])
        assert inf[i]["status"] == X.OK and inf[i]["basis_dim"] == k and inf[i]["iters"] == 0
        assert np.abs(cpu(specs[i].x) - x0o).max() <= 1e-9 * np.abs(x0o).max(), (H, bi)
        x0s.append(x0o)
    # full solve
    ctx.target_project_solve(d, len(specs), len(seed_specs), bases.ptrs,
                             X.Context.params(m), info)
    torch.cuda.synchronize()
    inf = X.infos_to_numpy(info)
    for i, (H, bi, mt) in enumerate(tg):
        At = oracle.Operator(H, 1.0 / T, 0.5, mt)
        bt = oracle.rhs(At, mt)
        ro = oracle.gmres(At, bt, x0=x0s[i], m=m)
        assert inf[i]["status"] == X.OK and inf[i]["res_true"] <= 1e-8
        assert oracle.residual(At, bt, cpu(specs[i].x)) <= 1e-8
        assert abs(int(inf[i]["iters"]) - ro.iters) <= max(2, 0.05 * ro.iters), (H, bi)


def test_queue_with_fewer_workgroups_and_consecutive_launches(X):
    """Seven plain solves through a context with two workspace slots (each workgroup takes
    several systems from the queue), then a three-system launch on the same counters; every
    result equals the system solved alone."""
    import torch
    H, T, m = 28, 50, 20
    mts = [blob_pair(H, seed=40 + i, jitter=1.0)[1] for i in range(7)]
    ctx = X.Context(H * H, m, 2)
    P = X.Context.params(m, mode="none")

    def solve(ctx, idx):
        specs = [X.SystemSpec(H, 1.0 / T, 0.5, t64(mts[i]), b=zeros(H * H), x=zeros(H * H))
                 for i in idx]
        d = X.pack_systems(specs, dev())
        ctx.build_rhs(d, len(specs))
        info = ctx.new_infos(len(specs))
        ctx.target_project_solve(d, len(specs), 0, None, P, info)
        torch.cuda.synchronize()
        return [cpu(s.x) for s in specs], X.infos_to_numpy(info)

    xs, inf = solve(ctx, range(7))
    xs2, inf2 = solve(ctx, [6, 0, 3])
    for j, i in enumerate(range(7)):
        x1, i1 = solve(X.Context(H * H, m, 1), [i])
        assert np.array_equal(xs[j], x1[0]) and inf[j]["iters"] == i1[0]["iters"]
    for j, i in enumerate([6, 0, 3]):
        assert np.array_equal(xs2[j], xs[i]) and inf2[j]["iters"] == inf[i]["iters"]
    assert np.all(inf["status"] == X.OK) and np.all(inf2["status"] == X.OK)


def test_basis_mismatch_and_range_give_einval(X):
    import torch
    T, m = 100, 20
    specs, _ = seeds_batch(X, [32, 24], T, m)
    bases, _ = run_seeds(X, specs, m, 32 * 32)
    _, mt = blob_pair(32, seed=5)
    tspecs = [X.SystemSpec(32, 0.01, 0.5, t64(mt), b=zeros(1024), x=zeros(1024), basis_id=0),
              X.SystemSpec(32, 0.01, 0.5, t64(mt), b=zeros(1024), x=zeros(1024), basis_id=1),
              X.SystemSpec(32, 0.01, 0.5, t64(mt), b=zeros(1024), x=zeros(1024), basis_id=2),
              X.SystemSpec(32, 0.01, 0.5, t64(mt), b=zeros(1024), x=zeros(1024), basis_id=-1)]
    ctx = X.Context(1024, m, 4)
    d = X.pack_systems(tspecs, dev())
    ctx.build_rhs(d, 4)
    info = ctx.new_infos(4)
    ctx.target_project_solve(d, 4, 2, bases.ptrs, X.Context.params(m), info)
    torch.cuda.synchronize()
    inf = X.infos_to_numpy(info)
    assert inf[0]["status"] == X.OK and inf[0]["res_true"] <= 1e-8
    assert list(inf["status"][1:]) == [X.EINVAL] * 3


def test_polish_restart_length(X):
    """polish_m sets the targets' restart length (the seed basis keeps m columns): the
    iteration count follows the oracle's GMRES(polish_m) from the same projected guess."""
    import torch
    H, T, m, pm = 64, 100, 40, 12
    ms, mt = blob_pair(H, seed=8, jitter=2.0)
    specs = [X.SystemSpec(H, 1.0 / T, 0.5, t64(ms), b=zeros(H * H), x=zeros(H * H))]
    bases, _ = run_seeds(X, specs, m, H * H)
    ts = [X.SystemSpec(H, 1.0 / T, 0.5, t64(mt), b=zeros(H * H), x=zeros(H * H))]
    ctx = X.Context(H * H, m, 1)
    d = X.pack_systems(ts, dev())
    ctx.build_rhs(d, 1)
    info = ctx.new_infos(1)
    ctx.target_project_solve(d, 1, 1, bases.ptrs, X.Context.params(m, polish_m=pm), info)
    torch.cuda.synchronize()
    inf = X.infos_to_numpy(info)[0]
    At = oracle.Operator(H, 1.0 / T, 0.5, mt)
    bt = oracle.rhs(At, mt)
    k = bases.header(0)["k"]
    x0, _, _ = oracle.project(At, bt, cpu(bases.V(0))[:, :k + 1], cpu(bases.Hbar(0))[:k + 1, :k])
    ro = oracle.gmres(At, bt, x0=x0, m=pm)
    assert inf["status"] == X.OK and inf["restarts"] >= 1 and inf["basis_dim"] == k
    assert abs(int(inf["iters"]) - ro.iters) <= max(2, 0.05 * ro.iters)
    assert oracle.residual(At, bt, cpu(ts[0].x)) <= 1e-8


def uneven_batch(T, m, **kw):
    from paper_2511_17634_amd.driver import Batch, Group
    groups = []
    for H, C, N in ((32, 2, 2), (20, 1, 3)):
        seed = np.stack([blob_pair(H, seed=60 + H + c)[0] for c in range(C)])
        tg = np.stack([np.stack([blob_pair(H, seed=60 + H + c, jitter=0.5 + t)[1]
                                 for c in range(C)]) for t in range(N)])
        groups.append(Group(H, seed, tg))
    return Batch(groups, T, m, **kw), groups


def test_uneven_chain_matches_oracle(X):
    T, m = 12, 20
    b, groups = uneven_batch(T, m)
    b.run()
    s_inf, t_inf = b.all_infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.all(t_inf["res_true"] <= 1e-8)
    assert np.all(b.verify_last() <= 1e-8 * (1 + 1e-6))
    from oracle.chain import run_chain
    for gi, gr in enumerate(b.groups):
        ms_g, mt_g = b.group_states(gi)
        ms_g, mt_g = cpu(ms_g), cpu(mt_g)
        for c in range(gr.C):
            ms_o, mt_o, st = run_chain(gr.seed_m0[c], gr.target_m0[:, c], gr.H, T, m)
            bound = T * 1e-8 * max(np.linalg.norm(gr.seed_m0[c]),
                                   np.linalg.norm(gr.target_m0[:, c], axis=1).max())
            assert np.abs(ms_g[c] - ms_o).max() <= bound
            assert np.abs(mt_g[:, c] - mt_o).max() <= bound


def test_graph_replays_match_eager_chain(X):
    """The chain captured once as a HIP graph and replayed three times, with eager chains and
    host synchronisations in between: every replay reproduces the eager states and infos."""
    import torch
    T, m = 8, 20
    b, _ = uneven_batch(T, m)
    b.run()
    ref_s, ref_t = (cpu(v).copy() for v in b.state())
    ref_si, ref_ti = (a.copy() for a in b.all_infos())
    b.capture()
    for rep in range(3):
        b.replay()
        torch.cuda.synchronize()
        s, t = (cpu(v) for v in b.state())
        si, ti = b.all_infos()
        assert np.array_equal(s, ref_s) and np.array_equal(t, ref_t), rep
        assert np.array_equal(si, ref_si) and np.array_equal(ti, ref_ti), rep
        b.run()                                  # eager work between the replays
        torch.cuda.synchronize()
        assert np.array_equal(cpu(b.state()[1]), ref_t)


def test_autotune_picks_a_converging_candidate(X):
    from paper_2511_17634_amd.driver import Chain
    H, T, m = 64, 20, 40
    s0, _ = blob_pair(H, seed=90)
    t0 = np.stack([blob_pair(H, seed=90, jitter=1.0 + 0.5 * i)[1] for i in range(6)])
    ch = Chain(H, T, m, s0, t0)
    t = ch.autotune(steps=2)
    assert t.polish_m in (6, 8, 9, 10, 20, 30, 40) and t.wg_per_cu >= 1 and t.n_tried >= 7
    assert 0 < t.ms_best <= t.ms_default * 1.000001
    assert ch.params.polish_m == t.polish_m
    ch.run()
    _, ti = ch.all_infos()
    assert np.all(ti["status"] == X.OK) and np.all(ti["res_true"] <= 1e-8)
    assert np.all(ch.verify_last() <= 1e-8 * (1 + 1e-6))


def test_seed_autotune_keeps_results(X):
    """xkp_autotune_seeds on the seeds of an uneven batch: the chosen workgroup size leaves the
    seed iterations within one of the default launch's and the chain still verifies."""
    T, m = 6, 20
    b, groups = uneven_batch(T, m)
    b.run()
    s_ref, _ = b.all_infos()
    t = b.autotune(steps=2)
    st = b.seed_tuning
    assert st is not None and st.waves in (4, 8, 16) and st.wg_per_cu >= 1
    assert st.n_tried >= 2 and 0 < st.ms_best <= st.ms_default * 1.000001
    assert st.polish_m == m and t.polish_m in (6, 8, 9, 10, 15, 20)
    b.params.polish_m = 0          # compare the seeds under the restart length of the reference
    b.run()
    s_inf, t_inf = b.all_infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.abs(s_inf["iters"].astype(int) - s_ref["iters"].astype(int)).max() <= 1
    assert np.all(b.verify_last() <= 1e-8 * (1 + 1e-6))


def test_autotune_cache_reuses_choices(X, tmp_path):
    """Batch.autotune with a cache file: the first call tunes and stores the choices under the
    batch's key, a second batch of the same workload takes them from the file without timing,
    with the same launch choices, and its chain still verifies; a batch of another m is a miss."""
    import json
    T, m = 6, 20
    path = str(tmp_path / "tuning.json")
    b1, _ = uneven_batch(T, m)
    t1 = b1.autotune(steps=2, cache=path)
    assert not b1.tuned_from_cache
    rec1 = b1.tuning_record(t1)
    data = json.load(open(path))
    assert list(data) == [b1.tuning_key()] and data[b1.tuning_key()] == rec1
    del b1
    b2, _ = uneven_batch(T, m)
    t2 = b2.autotune(steps=2, cache=path)
    assert b2.tuned_from_cache and b2.tuning_record(t2) == rec1
    assert t2.n_tried == 0 and b2.params.polish_m == rec1["polish_m"]
    b2.run()
    s_inf, t_inf = b2.all_infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.all(b2.verify_last() <= 1e-8 * (1 + 1e-6))
    del b2
    b3, _ = uneven_batch(T, 16)
    assert b3.tuning_key() not in data
    b3.autotune(steps=2, cache=path)
    assert not b3.tuned_from_cache and len(json.load(open(path))) == 2


def test_uneven_mixed_precision_chain(X):
    """Mixed precision over an uneven two-size, two-channel batch: every solve meets the FP64
    tolerance and the states stay within the chain bound of the FP64 oracle."""
    T, m = 8, 20
    b, groups = uneven_batch(T, m, precision=X.MIXED)
    b.run()
    s_inf, t_inf = b.all_infos()
    assert np.all(s_inf["status"] == X.OK) and np.all(t_inf["status"] == X.OK)
    assert np.all(t_inf["res_true"] <= 1e-8)
    assert np.all(b.verify_last() <= 1e-8 * (1 + 1e-6))
    from oracle.chain import run_chain
    for gi, gr in enumerate(b.groups):
        _, mt_g = b.group_states(gi)
        mt_g = cpu(mt_g)
        for c in range(gr.C):
            _, mt_o, _ = run_chain(gr.seed_m0[c], gr.target_m0[:, c], gr.H, T, m)
            bound = T * 1e-8 * np.linalg.norm(gr.target_m0[:, c], axis=1).max()
            assert np.abs(mt_g[:, c] - mt_o).max() <= bound
