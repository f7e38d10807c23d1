"""The benchmark's algorithmic byte and flop models (bench.py), against hand counts: GMRES
bytes per Arnoldi step and cycle end, with restarts, two Gram-Schmidt passes and FP32 element
sizes; a target launch's bytes (per-target inputs and outputs, the seed basis once per launch)
and the projection's flops; the polish launch after the projection launches and their
matrix-core roofline; the scipy matrix of the CPU baseline is the oracle's operator; the
counter figures apply only to the sources they were taken with."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def step_bytes(n, j, passes):
    # Arnoldi step j: v_0..v_j read once per pass, v_{j+1} written, operator u, m~ -> w
    return 8 * passes * n * (j + 1) + 8 * n + 24 * n


def cycle_end_bytes(n, k):
    # x += V_k y, then the true residual
    return 8 * n * k + 48 * n


def test_gmres_bytes_one_cycle():
    n, k = 100, 7
    want = sum(step_bytes(n, j, 1) for j in range(k)) + cycle_end_bytes(n, k)
    assert bench.gmres_bytes(n, 10, [k], [0]) == want


def test_gmres_bytes_restarts_and_passes():
    n, m = 64, 5
    iters, restarts = 2 * m + 3, 2                     # cycles of 5, 5 and 3 steps
    want = 0
    for k in (m, m, 3):
        want += sum(step_bytes(n, j, 2) for j in range(k)) + cycle_end_bytes(n, k)
    assert bench.gmres_bytes(n, m, [iters], [restarts], passes=2) == want
    # a last cycle of zero steps adds no cycle-end bytes
    assert bench.gmres_bytes(n, m, [m], [1]) == bench.gmres_bytes(n, m, [m], [0])


def test_launch_bytes_and_flops_by_hand():
    n, pm = 4096, 10
    inf = {"basis_dim": np.array([[30, 30, 30], [25, 25, 25]]),
           "iters": np.array([[12, 10, 7], [9, 9, 11]]),
           "restarts": np.array([[1, 0, 0], [0, 0, 1]])}
    ns, bids = [n] * 3, [0] * 3
    b = bench.launch_alg_bytes(ns, bids, inf, pm, project=True)
    # per launch: each target's GMRES bytes, m~ and b read and x0 written (24 n), the seed
    # basis V_k read once (8 n k); averaged over the two launches
    want = sum(bench.gmres_bytes(n, pm, [inf["iters"][t, i]], [inf["restarts"][t, i]])
               for t in range(2) for i in range(3))
    want += 2 * 3 * 24 * n + 8 * n * 30 + 8 * n * 25
    assert b == want / 2
    # plain GMRES: the GMRES bytes only; a warm start also reads x_base (8 n)
    assert bench.launch_alg_bytes(ns, bids, inf, pm, project=False) == \
        sum(bench.gmres_bytes(n, pm, inf["iters"][:, i], inf["restarts"][:, i])
            for i in range(3)) / 2
    assert bench.launch_alg_bytes(ns, bids, inf, pm, project=True, warm=True) == \
        want / 2 + 3 * 8 * n
    # two bases (uneven sizes) are each read once per launch
    b2 = bench.launch_alg_bytes([n, n, 1024], [0, 0, 1], inf, pm, project=True)
    assert b2 < b
    # V_k^T [A'V_k | r]: 2 n k (k + 1) flops per target
    assert bench.projection_flops(ns, inf) == (3 * 2 * n * 30 * 31 + 3 * 2 * n * 25 * 26) / 2


def test_mixed_gmres_bytes_use_element_sizes():
    n, m = 1000, 8
    # FP32 basis (4 bytes) and FP32 operator (12 n): the basis part halves, the cycle end keeps
    # its FP64 residual
    k = 5
    want = sum(4 * n * (j + 1) + 4 * n + 12 * n for j in range(k)) + 4 * n * k + 48 * n
    assert bench.gmres_bytes(n, m, [k], [0], sv=4, sop=12) == want


def test_scipy_matrix_is_the_operator(olib):
    import oracle
    rng = np.random.default_rng(3)
    for H in (3, 8, 13):
        A = oracle.Operator(H, 0.01, 0.5, rng.uniform(0, 1, H * H))
        u = rng.normal(size=H * H)
        M = bench.scipy_matrix(A)
        assert np.abs(M @ u - oracle.apply(A, u)).max() <= 1e-12 * np.abs(oracle.apply(A, u)).max()


def test_traffic_only_for_the_sources_it_was_taken_with(monkeypatch):
    monkeypatch.setitem(bench.TRAFFIC, "probe", {"csrc_digest": bench.csrc_digest(),
                                                 "fetch_kib": 1.0, "write_kib": 2.0,
                                                 "fetch_scale": 2.0, "write_scale": 1.0,
                                                 "polish_m": 10})
    assert bench.traffic_bytes("probe", 10) == 1024 * 4
    assert bench.traffic_bytes("probe", 20) is None
    assert bench.traffic_bytes("missing", 10) is None
    monkeypatch.setitem(bench.TRAFFIC["probe"], "csrc_digest", "0" * 16)
    assert bench.traffic_bytes("probe", 10) is None


def test_traffic_only_for_the_launch_choices_it_was_taken_with(monkeypatch):
    """A counter record applies only to the workgroup size, projection placement and (where it
    has one) seed basis dimension m that the leg runs with."""
    rec = {"csrc_digest": bench.csrc_digest(), "fetch_kib": 1.0, "write_kib": 2.0,
           "fetch_scale": 2.0, "write_scale": 1.0, "polish_m": 9, "waves": 8, "split": 0, "m": 30}
    monkeypatch.setitem(bench.TRAFFIC, "probe", rec)
    tuned = {"polish_m": 9, "waves": 8, "wg_per_cu": 1, "split": 0, "seed_waves": 8,
             "seed_wg_per_cu": 1, "seed_rows_per_thread": 0, "m": 30}
    monkeypatch.setitem(bench.TUNED, "probe", dict(tuned))
    assert bench.traffic_bytes("probe", 9) == 1024 * 4
    for k, v in (("m", 40), ("waves", 4), ("split", -1)):
        monkeypatch.setitem(bench.TUNED, "probe", {**tuned, k: v})
        assert bench.traffic_bytes("probe", 9) is None, k
    # any non-negative split is the same placement (launches of their own)
    monkeypatch.setitem(bench.TUNED, "probe", {**tuned, "split": 7})
    assert bench.traffic_bytes("probe", 9) == 1024 * 4
    # a leg without an m of its own matches a record without one
    rec2 = {k: v for k, v in rec.items() if k != "m"}
    monkeypatch.setitem(bench.TRAFFIC, "probe", rec2)
    monkeypatch.setitem(bench.TUNED, "probe", {k: v for k, v in tuned.items() if k != "m"})
    assert bench.traffic_bytes("probe", 9) == 1024 * 4


def test_polish_bytes_and_projection_roofline_by_hand():
    """The polish launch after the projection launches: GMRES bytes plus x0 and b read (16 n)
    per target; the projection launches against the FP64 (or BF16) matrix-core peak."""
    n, pm = 4096, 10
    inf = {"basis_dim": np.array([[30, 30, 30], [25, 25, 25]]),
           "iters": np.array([[12, 10, 7], [9, 9, 11]]),
           "restarts": np.array([[1, 0, 0], [0, 0, 1]])}
    want = sum(bench.gmres_bytes(n, pm, [inf["iters"][t, i]], [inf["restarts"][t, i]])
               for t in range(2) for i in range(3)) + 2 * 3 * 16 * n
    assert bench.polish_alg_bytes([n] * 3, inf, pm) == want / 2
    fl = bench.projection_flops([n] * 3, inf)
    rp = bench.projection_roofline("p", [n] * 3, inf, 2e-5)
    assert rp["bound"] == "mfma" and rp["peak"] == 78.6 and rp["unit"] == "TFLOP/s"
    assert rp["achieved"] == round(fl / 2e-5 / 1e12, 3) and rp["flops_per_launch"] == int(fl)
    assert bench.projection_roofline("p", [n] * 3, inf, 2e-5, mixed=True)["peak"] == 2500.0


def test_paper_context_ratios():
    """The paper's Table 4 reductions are quoted as given, and this run's ratios follow from the
    record: projection over plain GMRES, and the oracle's projection against its banded LU."""
    import bench
    out = {"value": 150.0, "plain_gmres": {"value": 300.0},
           "cpu_baseline": {"per_system_ms_one_core": {"banded_lu_ms": 10.0,
                                                       "projection_polish_ms": 7.5}}}
    ctx = bench.paper_context(out)
    assert ctx["reduction"] == {"32x32": 0.158, "64x64": 0.298, "128x128": 0.437}
    assert ctx["this_run"]["gpu_projection_over_plain_gmres"] == 0.5
    assert ctx["this_run"]["cpu_oracle_projection_vs_banded_lu_reduction"] == 0.25
    assert "cpu_oracle_projection_vs_banded_lu_reduction" not in bench.paper_context(
        {"value": 1.0, "plain_gmres": {"value": 2.0}})["this_run"]


def test_uneven_m_probe_is_skipped_where_m_is_given(monkeypatch):
    """pick_uneven_m times candidates only when several are given, the leg is autotuned and no
    stored record fixes m: a stored m wins, a single candidate is taken as is, and without
    autotuning the workload's own m stays."""
    from types import SimpleNamespace
    cfg = SimpleNamespace(m=40)
    args = SimpleNamespace(uneven_m="30,40,60", no_tune=False, m_probe_steps=10,
                           tuning_cache=None, reorth="auto")
    monkeypatch.setitem(bench.FIXED_TUNING, "uneven_project", {"m": 60})
    assert bench.pick_uneven_m(args, cfg, []) == (60, {})
    monkeypatch.delitem(bench.FIXED_TUNING, "uneven_project")
    assert bench.pick_uneven_m(SimpleNamespace(**{**vars(args), "uneven_m": "30"}), cfg, []) == (30, {})
    assert bench.pick_uneven_m(SimpleNamespace(**{**vars(args), "no_tune": True}), cfg, []) == (40, {})
