"""The benchmark's algorithmic byte and flop models (bench.py), against hand counts: GMRES
bytes per Arnoldi step and cycle end, with restarts and two Gram-Schmidt passes; the projected
launch's bytes and FP64 matrix-core products at kept basis dimensions of one and two passes over
the column tiles; the counter figures apply only to the sources they were taken with."""
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


def test_projected_bytes_flops_by_hand():
    n, pm = 4096, 10
    inf = {"basis_dim": np.array([[30, 40, 0]]), "iters": np.array([[12, 10, 7]]),
           "restarts": np.array([[1, 0, 0]])}
    b, f = bench.projected_bytes_flops(n, pm, inf)
    # k = 30: 2 row tiles, 2 column tiles of [A'V | r] (31 columns), one pass over them;
    # k = 40: 3 and 3 tiles, two passes (at most two column tiles each); k = 0: no projection
    proj = 8 * n * (30 + 31 + 1 * 30 + 31 + 30 + 1) + 8 * n * (40 + 41 + 2 * 40 + 41 + 40 + 1)
    assert b == proj + bench.gmres_bytes(n, pm, inf["iters"], inf["restarts"], 1)
    # one 16x16x4 product (2048 flops) per 4 rows and tile pair
    assert f == 2048 * (n // 4) * (2 * 2 + 3 * 3)


def test_traffic_only_for_the_sources_it_was_taken_with(monkeypatch):
    assert bench.traffic_bytes() is not None or bench.csrc_digest() != bench.TRAFFIC["csrc_digest"]
    monkeypatch.setitem(bench.TRAFFIC, "csrc_digest", "0" * 16)
    assert bench.traffic_bytes() is None
    tp = dict(bench.TRAFFIC_PROJECTED, csrc_digest="0" * 16)
    assert bench.traffic_bytes(tp) is None
