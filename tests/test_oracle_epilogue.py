"""Pins of the oracle's score and probability-flow step: exactness on linear fields, second-order
convergence on a Gaussian log-density (which separates the 2h divisor from a divisor of 2), the
zero-padding boundary rows, the flow's sign and scale, and the drift term."""
import numpy as np

from oracle import epilogue as E


def grid(H):
    h = 1.0 / H
    i, j = np.meshgrid(np.arange(H), np.arange(H), indexing="ij")
    return (i * h).reshape(-1), (j * h).reshape(-1)


def test_linear_field_is_exact_inside():
    H = 12
    x, y = grid(H)
    m = 3.0 * x - 2.0 * y + 0.5
    sx, sy = E.score(H, m)
    inner = np.zeros((H, H), dtype=bool)
    inner[1:-1, 1:-1] = True
    inner = inner.reshape(-1)
    assert np.allclose(sx[inner], 3.0, rtol=0, atol=1e-12)
    assert np.allclose(sy[inner], -2.0, rtol=0, atol=1e-12)


def test_zero_padding_rows():
    """On the first and last grid lines the missing neighbour counts as zero."""
    H = 6
    m = np.arange(H * H, dtype=np.float64) + 1.0
    M = m.reshape(H, H)
    sx, sy = E.score(H, m)
    SX, SY = sx.reshape(H, H), sy.reshape(H, H)
    h = 1.0 / H
    assert np.allclose(SX[0], (M[1] - 0.0) / (2 * h))
    assert np.allclose(SX[-1], (0.0 - M[-2]) / (2 * h))
    assert np.allclose(SY[:, 0], (M[:, 1] - 0.0) / (2 * h))
    assert np.allclose(SY[:, -1], (0.0 - M[:, -2]) / (2 * h))


def test_gaussian_log_density_converges_at_second_order():
    """m = log of a Gaussian: grad m = -(x - mu) / sigma^2 exactly; the interior error of the
    central difference falls by 4 when h halves."""
    errs = []
    for H in (32, 64, 128):
        x, y = grid(H)
        mu, s2 = 0.5, 0.02
        m = -((x - mu) ** 2 + (y - mu) ** 2) / (2 * s2) + np.sin(3 * x) * np.cos(2 * y)
        gx = -(x - mu) / s2 + 3 * np.cos(3 * x) * np.cos(2 * y)
        gy = -(y - mu) / s2 - 2 * np.sin(3 * x) * np.sin(2 * y)
        sx, sy = E.score(H, m)
        inner = np.zeros((H, H), dtype=bool)
        inner[1:-1, 1:-1] = True
        inner = inner.reshape(-1)
        errs.append(max(np.abs(sx - gx)[inner].max(), np.abs(sy - gy)[inner].max()))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


def test_flow_sign_scale_and_drift():
    """With a constant score s the displacement after T steps of dt = 1/T is -g^2/2 s; a
    constant drift adds f."""
    H, T, g = 10, 100, 0.5
    x, y = grid(H)
    m = 4.0 * x + 1.0 * y
    inner = np.zeros((H, H), dtype=bool)
    inner[1:-1, 1:-1] = True
    inner = inner.reshape(-1)
    d = np.zeros((2, H * H))
    for _ in range(T):
        d = E.flow_step(d, H, m, g, 1.0 / T)
    assert np.allclose(d[0][inner], -0.5 * g * g * 4.0, rtol=1e-12, atol=0)
    assert np.allclose(d[1][inner], -0.5 * g * g * 1.0, rtol=1e-12, atol=0)
    d2 = E.flow_step(np.zeros((2, H * H)), H, m, g, 0.1, fx=np.full(H * H, 2.0),
                     fy=np.full(H * H, -1.0))
    assert np.allclose(d2[0][inner], (2.0 - 0.5 * g * g * 4.0) * 0.1)
    assert np.allclose(d2[1][inner], (-1.0 - 0.5 * g * g * 1.0) * 0.1)
