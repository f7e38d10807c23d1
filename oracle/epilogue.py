"""Score and probability-flow embedding of a solved log-density (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU baseline use this module; it shares
nothing with the HIP library.

Section 2.3 (after the linear solve): the score is the central difference of the log-density,
  s_x[i, j] = (m[i+1, j] - m[i-1, j]) / (2h),   s_y[i, j] = (m[i, j+1] - m[i, j-1]) / (2h),
with h = 1/H and m = 0 outside the grid (zero padding); the divisor 2h is the reading that
matches the gradient used in the discretised PDE of the same section.
Section 4 (score embedding): the probability-flow ODE dx/dt = f - g^2/2 grad m, discretised with
the same timestep, x^n = x^{n-1} + alpha^{n-1} dt, alpha^{n-1} = f^{n-1} - g^2/2 s^{n-1}; applied per
pixel as a two-component displacement field.
Arrays are flat in the unknown ordering p = i*H + j (i the x index, j the y index).
"""
from __future__ import annotations

import numpy as np


def score(H: int, m) -> tuple[np.ndarray, np.ndarray]:
    """(s_x, s_y), each flat of H*H values, by central differences with zero padding."""
    M = np.zeros((H + 2, H + 2))
    M[1:-1, 1:-1] = np.asarray(m, dtype=np.float64).reshape(H, H)
    h = 1.0 / H
    sx = (M[2:, 1:-1] - M[:-2, 1:-1]) / (2.0 * h)
    sy = (M[1:-1, 2:] - M[1:-1, :-2]) / (2.0 * h)
    return sx.reshape(-1), sy.reshape(-1)


def flow_step(disp, H: int, m, g: float, dt: float, fx=None, fy=None) -> np.ndarray:
    """One explicit Euler step of the probability flow: returns disp + (f - g^2/2 grad m) dt,
    disp being (2, H*H) (x then y components) and f = 0 where not given."""
    sx, sy = score(H, m)
    n = H * H
    fx = np.zeros(n) if fx is None else np.asarray(fx, dtype=np.float64).reshape(-1)
    fy = np.zeros(n) if fy is None else np.asarray(fy, dtype=np.float64).reshape(-1)
    out = np.array(disp, dtype=np.float64).reshape(2, n).copy()
    out[0] += (fx - 0.5 * g * g * sx) * dt
    out[1] += (fy - 0.5 * g * g * sy) * dt
    return out
