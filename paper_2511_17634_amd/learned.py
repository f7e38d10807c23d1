"""Learned starting guess: training data from the method's own solves, training with the
library's network kernels, and the regression target.

For every target t and timestep n the best guess inside the seed subspace is V_n alpha*_{t,n},
alpha* = V_n^T x*_{t,n} (the 2-norm fit to the target's converged solution).  The network learns
it in residual coordinates, zeta*_{t,n} = Hbar_n alpha*_{t,n} / beta_n (Hbar_n, beta_n: the
seed's kept Arnoldi cycle at step n), from the target's initial image and n: since
A_seed V_n = V_{n,k+1} Hbar_n, an error in zeta is (for targets close to the seed) the error of
the guess's relative residual, so the squared loss measures what the guess is judged by, and
the solve recovers alpha by the Hessenberg least-squares problem.  zeta* is order one (its first
entry is about ||b_t|| / ||b_seed||), so no further scaling is applied.

The correction variant learns zeta* - zeta_P instead, zeta_P the coordinates of the target's
projected guess on the same basis (xkp_learned_correction_solve adds the prediction to the
projection and keeps it only where it lowers the guess's residual).
"""
from __future__ import annotations

import numpy as np

from . import xkp
from .driver import Batch, Group


def init_params(k, rng):
    """Initial FP32 parameters of a network with k outputs (the layout of xkp_cnn_param_count):
    normal weights with variance 2 / fan-in, zero biases."""
    shapes = [(16, 9), (16,), (32, 144), (32,), (64, 288), (64,), (k, 96), (k,)]
    parts = []
    for s in shapes:
        if len(s) == 1:
            parts.append(np.zeros(s))
        else:
            parts.append(rng.standard_normal(s).reshape(-1) * np.sqrt(2.0 / s[1]))
    return np.concatenate(parts).astype(np.float32)


def generate(seed_m0, target_m0, T, m, device=0, with_projection=False):
    """Run the chain (seeds with kept bases, targets by plain GMRES to 1e-8) and collect
    zeta*[t][i] = Hbar_{t+1} V_{t+1}^T x*_{i,t+1} / beta_{t+1} (float64 device tensor
    (T, N, m + 1)).  with_projection: also the same coordinates of each target's
    target-Galerkin guess x0_P on the same basis (the correction target is zeta* - zeta_P);
    returns (zeta*, zeta_P, ok) then, else (zeta*, ok)."""
    import torch
    gr = Group(64, np.asarray(seed_m0).reshape(1, -1), np.asarray(target_m0).reshape(-1, 1, 4096))
    b = Batch([gr], T, m, method="plain", with_seeds=True, pipeline=False, device=device)
    alpha = torch.empty((T, b.N, m + 1), dtype=torch.float64, device=b.dev)
    alpha_p = torch.empty_like(alpha) if with_projection else None
    if with_projection:
        # the projected guess of each target into a scratch iterate: the polish stops before
        # its first step (tolerance 1e300)
        scratch = torch.zeros_like(b.mt[0])
        pdesc = [b._desc(b.tgt_sys, b.mt, b.bt, par, x_from=scratch) for par in (0, 1)]
        pparams = xkp.Context.params(m, tol=1e300, mode=xkp.TARGET_GALERKIN)
        pinf = b.ctx.new_infos(b.N)

    def hook(par, bases, t):
        b.ctx.basis_coeffs(b.tgt_desc[par], b.N, b.S, bases, m + 1, alpha[t], kind=1)
        if with_projection:
            b.ctx.target_project_solve(pdesc[par], b.N, b.S, bases, pparams, pinf)
            b.ctx.basis_coeffs(pdesc[par], b.N, b.S, bases, m + 1, alpha_p[t], kind=1)

    b.reset()
    for t in range(T):
        b.step(after_targets=lambda par, bases, t=t: hook(par, bases, t))
    s_inf, t_inf = b.all_infos()
    ok = bool((s_inf["status"] == 0).all() and (t_inf["status"] == 0).all())
    torch.cuda.synchronize()
    if with_projection:
        return alpha, alpha_p, ok
    return alpha, ok


def train(net, images, alpha_star, epochs, batch, lr, seed=0, log=None):
    """Adam on the mean squared error between the network's outputs for (image i, timestep t+1)
    and zeta*[t][i], every (i, t) once per epoch in a random order.  Returns the per-epoch mean
    loss."""
    import torch
    T, N, m = alpha_star.shape
    rows = alpha_star.reshape(T * N, m)
    scale = 1.0
    dev = alpha_star.device
    rng = np.random.default_rng(seed)
    out = torch.empty((batch, net.k), dtype=torch.float32, device=dev)
    hist = []
    for ep in range(epochs):
        perm = rng.permutation(T * N).astype(np.int32)
        img_idx = torch.from_numpy(perm % N).to(dev)
        steps = torch.from_numpy(perm // N + 1).to(dev)
        tidx = torch.from_numpy(perm).to(dev)
        losses = torch.zeros((T * N) // batch, dtype=torch.float32, device=dev)
        for j, s0 in enumerate(range(0, T * N - batch + 1, batch)):
            net.backward(images, steps[s0:s0 + batch], rows, out, image_idx=img_idx[s0:s0 + batch],
                         target_idx=tidx[s0:s0 + batch], target_scale=scale)
            net.adam(lr)
            losses[j:j + 1].copy_(net.loss)
        hist.append(float(losses.mean()))
        if log:
            log(f"epoch {ep}: mean loss {hist[-1]:.5f}")
    return hist


def span_floor(b, picks, steps):
    """The smallest relative residual the seed subspace allows each picked target of a
    one-group chain b at the given timesteps, min_a ||b' - A' V a|| / ||b'|| (A', b' the
    target's operator and right-hand side, V the seed's kept basis at that step): A'V formed by
    the library's operator (xkp_apply, one system per basis column), the least-squares problem
    solved on the GPU in FP64.  Runs one eager chain; returns {(t, i): floor}."""
    import torch
    H = b.groups[0].H
    n = H * H
    out = {}

    def hook(par, bases, t):
        if t not in steps:
            return
        torch.cuda.synchronize(b.dev)
        for i in picks:
            _, off, bid = b.tgt_sys[i]
            j = par * b.S + bid
            k = b.bases.header(j)["k"]
            if k < 1:
                continue
            V = b.bases.V(j)
            W = torch.empty((k, n), dtype=torch.float64, device=b.dev)
            a = np.zeros(k, dtype=xkp.SYSTEM_DTYPE)
            mt = b.mt[par].data_ptr() + 8 * off
            bp = b.bt.data_ptr() + 8 * off
            for c in range(k):
                a[c] = (H, 0, b.dt, b.g, mt, 0, 0, bp, V[:, c].data_ptr(), W[c].data_ptr())
            d = torch.from_numpy(a.view(np.uint8).copy()).to(b.dev)
            b.ctx.apply(d, k)
            rhs = b.bt[off:off + n]
            sol = torch.linalg.lstsq(W.T, rhs[:, None]).solution
            out[(t, i)] = float(torch.linalg.norm(rhs - W.T @ sol[:, 0]) / torch.linalg.norm(rhs))

    b.reset()
    for t in range(b.T):
        b.step(after_targets=lambda par, bases, t=t: hook(par, bases, t))
    torch.cuda.synchronize(b.dev)
    return out
