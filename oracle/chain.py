"""Timestep chain of the method on the CPU oracle (test infrastructure only).

For n = 1..T (Section 2.3: one implicit solve per timestep, dt = 1/T; one linearisation pass,
m~ = m^{n-1}):
  seed:    A_s m = b_s solved by restarted GMRES from 0 (or from m^{n-1}); the first cycle's
           basis V^n and Hessenberg matrix are kept (Section 3, Phase 1).
  targets: each target is projected onto V^n and the result polished by GMRES to the
           tolerance (Section 3, Phase 2); "plain" runs the same GMRES from x_base instead,
           "direct" uses the banded LU.
  commit:  m^n <- x for every system.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import TARGET_GALERKIN, Operator, accumulate, banded_solve, gmres, project, residual, rhs


@dataclass
class ChainStats:
    seed_iters: list = field(default_factory=list)
    iters: list = field(default_factory=list)          # [step][target] polish / plain iterations
    restarts: list = field(default_factory=list)
    status: list = field(default_factory=list)
    res_true: list = field(default_factory=list)
    guess_res: list = field(default_factory=list)      # [step][target] ||b-Ax0||/||b||
    basis_dim: list = field(default_factory=list)
    picard_iters: list = field(default_factory=list)   # [step][k - 2][target]


def run_chain(seed_m0, target_m0, H, T, m, g=0.5, tol=1e-8, method="project",
              mode=TARGET_GALERKIN, warm=False, steps=None, max_restarts=1000, reorth="auto",
              on_step=None, picard=1):
    """Advance the seed and every target through `steps` (default T) timesteps.

    seed_m0: (n,) initial state of the seed; target_m0: (N, n).  Returns (m_seed, m_targets,
    stats).  With method "plain" or "direct" the seed chain is not solved.  reorth "auto": two
    Gram-Schmidt passes in the seed solves (their first-cycle basis is kept), one in the target
    solves (their basis is discarded); "always": two passes everywhere.  on_step(n, ms, mt), if
    given, sees the states m^{n-1} before the solves of step n (n = 1, 2, ...).  picard = K > 1
    repeats each step's linearisation (Section 2.3: m~^{(k)} = m^{(k-1)}): after the first solve,
    every system is solved K - 1 more times with its operator built from its previous iterate,
    the right-hand side kept at m^{n-1}/dt - div f, GMRES started from the previous iterate;
    the result of the K-th solve is m^n.  stats.iters then holds the first solves' counts and
    stats.picard_iters[step][k][target] those of the later ones.
    """
    if picard < 1:
        raise ValueError("picard must be >= 1")
    if reorth not in ("auto", "always"):
        raise ValueError("reorth must be 'auto' or 'always'")
    tpasses = 1 if reorth == "auto" else 2
    dt = 1.0 / T
    ms = np.array(seed_m0, dtype=np.float64).reshape(-1)
    mt = np.array(target_m0, dtype=np.float64).reshape(len(target_m0), -1)
    st = ChainStats()
    for step in range(T if steps is None else steps):
        if on_step is not None:
            on_step(step + 1, ms, mt)
        basis = None
        if method == "project":
            As = Operator(H, dt, g, ms)
            bs = rhs(As, ms)
            sr = gmres(As, bs, x0=ms if warm else None, m=m, tol=tol, keep_basis=True,
                       max_restarts=max_restarts)
            basis = sr
            st.seed_iters.append(sr.iters)
            st.basis_dim.append(sr.basis_dim)
        it_row, rs_row, stt_row, res_row, g_row = [], [], [], [], []
        new = np.empty_like(mt)
        for t in range(mt.shape[0]):
            At = Operator(H, dt, g, mt[t])
            bt = rhs(At, mt[t])
            xb = mt[t] if warm else None
            if method == "direct":
                x, s = banded_solve(At, bt)
                it_row.append(0); rs_row.append(0); stt_row.append(s)
                res_row.append(residual(At, bt, x)); g_row.append(np.nan)
            else:
                if method == "project":
                    x0, _, _ = project(At, bt, basis.V, basis.Hbar, mode=mode, x_base=xb)
                else:
                    x0 = xb
                g_row.append(residual(At, bt, x0) if x0 is not None else 1.0)
                r = gmres(At, bt, x0=x0, m=m, tol=tol, max_restarts=max_restarts,
                          passes=tpasses)
                x = r.x
                it_row.append(r.iters); rs_row.append(r.restarts); stt_row.append(r.status)
                res_row.append(r.res_true)
            new[t] = x
        new_s = basis.x if basis is not None else None
        pic_rows = []
        for _ in range(picard - 1):
            # the linearisation again, around the previous iterate
            if new_s is not None:
                As = Operator(H, dt, g, new_s)
                sr = gmres(As, rhs(As, ms), x0=new_s, m=m, tol=tol, max_restarts=max_restarts,
                           passes=tpasses)
                new_s = sr.x
            row = []
            for t in range(mt.shape[0]):
                At = Operator(H, dt, g, new[t])
                if method == "direct":
                    new[t], _ = banded_solve(At, rhs(At, mt[t]))
                    row.append(0)
                else:
                    r = gmres(At, rhs(At, mt[t]), x0=new[t], m=m, tol=tol,
                              max_restarts=max_restarts, passes=tpasses)
                    new[t] = r.x
                    row.append(r.iters)
                    res_row[t] = r.res_true
            pic_rows.append(row)
        if new_s is not None:
            ms = new_s
        mt = new
        st.iters.append(it_row); st.restarts.append(rs_row); st.status.append(stt_row)
        st.res_true.append(res_row); st.guess_res.append(g_row)
        st.picard_iters.append(pic_rows)
    return ms, mt, st


def run_cycle_chain(blocks, H, T, m, per_source, g=0.5, tol=1e-8, steps=None,
                    max_restarts=1000):
    """The image-cycle protocol (Experiment 2): `blocks` is a list of (seed_m0 (n,), targets_m0
    (N_g, n)); per timestep every block's seed is solved (first-cycle basis kept, two
    Gram-Schmidt passes), the basis of block g is gathered from the seeds of blocks 0..g
    (`accumulate`, at most per_source columns each, m in total), and block g's targets are
    projected on it (target Galerkin) and polished by GMRES(m) with one pass.
    Returns (seed states, target states per block, stats with iters[step][target])."""
    dt = 1.0 / T
    ms = [np.array(s0, dtype=np.float64).reshape(-1) for s0, _ in blocks]
    mt = [np.array(t0, dtype=np.float64).reshape(len(t0), -1) for _, t0 in blocks]
    st = ChainStats()
    for _ in range(T if steps is None else steps):
        srcs, new_s = [], []
        for b in range(len(blocks)):
            As = Operator(H, dt, g, ms[b])
            sr = gmres(As, rhs(As, ms[b]), m=m, tol=tol, keep_basis=True,
                       max_restarts=max_restarts)
            srcs.append(sr.V[:, :sr.basis_dim])
            new_s.append(sr.x)
            st.seed_iters.append(sr.iters)
        it_row, res_row, g_row = [], [], []
        new_t = []
        for b in range(len(blocks)):
            V = accumulate(srcs[:b + 1], per_source, m)
            k = V.shape[1]
            Vp = np.concatenate([V, np.zeros((V.shape[0], 1))], axis=1)
            out = np.empty_like(mt[b])
            for t in range(mt[b].shape[0]):
                At = Operator(H, dt, g, mt[b][t])
                bt = rhs(At, mt[b][t])
                x0, _, _ = project(At, bt, Vp, np.zeros((k + 1, k)), mode=TARGET_GALERKIN)
                g_row.append(residual(At, bt, x0))
                r = gmres(At, bt, x0=x0, m=m, tol=tol, max_restarts=max_restarts, passes=1)
                out[t] = r.x
                it_row.append(r.iters)
                res_row.append(r.res_true)
            new_t.append(out)
        ms, mt = new_s, new_t
        st.iters.append(it_row)
        st.res_true.append(res_row)
        st.guess_res.append(g_row)
    return ms, mt, st
