"""Timestep chain of the method on the GPU, built only from libxkp calls.

Per timestep n (Section 2.3: one implicit solve per image and timestep, dt = 1/T, one
linearisation pass m~ = m^{n-1}; Section 3: seed phase then target phase):
  xkp_build_rhs            b = m^{n-1}/dt for the seed and every target
  xkp_seed_build           seed GMRES, first-cycle basis V^n kept       (projection only)
  xkp_target_project_solve projection onto V^n + GMRES polish, or plain GMRES
and the solution buffers become the next step's m^{n-1} (double buffering, no copies).
"""
from __future__ import annotations

import numpy as np

from . import xkp


class Chain:
    """Seed and targets of one grid size advanced together through the timesteps.

    With `pipeline` (projection only) the seed runs on its own stream and context one timestep
    ahead of the targets: the seed of step n+1 overlaps the targets of step n.  The seed basis is
    double-buffered; events order seed n before targets n, and targets n before seed n+2 (which
    overwrites the basis targets n read).  All streams keep the default priority.
    """

    def __init__(self, H, T, m, seed_m0, target_m0, g=0.5, tol=1e-8, method="project",
                 mode="target_galerkin", warm=False, max_restarts=1000, device=0, ctx=None,
                 precision=xkp.FP64, pipeline=True):
        import torch
        self.H, self.T, self.m, self.g, self.tol = H, T, m, g, tol
        self.n = n = H * H
        self.method = method
        self.dev = torch.device(f"cuda:{device}")
        tgt = np.ascontiguousarray(np.asarray(target_m0, dtype=np.float64).reshape(-1, n))
        self.N = N = tgt.shape[0]
        self.ctx = ctx or xkp.Context(n, m, max(N, 1), device=device)
        self.pipeline = pipeline and method == "project"
        if self.pipeline:
            self.s_seed = torch.cuda.Stream(device=self.dev)
            self.ctx_seed = xkp.Context(n, m, 1, device=device, stream=self.s_seed)
            self.ev_seed = [torch.cuda.Event(), torch.cuda.Event()]
            self.ev_tgt = [torch.cuda.Event(), torch.cuda.Event()]
            self.ev_reset = torch.cuda.Event()
        else:
            self.ctx_seed = self.ctx
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.ms = [torch.tensor(np.asarray(seed_m0, dtype=np.float64).reshape(1, n), **f64),
                   torch.empty((1, n), **f64)]
        self.mt = [torch.tensor(tgt, **f64), torch.empty((N, n), **f64)]
        self.bs = torch.empty((1, n), **f64)
        self.bt = torch.empty((N, n), **f64)
        self.bases = xkp.Bases(2, n, m, device=device)
        dt = 1.0 / T
        mode_id = xkp.NONE if method == "plain" else xkp.MODES[mode]
        self.params = xkp.Context.params(m, tol=tol, max_restarts=max_restarts,
                                         precision=precision, mode=mode_id, batch_max_n=n)
        self.seed_desc, self.tgt_desc = [], []
        for par in (0, 1):
            sd = xkp.pack_batch(H, dt, g, self.ms[par], self.bs, self.ms[1 - par],
                                x0=self.ms[par] if warm else None)
            td = xkp.pack_batch(H, dt, g, self.mt[par], self.bt, self.mt[1 - par],
                                x0=self.mt[par] if warm else None, basis_id=0)
            self.seed_desc.append(sd)
            self.tgt_desc.append(td)
        # one info record per system and timestep, so that every solve can be verified
        self.info_s_all = self.ctx.new_infos(T)
        self.info_t_all = self.ctx.new_infos(T * N)
        self.m0 = (self.ms[0].clone(), self.mt[0].clone())
        self.step_no = 0

    def reset(self):
        """Back to the initial images (a device-to-device copy of the state)."""
        import torch
        if self.pipeline:
            # the seed stream may still be a step ahead: let the copies wait for it
            torch.cuda.current_stream(self.dev).wait_stream(self.s_seed)
        self.ms[0].copy_(self.m0[0])
        self.mt[0].copy_(self.m0[1])
        if self.pipeline:
            self.ev_reset.record(torch.cuda.current_stream(self.dev))
            self.s_seed.wait_event(self.ev_reset)
        self.step_no = 0

    def _info_slices(self, t):
        w = xkp.INFO_DTYPE.itemsize
        return (self.info_s_all[t * w:(t + 1) * w],
                self.info_t_all[t * self.N * w:(t + 1) * self.N * w])

    @property
    def info_s(self):
        return self._info_slices((self.step_no - 1) % self.T)[0]

    @property
    def info_t(self):
        return self._info_slices((self.step_no - 1) % self.T)[1]

    def step(self, events=None):
        """Enqueue one timestep on the context's stream.  `events`, if given, is a pair of
        HIP events recorded around the target call."""
        par = self.step_no & 1
        c = self.ctx
        inf_s, inf_t = self._info_slices(self.step_no % self.T)
        basis = self.bases.ptrs[par:par + 1]
        if self.method == "project":
            cs = self.ctx_seed
            if self.pipeline and self.step_no >= 2:
                self.s_seed.wait_event(self.ev_tgt[par])   # targets n-2 done with this basis
            cs.build_rhs(self.seed_desc[par], 1)
            cs.seed_build(self.seed_desc[par], 1, basis, self.params, inf_s)
            if self.pipeline:
                self.ev_seed[par].record(self.s_seed)
                c.stream.wait_event(self.ev_seed[par])
        c.build_rhs(self.tgt_desc[par], self.N)
        if events is not None:
            events[0].record(c.stream)
        c.target_project_solve(self.tgt_desc[par], self.N, 1, basis, self.params, inf_t)
        if events is not None:
            events[1].record(c.stream)
        if self.pipeline:
            self.ev_tgt[par].record(c.stream)
        self.step_no += 1

    def all_infos(self):
        """(seed infos [T], target infos [T, N]) of the last full chain."""
        s = xkp.infos_to_numpy(self.info_s_all)
        t = xkp.infos_to_numpy(self.info_t_all).reshape(self.T, self.N)
        return s, t

    @property
    def seed_state(self):
        return self.ms[self.step_no & 1][0]

    @property
    def target_state(self):
        return self.mt[self.step_no & 1]

    def infos(self):
        return xkp.infos_to_numpy(self.info_s), xkp.infos_to_numpy(self.info_t)
