"""Timestep chain of the method on the GPU, built only from libxkp calls.

Per timestep n (Section 2.3: one implicit solve per image, channel and timestep, dt = 1/T, one
linearisation pass m~ = m^{n-1}; Section 3: seed phase then target phase):
  xkp_build_rhs            b = m^{n-1}/dt for every seed and every target
  xkp_seed_build           all seeds in one launch, first-cycle bases V^n kept (projection only)
  xkp_target_project_solve all targets in one launch: projection onto their seed's V^n + GMRES
                           polish, or plain GMRES
and the solution buffers become the next step's m^{n-1} (double buffering, no copies).

A batch holds one or more groups; a group is one grid size with C channels, one seed image and
N target images.  Every channel of every image is its own system (C seeds and N*C targets per
group); a target uses the basis of its own group's seed in the same channel.  Targets are laid
out largest grid first, the order in which the work queue hands them out.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import xkp

# fields of a cached launch-choice record (Batch.tuning_record)
TUNING_FIELDS = ("polish_m", "waves", "wg_per_cu", "split", "seed_waves", "seed_wg_per_cu",
                 "seed_rows_per_thread")


def load_tuning_cache(path):
    """Launch-choice records by key from a JSON cache file ({} if it does not exist); records
    that lack a field are left out."""
    try:
        with open(path) as f:
            data = json.load(f)
    except FileNotFoundError:
        return {}
    if not isinstance(data, dict):
        raise ValueError(f"tuning cache {path}: not a JSON object")
    return {k: v for k, v in data.items()
            if isinstance(v, dict) and all(f in v for f in TUNING_FIELDS)}


def store_tuning_cache(path, key, rec):
    """Adds (or replaces) one record in the JSON cache file; the file is rewritten through a
    temporary file and a rename, so a reader never sees it half written."""
    missing = [f for f in TUNING_FIELDS if f not in rec]
    if missing:
        raise ValueError(f"tuning record lacks {missing}")
    try:
        with open(path) as f:
            data = json.load(f)
        if not isinstance(data, dict):
            data = {}
    except (FileNotFoundError, json.JSONDecodeError):
        data = {}
    data[key] = {f: rec[f] for f in TUNING_FIELDS}
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


class Group:
    """One grid size: seed_m0 (C, n) and target_m0 (N, C, n) initial states, n = H*H."""

    def __init__(self, H, seed_m0, target_m0):
        n = H * H
        self.H, self.n = H, n
        s = np.asarray(seed_m0, dtype=np.float64)
        self.C = s.size // n
        self.seed_m0 = np.ascontiguousarray(s.reshape(self.C, n))
        t = np.asarray(target_m0, dtype=np.float64)
        self.target_m0 = np.ascontiguousarray(t.reshape(-1, self.C, n))
        self.N = self.target_m0.shape[0]


class Batch:
    """Seeds and targets of several grid sizes advanced together through the timesteps.

    With `pipeline` (projection only) the seeds run on their own stream and context one timestep
    ahead of the targets: the seeds of step n+1 overlap the targets of step n.  The bases are
    double-buffered; events order seeds n before targets n, and targets n before seeds n+2
    (which overwrite the bases targets n read).  All streams keep the default priority.

    The work of one full chain (reset + T steps) can be captured once in a HIP graph
    (`capture`) and replayed (`replay`); the eager `run` enqueues the same calls.
    """

    def __init__(self, groups, T, m, g=0.5, tol=1e-8, method="project",
                 mode="target_galerkin", warm=False, max_restarts=1000, device=0,
                 precision=xkp.FP64, pipeline=True, polish_m=0, with_seeds=None, learned=None,
                 reorth="auto", accumulate=None, embed=False, picard=1):
        """method: "project" (projection + polish), "plain" (GMRES from x_base) or "learned"
        (the network's guess behind the residual gate, projection as fallback; `learned` =
        dict(params=FP32 parameters of a network with m + 1 outputs, scale=output scale,
        gate=residual gate, correction=False), single 64x64 group of one channel; with
        correction=True the network corrects the projected guess instead, kept when it lowers
        the guess's residual).  with_seeds: also solve the
        seeds with plain targets.  reorth: "auto" (two Gram-Schmidt passes only while a seed's
        basis is kept) or "always".  accumulate: per-source column count a of the image-cycle
        subspace expansion: the groups (one grid size, one channel) are consecutive blocks of
        one image cycle, and the targets of block g are projected on the basis gathered from
        the seeds of blocks 0..g (at most a columns each, m in total) at every timestep.
        embed: after each step's target call, the score of every target's state before the
        step (m^{n-1}) goes to `score_t` and one probability-flow step to the displacement
        `disp_t` (both (N, 2, n) per target of one grid size; reset with the chain).
        picard: K linearisation passes per timestep: after the seed and target calls every
        system is solved K - 1 more times by plain GMRES, the operator built from its previous
        iterate (m~ = m^{n,(k-1)}), the right-hand side kept, started from that iterate."""
        import torch
        self.groups = sorted(groups, key=lambda gr: -gr.n)      # largest grid first
        self.T, self.m, self.g, self.tol = T, m, g, tol
        self.method = method
        self.with_seeds = (method != "plain") if with_seeds is None else with_seeds
        self.dev = torch.device(f"cuda:{device}")
        self.nmax = max(gr.n for gr in self.groups)
        self.S = sum(gr.C for gr in self.groups)
        self.N = sum(gr.N * gr.C for gr in self.groups)
        self.s_main = torch.cuda.Stream(device=self.dev)
        self.ctx = xkp.Context(self.nmax, m, max(self.N, 1), device=device, stream=self.s_main)
        self.pipeline = pipeline and self.with_seeds
        if self.pipeline:
            self.s_seed = torch.cuda.Stream(device=self.dev)
            self.ctx_seed = xkp.Context(self.nmax, m, self.S, device=device, stream=self.s_seed)
            self.ev_seed = [torch.cuda.Event(), torch.cuda.Event()]
            self.ev_tgt = [torch.cuda.Event(), torch.cuda.Event()]
            self.ev_reset = torch.cuda.Event()
        else:
            self.ctx_seed = self.ctx
        # flat storage: seed systems (group, channel) then target systems (group, target, channel)
        so = to = 0
        self.seed_sys, self.tgt_sys = [], []       # (H, offset, basis id)
        for gr in self.groups:
            base_id = len(self.seed_sys)
            for c in range(gr.C):
                self.seed_sys.append((gr.H, so, base_id + c))
                so += gr.n
            for t in range(gr.N):
                for c in range(gr.C):
                    self.tgt_sys.append((gr.H, to, base_id + c))
                    to += gr.n
        f64 = dict(dtype=torch.float64, device=self.dev)
        s0 = np.concatenate([gr.seed_m0.reshape(-1) for gr in self.groups])
        t0 = np.concatenate([gr.target_m0.reshape(-1) for gr in self.groups])
        self.m0 = (torch.tensor(s0, **f64), torch.tensor(t0, **f64))
        self.ms = [self.m0[0].clone(), torch.empty_like(self.m0[0])]
        self.mt = [self.m0[1].clone(), torch.empty_like(self.m0[1])]
        self.bs = torch.empty_like(self.m0[0])
        self.bt = torch.empty_like(self.m0[1])
        ns = [H * H for H, _, _ in self.seed_sys]
        self.bases = xkp.Bases(2 * self.S, ns * 2, m, device=device)
        # a seed spread over workgroups (256 rows each) runs beside the previous target call
        # only where its workgroups and one per target fit the chip's compute units together
        self.seed_blocks = sum((n + 255) // 256 for n in ns)
        self.cus = torch.cuda.get_device_properties(self.dev).multi_processor_count
        self.dt = 1.0 / T
        mode_id = xkp.NONE if method == "plain" else xkp.MODES[mode]
        self.learned = None
        if method == "learned":
            assert len(self.groups) == 1 and self.groups[0].H == 64 and self.groups[0].C == 1
            gr = self.groups[0]
            k = m + 1                      # residual coordinates of an m-column basis
            self.learned = dict(learned)
            self.net = xkp.Net(self.ctx, k, self.N, learned["params"])
            self.images = torch.tensor(gr.target_m0.reshape(self.N, -1), **f64)
            steps = np.repeat(np.arange(1, T + 1, dtype=np.int32)[:, None], self.N, axis=1)
            self.steps_all = torch.from_numpy(steps).to(self.dev)
            self.alpha_l = torch.empty((self.N, k), dtype=torch.float32, device=self.dev)
        self.embed = bool(embed)
        if self.embed:
            assert len({gr.H for gr in self.groups}) == 1
            self.score_t = torch.zeros((self.N, 2, self.nmax), **f64)
            self.disp_t = torch.zeros((self.N, 2, self.nmax), **f64)
            rows = 2 * self.nmax * 8 * np.arange(self.N, dtype=np.int64)
            self.score_ptrs = torch.tensor(self.score_t.data_ptr() + rows, device=self.dev)
            self.disp_ptrs = torch.tensor(self.disp_t.data_ptr() + rows, device=self.dev)
        self.acc = None
        if accumulate is not None:
            assert method == "project" and mode == "target_galerkin"
            assert len({gr.H for gr in self.groups}) == 1 and all(gr.C == 1 for gr in self.groups)
            self.acc = int(accumulate)
            self.acc_bases = xkp.Bases(2 * self.S, self.nmax, m, device=device)
        self.params = xkp.Context.params(m, tol=tol, max_restarts=max_restarts,
                                         precision=precision, mode=mode_id,
                                         batch_max_n=self.nmax, polish_m=polish_m,
                                         reorth=reorth)
        self.config = dict(m=m, precision=int(precision), method=method,
                           mode=mode if method != "plain" else "none", reorth=reorth,
                           pipeline=bool(self.pipeline), picard=int(picard),
                           accumulate=self.acc)
        self.tuned_from_cache = False
        self.seed_tuning = None
        self.warm = warm
        self.K = int(picard)
        assert self.K >= 1
        if self.K > 1:
            self.ms_pic = torch.empty_like(self.ms[0])
            self.mt_pic = torch.empty_like(self.mt[0])
            self.params_plain = xkp.Context.params(m, tol=tol, max_restarts=max_restarts,
                                                   precision=precision, mode=xkp.NONE,
                                                   batch_max_n=self.nmax, polish_m=polish_m,
                                                   reorth=reorth)
            self.info_ps = self.ctx.new_infos(T * (self.K - 1) * self.S)
            self.info_pt = self.ctx.new_infos(T * (self.K - 1) * self.N)
        self.seed_desc = [self._desc(self.seed_sys, self.ms, self.bs, par,
                                     x_from=self._out(1, par, True)) for par in (0, 1)]
        self.tgt_desc = [self._desc(self.tgt_sys, self.mt, self.bt, par,
                                    x_from=self._out(1, par, False)) for par in (0, 1)]
        # Picard passes k = 2..K: m~ = x0 = iterate k-1, result into iterate k
        self.seed_pic = [[self._desc_raw(self.seed_sys, self._out(k - 1, par, True), self.bs,
                                         self._out(k, par, True), self._out(k - 1, par, True))
                          for k in range(2, self.K + 1)] for par in (0, 1)]
        self.tgt_pic = [[self._desc_raw(self.tgt_sys, self._out(k - 1, par, False), self.bt,
                                        self._out(k, par, False), self._out(k - 1, par, False))
                         for k in range(2, self.K + 1)] for par in (0, 1)]
        # one info record per system and timestep, so that every solve can be verified
        self.info_s_all = self.ctx.new_infos(T * self.S)
        self.info_t_all = self.ctx.new_infos(T * self.N)
        self.step_no = 0
        self.graph = None
        torch.cuda.synchronize(self.dev)     # inputs copied on the current stream are in place

    def _out(self, k, par, seeds):
        """Where Picard pass k of a step of parity par writes: passes alternate between the
        scratch iterate and the next state so that pass K lands in the state."""
        state = self.ms if seeds else self.mt
        if (self.K - k) % 2 == 0:
            return state[1 - par]
        return self.ms_pic if seeds else self.mt_pic

    def _desc_raw(self, systems, mt, b, x, x0):
        """Descriptors with explicit m~ (coefficients), b, x and x0 tensors."""
        import torch
        a = np.zeros(len(systems), dtype=xkp.SYSTEM_DTYPE)
        for i, (H, off, bid) in enumerate(systems):
            o = 8 * off
            a[i] = (H, bid, self.dt, self.g, mt.data_ptr() + o, 0, 0, b.data_ptr() + o,
                    x0.data_ptr() + o, x.data_ptr() + o)
        d = torch.from_numpy(a.view(np.uint8).copy()).to(self.dev)
        d._xkp_keep = [mt, b, x, x0]
        return d

    def _desc(self, systems, state, b, par, x_from=None):
        """Descriptors of `systems` at a step of parity par: m~ = state[par], solution into
        state[1 - par] (or x_from)."""
        import torch
        a = np.zeros(len(systems), dtype=xkp.SYSTEM_DTYPE)
        mt = state[par].data_ptr()
        x = (x_from if x_from is not None else state[1 - par]).data_ptr()
        bp = b.data_ptr()
        for i, (H, off, bid) in enumerate(systems):
            o = 8 * off
            a[i] = (H, bid, self.dt, self.g, mt + o, 0, 0, bp + o,
                    (mt + o) if self.warm else 0, x + o)
        d = torch.from_numpy(a.view(np.uint8).copy()).to(self.dev)
        d._xkp_keep = [state[0], state[1], b]
        return d

    # -- eager enqueue --------------------------------------------------------------------

    def reset(self, join_seed=True):
        """Back to the initial images (device-to-device copies on the main stream)."""
        import torch
        with torch.cuda.stream(self.s_main):
            if self.pipeline and join_seed:
                # the seed stream may still be a step ahead: let the copies wait for it
                self.s_main.wait_stream(self.s_seed)
            self.ms[0].copy_(self.m0[0])
            self.mt[0].copy_(self.m0[1])
            if self.embed:
                self.disp_t.zero_()
            if self.pipeline:
                self.ev_reset.record(self.s_main)
                self.s_seed.wait_event(self.ev_reset)
        self.step_no = 0

    def _info_slices(self, t):
        w = xkp.INFO_DTYPE.itemsize
        return (self.info_s_all[t * self.S * w:(t + 1) * self.S * w],
                self.info_t_all[t * self.N * w:(t + 1) * self.N * w])

    def step(self, events=None, after_targets=None, seed_events=None):
        """Enqueue one timestep.  `events`, if given, is a pair of HIP events recorded on the
        main stream around the target call (`seed_events`: on the seed stream around the seed
        call); `after_targets(par, bases)` is called after the target call is enqueued."""
        par = self.step_no & 1
        c = self.ctx
        inf_s, inf_t = self._info_slices(self.step_no % self.T)
        bases = self.bases.ptrs[par * self.S:(par + 1) * self.S]
        if self.with_seeds:
            cs = self.ctx_seed
            if self.pipeline and self.step_no >= 2:
                self.s_seed.wait_event(self.ev_tgt[par])   # targets n-2 done with these bases
            if (self.pipeline and self.step_no >= 1 and self.ctx_seed_rows() > 0
                    and self.N + self.seed_blocks > self.cus):
                # a seed spread over several workgroups needs them resident together: beside a
                # target call that fills the chip it would wait for it anyway, so it runs after
                self.s_seed.wait_event(self.ev_tgt[1 - par])
            cs.build_rhs(self.seed_desc[par], self.S)
            if seed_events is not None:
                seed_events[0].record(cs.stream)
            cs.seed_build(self.seed_desc[par], self.S, bases, self.params, inf_s)
            if seed_events is not None:
                seed_events[1].record(cs.stream)
            bases = self._accumulate(par, bases)
            if self.pipeline:
                self.ev_seed[par].record(self.s_seed)
                c.stream.wait_event(self.ev_seed[par])
            t = self.step_no % self.T
            w = xkp.INFO_DTYPE.itemsize
            for k in range(2, self.K + 1):
                o = ((t * (self.K - 1) + k - 2) * self.S) * w
                cs.target_project_solve(self.seed_pic[par][k - 2], self.S, 0, None,
                                        self.params_plain, self.info_ps[o:o + self.S * w])
        c.build_rhs(self.tgt_desc[par], self.N)
        if events is not None:
            events[0].record(c.stream)
        if self.learned is not None:
            t = self.step_no % self.T
            self.net.forward(self.images, self.steps_all[t], self.alpha_l)
            solve = (c.learned_correction_solve if self.learned.get("correction")
                     else c.learned_solve)
            solve(self.tgt_desc[par], self.N, self.S, bases, self.params, self.alpha_l,
                  self.m + 1, self.learned["scale"], self.learned["gate"], inf_t)
        else:
            c.target_project_solve(self.tgt_desc[par], self.N, self.S, bases, self.params, inf_t)
        if events is not None:
            events[1].record(c.stream)
        t = self.step_no % self.T
        w = xkp.INFO_DTYPE.itemsize
        for k in range(2, self.K + 1):
            o = ((t * (self.K - 1) + k - 2) * self.N) * w
            c.target_project_solve(self.tgt_pic[par][k - 2], self.N, 0, None, self.params_plain,
                                   self.info_pt[o:o + self.N * w])
        if self.embed:
            c.score_flow(self.tgt_desc[par], self.N, xkp.FIELD_MT, self.score_ptrs,
                         self.disp_ptrs)
        if after_targets is not None:
            after_targets(par, bases)
        if self.pipeline:
            self.ev_tgt[par].record(c.stream)
        self.step_no += 1

    def _accumulate(self, par, bases):
        """The targets' bases of this step: the seeds' own, or (image cycle) the bases gathered
        from the seeds of blocks 0..g, built on the seed context's stream."""
        if self.acc is None:
            return bases
        acc = self.acc_bases.ptrs[par * self.S:(par + 1) * self.S]
        self.ctx_seed.basis_accumulate(self.nmax, self.S, bases, acc, self.acc, self.m)
        return acc

    def run(self):
        """One full chain, eagerly enqueued."""
        self.reset()
        for _ in range(self.T):
            self.step()

    # -- graph ----------------------------------------------------------------------------

    def capture(self):
        """Capture reset + T steps as one HIP graph (run the chain eagerly once before, so that
        every kernel attribute is set outside the capture)."""
        import torch
        torch.cuda.synchronize(self.dev)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.s_main):
            self.reset(join_seed=False)
            for _ in range(self.T):
                self.step()
            if self.pipeline:
                # seed work after the last step's basis event (Picard passes) joins the capture
                self.s_main.wait_stream(self.s_seed)
        self.graph = g
        return g

    def replay(self):
        """Replay the captured chain on the main stream."""
        import torch
        self.s_main.wait_stream(torch.cuda.current_stream(self.dev))
        with torch.cuda.stream(self.s_main):
            self.graph.replay()
        self.step_no = self.T

    # -- tuning and results -----------------------------------------------------------------

    def autotune(self, steps=2, cache=None):
        """Advance `steps` timesteps eagerly, then time the target call of the next timestep
        over the candidates of xkp_autotune on its real inputs; the chosen polish restart length
        goes into the params, the workgroup count into the context.  With a seed context of
        its own (pipelined chains), the seed call of that timestep is tuned too
        (xkp_autotune_seeds; the result is in `self.seed_tuning`), and a spread-out seed width
        is kept only if the pipelined chain steps are faster with it.  Resets the chain.

        cache: path of a JSON file of launch choices keyed by `tuning_key()` (device, grid
        sizes and system counts, m, precision, method).  A hit applies the stored choices
        without timing anything (`tuned_from_cache` is then True); a miss tunes and adds the
        choices to the file."""
        import torch
        key = self.tuning_key() if cache is not None else None
        if key is not None:
            rec = load_tuning_cache(cache).get(key)
            if rec is not None:
                t = self.apply_tuning(rec)
                self.tuned_from_cache = True
                return t
        self.tuned_from_cache = False
        t = self._autotune(steps)
        if key is not None:
            store_tuning_cache(cache, key, self.tuning_record(t))
        return t

    def tuning_key(self):
        """Cache key of this batch's launch choices: the device's architecture and compute
        units, every group's grid side, channels and targets, and the solver configuration."""
        import torch
        p = torch.cuda.get_device_properties(self.dev)
        arch = getattr(p, "gcnArchName", "") or p.name
        shape = "+".join(f"{gr.H}x{gr.C}x{gr.N}" for gr in self.groups)
        c = self.config
        return (f"{arch}/cu{p.multi_processor_count}/{shape}/m{c['m']}/prec{c['precision']}/"
                f"{c['method']}/{c['mode']}/{c['reorth']}/"
                f"{'pipe' if c['pipeline'] else 'serial'}/K{c['picard']}/acc{c['accumulate']}")

    def tuning_record(self, t):
        """The launch choices the batch runs with (JSON-able): polish restart length, target
        launch shape and projection placement, the seed context's launch shape and seed
        width."""
        ts = self.seed_tuning
        return {"polish_m": int(self.params.polish_m), "waves": int(t.waves),
                "wg_per_cu": int(t.wg_per_cu), "split": int(getattr(self.ctx, "split", -1)),
                "seed_waves": None if ts is None else int(ts.waves),
                "seed_wg_per_cu": None if ts is None else int(ts.wg_per_cu),
                "seed_rows_per_thread": None if ts is None else int(ts.seed_rows)}

    def apply_tuning(self, rec):
        """Set the launch choices of a `tuning_record` instead of timing candidates; returns
        the Tuning the autotuner would have."""
        self.params.polish_m = rec["polish_m"]
        self.ctx.set_launch(rec["waves"], rec["wg_per_cu"])
        self.ctx.set_projection_split(rec["split"])
        self.seed_tuning = None
        if rec.get("seed_waves") is not None and self.with_seeds and self.ctx_seed is not self.ctx:
            self.ctx_seed.set_launch(rec["seed_waves"], rec["seed_wg_per_cu"])
            self.ctx_seed.set_seed_width(rec["seed_rows_per_thread"])
            self.seed_tuning = xkp.Tuning(waves=rec["seed_waves"],
                                          wg_per_cu=rec["seed_wg_per_cu"],
                                          seed_rows=rec["seed_rows_per_thread"])
        return xkp.Tuning(polish_m=rec["polish_m"], wg_per_cu=rec["wg_per_cu"],
                          waves=rec["waves"], split=rec["split"])

    def _autotune(self, steps):
        import torch
        self.reset()
        for _ in range(steps):
            self.step()
        par = self.step_no & 1
        bases = self.bases.ptrs[par * self.S:(par + 1) * self.S]
        inf_s, inf_t = self._info_slices(self.step_no % self.T)
        self.seed_tuning = None
        if self.with_seeds:
            self.ctx_seed.build_rhs(self.seed_desc[par], self.S)
            if self.ctx_seed is not self.ctx:
                torch.cuda.synchronize(self.dev)
                self.seed_tuning = self.ctx_seed.autotune_seeds(self.seed_desc[par], self.S,
                                                                bases, self.params, inf_s)
            else:
                self.ctx_seed.seed_build(self.seed_desc[par], self.S, bases, self.params, inf_s)
            bases = self._accumulate(par, bases)
        self.ctx.build_rhs(self.tgt_desc[par], self.N)
        torch.cuda.synchronize(self.dev)
        t = self.ctx.autotune(self.tgt_desc[par], self.N, self.S, bases, self.params, inf_t)
        self.params.polish_m = t.polish_m
        if self.seed_tuning is not None and self.seed_tuning.seed_rows == 1:
            # the seed call was timed alone; beside the target launches (projection launches
            # that fill the chip) a seed spread over workgroups must wait until all of them are
            # resident, so the width whose chain steps run faster is kept
            self.seed_tuning.seed_rows = self._pick_seed_width()
        self.reset()
        torch.cuda.synchronize(self.dev)
        return t

    def _chain_ms(self):
        """Host time of one replay of the whole chain, captured now and replayed once before."""
        import time
        import torch
        self.capture()
        self.replay()
        self._join()
        torch.cuda.synchronize(self.dev)
        t0 = time.perf_counter()
        self.replay()
        self._join()
        torch.cuda.synchronize(self.dev)
        self.graph = None
        return (time.perf_counter() - t0) * 1e3

    def _pick_seed_width(self, reps=2):
        """Seed width (1: spread over workgroups, 0: one workgroup per seed) whose replayed
        chain is faster, the better of `reps` alternating timings each; sets it in the seed
        context and returns it."""
        best = {0: float("inf"), 1: float("inf")}
        for _ in range(reps):
            for w in (1, 0):
                self.ctx_seed.set_seed_width(w)
                best[w] = min(best[w], self._chain_ms())
        w = 1 if best[1] < best[0] else 0
        self.ctx_seed.set_seed_width(w)
        return w

    def ctx_seed_rows(self):
        """1 if the seed context spreads each seed over several workgroups, else 0."""
        return int(getattr(self.ctx_seed, "seed_width", 0))

    def _join(self):
        """Order the current stream after everything enqueued on the chain's streams."""
        import torch
        cur = torch.cuda.current_stream(self.dev)
        cur.wait_stream(self.s_main)
        if self.pipeline:
            cur.wait_stream(self.s_seed)

    def all_infos(self):
        """(seed infos [T, S], target infos [T, N]) of the last full chain."""
        self._join()
        s = xkp.infos_to_numpy(self.info_s_all).reshape(self.T, self.S)
        t = xkp.infos_to_numpy(self.info_t_all).reshape(self.T, self.N)
        return s, t

    def picard_infos(self):
        """(seed infos [T, K-1, S], target infos [T, K-1, N]) of the later Picard passes."""
        self._join()
        s = xkp.infos_to_numpy(self.info_ps).reshape(self.T, self.K - 1, self.S)
        t = xkp.infos_to_numpy(self.info_pt).reshape(self.T, self.K - 1, self.N)
        return s, t

    def infos(self):
        """(seed infos [S], target infos [N]) of the last step."""
        self._join()
        s, t = self._info_slices((self.step_no - 1) % self.T)
        return xkp.infos_to_numpy(s), xkp.infos_to_numpy(t)

    def state(self, par=None):
        """(seed states [S*n...], target states) flat tensors after the last step."""
        self._join()
        p = (self.step_no & 1) if par is None else par
        return self.ms[p], self.mt[p]

    def group_states(self, gi):
        """(seed (C, n), targets (N, C, n)) views of group gi's current state."""
        gr = self.groups[gi]
        ms, mt = self.state()
        so = sum(g.C * g.n for g in self.groups[:gi])
        to = sum(g.N * g.C * g.n for g in self.groups[:gi])
        return (ms[so:so + gr.C * gr.n].view(gr.C, gr.n),
                mt[to:to + gr.N * gr.C * gr.n].view(gr.N, gr.C, gr.n))

    def verify_chain(self):
        """One eager chain in which every target solve is checked as soon as it is enqueued:
        the FP64 relative residual of each target's solution with the operator and right-hand
        side rebuilt from that step's m^{n-1} through the library (xkp_build_rhs into a scratch
        buffer, xkp_residual, whose operator is formed from m~ on the fly).  Returns rel [T, N].
        One linearisation pass per step."""
        import torch
        assert self.K == 1
        bt = torch.empty_like(self.bt)
        dv = [self._desc(self.tgt_sys, self.mt, bt, par) for par in (0, 1)]
        rel = torch.empty((self.T, self.N), dtype=torch.float64, device=self.dev)

        def hook(par, bases):
            t = self.step_no % self.T
            self.ctx.build_rhs(dv[par], self.N)
            self.ctx.residual(dv[par], self.N, rel[t])
        self.s_main.wait_stream(torch.cuda.current_stream(self.dev))
        self.reset()
        for _ in range(self.T):
            self.step(after_targets=hook)
        self._join()
        return rel.cpu().numpy()

    def record_chain(self, picks):
        """One eager chain that copies the solutions of targets `picks` after every timestep:
        returns a [T, len(picks), nmax] float64 tensor (row t = m^{t+1}; a target of a smaller
        grid fills the first n entries).  One linearisation pass per step."""
        import torch
        assert self.K == 1
        rec = torch.zeros((self.T, len(picks), self.nmax), dtype=torch.float64, device=self.dev)

        def hook(par, bases):
            t = self.step_no % self.T
            with torch.cuda.stream(self.s_main):
                for j, i in enumerate(picks):
                    H, off, _ = self.tgt_sys[i]
                    rec[t, j, :H * H].copy_(self.mt[1 - par][off:off + H * H])
        self.s_main.wait_stream(torch.cuda.current_stream(self.dev))
        self.reset()
        for _ in range(self.T):
            self.step(after_targets=hook)
        self._join()
        torch.cuda.synchronize(self.dev)
        return rec

    def verify_last(self):
        """FP64 relative residual of every target's last solution (operator and right-hand side
        of the last timestep rebuilt through the library)."""
        import torch
        par = self.step_no & 1
        prev = 1 - par                       # m^{T-1} defined the last solve
        bt = torch.empty_like(self.bt)
        d = self._desc(self.tgt_sys, self.mt, bt, prev)
        # with Picard passes the last solve's operator came from the iterate before it
        dr = d if self.K == 1 else self._desc_raw(self.tgt_sys, self._out(self.K - 1, prev, False),
                                                  bt, self.mt[par], self.mt[par])
        rel = torch.empty(self.N, dtype=torch.float64, device=self.dev)
        self.s_main.wait_stream(torch.cuda.current_stream(self.dev))   # the descriptors' copy
        with torch.cuda.stream(self.s_main):
            self.ctx.build_rhs(d, self.N)
            self.ctx.residual(dr, self.N, rel)
        self.s_main.synchronize()
        return rel.cpu().numpy()


def cluster_groups(images, H, assign, seeds):
    """Groups of a clustered image set: for every non-empty cluster c, its seed image
    images[seeds[c]] and the other members, in index order, as its targets (one channel)."""
    images = np.asarray(images, dtype=np.float64).reshape(len(images), -1)
    assign = np.asarray(assign)
    groups = []
    for c, s in enumerate(np.asarray(seeds)):
        if s < 0:
            continue
        members = [i for i in np.nonzero(assign == c)[0] if i != s]
        if not members:
            continue
        groups.append(Group(H, images[s][None], images[members][:, None]))
    return groups


class Chain(Batch):
    """One grid size, one channel: seed_m0 (n,), target_m0 (N, n)."""

    def __init__(self, H, T, m, seed_m0, target_m0, **kw):
        n = H * H
        t = np.asarray(target_m0, dtype=np.float64).reshape(-1, 1, n)
        super().__init__([Group(H, np.asarray(seed_m0).reshape(1, n), t)], T, m, **kw)
        self.H, self.n = H, n

    @property
    def seed_state(self):
        return self.state()[0]

    @property
    def target_state(self):
        return self.state()[1].view(self.N, self.n)
