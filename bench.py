"""Benchmark: target systems solved per second at FP64-verified relative residual 1e-8.

Workload (one GPU): 64x64 grid (4096 unknowns), 1 seed + 63 targets (blob images, seed blobs
jittered by N(0, 2 px), amplitudes scaled by U[0.9, 1.1]), T = 100 timesteps, seed basis
dimension m = 40, tol 1e-8, FP64.  One step = the whole hot path over the batch: for each of the
100 timesteps, the right-hand sides, the seed GMRES with its kept basis, and the projection +
GMRES polish of all 63 targets, one persistent launch each.  value = 63 * 100 * steps / elapsed
seconds for the projection path (target-Galerkin mode); the same chain with plain GMRES and with
the seed-Galerkin mode is timed beside it.  Each chain is captured once as a HIP graph and
replayed (--eager: enqueued call by call); the polish restart length and workgroups per compute
unit come from the library's autotuner, run on the chain's own inputs before the timed region
(--no-tune: restart length m).  Inputs are resident in device memory before the timed region.

Also timed (--no-uneven skips it): the uneven batch, 32x32 / 64x64 / 128x128 grids with 3
channels each (3072 target systems, 9 seeds) in one launch per timestep; (--no-mixed skips
it) the 128x128 workload (1 seed + 255 targets, m = 60) in mixed and FP64 precision, with each
target's error against the FP64 path; and (--no-learned skips it) the learned-guess workload:
training data from the method's own 64x64 chain (4096 targets), training, and 1024 held-out
targets solved with the learned guess behind residual gates beside projection and plain GMRES.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "target systems solved/sec @ rel-residual 1e-8; projected vs plain GMRES"
HBM_PEAK_GBS = 8000.0

# HBM traffic of target launches (solve_kernel), from two rocprofv3 --pmc runs of this file per
# launch kind (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch averaged over the chain's target
# launches), each scaled by what the same counter reads for a plain device copy of known size in
# the same run (--copy-probe).  A record applies only to the kernel sources it was taken with
# (digest), the restart length, workgroup size and projection placement it was taken at.
TRAFFIC = {
    # means over the last 100 dispatches of each launch kind in counter runs of this file with
    # the launch choices of an unprofiled run (--tuning-from); copy probe: three 256 MiB copies
    # read about 131086 KiB (FETCH_SIZE) and wrote 262144 KiB (WRITE_SIZE) each
    "c2_project": {"csrc_digest": "b82947a142d54c38", "polish_m": 8, "waves": 4, "split": 0,
        "fetch_kib": 8312.19, "write_kib": 15314.77, "fetch_scale": 1.99978, "write_scale": 1.0},
    "c2_plain": {"csrc_digest": "b82947a142d54c38", "polish_m": 6, "waves": 4, "split": -1,
        "fetch_kib": 8074.26, "write_kib": 15234.25, "fetch_scale": 1.99978, "write_scale": 1.0},
    "c3_project_mixed": {"csrc_digest": "b82947a142d54c38", "polish_m": 15, "waves": 8, "split": -1,
        "fetch_kib": 9600652.47, "write_kib": 2493507.40, "fetch_scale": 1.9998, "write_scale": 1.0},
    "c3_project_fp64": {"csrc_digest": "b82947a142d54c38", "polish_m": 9, "waves": 16, "split": 0,
        "fetch_kib": 16500537.72, "write_kib": 5064994.66, "fetch_scale": 1.9998, "write_scale": 1.0},
    "c3_plain_mixed": {"csrc_digest": "b82947a142d54c38", "polish_m": 15, "waves": 8, "split": -1,
        "fetch_kib": 6675145.78, "write_kib": 1634356.40, "fetch_scale": 1.9998, "write_scale": 1.0},
    "c3_plain_fp64": {"csrc_digest": "b82947a142d54c38", "polish_m": 9, "waves": 16, "split": -1,
        "fetch_kib": 12545493.88, "write_kib": 3936355.23, "fetch_scale": 1.9998, "write_scale": 1.0},
    "uneven_project": {"csrc_digest": "b82947a142d54c38", "polish_m": 9, "waves": 8, "split": 0,
        "m": 30, "fetch_kib": 74526416.47, "write_kib": 22978637.78, "fetch_scale": 1.9998,
        "write_scale": 1.0},
    "uneven_plain": {"csrc_digest": "b82947a142d54c38", "polish_m": 10, "waves": 8, "split": -1,
        "fetch_kib": 57597886.69, "write_kib": 17150009.10, "fetch_scale": 1.9998, "write_scale": 1.0},
}


def csrc_digest():
    """Digest of the sources the solve and projection kernels are built from, to tell whether
    stored counter figures still apply."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2511_17634_amd", "csrc")
    for f in ("xkp_device.h", "xkp_internal.h", "xkp_kernels.hip", "xkp_project.hip"):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(name, polish_m):
    """HBM bytes per launch of the launch kind `name` from its stored counter record, or None if
    there is none, the sources have changed, or the restart length, launch shape, projection
    placement or (where the record has one) the seeds' basis dimension m differs."""
    tr = TRAFFIC.get(name)
    if tr is None or csrc_digest() != tr["csrc_digest"] or tr["polish_m"] != polish_m:
        return None
    tu = TUNED.get(name)
    if tu is not None and (tu["waves"] != tr["waves"] or (tu["split"] >= 0) != (tr["split"] >= 0)
                           or tu.get("m", tr.get("m")) != tr.get("m")):
        return None
    return int(1024 * (tr["fetch_kib"] * tr["fetch_scale"]
                       + tr["write_kib"] * tr["write_scale"]))


def roofline(kernel, byts, launch_s, traffic=None, **extra):
    """HBM roofline object of one launch kind: algorithmic bytes per launch over its measured
    duration against the 8 TB/s peak."""
    ach = byts / launch_s / 1e9
    r = {"kernel": kernel, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
         "bytes_per_launch": int(byts), "launch_ms": round(launch_s * 1e3, 4)}
    r.update(extra)
    return r


def gmres_bytes(n, m, iters, restarts, passes=1, sv=8, sop=24):
    """Algorithmic HBM bytes of restarted GMRES(m) with `passes` Gram-Schmidt passes: Arnoldi
    step j reads v_0..v_j once per pass (sv n (j+1) each, sv = bytes per basis element), writes
    v_{j+1} (sv n) and applies the operator (read u and m~, write w: sop n); each cycle end forms
    x += V y (sv n k) and the FP64 true residual (48 n)."""
    iters = np.asarray(iters, dtype=np.int64)
    restarts = np.asarray(restarts, dtype=np.int64)
    total = 0
    for it, rs in zip(iters.ravel(), restarts.ravel()):
        cycles = [m] * int(rs) + [int(it) - int(rs) * m]
        for k in cycles:
            if k <= 0:
                continue
            total += passes * sv * n * k * (k + 1) // 2 + k * (sv * n + sop * n)
            total += sv * n * k + 48 * n
    return total


def launch_alg_bytes(ns, bids, inf, polish_m, project, warm=False, sv=8, sop=24, sbv=0,
                     passes=1):
    """Algorithmic HBM bytes of one target launch, averaged over a chain's launches (inf: target
    infos [T, N]; ns, bids: unknowns and basis id of each target).  Per target: its GMRES bytes
    (gmres_bytes); projected targets also read m~' and b' and write x0 (24 n, + 8 n for x_base
    with a warm start); per launch every seed basis V_k used is read once (8 n k, + sbv n k for
    its low-precision copy)."""
    iters, rest, kd = inf["iters"], inf["restarts"], inf["basis_dim"]
    T, N = iters.shape
    total = 0
    for i in range(N):
        total += gmres_bytes(ns[i], polish_m, iters[:, i], rest[:, i], passes, sv, sop)
        if project:
            total += T * (24 + (8 if warm else 0)) * ns[i]
    if project:
        for t in range(T):
            used = {}
            for i in range(N):
                used[bids[i]] = (ns[i], int(kd[t, i]))
            total += sum((8 + sbv) * n * k for n, k in used.values())
    return total / T


def polish_alg_bytes(ns, inf, polish_m, sv=8, sop=24, passes=1):
    """Algorithmic HBM bytes of one solve launch that polishes projected guesses made by the
    projection launches, averaged over a chain: per target its GMRES bytes and the guess x0
    and b read (16 n)."""
    iters, rest = inf["iters"], inf["restarts"]
    T, N = iters.shape
    total = 0
    for i in range(N):
        total += gmres_bytes(ns[i], polish_m, iters[:, i], rest[:, i], passes, sv, sop)
        total += T * 16 * ns[i]
    return total / T


def projection_roofline(label, ns, inf, proj_s, mixed=False):
    """The projection launches (Gram shares on the matrix cores, the small solves, x0) against
    the matrix-core peak of their contraction's type: FP64, or BF16 in mixed precision."""
    fl = projection_flops(ns, inf)
    peak = 2500.0 if mixed else 78.6
    ach = fl / proj_s / 1e12
    return {"kernel": label, "bound": "mfma", "achieved": round(ach, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(ach / peak, 4), "traffic": None,
            "flops_per_launch": int(fl), "launch_ms": round(proj_s * 1e3, 4)}


def target_rooflines(b, label, r, project, lm, warm=False, mixed=False, traffic_key=None):
    """Roofline objects of a chain's target call.  With the projection inside the solve launch
    (or plain GMRES): the one solve launch against HBM, launch_alg_bytes over the call's measured
    duration lm (ms per timestep).  With the projection in launches of its own (the context's
    autotuned choice): the solve launch (the polish) against HBM and the projection launches
    against the matrix-core peak, each over its own duration from the library's phase events.
    Returns (solve-launch roofline, projection roofline or None, phase figures)."""
    ns, bids = chain_shape(b)
    sv, sop, sbv = (4, 12, 2) if mixed else (8, 24, 0)
    traffic = traffic_bytes(traffic_key, r["polish_m"]) if traffic_key else None
    if project and getattr(b.ctx, "split", -1) >= 0:
        pj, so = target_phase_ms(b)
        byts = polish_alg_bytes(ns, r["infos"], r["polish_m"], sv, sop)
        ro = roofline(f"solve_kernel (polish from the projected guess, {label})", byts,
                      np.mean(so) / 1e3, traffic)
        rp = projection_roofline(f"gram_kernel + x0_kernel (target projection, {label})", ns,
                                 r["infos"], np.mean(pj) / 1e3, mixed)
        return ro, rp, {"projection": "own launches", "split_tiles": int(b.ctx.split),
                        "projection_launch_ms": round(float(np.mean(pj)), 4),
                        "solve_launch_ms": round(float(np.mean(so)), 4)}
    byts = launch_alg_bytes(ns, bids, r["infos"], r["polish_m"], project, warm=warm, sv=sv,
                            sop=sop, sbv=sbv)
    ls = np.mean(lm) / 1e3
    ro = roofline(f"solve_kernel ({'projection + polish' if project else 'plain GMRES'}, "
                  f"{label})", byts, ls, traffic)
    if project:
        fl = projection_flops(ns, r["infos"])
        ro["projection_flops_per_launch"] = int(fl)
        ro["projection_tflops"] = round(fl / ls / 1e12, 3)
        return ro, None, {"projection": "inside the solve launch"}
    return ro, None, {}


def projection_flops(ns, inf):
    """Algorithmic flops of the target-Galerkin products V_k^T [A'V_k | r_base] per launch,
    averaged over a chain: 2 n k (k + 1) per target."""
    kd = np.asarray(inf["basis_dim"], dtype=np.int64)
    n = np.asarray(ns, dtype=np.int64)[None, :]
    return float((2 * n * kd * (kd + 1)).sum()) / kd.shape[0]


def build_c2():
    from synth import CONFIGS, config_images, initial_state
    cfg = CONFIGS["c2"]
    seed, tg = config_images(cfg, 0)
    s0 = initial_state(seed[0])
    t0 = np.stack([initial_state(t[0]) for t in tg])
    return cfg, s0, t0


def build_c4():
    """Groups of the uneven workload: 32x32, 64x64 and 128x128, 3 channels each."""
    from paper_2511_17634_amd.driver import Group
    from synth import CONFIGS, config_images
    cfg = CONFIGS["c4"]
    groups = []
    for gi, gr in enumerate(cfg.groups):
        seed, tg = config_images(cfg, gi)
        groups.append(Group(gr.H, seed.reshape(cfg.channels, -1),
                            tg.reshape(tg.shape[0], cfg.channels, -1)))
    return cfg, groups


def build_c3():
    from synth import CONFIGS, config_images, initial_state
    cfg = CONFIGS["c3"]
    seed, tg = config_images(cfg, 0)
    return cfg, initial_state(seed[0]), np.stack([initial_state(t[0]) for t in tg])


class OracleRecord:
    """The FP64 oracle chain (seed chain, then projection + polish chains) of a few sampled
    targets over all T timesteps, computed in background threads while the GPU legs run; its
    states [T, picks, n] are the reference of the per-target error of the GPU legs."""

    def __init__(self, H, T, m, s0, t0, picks):
        from concurrent.futures import ThreadPoolExecutor
        self.H, self.T, self.m, self.picks = H, T, m, list(picks)
        self._ex = ThreadPoolExecutor(1)
        self._fut = self._ex.submit(self._run, np.array(s0), np.array(t0[self.picks]))

    def _run(self, s0, tp):
        H, T, m = self.H, self.T, self.m
        bases = oracle_seed_chain(H, T, m, s0, T)

        def one(t):
            rec = np.empty((T, H * H))
            oracle_target_chain(H, T, m, t, bases, T, "project",
                                record=lambda k, x: rec.__setitem__(k, x))
            return rec
        return np.stack(_pool(one, list(tp), len(tp)), axis=1)

    def result(self):
        return self._fut.result()


def err_vs_oracle(rec_gpu, rec_o):
    """Per sampled target: max over timesteps of max|x - x_o| / max|x_o|, and of max|x - x_o|
    (states after each timestep, GPU against the FP64 oracle chain)."""
    g = rec_gpu[:, :, :rec_o.shape[2]]
    num = np.abs(g - rec_o).max(axis=2)
    den = np.abs(rec_o).max(axis=2)
    return (num / den).max(axis=0), num.max(axis=0)


def pick_uneven_m(args, cfg4, groups):
    """The seeds' basis dimension m of the projected uneven batch, which the workload leaves
    open: each candidate (--uneven-m) is autotuned, then its first --m-probe-steps timesteps
    are timed eagerly after one untimed step; the fastest is kept.  Returns (m, {m: ms per
    timestep})."""
    import torch
    from paper_2511_17634_amd.driver import Batch
    cands = [int(v) for v in args.uneven_m.split(",") if v.strip()]
    fixed = FIXED_TUNING.get("uneven_project", {}).get("m")
    if fixed is not None or len(cands) == 1 or args.no_tune:
        return (int(fixed) if fixed is not None else (cands[0] if len(cands) == 1 else cfg4.m)), {}
    ms = {}
    for m in cands:
        b = Batch(groups, cfg4.T, m, method="project", mode="target_galerkin",
                  reorth=args.reorth)
        b.autotune(cache=args.tuning_cache)
        b.reset()
        b.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.m_probe_steps):
            b.step()
        torch.cuda.synchronize()
        ms[m] = round((time.perf_counter() - t0) * 1e3 / args.m_probe_steps, 3)
        del b
    best = min(ms, key=ms.get)
    print(f"# uneven m probe (ms per timestep): {ms}, m = {best}", file=sys.stderr, flush=True)
    return best, ms


def uneven_leg(args):
    """Uneven batch: 32x32 / 64x64 / 128x128 x 3 channels, one launch per timestep."""
    from paper_2511_17634_amd.driver import Batch
    graph = not args.eager
    cfg4, groups = build_c4()
    m_proj, m_probe = pick_uneven_m(args, cfg4, groups)
    un = {}
    for name, method in (("project", "project"), ("plain", "plain")):
        m = m_proj if method == "project" else cfg4.m
        b = Batch(groups, cfg4.T, m, method=method, mode="target_galerkin",
                  reorth=args.reorth)
        tu = None if args.no_tune else tune(b, args, f"uneven_{name}")
        if method == "project" and f"uneven_{name}" in TUNED:
            TUNED[f"uneven_{name}"]["m"] = m
        r = time_chain(b, args, args.uneven_steps, 1, graph)
        lm = target_call_ms(b)
        ro, rp, ph = target_rooflines(b, f"{b.N} systems of three sizes per launch", r,
                                      method == "project", lm,
                                      traffic_key=f"uneven_{name}")
        un[name] = {"value": round(b.N * cfg4.T / r["per_chain_s"], 2),
                    "m": m,
                    "ms_per_chain": round(r["per_chain_s"] * 1e3, 2),
                    "target_phase_value": round(b.N * cfg4.T / (sum(lm) / 1e3), 2),
                    "mean_iters": round(r["iters_mean"], 2), "verified": r["ok"],
                    "verified_solves": r["verified_solves"],
                    "polish_m": r["polish_m"],
                    "wg_per_cu": None if tu is None else tu.wg_per_cu,
                    "waves": None if tu is None else tu.waves,
                    "seed_waves": None if tu is None or b.seed_tuning is None
                    else b.seed_tuning.waves,
                    "roofline": ro, **ph}
        if rp is not None:
            un[name]["roofline_projection"] = rp
        print(f"# uneven {name}: {r['per_chain_s'] * 1e3:.1f} ms/chain, ok={r['ok']}, "
              f"launch {np.mean(lm):.3f} ms, frac {un[name]['roofline']['frac']}",
              file=sys.stderr, flush=True)
        del b
    return {"workload": cfg4.name, "targets": sum(g.N * g.C for g in groups),
            "seeds": sum(g.C for g in groups), "timesteps": cfg4.T, "m": m_proj,
            "m_probe_ms_per_step": m_probe, "unit": "target systems/s", **un}


def mixed_leg(args, orc=None):
    """128x128, 1 seed + 255 targets, m = 60, mixed and FP64 precision: throughput, launch
    rooflines, and each sampled target's error against the FP64 oracle chain at every
    timestep."""
    from paper_2511_17634_amd import xkp
    from paper_2511_17634_amd.driver import Chain
    graph = not args.eager
    cfg3, s3, t3 = build_c3()
    H3 = cfg3.groups[0].H
    picks = [0, 127, 254]
    if orc is None and not args.no_oracle_mixed:
        orc = OracleRecord(H3, cfg3.T, cfg3.m, s3, t3, picks)
    mx = {}
    for name, method, prec in (("project_mixed", "project", xkp.MIXED),
                               ("project_fp64", "project", xkp.FP64),
                               ("plain_mixed", "plain", xkp.MIXED),
                               ("plain_fp64", "plain", xkp.FP64)):
        b = Chain(H3, cfg3.T, cfg3.m, s3, t3, method=method, precision=prec,
                  reorth=args.reorth)
        tu = None if args.no_tune else tune(b, args, f"c3_{name}")
        r = time_chain(b, args, args.mixed_steps, 1, graph)
        lm = target_call_ms(b)
        mixed = prec == xkp.MIXED
        ro, rp, ph = target_rooflines(b, f"{b.N} systems per launch", r, method == "project",
                                      lm, mixed=mixed, traffic_key=f"c3_{name}")
        rec = b.record_chain(picks).cpu().numpy() if orc is not None else None
        sms = None
        if method == "project":
            sms = {"alone": round(seed_call_ms(b, True), 4),
                   "beside_targets": round(seed_call_ms(b, False), 4),
                   "rows_per_thread": b.seed_tuning.seed_rows if b.seed_tuning else None}
        mx[name] = {"value": round(b.N * cfg3.T / r["per_chain_s"], 2),
                    "ms_per_chain": round(r["per_chain_s"] * 1e3, 2),
                    "target_phase_value": round(b.N * cfg3.T / (sum(lm) / 1e3), 2),
                    "mean_iters": round(r["iters_mean"], 2), "verified": r["ok"],
                    "verified_solves": r["verified_solves"],
                    "polish_m": r["polish_m"],
                    "waves": None if tu is None else tu.waves,
                    "seed_waves": None if tu is None or b.seed_tuning is None
                    else b.seed_tuning.waves,
                    "mean_guess_residual": round(r["guess_res_mean"], 4),
                    "seed_call_ms": sms, "seeds_redone": r["seeds_redone"],
                    "roofline": ro, **ph}
        if rp is not None:
            mx[name]["roofline_projection"] = rp
        if rec is not None:
            mx[name]["_rec"] = rec
        print(f"# 128x128 {name}: {r['per_chain_s'] * 1e3:.1f} ms/chain, ok={r['ok']}, "
              f"mean iters {r['iters_mean']:.1f}, launch {np.mean(lm):.3f} ms, "
              f"frac {mx[name]['roofline']['frac']}", file=sys.stderr, flush=True)
        del b
    if orc is not None:
        ro = orc.result()
        # each step's solution is within dt ||r||_inf <= tol ||m^{n-1}||_2 of the exact one
        # (Varah), and the step map does not amplify differences in the max norm
        bound = cfg3.T * args.tol * max(np.linalg.norm(s3), np.linalg.norm(t3, axis=1).max())
        for name, v in mx.items():
            e, ea = err_vs_oracle(v.pop("_rec"), ro)
            v["err_vs_oracle"] = [float(f"{x:.3e}") for x in e]
            v["verified"] = v["verified"] and bool((ea <= bound).all())
    return {"workload": cfg3.name, "targets": len(t3), "seeds": 1,
            "timesteps": cfg3.T, "m": cfg3.m, "unit": "target systems/s",
            "err_note": f"targets {picks}: max over the {cfg3.T} timesteps of "
                        "max|x - x_oracle| / max|x_oracle|, x_oracle = the FP64 CPU oracle's "
                        "own chain (seed chain, target-Galerkin projection, GMRES(m) polish); "
                        "both solve every step to 1e-8, so they agree to about T x 1e-8",
            **mx}


def learned_leg(args):
    """64x64 learned-guess workload: training data from the method's own chain (seed + 4096
    targets x 100 timesteps), training on the GPU, then 1024 held-out targets solved by plain
    GMRES, projection + polish, the learned guess behind residual gates 1e-6, 1e-4, 1e-2 and
    none, and the learned correction of the projection (a second network trained on the
    projected guess's coordinate error, kept where it lowers the guess's residual).  Each leg
    is compared with the projection (polish iterations, guess residual, throughput), and a
    sample of held-out targets gets the smallest residual the seed subspace allows (the floor
    no guess built from it can pass)."""
    import torch
    from paper_2511_17634_amd import learned, xkp
    from paper_2511_17634_amd.driver import Batch, Group
    from synth import CONFIGS, config_images, initial_state
    from synth.configs import ROLE_EVAL
    cfg = CONFIGS["c5"]
    T, m = cfg.T, cfg.m
    seed, tg = config_images(cfg, 0)
    s0 = initial_state(seed[0])
    t0 = np.stack([initial_state(t[0]) for t in tg])
    _, ev = config_images(cfg, 0, 0, 1024, role=ROLE_EVAL)
    e0 = np.stack([initial_state(t[0]) for t in ev])
    torch.cuda.synchronize()
    t_gen = time.perf_counter()
    zeta, zeta_p, gen_ok = learned.generate(s0, t0, T, m, with_projection=True)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    ctx = xkp.Context(4096, m, 1)
    imgs = torch.tensor(t0, dtype=torch.float64, device="cuda")
    nets, hists, t_tr = {}, {}, {}
    for name, target in (("full", zeta), ("correction", zeta - zeta_p)):
        nets[name] = xkp.Net(ctx, m + 1, 512, learned.init_params(m + 1, np.random.default_rng(0)))
        t1 = time.perf_counter()
        hists[name] = learned.train(nets[name], imgs, target, args.learned_epochs, 512, 2e-3)
        torch.cuda.synchronize()
        t_tr[name] = round(time.perf_counter() - t1, 2)
    legs, infos, polish_m = {}, {}, 0
    for name, kw in (("project", dict(method="project")), ("plain", dict(method="plain")),
                     ("learned_gate_1e-6", dict(method="learned", gate=1e-6)),
                     ("learned_gate_1e-4", dict(method="learned", gate=1e-4)),
                     ("learned_gate_1e-2", dict(method="learned", gate=1e-2)),
                     ("learned_gate_inf", dict(method="learned", gate=1e300)),
                     ("learned_correction", dict(method="learned", gate=1e300, correction=True))):
        if kw["method"] == "learned":
            net = nets["correction" if kw.get("correction") else "full"]
            kw = dict(method="learned", polish_m=polish_m,
                      learned=dict(params=net.params, scale=1.0, gate=kw["gate"],
                                   correction=bool(kw.get("correction"))))
        b = Batch([Group(64, s0[None], e0[:, None])], T, m, reorth=args.reorth, **kw)
        if kw["method"] == "project" and not args.no_tune:
            polish_m = tune(b, args, f"learned_{name}").polish_m
        elif kw["method"] == "plain" and not args.no_tune:
            tune(b, args, f"learned_{name}")
        r = time_chain(b, args, 1, 1, not args.eager)
        _, ti = b.all_infos()
        infos[name] = ti.copy()
        legs[name] = {"value": round(b.N * T / r["per_chain_s"], 2),
                      "ms_per_chain": round(r["per_chain_s"] * 1e3, 2),
                      "mean_iters": round(r["iters_mean"], 2),
                      "median_guess_residual": float(f"{np.median(ti['guess_res']):.4g}"),
                      "mean_guess_residual": float(f"{np.mean(ti['guess_res']):.4g}"),
                      "accepted": round(float((ti["guess_source"] >= 2).mean()), 4),
                      "polish_m": r["polish_m"], "verified": r["ok"] and gen_ok}
        if name == "project":
            # the floor of the seed subspace on a sample: 16 held-out targets at 4 timesteps
            picks, steps = list(range(0, b.N, b.N // 16))[:16], (0, 9, 49, 99)
            floor = learned.span_floor(b, picks, steps)
        print(f"# learned workload {name}: {r['per_chain_s'] * 1e3:.1f} ms/chain, "
              f"mean iters {r['iters_mean']:.1f}, accepted {legs[name]['accepted']:.3f}",
              file=sys.stderr, flush=True)
        del b
    # every leg against the projection, target by target and timestep by timestep
    tp = infos["project"]
    for name, v in legs.items():
        if name == "project":
            continue
        ti = infos[name]
        v["vs_projection"] = {
            "iters_delta": round(float(ti["iters"].mean() - tp["iters"].mean()), 3),
            "value_ratio": round(v["value"] / legs["project"]["value"], 4),
            "guess_better_frac": round(float((ti["guess_res"] < tp["guess_res"]).mean()), 4)}
    keys = sorted(floor)
    fl = np.array([floor[q] for q in keys])
    fin = fl[np.isfinite(fl)]
    at = lambda inf: np.array([inf["guess_res"][t, i] for t, i in keys])
    sample = {"targets": len({i for _, i in keys}), "timesteps": sorted({t + 1 for t, _ in keys}),
              # a least-squares solve that returned a non-finite value is left out and counted
              "median_floor": float(f"{np.median(fin):.4g}") if fin.size else None,
              "min_floor": float(f"{fin.min():.4g}") if fin.size else None,
              "non_finite_floors": int(fl.size - fin.size),
              "median_projection": float(f"{np.median(at(tp)):.4g}"),
              "median_learned": float(f"{np.median(at(infos['learned_gate_inf'])):.4g}"),
              "median_correction": float(f"{np.median(at(infos['learned_correction'])):.4g}"),
              "note": "min over a of ||b - A V a|| / ||b|| on the seed basis V of that timestep "
                      "(A, b the target's): no guess x_base + V a can have a lower residual, so "
                      "a gate below the floor accepts nothing"}
    return {"workload": cfg.name, "train_targets": len(t0), "eval_targets": len(e0),
            "timesteps": T, "m": m, "unit": "target systems/s",
            "generate_s": round(t_gen, 2), "train_s": t_tr,
            "epochs": args.learned_epochs,
            "loss_per_epoch": {k: [float(f"{v:.4g}") for v in h] for k, h in hists.items()},
            "subspace_floor": sample, "legs": legs}


def copy_gbs():
    """A plain device copy for scale: torch copying 1 GiB device-to-device (read + write bytes),
    timed with HIP events, best of five (a lower bound on the achievable HBM bandwidth; the
    library's own streaming kernels exceed it)."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2 * 8 * (1 << 27) / best / 1e6


def cycle_leg(args):
    """Image cycle (Experiment 2's protocol, 64x64): 100 similar images, a new seed every 50
    images; block 1's targets projected on the basis gathered from both seeds (a = 20 columns
    per seed), against each block's own seed, one seed for all 99 images, and plain GMRES."""
    from paper_2511_17634_amd.driver import Batch, Group
    from synth import CONFIGS, cycle_blocks
    cfg = CONFIGS["c6"]
    H, T, m, a, h = cfg.groups[0].H, cfg.T, cfg.m, 20, 50
    blocks = cycle_blocks(cfg, h)
    groups = [Group(H, s, t) for s, t in blocks]
    one = Group(H, blocks[0][0], np.concatenate([blocks[0][1], blocks[1][0][None],
                                                  blocks[1][1]]))
    legs = {}
    for name, gr, kw in (("accumulate", groups, dict(accumulate=a)),
                         ("seed_per_block", groups, {}),
                         ("one_seed", [one], {}),
                         ("plain", groups, dict(method="plain"))):
        b = Batch(gr, T, m, reorth=args.reorth, **kw)
        if not args.no_tune:
            tune(b, args, f"cycle_{name}")
        r = time_chain(b, args, 1, 1, not args.eager)
        _, ti = b.all_infos()
        legs[name] = {"value": round(b.N * T / r["per_chain_s"], 2),
                      "ms_per_chain": round(r["per_chain_s"] * 1e3, 2),
                      "targets": b.N, "mean_iters": round(r["iters_mean"], 2),
                      "mean_guess_residual": round(r["guess_res_mean"], 4),
                      "mean_basis_dim": round(float(ti["basis_dim"].mean()), 2),
                      "polish_m": r["polish_m"], "verified": r["ok"]}
        print(f"# cycle {name}: {r['per_chain_s'] * 1e3:.1f} ms/chain, mean iters "
              f"{r['iters_mean']:.1f}, guess residual {r['guess_res_mean']:.4f}",
              file=sys.stderr, flush=True)
        del b
    return {"workload": cfg.name, "images": 100, "cycle": h, "a": a, "timesteps": T, "m": m,
            "unit": "target systems/s", "legs": legs}


def cluster_leg(args):
    """Diverse set: 200 images at 64x64 from 4 prototypes, interleaved.  k-means seed selection
    (K = 4 on 8x8 block means) against one seed for all images: projected-guess quality, polish
    iterations and throughput of the chains."""
    import torch
    from paper_2511_17634_amd import xkp
    from paper_2511_17634_amd.driver import Batch, Group, cluster_groups
    from synth import CONFIGS, interleaved_images
    cfg = CONFIGS["c7"]
    H, T, m, K = 64, cfg.T, cfg.m, 4
    imgs = interleaved_images(cfg)
    ctx = xkp.Context(H * H, 8, 1)
    dimg = torch.tensor(imgs, dtype=torch.float64, device="cuda")
    ctx.cluster_seeds(dimg, H, 8, K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, sd, it = ctx.cluster_seeds(dimg, H, 8, K)
    cl_ms = (time.perf_counter() - t0) * 1e3
    groups = cluster_groups(imgs, H, a.cpu().numpy(), sd.cpu().numpy())
    legs = {}
    for name, gr in (("clustered", groups),
                     ("one_seed", [Group(H, imgs[0][None], imgs[1:][:, None])])):
        b = Batch(gr, T, m, reorth=args.reorth)
        if not args.no_tune:
            tune(b, args, f"cluster_{name}")
        r = time_chain(b, args, 1, 1, not args.eager)
        legs[name] = {"value": round(b.N * T / r["per_chain_s"], 2),
                      "ms_per_chain": round(r["per_chain_s"] * 1e3, 2), "targets": b.N,
                      "seeds": b.S, "mean_iters": round(r["iters_mean"], 2),
                      "mean_guess_residual": round(r["guess_res_mean"], 4),
                      "verified": r["ok"]}
        print(f"# cluster {name}: {r['per_chain_s'] * 1e3:.1f} ms/chain, mean iters "
              f"{r['iters_mean']:.1f}, guess residual {r['guess_res_mean']:.4f}",
              file=sys.stderr, flush=True)
        del b
    return {"workload": cfg.name, "K": K, "pool": 8, "cluster_ms": round(cl_ms, 2),
            "lloyd_assignments": it, "unit": "target systems/s", "legs": legs}


def picard_leg(args):
    """64x64 benchmark chain with K = 2 and 3 linearisation passes per timestep (projection for
    the first pass, plain GMRES from the previous iterate for the later ones)."""
    from paper_2511_17634_amd.driver import Chain
    cfg, s0, t0 = build_c2()
    H, T, m = cfg.groups[0].H, cfg.T, cfg.m
    legs = {}
    for K in (2, 3):
        b = Chain(H, T, m, s0, t0, picard=K, reorth=args.reorth)
        if not args.no_tune:
            tune(b, args, f"picard_K{K}")
        r = time_chain(b, args, 1, 1, not args.eager)
        _, pt = b.picard_infos()
        ok = r["ok"] and bool((pt["status"] == 0).all() and (pt["res_true"] <= args.tol).all())
        legs[f"K{K}"] = {"value": round(b.N * T / r["per_chain_s"], 2),
                         "ms_per_chain": round(r["per_chain_s"] * 1e3, 2),
                         "mean_iters_first_pass": round(r["iters_mean"], 2),
                         "mean_iters_later_passes": [round(float(pt["iters"][:, k].mean()), 2)
                                                     for k in range(K - 1)],
                         "verified": ok}
        print(f"# picard K={K}: {r['per_chain_s'] * 1e3:.1f} ms/chain, iters {r['iters_mean']:.1f}"
              f" then {legs[f'K{K}']['mean_iters_later_passes']}", file=sys.stderr, flush=True)
        del b
    return {"workload": cfg.name, "unit": "target systems/s (one per target and timestep)",
            "legs": legs}


def epilogue_leg(args):
    """Score + probability-flow pass over 255 systems of 128x128 (the size of the mixed
    workload), timed with HIP events on the context's stream; HBM roofline with algorithmic
    bytes 8n (read m) + 16n (write the score) + 32n (update the displacement) per system."""
    import torch
    from paper_2511_17634_amd import xkp
    H, N, reps = 128, 255, 20
    n = H * H
    st = torch.cuda.Stream()
    ctx = xkp.Context(n, 8, N, stream=st)
    rng = np.random.default_rng(5)
    m = torch.tensor(rng.uniform(0, 1, (N, n)), dtype=torch.float64, device="cuda")
    b = torch.zeros_like(m)
    score = torch.zeros((N, 2, n), dtype=torch.float64, device="cuda")
    disp = torch.zeros_like(score)
    d = xkp.pack_batch(H, 0.01, 0.5, m, b, m)
    rows = 2 * n * 8 * np.arange(N, dtype=np.int64)
    sp = torch.tensor(score.data_ptr() + rows, device="cuda")
    dp = torch.tensor(disp.data_ptr() + rows, device="cuda")
    torch.cuda.synchronize()
    ctx.score_flow(d, N, xkp.FIELD_MT, sp, dp)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        ctx.score_flow(d, N, xkp.FIELD_MT, sp, dp)
    e1.record(st)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    byts = 56 * n * N
    return {"workload": f"{N} systems of {H}x{H}", "launch_us": round(us, 2),
            "roofline": {"kernel": "score_flow_kernel", "bound": "hbm",
                         "achieved": round(byts / us / 1e3, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(byts / us / 1e3 / HBM_PEAK_GBS, 4),
                         "bytes_per_launch": byts}}


# launch choices per leg (keys as in TRAFFIC): written by --tuning-out, applied by --tuning-from
TUNED = {}
FIXED_TUNING = {}
# legs whose launch choices came from / were added to the --tuning-cache file
CACHE_HITS, CACHE_MISSES = [], []


def tuning_record(b, t):
    """The launch choices a leg runs with (Batch.tuning_record)."""
    return b.tuning_record(t)


def apply_tuning(b, rec):
    """Set a leg's launch choices from a record of tuning_record instead of autotuning (runs
    under a counter profiler, whose serialised dispatches would mislead the autotuners).
    Returns the Tuning the autotuner would have."""
    return b.apply_tuning(rec)


def paper_context(out):
    """The paper's own reductions (Table 4: total time of 100 images over T = 100 steps, the
    cross-matrix projection against a direct sparse solver), quoted with the hardware and
    accuracy it states, beside this run's corresponding ratios; context, not a target."""
    ctx = {"source": "Table 4: total time for 100 images, cross-matrix projection vs a direct "
                     "sparse solver",
           "hardware": "M4 CPU, Python; loose accuracy (average L2 relative error "
                       "0.056 / 0.077 / 0.095), not a fixed residual",
           "reduction": {"32x32": 0.158, "64x64": 0.298, "128x128": 0.437}}
    mine = {"gpu_projection_over_plain_gmres": round(out["value"] / out["plain_gmres"]["value"], 3)}
    ps = (out.get("cpu_baseline") or {}).get("per_system_ms_one_core") or {}
    if ps.get("banded_lu_ms") and ps.get("projection_polish_ms"):
        # the same comparison on the oracle, one core, 64x64, tol 1e-8
        mine["cpu_oracle_projection_vs_banded_lu_reduction"] = round(
            1.0 - ps["projection_polish_ms"] / ps["banded_lu_ms"], 3)
    ctx["this_run"] = mine
    return ctx


def finite(o):
    """The record with every non-finite float replaced by None (strict JSON)."""
    if isinstance(o, float):
        return o if np.isfinite(o) else None
    if isinstance(o, dict):
        return {k: finite(v) for k, v in o.items()}
    if isinstance(o, (list, tuple)):
        return [finite(v) for v in o]
    return o


def save_tuning(args):
    if args.tuning_out:
        with open(args.tuning_out, "w") as f:
            json.dump(TUNED, f, indent=1)


def tune(b, args, key):
    """The library's autotuners on a driver Batch (see Batch.autotune); with --split off the
    projection then stays inside the solve launch.  With --tuning-from the leg `key` takes the
    stored choices instead (a leg the file does not hold is tuned as usual)."""
    if key in FIXED_TUNING:
        t = apply_tuning(b, FIXED_TUNING[key])
    else:
        t = b.autotune(cache=args.tuning_cache)
        (CACHE_HITS if b.tuned_from_cache else CACHE_MISSES).append(key)
        if args.split == "off":
            b.ctx.set_projection_split(-1)
    TUNED[key] = tuning_record(b, t)
    return t


def time_chain(b, args, steps, warmup, graph=True, verify_all=True):
    """Time `steps` full chains (reset + T timesteps) of a driver Batch, replayed from one
    captured graph (or enqueued eagerly); then verify every solve: the kernels' own statuses and
    FP64 true residuals of the last timed chain, and (verify_all) one more eager chain in which
    every target solution of every timestep is re-checked through xkp_residual, whose operator
    is rebuilt from m~ independently of the solve kernel's coefficient arrays."""
    import torch
    for _ in range(warmup):
        b.run()
    torch.cuda.synchronize()
    if graph:
        b.capture()
    t0 = time.perf_counter()
    for _ in range(steps):
        if graph:
            b.replay()
        else:
            b.run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    seed_inf, tgt_inf = b.all_infos()
    checks = {"target status": bool((tgt_inf["status"] == 0).all()),
              "target res_true": bool((tgt_inf["res_true"] <= args.tol).all())}
    if b.with_seeds:
        checks["seed status"] = bool((seed_inf["status"] == 0).all())
    if verify_all and b.K == 1:
        rel = b.verify_chain()
        _, tgt2 = b.all_infos()
        # the eager chain repeats the replayed one: same iteration counts
        checks["eager = replay iterations"] = bool(np.array_equal(tgt2["iters"], tgt_inf["iters"]))
    else:
        rel = b.verify_last()[None]
    checks["xkp_residual"] = bool((rel <= args.tol * (1 + 1e-6)).all())
    ok = all(checks.values())
    if not ok:
        bad = [k for k, v in checks.items() if not v]
        extra = ""
        if b.with_seeds and not checks["seed status"]:
            extra = f" seed statuses {np.unique(seed_inf['status']).tolist()}"
        if not checks["target status"]:
            extra += f" target statuses {np.unique(tgt_inf['status']).tolist()}"
        print(f"# verification failed: {bad}{extra}", file=sys.stderr, flush=True)
    return {
        "elapsed": elapsed, "ok": ok, "per_chain_s": elapsed / steps,
        "iters_mean": float(tgt_inf["iters"].mean()),
        "restarts": tgt_inf["restarts"], "iters": tgt_inf["iters"], "infos": tgt_inf,
        "seed_iters_total": int(seed_inf["iters"].sum()) if b.with_seeds else 0,
        # seeds whose spread-out solve gave up and one workgroup solved again
        "seeds_redone": int((seed_inf["guess_source"] == 4).sum()) if b.with_seeds else 0,
        "guess_res_mean": float(np.mean(tgt_inf["guess_res"])),
        "max_res": float(max(tgt_inf["res_true"].max(), rel.max())),
        "verified_solves": int(rel.size),
        "N": b.N, "polish_m": int(b.params.polish_m) or b.m,
    }


def target_call_ms(b):
    """Per-timestep duration of the target launch (HIP events on the launch's stream) over one
    eager chain."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(b.T)]
    b.reset()
    for t in range(b.T):
        b.step(events=ev[t])
    torch.cuda.synchronize()
    return [a.elapsed_time(e) for a, e in ev]


def target_phase_ms(b):
    """Per-timestep durations (ms) of the target call's projection launches and of its solve
    launch, from the phase events the library records on the call's stream
    (xkp_ctx_set_timing), over one eager chain."""
    import torch
    b.ctx.set_timing(True)
    b.reset()
    pj, sv = [], []
    for _ in range(b.T):
        b.step()
        a, c = b.ctx.last_timing()
        pj.append(a)
        sv.append(c)
    b.ctx.set_timing(False)
    torch.cuda.synchronize()
    return pj, sv


def seed_call_ms(b, alone=True):
    """Mean duration of the seed call (HIP events on the seed stream): over one eager chain in
    which every timestep's target call waits for its seed call to end (alone), or over the
    ordinary pipelined chain (seed n+1 beside targets n)."""
    import torch
    if not b.with_seeds:
        return None
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(b.T)]
    b.reset()
    for t in range(b.T):
        if alone and b.pipeline:
            b.s_seed.wait_stream(b.s_main)
        b.step(seed_events=ev[t])
        if alone and b.pipeline:
            b.s_main.wait_stream(b.s_seed)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(e) for a, e in ev]))


def chain_shape(b):
    """(unknowns, basis id) of every target of a driver Batch."""
    return [H * H for H, _, _ in b.tgt_sys], [bid for _, _, bid in b.tgt_sys]


def per_step_log(inf, digits=4):
    """Mean guess residual and mean iterations of every timestep (rows of infos [T, N])."""
    return {"guess_res_mean": [float(f"{v:.{digits}g}") for v in inf["guess_res"].mean(axis=1)],
            "iters_mean": [round(float(v), 2) for v in inf["iters"].mean(axis=1)]}


def _pool(fn, items, workers):
    """map fn over items with `workers` threads (the oracle's C calls release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    if workers <= 1:
        return [fn(x) for x in items]
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(fn, items))


def oracle_seed_chain(H, T, m, s0, steps, g=0.5, tol=1e-8):
    """The seed chain on the oracle (Section 3, Phase 1): per timestep the seed's GMRES(m) solve
    from 0 and its kept first-cycle basis; returns [(V, Hbar)] per step."""
    import oracle
    dt, ms, out = 1.0 / T, np.array(s0, dtype=np.float64), []
    for _ in range(steps):
        A = oracle.Operator(H, dt, g, ms)
        r = oracle.gmres(A, oracle.rhs(A, ms), m=m, tol=tol, keep_basis=True)
        out.append((r.V, r.Hbar))
        ms = r.x
    return out


def oracle_target_chain(H, T, m, t0, bases, steps, method, g=0.5, tol=1e-8, record=None):
    """One target through `steps` timesteps on the oracle: target-Galerkin projection on the
    step's seed basis then GMRES(m) polish (one Gram-Schmidt pass), or plain GMRES(m) from 0.
    Returns (final state, polish iterations per step); record(step, x) sees every solution."""
    import oracle
    dt, mt, its = 1.0 / T, np.array(t0, dtype=np.float64), []
    for n in range(steps):
        A = oracle.Operator(H, dt, g, mt)
        b = oracle.rhs(A, mt)
        x0 = None
        if method == "project":
            V, Hb = bases[n]
            x0, _, _ = oracle.project(A, b, V, Hb)
        r = oracle.gmres(A, b, x0=x0, m=m, tol=tol, passes=1)
        its.append(r.iters)
        mt = r.x
        if record is not None:
            record(n, mt)
    return mt, its


def scipy_matrix(A):
    """The five-point matrix of an oracle operator as a scipy CSR matrix (coefficients from the
    oracle; the paper's Python direct-solver baseline factorises such a matrix)."""
    import scipy.sparse as sp
    import oracle
    cd, ce, cw, cn, cs = oracle.coeffs(A)
    n, H = A.n, A.H
    j = np.arange(n) % H
    cn = np.where(j + 1 < H, cn, 0.0)[:n - 1]
    cs = np.where(j >= 1, cs, 0.0)[1:]
    return sp.diags([cd, ce[:n - H], cw[H:], cn, cs], [0, H, -H, 1, -1], format="csc")


def cpu_baseline(H, T, m, s0, t0, one_core_targets, steps):
    """The oracle (plain C, FP64) timed on this host's cores on bounded samples of the 64x64
    chain: the projection chain (seed chain, then every target's chain; targets in a thread pool
    over all cores, and on one core for a subset), and per-system times of the banded LU (the
    direct-solver analogue of the paper's SpSolve), plain GMRES(m), projection + polish, and
    scipy's sparse direct solve single-threaded."""
    import oracle
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    workers = max(1, min(ncores, 16))
    tic = time.perf_counter()
    bases = oracle_seed_chain(H, T, m, s0, steps)
    t_seed = time.perf_counter() - tic
    tic = time.perf_counter()
    _pool(lambda t: oracle_target_chain(H, T, m, t, bases, steps, "project"), list(t0), workers)
    t_all = time.perf_counter() - tic
    sub = t0[:one_core_targets]
    tic = time.perf_counter()
    for t in sub:
        oracle_target_chain(H, T, m, t, bases, steps, "project")
    t_one = time.perf_counter() - tic
    # per-system times at timestep 1, one thread
    dt, per = 1.0 / T, {}
    systems = []
    for t in t0[:16]:
        A = oracle.Operator(H, dt, 0.5, t)
        systems.append((A, oracle.rhs(A, t)))

    def timed(fn):
        tic = time.perf_counter()
        for A, b in systems:
            fn(A, b)
        return (time.perf_counter() - tic) / len(systems) * 1e3
    per["banded_lu_ms"] = timed(lambda A, b: oracle.banded_solve(A, b))
    per["plain_gmres_ms"] = timed(lambda A, b: oracle.gmres(A, b, m=m, passes=1))
    V0, H0 = bases[0]
    per["projection_polish_ms"] = timed(
        lambda A, b: oracle.gmres(A, b, x0=oracle.project(A, b, V0, H0)[0], m=m, passes=1))
    try:
        import scipy.sparse.linalg as spl
        mats = [(scipy_matrix(A), b) for A, b in systems[:8]]
        tic = time.perf_counter()
        for M, b in mats:
            spl.spsolve(M, b)
        per["scipy_spsolve_ms"] = (time.perf_counter() - tic) / len(mats) * 1e3
    except ImportError:
        per["scipy_spsolve_ms"] = None
    N = len(t0)
    value = N * steps / (t_seed + t_all)
    return {"value": round(value, 2), "unit": "target systems/s", "cores": workers,
            "kind": "oracle", "nproc": ncores,
            "sample": f"all {N} targets x {steps} of {T} timesteps of the 64x64 chain: the seed "
                      f"chain ({t_seed:.1f} s, one core), then the targets' projection + "
                      f"GMRES({m}) chains in {workers} threads ({t_all:.1f} s)",
            "one_core": {"value": round(len(sub) * steps / (t_seed + t_one), 2),
                         "sample": f"{len(sub)} targets x {steps} timesteps, seed chain "
                                   f"included, {t_seed + t_one:.1f} s"},
            "per_system_ms_one_core": {k: (None if v is None else round(v, 3))
                                       for k, v in per.items()},
            "per_system_note": "timestep 1 of 16 targets (8 for scipy), 64x64, one thread: "
                               "banded LU with partial pivoting (the paper's SpSolve analogue), "
                               "GMRES(m) from 0, target-Galerkin projection + GMRES(m), "
                               "scipy.sparse.linalg.spsolve (SuperLU)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-size batch")
    ap.add_argument("--no-tune", action="store_true", help="default launch parameters")
    ap.add_argument("--eager", action="store_true", help="enqueue eagerly instead of a graph")
    ap.add_argument("--polish-m", type=int, default=0,
                    help="fixed polish restart length (implies --no-tune)")
    ap.add_argument("--uneven-steps", type=int, default=1)
    ap.add_argument("--no-mixed", action="store_true", help="skip the 128x128 mixed workload")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-guess workload")
    ap.add_argument("--learned-epochs", type=int, default=4)
    ap.add_argument("--no-cycle", action="store_true", help="skip the image-cycle workload")
    ap.add_argument("--no-picard", action="store_true", help="skip the Picard-pass legs")
    ap.add_argument("--no-cluster", action="store_true", help="skip the clustered-seed legs")
    ap.add_argument("--only", choices=("uneven", "mixed", "learned", "cycle", "epilogue",
                                       "picard", "cluster"),
                    help="run one of the other workloads alone and print its record (profiling)")
    ap.add_argument("--mixed-steps", type=int, default=1)
    ap.add_argument("--no-oracle-mixed", action="store_true",
                    help="skip the 128x128 oracle chain (per-target error of the mixed legs)")
    ap.add_argument("--legs", default="project,project_seed_galerkin,plain,project_warm,plain_warm",
                    help="comma list of the 64x64 legs to run (profiling runs take one)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--reorth", choices=("auto", "always"), default="auto",
                    help="Gram-Schmidt passes: two only while a seed basis is kept, or always")
    ap.add_argument("--cpu-targets", type=int, default=6,
                    help="targets of the one-core oracle sample")
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--tuning-out", metavar="PATH",
                    help="write every leg's launch choices (JSON) to PATH")
    ap.add_argument("--tuning-from", metavar="PATH",
                    help="take every leg's launch choices from a --tuning-out file instead of "
                         "autotuning (for runs under a counter profiler)")
    ap.add_argument("--tuning-cache", metavar="PATH",
                    help="launch choices cached by device and workload (JSON): a leg found "
                         "there is not autotuned, a leg that is not is autotuned and added")
    ap.add_argument("--uneven-m", default="30,40,60",
                    help="candidates of the seeds' basis dimension m for the projected uneven "
                         "batch (one value: no probe)")
    ap.add_argument("--m-probe-steps", type=int, default=10,
                    help="timesteps timed per m candidate")
    ap.add_argument("--split", choices=("auto", "off"), default="auto",
                    help="projection placement: autotuned (inside the solve launch or in "
                         "launches of its own), or always inside the solve launch")
    args = ap.parse_args()
    if args.tuning_from:
        with open(args.tuning_from) as f:
            FIXED_TUNING.update(json.load(f))
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the path is "
              "built and measured on one GPU only)", file=sys.stderr)
        sys.exit(2)

    from paper_2511_17634_amd import xkp
    from paper_2511_17634_amd.driver import Batch, Chain

    xkp.load()
    if args.copy_probe:
        # a device copy of known size, the scale of the HBM counters of a --pmc run
        import torch
        src = torch.ones(args.copy_probe << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy probe: 3 copies of {args.copy_probe} MiB", file=sys.stderr, flush=True)
        del src, dst
    if args.only:
        rec = {"uneven": uneven_leg, "mixed": mixed_leg, "learned": learned_leg,
               "cycle": cycle_leg, "epilogue": epilogue_leg, "picard": picard_leg,
               "cluster": cluster_leg}[args.only](args)
        save_tuning(args)
        print(json.dumps(finite(rec)), flush=True)
        return
    cfg, s0, t0 = build_c2()
    H, T, m = cfg.groups[0].H, cfg.T, cfg.m
    n = H * H
    graph = not args.eager
    # the FP64 oracle of the 128x128 workload's sampled targets runs on the host meanwhile
    orc = None
    if not args.no_mixed and not args.no_oracle_mixed:
        cfg3, s3, t3 = build_c3()
        orc = OracleRecord(cfg3.groups[0].H, cfg3.T, cfg3.m, s3, t3, [0, 127, 254])

    wanted = args.legs.split(",")
    legs, tunings, launch, roofs = {}, {}, {}, {}
    for name, method, mode, warm in (("project", "project", "target_galerkin", False),
                                     ("project_seed_galerkin", "project", "seed_galerkin", False),
                                     ("plain", "plain", "none", False),
                                     ("project_warm", "project", "target_galerkin", True),
                                     ("plain_warm", "plain", "none", True)):
        if name not in wanted:
            continue
        ch = Chain(H, T, m, s0, t0, method=method, mode=mode, polish_m=args.polish_m,
                   reorth=args.reorth, warm=warm)
        if not args.no_tune and not args.polish_m:
            tunings[name] = (tune(ch, args, f"c2_{name}"), ch.seed_tuning)
        legs[name] = time_chain(ch, args, args.steps, args.warmup, graph)
        if name in ("project", "plain", "project_warm", "plain_warm"):
            launch[name] = target_call_ms(ch)
            roofs[name] = target_rooflines(
                ch, f"{ch.N} systems per launch", legs[name], method == "project", launch[name],
                warm=warm, traffic_key=f"c2_{name}" if args.reorth == "auto" else None)
        if method == "project":
            legs[name]["seed_ms"] = {"alone": round(seed_call_ms(ch, True), 4),
                                     "beside_targets": round(seed_call_ms(ch, False), 4)}
            if name == "project":
                # the same seed call on one workgroup and spread over ceil(n / 256) workgroups,
                # alone and beside the target calls, whichever width the chain runs with
                rows = ch.ctx_seed_rows()
                for w, key in ((0, "one_workgroup"), (1, "spread")):
                    ch.ctx_seed.set_seed_width(w)
                    legs[name]["seed_ms"][f"{key}_alone"] = round(seed_call_ms(ch, True), 4)
                    legs[name]["seed_ms"][f"{key}_beside_targets"] = round(
                        seed_call_ms(ch, False), 4)
                ch.ctx_seed.set_seed_width(rows)
                legs[name]["seed_ms"]["width_used"] = "spread" if rows else "one_workgroup"
        print(f"# {name}: {legs[name]['per_chain_s'] * 1e3:.1f} ms/chain, ok={legs[name]['ok']}, "
              f"mean iters {legs[name]['iters_mean']:.1f}, polish_m {legs[name]['polish_m']}",
              file=sys.stderr, flush=True)
        del ch

    if "project" not in legs or "plain" not in legs:
        # a partial run (profiling): one line per leg, not the benchmark record
        save_tuning(args)
        for k, v in legs.items():
            print(json.dumps({"leg": k, "ms_per_chain": round(v["per_chain_s"] * 1e3, 3),
                              "verified": v["ok"], "mean_iters": round(v["iters_mean"], 2)}))
        return
    N = legs["project"]["N"]
    ns, bids = [n] * N, [0] * N
    per_step = {k: v["per_chain_s"] for k, v in legs.items()}
    value = N * T / per_step["project"]

    def leg_roof(name, project, warm=False):
        ro, rp, ph = roofs[name]
        out_ro = dict(ro)
        if rp is not None:
            out_ro["projection_launches"] = rp
        return out_ro

    def summary(name):
        r = legs[name]
        d = {"value": round(N * T / per_step[name], 2),
             "ms_per_step": round(per_step[name] * 1e3, 3),
             "mean_iters": round(r["iters_mean"], 2), "polish_m": r["polish_m"],
             "mean_guess_residual": round(r["guess_res_mean"], 4),
             "verified": r["ok"], "verified_solves": r["verified_solves"]}
        if name in launch:
            d["target_phase_value"] = round(N * T / (sum(launch[name]) / 1e3), 2)
            d["target_call_ms"] = round(float(np.mean(launch[name])), 4)
            d.update(roofs[name][2])
        if "seed_ms" in r:
            d["seed_call_ms"] = r["seed_ms"]
        return d

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "target systems/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(per_step["project"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg.name, "grid": f"{H}x{H}", "n": n, "targets": N, "seeds": 1,
                   "timesteps": T, "m": m, "tol": args.tol, "projection": "target_galerkin",
                   "polish_m": legs["project"]["polish_m"], "graph": graph,
                   "reorth": args.reorth},
        "verified": all(v["ok"] for v in legs.values()),
        "project": summary("project"),
        "plain_gmres": summary("plain"),
        "autotune": {k: {"polish_m": t.polish_m, "wg_per_cu": t.wg_per_cu, "waves": t.waves,
                         "split": t.split,
                         "ms_best": round(t.ms_best, 4), "ms_default": round(t.ms_default, 4),
                         "seed_waves": None if ts is None else ts.waves,
                         "seed_rows_per_thread": None if ts is None else ts.seed_rows}
                     for k, (t, ts) in tunings.items()},
        # the headline chain's own target launch: projection + polish of the 63 targets
        "roofline": leg_roof("project", True),
        "roofline_plain": leg_roof("plain", False),
        "per_timestep": {"project": per_step_log(legs["project"]["infos"]),
                         "plain_iters_mean": per_step_log(legs["plain"]["infos"])["iters_mean"]},
    }
    out["project"]["seed_iters_per_chain"] = legs["project"]["seed_iters_total"]
    out["project"]["seeds_redone"] = legs["project"]["seeds_redone"]
    if "project_seed_galerkin" in legs:
        out["seed_galerkin"] = summary("project_seed_galerkin")
    if "project_warm" in legs and "plain_warm" in legs:
        out["warm_start"] = {"note": "x_base = m^{n-1} for targets and seed start m^{n-1}",
                             "project": summary("project_warm"),
                             "plain_gmres": summary("plain_warm"),
                             "roofline": leg_roof("project_warm", True, True)}
        out["per_timestep"]["project_warm"] = per_step_log(legs["project_warm"]["infos"])
        out["per_timestep"]["plain_warm_iters_mean"] = \
            per_step_log(legs["plain_warm"]["infos"])["iters_mean"]
    cg = copy_gbs()
    out["roofline"]["torch_copy_gbs"] = round(cg, 1)
    if not args.no_uneven:
        out["uneven"] = uneven_leg(args)
        out["verified"] = out["verified"] and all(
            v["verified"] for k, v in out["uneven"].items() if k in ("project", "plain"))
    if not args.no_mixed:
        out["mixed"] = mixed_leg(args, orc)
        out["verified"] = out["verified"] and all(
            v["verified"] for v in out["mixed"].values() if isinstance(v, dict))
    if not args.no_learned:
        out["learned"] = learned_leg(args)
        out["verified"] = out["verified"] and all(
            v["verified"] for v in out["learned"]["legs"].values())
    out["epilogue"] = epilogue_leg(args)
    out["epilogue"]["roofline"]["torch_copy_gbs"] = round(cg, 1)
    if not args.no_cluster:
        out["cluster"] = cluster_leg(args)
        out["verified"] = out["verified"] and all(
            v["verified"] for v in out["cluster"]["legs"].values())
    if not args.no_picard:
        out["picard"] = picard_leg(args)
        out["verified"] = out["verified"] and all(
            v["verified"] for v in out["picard"]["legs"].values())
    if not args.no_cycle:
        out["cycle"] = cycle_leg(args)
        out["verified"] = out["verified"] and all(
            v["verified"] for v in out["cycle"]["legs"].values())
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(H, T, m, s0, t0, args.cpu_targets, args.cpu_steps)
    out["paper_context"] = paper_context(out)
    if args.tuning_cache:
        out["tuning_cache"] = {"path": args.tuning_cache, "hits": CACHE_HITS,
                               "tuned_and_added": CACHE_MISSES}
    save_tuning(args)
    print(json.dumps(finite(out)), flush=True)


if __name__ == "__main__":
    main()
