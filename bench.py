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

# HBM traffic of the roofline kernel (solve_kernel, plain leg, polish restart 10, 63 systems per
# launch), from two rocprofv3 --pmc runs of this file (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch averaged over the 200 target launches).  FETCH_SIZE read 131087 KiB for a 262144 KiB
# device copy in the same runs (WRITE_SIZE read 262144 KiB): fetch figures are scaled by
# 262144 / 131087.  Valid only for the kernel sources they were taken with (digest below) and
# the restart length they were taken at.
TRAFFIC = {"csrc_digest": "298c3feb44a194ae", "fetch_kib": 35233.5, "write_kib": 95945.5,
           "fetch_scale": 262144.0 / 131086.8, "write_scale": 1.0, "polish_m": 10}


# The same for the projected target launch of the headline chain (target Galerkin, polish
# restart 10, 8 waves, 63 systems), from two more --pmc runs of this file (--legs project).
TRAFFIC_PROJECTED = {"csrc_digest": TRAFFIC["csrc_digest"], "fetch_kib": 88935.4,
                     "write_kib": 196923.1, "fetch_scale": 262144.0 / 131085.1,
                     "write_scale": 1.0, "polish_m": 10}


def csrc_digest():
    """Digest of the sources the solve kernel is built from, to tell whether stored counter
    figures still apply."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2511_17634_amd", "csrc")
    for f in ("xkp_device.h", "xkp_internal.h", "xkp_kernels.hip"):
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(tr=None):
    """HBM bytes per launch of the roofline kernel (or of the launch `tr` describes), or None
    if the sources have changed."""
    tr = TRAFFIC if tr is None else tr
    if csrc_digest() != tr["csrc_digest"]:
        return None
    return int(1024 * (tr["fetch_kib"] * tr["fetch_scale"]
                       + tr["write_kib"] * tr["write_scale"]))


def gmres_bytes(n, m, iters, restarts, passes=1):
    """Algorithmic HBM bytes of restarted GMRES(m) with `passes` Gram-Schmidt passes, FP64:
    Arnoldi step j reads v_0..v_j once per pass (8 n (j+1) each), writes v_{j+1} (8 n) and
    applies the operator (read u and m~, write w: 24 n); each cycle end forms x += V y (8 n k)
    and the true residual (48 n)."""
    iters = np.asarray(iters, dtype=np.int64)
    restarts = np.asarray(restarts, dtype=np.int64)
    total = 0
    for it, rs in zip(iters.ravel(), restarts.ravel()):
        cycles = [m] * int(rs) + [int(it) - int(rs) * m]
        for k in cycles:
            if k <= 0:
                continue
            total += sum(8 * passes * n * (j + 1) + 8 * n + 24 * n for j in range(k))
            total += 8 * n * k + 48 * n
    return total


def projected_bytes_flops(n, polish_m, inf, ntc_max=2):
    """Algorithmic HBM bytes and FP64 matrix-core flops of the projected target launches
    (target Galerkin, FP64, x_base = 0), summed over the solves in `inf` (target infos of a
    chain).  Per target with a kept basis of k columns: A'V_k reads V_k (8 n k) and writes
    W = [A'V_k | r_base] (8 n (k+1)); the Gram reads V_k once per pass over at most ntc_max
    16-wide column tiles of W and W once (8 n k passes + 8 n (k+1)); x0 = V_k alpha reads V_k and
    writes x0 (8 n k + 8 n); then the polish's GMRES bytes (gmres_bytes, one Gram-Schmidt pass).
    Flops: one 16x16x4 product (2048 flops) per 4 rows for every pair of 16-wide row tiles of
    V_k and column tiles of W, as executed (tiles padded)."""
    byts, flops = 0, 0
    ngroups = (n + 7) // 8
    for k in np.asarray(inf["basis_dim"], dtype=np.int64).ravel():
        k = int(k)
        if k <= 0:
            continue
        ktr, ktc = (k + 15) // 16, (k + 16) // 16
        passes = (ktc + ntc_max - 1) // ntc_max
        byts += 8 * n * (k + (k + 1) + passes * k + (k + 1) + k + 1)
        flops += 2048 * 2 * ngroups * ktr * ktc
    byts += gmres_bytes(n, polish_m, inf["iters"], inf["restarts"], 1)
    return byts, flops


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


def err_vs_fp64(b, tol=1e-12):
    """Per-target max |x - x64| / max |x64| of the chain's last solutions against the same
    systems solved again by the FP64 path (plain GMRES to `tol`)."""
    import torch
    from paper_2511_17634_amd import xkp
    par = b.step_no & 1
    prev = 1 - par
    bt = torch.empty_like(b.bt)
    x64 = torch.empty_like(b.bt)
    d = b._desc(b.tgt_sys, b.mt, bt, prev, x_from=x64)
    ctx = xkp.Context(b.nmax, b.m, b.N, stream=b.s_main)
    info = ctx.new_infos(b.N)
    b.s_main.wait_stream(torch.cuda.current_stream())
    P = xkp.Context.params(b.m, tol=tol, mode="none", batch_max_n=b.nmax)
    ctx.build_rhs(d, b.N)
    ctx.target_project_solve(d, b.N, 0, None, P, info)
    b.s_main.synchronize()
    x = b.state()[1]
    errs = []
    for H, off, _ in b.tgt_sys:
        n = H * H
        ref = x64[off:off + n]
        errs.append(float((x[off:off + n] - ref).abs().max() / ref.abs().max()))
    ok = bool((xkp.infos_to_numpy(info)["status"] == 0).all())
    return np.array(errs), ok


def uneven_leg(args):
    """Uneven batch: 32x32 / 64x64 / 128x128 x 3 channels, one launch per timestep."""
    from paper_2511_17634_amd.driver import Batch
    graph = not args.eager
    cfg4, groups = build_c4()
    un = {}
    for name, method in (("project", "project"), ("plain", "plain")):
        b = Batch(groups, cfg4.T, cfg4.m, method=method, mode="target_galerkin",
                  reorth=args.reorth)
        tu = None if args.no_tune else b.autotune()
        r = time_chain(b, args, args.uneven_steps, 1, graph)
        un[name] = {"value": round(b.N * cfg4.T / r["per_chain_s"], 2),
                    "ms_per_chain": round(r["per_chain_s"] * 1e3, 2),
                    "mean_iters": round(r["iters_mean"], 2), "verified": r["ok"],
                    "polish_m": r["polish_m"],
                    "wg_per_cu": None if tu is None else tu.wg_per_cu,
                    "waves": None if tu is None else tu.waves,
                    "seed_waves": None if tu is None or b.seed_tuning is None
                    else b.seed_tuning.waves}
        print(f"# uneven {name}: {r['per_chain_s'] * 1e3:.1f} ms/chain, ok={r['ok']}",
              file=sys.stderr, flush=True)
        del b
    return {"workload": cfg4.name, "targets": sum(g.N * g.C for g in groups),
            "seeds": sum(g.C for g in groups), "timesteps": cfg4.T, "m": cfg4.m,
            "unit": "target systems/s", **un}


def mixed_leg(args):
    """128x128, 1 seed + 255 targets, m = 60, mixed and FP64 precision."""
    from paper_2511_17634_amd import xkp
    from paper_2511_17634_amd.driver import Chain
    graph = not args.eager
    cfg3, s3, t3 = build_c3()
    H3 = cfg3.groups[0].H
    mx = {}
    for name, method, prec in (("project_mixed", "project", xkp.MIXED),
                               ("project_fp64", "project", xkp.FP64),
                               ("plain_mixed", "plain", xkp.MIXED),
                               ("plain_fp64", "plain", xkp.FP64)):
        b = Chain(H3, cfg3.T, cfg3.m, s3, t3, method=method, precision=prec,
                  reorth=args.reorth)
        tu = None if args.no_tune else b.autotune()
        r = time_chain(b, args, args.mixed_steps, 1, graph)
        roof = None
        if name == "plain_fp64":
            # the same kernel roofline as the 64x64 record, here on the HBM-bound size
            lm = target_call_ms(b)
            n3 = H3 * H3
            passes = 1 if args.reorth == "auto" else 2
            byts = gmres_bytes(n3, r["polish_m"], r["iters"], r["restarts"], passes) / cfg3.T
            ls = sum(lm) / 1e3 / cfg3.T
            roof = {"kernel": f"solve_kernel (plain GMRES, {len(t3)} systems per launch)",
                    "bound": "hbm", "achieved": round(byts / ls / 1e9, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(byts / ls / 1e9 / HBM_PEAK_GBS, 4),
                    "bytes_per_launch": int(byts), "launch_ms": round(ls * 1e3, 4)}
        e, eok = err_vs_fp64(b)
        mx[name] = {"value": round(b.N * cfg3.T / r["per_chain_s"], 2),
                    "ms_per_chain": round(r["per_chain_s"] * 1e3, 2),
                    "mean_iters": round(r["iters_mean"], 2), "verified": r["ok"] and eok,
                    "polish_m": r["polish_m"],
                    "waves": None if tu is None else tu.waves,
                    "seed_waves": None if tu is None or b.seed_tuning is None
                    else b.seed_tuning.waves,
                    "mean_guess_residual": round(r["guess_res_mean"], 4),
                    "err_vs_fp64_max": float(f"{e.max():.3e}"),
                    "err_vs_fp64_median": float(f"{np.median(e):.3e}")}
        if roof is not None:
            mx[name]["roofline"] = roof
        print(f"# 128x128 {name}: {r['per_chain_s'] * 1e3:.1f} ms/chain, ok={r['ok']}, "
              f"mean iters {r['iters_mean']:.1f}, max err vs fp64 {e.max():.2e}",
              file=sys.stderr, flush=True)
        del b
    return {"workload": cfg3.name, "targets": len(t3), "seeds": 1,
            "timesteps": cfg3.T, "m": cfg3.m, "unit": "target systems/s",
            "err_note": "per-target max |x - x_fp64| / max |x_fp64| at the last timestep, "
                        "x_fp64 = the same systems re-solved by the FP64 path to 1e-12", **mx}


def learned_leg(args):
    """64x64 learned-guess workload: training data from the method's own chain (seed + 4096
    targets x 100 timesteps), training on the GPU, then 1024 held-out targets solved by plain
    GMRES, projection + polish and the learned guess behind residual gates 1e-6, 1e-2, 1e300."""
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
    zeta, gen_ok = learned.generate(s0, t0, T, m)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    ctx = xkp.Context(4096, m, 1)
    net = xkp.Net(ctx, m + 1, 512, learned.init_params(m + 1, np.random.default_rng(0)))
    imgs = torch.tensor(t0, dtype=torch.float64, device="cuda")
    t_tr = time.perf_counter()
    hist = learned.train(net, imgs, zeta, args.learned_epochs, 512, 2e-3)
    torch.cuda.synchronize()
    t_tr = time.perf_counter() - t_tr
    legs, polish_m = {}, 0
    for name, kw in (("project", dict(method="project")), ("plain", dict(method="plain")),
                     ("learned_gate_1e-6", dict(method="learned", gate=1e-6)),
                     ("learned_gate_1e-2", dict(method="learned", gate=1e-2)),
                     ("learned_gate_inf", dict(method="learned", gate=1e300))):
        if kw["method"] == "learned":
            kw = dict(method="learned", polish_m=polish_m,
                      learned=dict(params=net.params, scale=1.0, gate=kw["gate"]))
        b = Batch([Group(64, s0[None], e0[:, None])], T, m, reorth=args.reorth, **kw)
        if kw["method"] == "project" and not args.no_tune:
            polish_m = b.autotune().polish_m
        elif kw["method"] == "plain" and not args.no_tune:
            b.autotune()
        r = time_chain(b, args, 1, 1, not args.eager)
        _, ti = b.all_infos()
        legs[name] = {"value": round(b.N * T / r["per_chain_s"], 2),
                      "ms_per_chain": round(r["per_chain_s"] * 1e3, 2),
                      "mean_iters": round(r["iters_mean"], 2),
                      "median_guess_residual": float(f"{np.median(ti['guess_res']):.4g}"),
                      "accepted": round(float((ti["guess_source"] == 2).mean()), 4),
                      "polish_m": r["polish_m"], "verified": r["ok"] and gen_ok}
        print(f"# learned workload {name}: {r['per_chain_s'] * 1e3:.1f} ms/chain, "
              f"mean iters {r['iters_mean']:.1f}, accepted {legs[name]['accepted']:.3f}",
              file=sys.stderr, flush=True)
        del b
    return {"workload": cfg.name, "train_targets": len(t0), "eval_targets": len(e0),
            "timesteps": T, "m": m, "unit": "target systems/s",
            "generate_s": round(t_gen, 2), "train_s": round(t_tr, 2),
            "epochs": args.learned_epochs, "loss_per_epoch": [float(f"{v:.4g}") for v in hist],
            "legs": legs}


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
            b.autotune()
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
            b.autotune()
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
            b.autotune()
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


def time_chain(b, args, steps, warmup, graph=True):
    """Time `steps` full chains (reset + T timesteps) of a driver Batch, replayed from one
    captured graph (or enqueued eagerly), then verify every solve of the last chain."""
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
    ok = bool((tgt_inf["status"] == 0).all() and (tgt_inf["res_true"] <= args.tol).all())
    if b.with_seeds:
        ok = ok and bool((seed_inf["status"] == 0).all())
    # independent FP64 check of the last timestep through the residual entry point
    rel = b.verify_last()
    ok = ok and bool((rel <= args.tol * (1 + 1e-6)).all())
    return {
        "elapsed": elapsed, "ok": ok, "per_chain_s": elapsed / steps,
        "iters_mean": float(tgt_inf["iters"].mean()),
        "restarts": tgt_inf["restarts"], "iters": tgt_inf["iters"],
        "seed_iters_total": int(seed_inf["iters"].sum()) if b.with_seeds else 0,
        "guess_res_mean": float(np.mean(tgt_inf["guess_res"])),
        "max_res": float(max(tgt_inf["res_true"].max(), rel.max())),
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


def cpu_baseline(H, T, m, s0, t0, n_targets, steps, reorth="auto"):
    """The oracle (single-threaded C, FP64) on a bounded sample of the same chain."""
    from oracle.chain import run_chain
    t = time.perf_counter()
    _, _, st = run_chain(s0, t0[:n_targets], H, T, m, method="project", steps=steps,
                         reorth=reorth)
    el = time.perf_counter() - t
    return {"value": n_targets * steps / el, "unit": "target systems/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_targets} of 63 targets x {steps} of {T} timesteps of the same "
                      f"64x64 chain (seed chain included), target-Galerkin projection + "
                      f"GMRES({m}) polish, {el:.1f} s"}


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
    ap.add_argument("--legs", default="project,project_seed_galerkin,plain",
                    help="comma list of the 64x64 legs to run (profiling runs take one)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--reorth", choices=("auto", "always"), default="auto",
                    help="Gram-Schmidt passes: two only while a seed basis is kept, or always")
    ap.add_argument("--cpu-targets", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is described in DESIGN.md, not run)", file=sys.stderr)
        sys.exit(2)

    from paper_2511_17634_amd import xkp
    from paper_2511_17634_amd.driver import Batch, Chain

    xkp.load()
    if args.only:
        rec = {"uneven": uneven_leg, "mixed": mixed_leg, "learned": learned_leg,
               "cycle": cycle_leg, "epilogue": epilogue_leg, "picard": picard_leg,
               "cluster": cluster_leg}[args.only](args)
        print(json.dumps(rec), flush=True)
        return
    cfg, s0, t0 = build_c2()
    H, T, m = cfg.groups[0].H, cfg.T, cfg.m
    n = H * H
    graph = not args.eager

    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy probe: 3 copies of {args.copy_probe} MiB", file=sys.stderr, flush=True)
        del src, dst
    wanted = args.legs.split(",")
    legs, tunings = {}, {}
    for name, method, mode in (("project", "project", "target_galerkin"),
                               ("project_seed_galerkin", "project", "seed_galerkin"),
                               ("plain", "plain", "none")):
        if name not in wanted:
            continue
        ch = Chain(H, T, m, s0, t0, method=method, mode=mode, polish_m=args.polish_m,
                   reorth=args.reorth)
        if not args.no_tune and not args.polish_m:
            tunings[name] = (ch.autotune(), ch.seed_tuning)
        legs[name] = time_chain(ch, args, args.steps, args.warmup, graph)
        if name == "plain":
            launch_ms = target_call_ms(ch)
            plain_chain = ch
        if name == "project":
            proj_launch_ms = target_call_ms(ch)
            proj_infos = ch.all_infos()[1]
        print(f"# {name}: {legs[name]['per_chain_s'] * 1e3:.1f} ms/chain, ok={legs[name]['ok']}, "
              f"mean iters {legs[name]['iters_mean']:.1f}, polish_m {legs[name]['polish_m']}",
              file=sys.stderr, flush=True)

    if "project" not in legs or "plain" not in legs:
        # a partial run (profiling): one line per leg, not the benchmark record
        for k, v in legs.items():
            print(json.dumps({"leg": k, "ms_per_chain": round(v["per_chain_s"] * 1e3, 3),
                              "verified": v["ok"], "mean_iters": round(v["iters_mean"], 2)}))
        return
    N = legs["project"]["N"]
    per_step = {k: v["per_chain_s"] for k, v in legs.items()}
    value = N * T / per_step["project"]
    # roofline of the dominant kernel: the batched solve kernel in the plain leg (GMRES only),
    # one launch per timestep, timed by HIP events on its stream
    pl = legs["plain"]
    passes = 1 if args.reorth == "auto" else 2
    byts = gmres_bytes(n, pl["polish_m"], pl["iters"], pl["restarts"], passes) / T  # per launch
    launch_s = sum(launch_ms) / 1e3 / T
    achieved = byts / launch_s / 1e9
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
        "plain_gmres": {"value": round(N * T / per_step["plain"], 2),
                        "ms_per_step": round(per_step["plain"] * 1e3, 3),
                        "mean_iters": round(pl["iters_mean"], 2), "restart": pl["polish_m"]},
        "seed_galerkin": None if "project_seed_galerkin" not in legs else {
            "value": round(N * T / per_step["project_seed_galerkin"], 2),
            "ms_per_step": round(per_step["project_seed_galerkin"] * 1e3, 3),
            "mean_iters": round(legs["project_seed_galerkin"]["iters_mean"], 2),
            "polish_m": legs["project_seed_galerkin"]["polish_m"]},
        "projection": {"mean_polish_iters": round(legs["project"]["iters_mean"], 2),
                       "mean_guess_residual": round(legs["project"]["guess_res_mean"], 4),
                       "seed_iters_per_chain": legs["project"]["seed_iters_total"]},
        "autotune": {k: {"polish_m": t.polish_m, "wg_per_cu": t.wg_per_cu, "waves": t.waves,
                         "ms_best": round(t.ms_best, 4), "ms_default": round(t.ms_default, 4),
                         "seed_waves": None if ts is None else ts.waves}
                     for k, (t, ts) in tunings.items()},
        "roofline": {"kernel": "solve_kernel (plain GMRES leg, 63 systems per launch)",
                     "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_bytes() if args.reorth == "auto"
                     and pl["polish_m"] == TRAFFIC["polish_m"] else None,
                     "bytes_per_launch": int(byts), "launch_ms": round(launch_s * 1e3, 4)},
    }
    # the headline chain's own target launch (projection + polish, 63 systems), the same
    # kernel: HBM roofline of its algorithmic bytes, and its FP64 matrix-core flops
    pb, pf = projected_bytes_flops(n, legs["project"]["polish_m"], proj_infos)
    pls = sum(proj_launch_ms) / 1e3 / T
    pach = pb / T / pls / 1e9
    out["roofline_projected"] = {
        "kernel": "solve_kernel (projection + polish, target Galerkin, 63 systems per launch)",
        "bound": "hbm", "achieved": round(pach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(pach / HBM_PEAK_GBS, 4),
        "traffic": traffic_bytes(TRAFFIC_PROJECTED) if args.reorth == "auto"
        and legs["project"]["polish_m"] == TRAFFIC_PROJECTED["polish_m"] else None,
        "bytes_per_launch": int(pb / T), "launch_ms": round(pls * 1e3, 4),
        "mfma_f64_flops_per_launch": int(pf / T),
        "mfma_f64_tflops": round(pf / T / pls / 1e12, 3), "mfma_f64_peak_tflops": 78.6}
    del plain_chain
    cg = copy_gbs()
    out["roofline"]["torch_copy_gbs"] = round(cg, 1)
    if not args.no_uneven:
        out["uneven"] = uneven_leg(args)
        out["verified"] = out["verified"] and all(
            v["verified"] for k, v in out["uneven"].items() if k in ("project", "plain"))
    if not args.no_mixed:
        out["mixed"] = mixed_leg(args)
        r128 = out["mixed"].get("plain_fp64", {}).get("roofline")
        if r128:
            r128["torch_copy_gbs"] = round(cg, 1)
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
        out["cpu_baseline"] = cpu_baseline(H, T, m, s0, t0, args.cpu_targets, args.cpu_steps,
                                           args.reorth)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
