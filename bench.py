#!/usr/bin/env python3
"""Throughput benchmark of the registration hot path on one MI355X.

Headline (the largest single-registration workload, lv224): a step is one
whole registration of the 224 x 208 x 176 ED LV masks -- prior draw, K = 40
filter iterations over N = 4096 particles (warp-and-score of every particle
over the whole target grid, update, normalise / estimate, systematic
resampling, prediction), reading the estimate -- then warp_apply of that
transform to all 20 mask frames (nearest) and all 20 speckle frames
(trilinear).  Inputs are resident in HBM before timing starts.

value = N x V x K x steps / wall time (particle x voxel evaluations per
second, V the nominal target grid).  The JSON line also carries

* roofline: the dominant kernel (mask warp-and-score), timed live with HIP
  events on the library's stream, against the published FP32 vector peak,
  on the particle x voxel pairs it evaluates (tile culling skips the pairs
  it proves add nothing; the library counts both);
  its gather probe (the same grid, coordinates and source loads and nothing
  else) timed on the particle sets of a real registration;
* cpu_baseline: the CPU oracle on a bounded sample of the same workload;
* nested lines for the other configurations: the 64-pair batch (one graph
  launch, and the same pairs run one after another), the 160^3 speckle image
  registration, time-to-Dice of the learned proposal over 16 held-out pairs,
  and the exhaustive-search baseline on the headline pair.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published dense FP32 vector peak: 256 CUs x 128 FP32 lanes x 2 flops
# (one FMA) per clock x 2.4 GHz = 157.3 TFLOP/s.  Method arithmetic is
# counted in the same unit: an FMA is 2, every other operation 1.
PEAK_FP32_TFLOPS = 256 * 128 * 2 * 2.4e9 / 1e12
# Algorithmic work of one particle x voxel evaluation, FMA counted as 2:
# masks (nearest): 3 coordinate FMAs (6), 3 round-to-index (3), 3 inside
# compares (3), 2 integer count updates (a, c) (2) = 14
OPS_PER_EVAL_MASK = 14.0
# images (trilinear): 3 coordinate FMAs (6), 7 lerps of a subtraction and an
# FMA (21), fixed-point scale-round and convert (2), moment updates n, s, t,
# s^2, t^2, s t (2 products + 6 additions = 8) = 37
OPS_PER_EVAL_IMAGE = 37.0
# source bytes gathered per evaluation (served from L1 / L2, not HBM)
GATHER_BYTES_MASK, GATHER_BYTES_IMAGE = 1.0, 8.0
# image launch configuration timed for speckle160 (layout, particles per
# workgroup, tile depth): the autotuner's choice on that workload
DEFAULT_IMAGE_TUNING = "5,4,256"
KERNEL_SOURCES = ["paper_2504_19930_amd/csrc/score.hip", "paper_2504_19930_amd/csrc/internal.h",
                  "paper_2504_19930_amd/csrc/common.h"]
PMC_MASK = os.path.join(ROOT, "profiles", "k_score_mask_lv224_pmc.md")
PMC_IMAGE = os.path.join(ROOT, "profiles", "k_score_image_speckle160_pmc.md")
GOLDEN = os.path.join(ROOT, "tests", "golden", "full_runs.json")
LV_FRAMES = 20


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_values(path):
    """Values recorded in a committed counter summary, or {} when it is
    missing or the kernel sources changed since it was taken."""
    if not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("    ") and ":" in line:
                k, v = line.strip().split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256") != kernel_sources_hash():
        return {}
    return vals


def pmc_traffic(path):
    """HBM-side bytes per launch (FETCH_SIZE + WRITE_SIZE, each scaled by its
    copy-kernel factor) from a counter summary, or None."""
    vals = pmc_values(path)
    try:
        return (float(vals["fetch_kib_per_dispatch"]) * float(vals["fetch_copy_factor"]) +
                float(vals["write_kib_per_dispatch"]) * float(vals["write_copy_factor"])) * 1024.0
    except (KeyError, ValueError):
        return None


def pmc_gather_path(path, launch_ms):
    """On-chip gather-path figures per launch from a counter summary, or None."""
    vals = pmc_values(path)
    keys = ("l1_tag_lookups_per_dispatch", "l2_read_requests_per_dispatch", "l1_lookups_per_cu_clock",
            "td_busy_frac", "ta_busy_frac", "valu_insts_per_cu_clock", "l2_hit_rate")
    out = {}
    for k in keys:
        try:
            out[k] = float(vals[k])
        except (KeyError, ValueError):
            pass
    if not out:
        return None
    if "l1_tag_lookups_per_dispatch" in out:
        out["l1_lines_GBs"] = out["l1_tag_lookups_per_dispatch"] * 128.0 / (launch_ms * 1e-3) / 1e9
    out["note"] = "from the committed rocprofv3 counter summary; lines of 128 B"
    return out


def roofline(kernel, ops_per_eval, evals_per_launch, launch_ms, launches, gather_bytes, pmc_path, probe):
    achieved = evals_per_launch * ops_per_eval / (launch_ms * 1e-3) / 1e12
    r = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
         "frac": achieved / PEAK_FP32_TFLOPS, "traffic": pmc_traffic(pmc_path), "kernel": kernel,
         "ops_per_eval": ops_per_eval, "evals_per_launch": evals_per_launch, "kernel_ms_per_launch": launch_ms,
         "launches": launches,
         "gather_GBs": evals_per_launch * gather_bytes / (launch_ms * 1e-3) / 1e9,
         "limiter": "on-chip source gathers (L1 / TA path); HBM traffic is first touch only",
         "gather_path": pmc_gather_path(pmc_path, launch_ms)}
    if probe is not None:
        r.update(probe)
    return r


def mask_roofline(launch_ms, launches, work, N, V, probe):
    """The mask kernel's roofline on the work its launches did: tile culling
    proves that a particle adds nothing to a tile whose image reaches no
    occupied source cell and skips it, so `achieved` counts the evaluated
    particle x voxel pairs only (the headline value counts every pair of the
    target grid, as the sums do)."""
    # the counters also cover the final estimate's own one-particle scoring:
    # per launch, the evaluated fraction of the launch's N + 1 particles
    grid = float(N + 1) * V
    frac_eval = work["evaluated"] / work["covered"] if work["covered"] else 1.0
    evaluated, covered = frac_eval * grid, grid
    r = roofline("k_score_mask (warp-and-score, nearest, Dice counts)", OPS_PER_EVAL_MASK, evaluated, launch_ms,
                 launches, GATHER_BYTES_MASK, PMC_MASK, probe)
    frac_int = work.get("interior", 0) / work["evaluated"] if work["evaluated"] else 0.0
    r.update({"evals_per_launch_covered": covered, "evaluated_fraction": frac_eval,
              "interior_fraction_of_evaluated": frac_int,
              "evals_note": "evals_per_launch = particle x voxel pairs evaluated per launch (the culled ones "
                            "excluded): the fraction the cull pre-pass counted over the timed registrations times "
                            "the launch's (N + 1) x V pairs"})
    return r


# ----------------------------------------------------------------- inputs
# Generated on the host before anything touches the GPU: the worker pool
# forks from a process that has not initialised HIP.

def _lv_frame(args):
    import synth
    seed, f = args
    s = synth.lv_sequence(seed=seed, n_frames=LV_FRAMES, frames=[f], speckle=True)
    return s["src_masks"][0], s["tgt_masks"][0], s["src_speckle"][0]


def _lv_ed(seed):
    import synth
    return synth.lv_sequence(seed=seed, frames=[0], speckle=False)


def _batch_pair(spec):
    import synth
    p = synth.make_batch_pair(spec)
    return dict(src=p["src"], tgt=p["tgt"], src_fov=p.get("src_fov"))


def _speckle(_):
    import synth
    return synth.speckle_pair(side=160, seed=2)


def make_inputs(args):
    import multiprocessing as mp

    import numpy as np

    import synth
    inp = {}
    workers = min(16, os.cpu_count() or 1)
    pool = mp.get_context("fork").Pool(workers)
    try:
        jobs = {}
        log(f"generating inputs on {workers} host processes ...")
        if args.only in (None, "lv224"):
            jobs["lv"] = pool.map_async(_lv_frame, [(3, f) for f in range(args.lv_frames)])
        if not args.no_speckle:
            jobs["speckle"] = pool.map_async(_speckle, [0])
        if not args.no_batch:
            inp["batch_specs"] = synth.batch_pairs(64, seed=4)
            jobs["batch"] = pool.map_async(_batch_pair, inp["batch_specs"])
        if not args.no_time_to_dice and args.ttd_pairs > 0:
            jobs["ttd"] = pool.map_async(_lv_ed, [900000 + i for i in range(args.ttd_pairs)])
        if "lv" in jobs:
            frames = jobs["lv"].get()
            inp["lv"] = dict(src_masks=np.stack([f[0] for f in frames]),
                             tgt_masks=np.stack([f[1] for f in frames]),
                             src_speckle=np.stack([f[2] for f in frames]))
        if "speckle" in jobs:
            inp["speckle"] = jobs["speckle"].get()[0]
        if "batch" in jobs:
            inp["batch"] = jobs["batch"].get()
        if "ttd" in jobs:
            inp["ttd"] = jobs["ttd"].get()
    except BaseException:
        pool.terminate()
        raise
    else:
        pool.close()  # workers exit on their own; nothing is terminated
    finally:
        pool.join()
    return inp


# ----------------------------------------------------------------- workloads

def dev(a):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gather_probe_run(reg, K, seed):
    """Probe and production launch times over the particle sets of one whole
    registration (each iteration's set, timed before that iteration runs)."""
    reg.reset(seed)
    tp = ts = 0.0
    for _ in range(K):
        p, s = reg.gather_probe(1)
        tp += p
        ts += s
        reg.step(1)
    return {"gather_probe_ms_per_launch": tp / K, "gather_probe_score_ms_per_launch": ts / K,
            "gather_frac": tp / ts,
            "gather_probe_note": "probe = the warp-and-score grid, culling, coordinates, offsets and source loads "
                                 "only (smc_gather_probe), timed with the production kernel on each particle set of "
                                 f"one {K}-iteration registration; gather_frac = probe time / production time"}


def exhaustive_run(reg, prm, V, smc_ms, smc_score, g=7):
    """The exhaustive-search baseline (EX) on the same pair: every point of a
    g^6 grid over the limits box scored once, argmax reported; timed beside
    one SMC registration (context for the EX-versus-filter comparison of
    Table 4)."""
    import numpy as np
    import torch
    lim, x0 = np.array(prm["limit"]), np.array(prm["x0"])
    lo, step = x0 - lim, 2.0 * lim / (g - 1)
    reg.exhaustive(lo, step, [g] * 6)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = reg.exhaustive(lo, step, [g] * 6)
    ms = (time.perf_counter() - t0) * 1e3
    n = g ** 6
    return {"grid": f"{g}^6 = {n} transforms over x0 +- limit", "ms": ms, "evals_per_s": float(n) * V / (ms * 1e-3),
            "best_score": r["score"], "smc_final_score": smc_score, "smc_ms_per_registration": smc_ms,
            "ex_over_smc_time": ms / smc_ms}


def lv224(inp, args):
    import torch

    from paper_2504_19930_amd import binding, config
    lv = inp["lv"]
    prm = config.workload_params("lv224")
    N, K = prm["n_particles"], prm["n_iters"]
    V = int(lv["tgt_masks"][0].size)
    reg = binding.Registration(dev(lv["src_masks"][0]), dev(lv["tgt_masks"][0]), prm)
    if args.mask_tuning:
        ppg, depth = (int(v) for v in args.mask_tuning.split(","))
        reg.tune(None, ppg, depth)
    sm, ss = dev(lv["src_masks"]), dev(lv["src_speckle"])
    F = len(lv["src_masks"])
    out_m = torch.empty_like(sm)
    out_s = torch.empty_like(ss)
    src_m, src_s = binding.volume(sm[0]), binding.volume(ss[0])

    def step(s):
        reg.reset(1000 + s)
        reg.step(K)
        est = reg.estimate()
        binding.warp_apply(src_m, est["matrix"], "nearest", out_m, n_frames=F, src_frame_stride=V,
                           dst_frame_stride=V)
        binding.warp_apply(src_s, est["matrix"], "trilinear", out_s, n_frames=F, src_frame_stride=V,
                           dst_frame_stride=V)
        return est

    for w in range(args.warmup):
        step(w)
    torch.cuda.synchronize()
    log(f"lv224: timing {args.steps} steps ...")
    reg.profile(True)
    reg.profile_read()
    reg.profile_work()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        est = step(args.warmup + s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = reg.profile_read()
    work = reg.profile_work()
    reg.profile(False)
    launch_ms = prof["score_ms"] / max(1, prof["score_launches"])
    probe = None if args.no_gather_probe else gather_probe_run(reg, K, 77)
    ex = None if args.no_exhaustive else exhaustive_run(reg, prm, V, wall * 1e3 / args.steps, est["score"])
    tuning = reg.tuning()
    reg.close()
    evals = float(N) * V * K * args.steps
    return dict(wall=wall, evals=evals, est=est, N=N, K=K, V=V, F=F, tuning=tuning, prm=prm, exhaustive=ex,
                roofline=mask_roofline(launch_ms, prof["score_launches"], work, N, V, probe),
                filter_ms=prof["filter_ms"] / max(1, prof["filter_launches"]))


def speckle160(inp, args):
    import torch

    from paper_2504_19930_amd import binding, config
    pair = inp["speckle"]
    prm = config.workload_params("speckle160")
    N, K, V = prm["n_particles"], prm["n_iters"], int(pair["tgt"].size)
    src, tgt, fov = dev(pair["src"]), dev(pair["tgt"]), dev(pair["src_fov"])
    out = torch.zeros_like(tgt)
    reg = binding.Registration(src, tgt, prm, src_fov=fov)
    lay, ppg, depth = (int(v) for v in args.image_tuning.split(","))
    reg.tune(lay, ppg, depth)
    src_vol = binding.volume(src)

    def step(s):
        reg.reset(1000 + s)
        reg.step(K)
        est = reg.estimate()
        binding.warp_apply(src_vol, est["matrix"], "trilinear", out)
        return est

    step(0)
    torch.cuda.synchronize()
    steps = args.speckle_steps
    log(f"speckle160: timing {steps} steps ...")
    reg.profile(True)
    reg.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        est = step(1 + s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = reg.profile_read()
    reg.profile(False)
    launch_ms = prof["score_ms"] / max(1, prof["score_launches"])
    probe = None if args.no_gather_probe else gather_probe_run(reg, K, 78)
    tuning = reg.tuning()
    reg.close()
    evals = float(N) * V * K * steps
    return {"value": evals / wall, "unit": "evals/s", "steps": steps, "warmup": 1, "ms_per_step": wall * 1e3 / steps,
            "workload": f"speckle160: 160^3 u8 speckle images, 60 deg apical-cone source FOV, N={N}, K={K}, NCC, "
                        "trilinear; one step = one registration + warp_apply",
            "tuning": tuning, "final_score": est["score"],
            "roofline": roofline("k_score_image (warp-and-score, trilinear)", OPS_PER_EVAL_IMAGE, float(N + 1) * V,
                                 launch_ms, prof["score_launches"], GATHER_BYTES_IMAGE, PMC_IMAGE, probe)}


def batch64(inp, args):
    import numpy as np
    import torch

    from paper_2504_19930_amd import binding, config
    specs, vols = inp["batch_specs"], inp["batch"]
    pairs, prms, evals = [], [], 0.0
    for spec, v in zip(specs, vols):
        if spec["kind"] == "mask":
            prm = config.default_params("dice", spec["n_particles"], 30, 15.0, 8.0 * spec["side"] / 64,
                                        seed=spec["pair"])
        else:
            prm = config.default_params("ncc", spec["n_particles"], 30, 20.0, 12.0 * spec["side"] / 160,
                                        seed=spec["pair"])
        q = dict(src=dev(v["src"]), tgt=dev(v["tgt"]), params=prm)
        if v["src_fov"] is not None:
            q["src_fov"] = dev(v["src_fov"])
        pairs.append(q)
        prms.append(prm)
        evals += spec["n_particles"] * v["tgt"].size * 30
    b = binding.Batch(pairs)
    log("batch64: autotuning ...")
    b.autotune(3)
    tunings = [binding.smc_get_tuning(b.pair(i)) for i in range(len(pairs))]
    log("batch64: one graph launch (warm-up), then one timed ...")
    b.set_seeds(np.arange(64) + 100)
    b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.set_seeds(np.arange(64) + 200)
    b.run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dice = [b.estimate(i)["score"] for i in range(len(pairs))]
    b.close()
    # the same registrations as single contexts, one after another, with the
    # tunings the batch applied (contexts built and warmed outside the clock)
    regs = []
    for q, prm, tu in zip(pairs, prms, tunings):
        r = binding.Registration(q["src"], q["tgt"], prm, src_fov=q.get("src_fov"))
        r.tune(tu["layout"], tu["particles_per_group"], tu["tile_depth"])
        regs.append(r)
    log("batch64: the same 64 registrations back to back ...")
    warmed = set()
    for i, (spec, tu, r) in enumerate(zip(specs, tunings, regs)):
        key = (spec["kind"], tu["layout"], tu["particles_per_group"], tu["tile_depth"])
        if key not in warmed:  # first launches of each kernel instance
            warmed.add(key)
            r.reset(100 + i)
            r.step(30)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, r in enumerate(regs):
        r.reset(200 + i)
        r.step(30)
    torch.cuda.synchronize()
    wall_single = time.perf_counter() - t0
    for r in regs:
        r.close()
    kinds = {}
    for spec, tu in zip(specs, tunings):
        kinds.setdefault(spec["kind"], tu)
    return {"value": evals / wall, "unit": "evals/s", "steps": 1, "warmup": 1, "ms_per_step": wall * 1e3,
            "workload": "batch64: 64 pairs, cubic sides 96..224, N in {1024..8192}, K=30, half shell masks (Dice) "
                        "and half speckle images (NCC); one step = one graph launch of every registration",
            "evals_per_step": evals, "tuning": kinds,
            "back_to_back_ms": wall_single * 1e3, "back_to_back_value": evals / wall_single,
            "batch_speedup_over_back_to_back": wall_single / wall,
            "median_final_score": {"mask": float(np.median(dice[0::2])), "image": float(np.median(dice[1::2]))}}


def time_to_dice(inp, args):
    import numpy as np

    from paper_2504_19930_amd import learned
    if not os.path.exists(learned.WEIGHTS):
        return None
    params = learned.load_weights()
    golden = {}
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as fh:
            golden = json.load(fh)
    rows = []
    log(f"time-to-Dice: learned proposal (N=512) vs plain filter (N=4096) on {len(inp['ttd'])} held-out pairs ...")
    for i, pair in enumerate(inp["ttd"]):
        rows.append(learned.time_to_dice(pair, params, seed=i))
    ratios = [r["ratio"] for r in rows if r["ratio"]]
    checked = []
    for i, r in enumerate(rows):
        g = golden.get(f"lv224_heldout{i}")
        if g is not None:
            checked.append(dict(pair=i, d_star_gpu=r["d_star"], d_star_oracle=g["trace_score"][-1],
                                equal=abs(r["d_star"] - g["trace_score"][-1]) <= 1e-12))
    return {"metric": "time to Dice >= plain final Dice - 0.005, plain (N=4096) / learned (N=512)",
            "median_ratio": float(np.median(ratios)) if ratios else None, "reached": len(ratios), "pairs": len(rows),
            "t_plain_ms": [r["t_plain_ms"] for r in rows], "t_learned_ms": [r["t_learned_ms"] for r in rows],
            "d_star": [r["d_star"] for r in rows], "d_star_oracle_checked": checked,
            "workload": "224x208x176 ED LV masks (held-out seeds 900000+), +-15 deg, +-16 voxels, K <= 40; the "
                        "learned clock includes downsampling and the network forward"}


def cpu_baseline(inp, prm, target_s: float):
    """The oracle's recipe-mode mask warp-and-score (>= 99 % of the path's
    work), timed on a bounded sample of the prior particles of the headline
    workload on the host's cores."""
    import oracle

    lv = inp["lv"]
    s = oracle.Volume(lv["src_masks"][0])
    t = oracle.Volume(lv["tgt_masks"][0])
    pb = oracle.Problem(s, t)
    x = oracle.init_particles(prm)
    V = int(lv["tgt_masks"][0].size)
    threads = oracle.num_threads()
    n = max(1, threads)
    t0 = time.perf_counter()
    pb.score(prm, x[:n])
    dt = time.perf_counter() - t0
    n2 = int(min(len(x), max(n, n * target_s / max(dt, 1e-3))))
    n2 = max(threads, (n2 // threads) * threads)
    t0 = time.perf_counter()
    pb.score(prm, x[:n2])
    dt = time.perf_counter() - t0
    oracle.set_threads(1)
    try:
        n1 = max(1, int(n2 / threads * 0.25))
        t0 = time.perf_counter()
        pb.score(prm, x[:n1])
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(value=n2 * V / dt, unit="evals/s", cores=threads, kind="oracle",
                sample=f"{n2} prior particles x {V} target voxels of the lv224 ED masks, one nearest-neighbour Dice "
                       f"evaluation each ({dt:.1f} s)",
                single_core_value=n1 * V / dt1, single_core_sample=f"{n1} particles ({dt1:.1f} s)",
                host_cpu=model, host_logical_cpus=os.cpu_count())


def copy_probe():
    import torch
    torch.cuda.set_device(0)
    a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda").fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b = a.clone()
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": a.numel(), "copies": 3, "checksum": int(b[::4096].sum().item())}))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-time-to-dice", action="store_true")
    ap.add_argument("--ttd-pairs", type=int, default=16)
    ap.add_argument("--no-batch", action="store_true", help="skip the nested batch64 line")
    ap.add_argument("--no-speckle", action="store_true", help="skip the nested speckle160 line")
    ap.add_argument("--speckle-steps", type=int, default=3)
    ap.add_argument("--no-gather-probe", action="store_true")
    ap.add_argument("--no-exhaustive", action="store_true", help="skip the exhaustive-search line")
    ap.add_argument("--mask-tuning", default=None,
                    help="particles_per_group,tile_depth of the lv224 mask launch (default: the library's)")
    ap.add_argument("--image-tuning", default=DEFAULT_IMAGE_TUNING,
                    help="layout,particles_per_group,tile_depth of the speckle160 warp-and-score launch")
    ap.add_argument("--lv-frames", type=int, default=LV_FRAMES,
                    help="frames of the lv224 sequence generated and warped (the workload has 20)")
    ap.add_argument("--only", choices=["lv224", "speckle160", "batch64", "ttd"], default=None,
                    help="run one workload alone and print its line (for profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 256 MiB (three times), to scale HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the registration path runs on a "
              f"single MI355X; sharding by pair or by particle is a design note, not built)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.only is not None:
        args.no_speckle = args.only != "speckle160"
        args.no_batch = args.only != "batch64"
        args.no_time_to_dice = args.only != "ttd"
        args.no_cpu_baseline = True

    inp = make_inputs(args)  # before anything initialises the GPU

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2504_19930_amd import binding
    binding.lib()
    torch.cuda.set_device(0)

    if args.only == "speckle160":
        print(json.dumps(dict(speckle160(inp, args), n_gpus=1)), flush=True)
        return
    if args.only == "batch64":
        print(json.dumps(dict(batch64(inp, args), n_gpus=1)), flush=True)
        return
    if args.only == "ttd":
        print(json.dumps(dict(time_to_dice(inp, args) or {}, n_gpus=1)), flush=True)
        return
    h = lv224(inp, args)
    line = {
        "metric": "particle×voxel evals/s",
        "value": h["evals"] / h["wall"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["wall"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"lv224: 224x208x176 u8 ED LV masks, N={h['N']} particles, K={h['K']} iterations, "
                               f"Dice, nearest; one step = one full registration + warp_apply of {h['F']} mask "
                               f"and {h['F']} speckle frames",
                   "particles": h["N"], "iterations": h["K"], "target_voxels": h["V"], "score": "dice",
                   "tuning": h["tuning"]},
        "roofline": dict(h["roofline"], filter_ms_per_launch=h["filter_ms"]),
        "final_score": h["est"]["score"],
    }
    if h["exhaustive"] is not None:
        line["exhaustive"] = h["exhaustive"]
    if not args.no_speckle:
        line["speckle160"] = speckle160(inp, args)
    if not args.no_batch:
        line["batch64"] = batch64(inp, args)
    if not args.no_time_to_dice and args.ttd_pairs > 0:
        ttd = time_to_dice(inp, args)
        if ttd is not None:
            line["time_to_dice"] = ttd
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        cb = cpu_baseline(inp, h["prm"], args.cpu_seconds)
        line["cpu_baseline"] = cb
        line["gpu_over_cpu"] = line["value"] / cb["value"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
