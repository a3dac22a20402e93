#!/usr/bin/env python3
"""Throughput benchmark of the registration hot path on one MI355X.

A step is one whole registration of the 160^3 speckle workload: prior draw,
K = 30 filter iterations over N = 2048 particles (warp-and-score of every
particle over the whole target grid, update, normalise / estimate,
systematic resampling, prediction), reading the estimate, and applying it to
the source with warp_apply.  Inputs are resident in HBM before timing starts.

value = N x V x K x steps / wall time (particle x voxel evaluations per
second, V the nominal target grid).  The JSON line also carries the roofline
of the dominant kernel (warp-and-score, timed live with HIP events on the
library's stream) and the CPU oracle timed on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import hashlib

# MI355X VALU issue: the published FP32 vector peak, 157.3 TFLOP/s, is 256
# CUs x 128 lane-FMAs per clock x 2.4 GHz x 2 flops; one 32-bit VALU lane
# operation per lane slot gives 78.6e12 operations per second
PEAK_VALU_TOPS = 256 * 128 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
# algorithmic ALU work of one trilinear particle x voxel evaluation: 3
# coordinate FMAs, 7 lerps of a subtraction and an FMA (14), fixed-point
# scale-round and convert (2), six sum updates (n, s, t, s^2, t^2, s t)
OPS_PER_EVAL = 25.0
# source gather: the 2 x 2 x 2 taps (served from L1 / L2, not HBM), plus the
# target byte shared by the particles of a workgroup
GATHER_BYTES_PER_EVAL = 8.0
# launch configuration timed by default (layout, particles per workgroup,
# tile depth): the fastest setting of the autotuner on this workload
DEFAULT_TUNING = "5,4,256"
# the committed hardware-counter summary of the warp-and-score kernel
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_score_image_speckle160_pmc.md")
KERNEL_SOURCES = ["paper_2504_19930_amd/csrc/score.hip", "paper_2504_19930_amd/csrc/internal.h",
                  "paper_2504_19930_amd/csrc/common.h"]


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_values():
    """The values recorded in the committed counter summary, or {} when it is
    missing or the kernel sources changed since it was taken."""
    if not os.path.exists(PMC_SUMMARY):
        return {}
    vals = {}
    with open(PMC_SUMMARY) as fh:
        for line in fh:
            if line.startswith("    ") and ":" in line:
                k, v = line.strip().split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256") != kernel_sources_hash():
        return {}
    return vals


def pmc_traffic():
    """HBM-side bytes per warp-and-score launch from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by its copy-kernel factor),
    or None when the summary is missing or the kernel sources changed since."""
    vals = pmc_values()
    try:
        return (float(vals["fetch_kib_per_dispatch"]) * float(vals["fetch_copy_factor"]) +
                float(vals["write_kib_per_dispatch"]) * float(vals["write_copy_factor"])) * 1024.0
    except (KeyError, ValueError):
        return None


def pmc_gather_path():
    """On-chip gather-path figures per warp-and-score launch from the same
    summary (L1 cache-line lookups, L1 -> L2 read requests, busy fractions), or
    None."""
    vals = pmc_values()
    keys = ("l1_tag_lookups_per_dispatch", "l2_read_requests_per_dispatch", "l1_lookups_per_cu_clock",
            "td_busy_frac", "ta_busy_frac", "valu_insts_per_cu_clock")
    try:
        return {k: float(vals[k]) for k in keys}
    except (KeyError, ValueError):
        return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(pair, prm, target_s: float):
    """The oracle's recipe-mode warp-and-score (>= 99 % of the path's work),
    timed on a bounded sample of the prior particles on the host's cores."""
    import numpy as np

    import oracle

    s = oracle.Volume(pair["src"], fov=pair["src_fov"])
    t = oracle.Volume(pair["tgt"])
    pb = oracle.Problem(s, t)
    # a larger draw from the same prior, so the sample is not capped at N
    x = oracle.init_particles(dict(prm, n_particles=16 * prm["n_particles"]))
    V = pair["tgt"].size
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
    # one core, on a sample a quarter as long
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
                sample=f"{n2} prior particles x {V} target voxels, one trilinear NCC evaluation each "
                       f"({dt:.1f} s)",
                single_core_value=n1 * V / dt1, single_core_sample=f"{n1} particles ({dt1:.1f} s)",
                host_cpu=model, host_logical_cpus=os.cpu_count())


def _batch_pair(spec):
    import synth
    p = synth.make_batch_pair(spec)
    return dict(src=p["src"], tgt=p["tgt"], src_fov=p.get("src_fov"))


def other_workload(name, steps, warmup):
    """The full-size mask registration (lv224) and the 64-pair batch
    (batch64), timed the same way; they document the other configurations and
    are not the headline line (that is the default workload)."""
    import numpy as np
    import torch

    import synth
    from paper_2504_19930_amd import binding, config
    binding.lib()
    torch.cuda.set_device(0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    if name == "lv224":
        log("generating the 224x208x176 LV sequence (20 frames, masks and speckle) ...")
        seq = synth.lv_sequence(seed=3, n_frames=20, speckle=True)
        prm = config.workload_params("lv224")
        N, K, V = prm["n_particles"], prm["n_iters"], seq["tgt"].size
        reg = binding.Registration(dev(seq["src"]), dev(seq["tgt"]), prm)
        sm, ss = dev(seq["src_masks"]), dev(seq["src_speckle"])
        out_m = torch.empty((20,) + seq["tgt"].shape, dtype=torch.uint8, device="cuda")
        out_s = torch.empty_like(out_m)

        def step(s):
            reg.reset(1000 + s)
            reg.step(K)
            est = reg.estimate()
            binding.warp_apply(binding.volume(sm[0]), est["matrix"], "nearest", out_m, n_frames=20,
                               src_frame_stride=V, dst_frame_stride=V)
            binding.warp_apply(binding.volume(ss[0]), est["matrix"], "trilinear", out_s, n_frames=20,
                               src_frame_stride=V, dst_frame_stride=V)
            return est

        for w in range(warmup):
            step(w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            est = step(warmup + s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        evals = float(N) * V * K * steps
        line = {"metric": "particle×voxel evals/s", "value": evals / wall, "unit": "evals/s", "n_gpus": 1,
                "steps": steps, "warmup": warmup, "ms_per_step": wall * 1e3 / steps, "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "u8 masks, fp32 coordinates", "data": "synthetic",
                "config": {"workload": "lv224: 224x208x176 ED LV masks, N=4096, K=40, Dice, nearest; one step = "
                                       "one registration + warp_apply of 20 mask and 20 speckle frames",
                           "tuning": reg.tuning()},
                "final_score": est["score"]}
        reg.close()
    else:
        import multiprocessing as mp
        specs = synth.batch_pairs(64, seed=4)
        log("generating the 64 batch pairs ...")
        with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
            vols = list(pool.imap(_batch_pair, specs))
        pairs, evals = [], 0.0
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
            evals += spec["n_particles"] * v["tgt"].size * 30
        b = binding.Batch(pairs)
        log("autotuning ...")
        b.autotune(3)
        kinds = {spec["kind"]: i for i, spec in reversed(list(enumerate(specs)))}
        tunings = {k: binding.smc_get_tuning(b.pair(i)) for k, i in kinds.items()}
        log(f"tunings: {tunings}")
        for w in range(warmup):
            b.set_seeds(np.arange(64) + 100 + w)
            b.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            b.set_seeds(np.arange(64) + 200 + s)
            b.run()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        line = {"metric": "particle×voxel evals/s", "value": evals * steps / wall, "unit": "evals/s", "n_gpus": 1,
                "steps": steps, "warmup": warmup, "ms_per_step": wall * 1e3 / steps, "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "u8, fp32 coordinates", "data": "synthetic",
                "config": {"workload": "batch64: 64 pairs, cubic sides 96..224, N in {1024..8192}, K=30, half "
                                       "shell masks (Dice) and half speckle images (NCC); one step = one graph "
                                       "launch of every registration", "evals_per_step": evals,
                           "tuning": tunings}}
        b.close()
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--score", default="ncc", choices=["ncc", "ssd"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-time-to-dice", action="store_true")
    ap.add_argument("--ttd-pairs", type=int, default=2)
    ap.add_argument("--tuning", default=DEFAULT_TUNING,
                    help="layout,particles_per_group,tile_depth of the warp-and-score launch")
    ap.add_argument("--autotune", action="store_true", help="autotune the launch instead of --tuning")
    ap.add_argument("--workload", default="speckle160", choices=["speckle160", "lv224", "batch64"],
                    help="speckle160 (the headline line); lv224 or batch64 time the other configurations")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 256 MiB (three times), to scale HBM byte counters")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        torch.cuda.set_device(0)
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda").fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b = a.clone()
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel(), "copies": 3, "checksum": int(b[::4096].sum().item())}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the registration path "
              f"runs on a single MI355X; sharding by pair or by particle is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    if args.workload != "speckle160":
        import torch
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            sys.exit(1)
        other_workload(args.workload, args.steps, args.warmup)
        return

    import numpy as np
    import torch

    import synth
    from paper_2504_19930_amd import binding, config

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    binding.lib()
    torch.cuda.set_device(0)

    log("generating the 160^3 speckle pair ...")
    pair = synth.speckle_pair(side=160, seed=2)
    prm = config.workload_params("speckle160")
    prm["score"] = args.score
    prm["sigma_score"] = config.SIGMA_SCORE[args.score]
    N, K = prm["n_particles"], prm["n_iters"]
    V = pair["tgt"].size

    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    src, tgt, fov = dev(pair["src"]), dev(pair["tgt"]), dev(pair["src_fov"])
    out = torch.zeros_like(tgt)
    stream = torch.cuda.current_stream()
    reg = binding.Registration(src, tgt, prm, src_fov=fov)
    src_vol = binding.volume(src)
    if args.autotune:
        tuning = reg.autotune(reps=2)
    else:
        lay, ppg, depth = (int(v) for v in args.tuning.split(","))
        reg.tune(lay, ppg, depth)
        tuning = reg.tuning()
    log(f"tuning: {tuning}")

    def step(s):
        reg.reset(1000 + s)
        reg.step(K)
        est = reg.estimate()
        binding.warp_apply(src_vol, est["matrix"], "trilinear", out)
        return est

    for w in range(args.warmup):
        step(w)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps ...")
    reg.profile(True)
    reg.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        est = step(args.warmup + s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = reg.profile_read()
    reg.profile(False)

    wall = t1 - t0
    evals = float(N) * V * K * args.steps
    value = evals / wall
    score_launch_ms = prof["score_ms"] / max(1, prof["score_launches"])
    evals_per_launch = float(N + 1) * V
    achieved_tops = evals_per_launch * OPS_PER_EVAL / (score_launch_ms * 1e-3) / 1e12
    gather_gbs = evals_per_launch * GATHER_BYTES_PER_EVAL / (score_launch_ms * 1e-3) / 1e9
    traffic = pmc_traffic()
    gpath = pmc_gather_path()
    line = {
        "metric": "particle×voxel evals/s",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"speckle160: 160^3 u8 speckle images, 60 deg apical-cone source FOV, "
                               f"N={N} particles, K={K} iterations, {args.score.upper()}, trilinear; "
                               f"one step = one full registration + warp_apply",
                   "particles": N, "iterations": K, "target_voxels": V, "score": args.score,
                   "tuning": {k: tuning[k] for k in ("layout", "particles_per_group", "tile_depth")}},
        "roofline": {"bound": "alu", "achieved": achieved_tops, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                     "frac": achieved_tops / PEAK_VALU_TOPS, "traffic": traffic,
                     "kernel": "k_score_image (warp-and-score, trilinear)",
                     "ops_per_eval": OPS_PER_EVAL, "evals_per_launch": evals_per_launch,
                     "kernel_ms_per_launch": score_launch_ms, "launches": prof["score_launches"],
                     "gather_GBs": gather_gbs,
                     "gather_path": None if gpath is None else dict(
                         gpath, l1_lines_GBs=gpath["l1_tag_lookups_per_dispatch"] * 128.0 / (score_launch_ms * 1e-3) / 1e9,
                         note="from the committed rocprofv3 counter summary; lines of 128 B"),
                     "filter_ms_per_launch": prof["filter_ms"] / max(1, prof["filter_launches"])},
        "final_score": est["score"],
    }
    if not args.no_time_to_dice:
        from paper_2504_19930_amd import learned
        if os.path.exists(learned.WEIGHTS):
            log("time-to-Dice: learned proposal (N=512) vs plain filter (N=4096) ...")
            params = learned.load_weights()
            rows = []
            for i in range(args.ttd_pairs):
                lvp = synth.lv_sequence(seed=900000 + i, frames=[0], speckle=False)
                rows.append(learned.time_to_dice(lvp, params, seed=i))
            ratios = [r["ratio"] for r in rows if r["ratio"]]
            line["time_to_dice"] = {
                "metric": "time to Dice >= plain final Dice - 0.005, plain (N=4096) / learned (N=512)",
                "median_ratio": float(np.median(ratios)) if ratios else None,
                "reached": len(ratios), "pairs": len(rows),
                "t_plain_ms": [r["t_plain_ms"] for r in rows], "t_learned_ms": [r["t_learned_ms"] for r in rows],
                "workload": "224x208x176 ED LV masks, +-15 deg, +-16 voxels, K <= 40"}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        cb = cpu_baseline(pair, prm, args.cpu_seconds)
        line["cpu_baseline"] = cb
        line["gpu_over_cpu"] = value / cb["value"]
    reg.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
