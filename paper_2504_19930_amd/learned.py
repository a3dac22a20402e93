"""Learned proposal: labels from the filter itself, training on the GPU with
the library's own forward / backward / Adam kernels, and its use as the
filter's proposal.

Every numerical step runs in ``libsmc.so``; this module orders the calls and
moves small host arrays (labels, outputs, parameters).

Units: the network predicts, per pair, a Gaussian over the transform in
units of the limits -- mean (x - x0) / L and log-variance log(var / L^2) --
so one network serves any limits box.

    python -m paper_2504_19930_amd.learned train --pairs 20000 --out weights.npz
    python -m paper_2504_19930_amd.learned eval --weights weights.npz --pairs 16
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import binding
from .config import default_params

PKG = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(PKG, "weights", "proposal.npz")
ROT_DEG, TRANS = 15.0, 16.0
N_PARAMS = binding.CNN_PARAMS


def _torch():
    import torch
    return torch


def init_params(seed: int) -> np.ndarray:
    """He-uniform convolution weights, a small head, zero biases."""
    rng = np.random.default_rng(seed)
    chans = (2, 16, 32, 64, 64)
    parts = []
    for ci, co in zip(chans[:-1], chans[1:]):
        lim = math.sqrt(6.0 / (ci * 27))
        parts += [rng.uniform(-lim, lim, co * ci * 27), np.zeros(co)]
    parts += [rng.uniform(-1, 1, 12 * 4096) * math.sqrt(1.0 / 4096), np.zeros(12)]
    out = np.concatenate(parts).astype(np.float32)
    assert out.size == N_PARAMS
    return out


# ------------------------------------------------------------------ data and labels

def _gen(seed):
    import synth
    p = synth.lv_train_pair(seed)
    return p["src"], p["tgt"], p["src_mask"], p["tgt_mask"], p["spacing"]


def make_training_set(n_pairs: int, seed0: int = 1_000_000, workers: int = 16, log=None):
    """Training pairs on the network's 64^3 grid (CPU, process pool)."""
    import multiprocessing as mp
    seeds = [seed0 + i for i in range(n_pairs)]
    shape = (n_pairs, 64, 64, 64)
    src, tgt = np.empty(shape, np.uint8), np.empty(shape, np.uint8)
    smask, tmask = np.empty(shape, np.uint8), np.empty(shape, np.uint8)
    spacing = None

    def put(i, r):
        nonlocal spacing
        src[i], tgt[i], smask[i], tmask[i], spacing = r
        if log and (i + 1) % 1000 == 0:
            log(f"generated {i + 1}/{n_pairs}")

    if workers > 1:
        with mp.get_context("fork").Pool(workers) as pool:
            for i, r in enumerate(pool.imap(_gen, seeds, chunksize=16)):
                put(i, r)
    else:
        for i, sd in enumerate(seeds):
            put(i, _gen(sd))
    return dict(src=src, tgt=tgt, src_mask=smask, tgt_mask=tmask, spacing=spacing)


def label_with_smc(data, n_particles=256, n_iters=15, batch_pairs=256, seed=7, log=None, var_floor=1e-4):
    """Run the plain filter on every training pair (batched, one graph launch
    per batch) and summarise its final weighted cloud (smc_cloud_moments):
    mean and variance in units of the limits, the variance floored."""
    torch = _torch()
    n = len(data["src_mask"])
    mean = np.zeros((n, 6))
    var = np.zeros((n, 6))
    sp = data["spacing"]
    for b0 in range(0, n, batch_pairs):
        idx = range(b0, min(n, b0 + batch_pairs))
        pairs = []
        for i in idx:
            prm = default_params("dice", n_particles, n_iters, ROT_DEG, TRANS, seed=seed + i, pair_id=i)
            pairs.append(dict(src=torch.from_numpy(data["src_mask"][i]).cuda(),
                              tgt=torch.from_numpy(data["tgt_mask"][i]).cuda(), params=prm, spacing=sp))
        batch = binding.Batch(pairs)
        batch.run()
        for q, i in enumerate(idx):
            mean[i], var[i] = binding.smc_cloud_moments(batch.pair(q), var_floor)
        batch.close()
        if log:
            log(f"labels {min(n, b0 + batch_pairs)}/{n}")
    return mean, var


# ------------------------------------------------------------------ training

def train(data, mean, var, epochs=8, batch=32, lr=1e-3, seed=0, holdout=512, log=None):
    torch = _torch()
    n = len(data["src"])
    src = torch.from_numpy(data["src"]).cuda()
    tgt = torch.from_numpy(data["tgt"]).cuda()
    target = np.concatenate([mean, var], axis=1).astype(np.float32)
    net = binding.Cnn(max_batch=batch)
    net.set_params(init_params(seed))
    rng = np.random.default_rng(seed)
    train_idx = np.arange(holdout, n)
    val_idx = np.arange(0, holdout)
    steps = epochs * (len(train_idx) // batch)
    step = 0
    hist = []

    def load(ids):
        for s, i in enumerate(ids):
            net.input(s, binding.volume(src[i]), binding.volume(tgt[i]), 1.0 / 255.0)

    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = rng.permutation(train_idx)
        losses = []
        for b in range(len(perm) // batch):
            ids = perm[b * batch:(b + 1) * batch]
            load(ids)
            losses.append(net.backward(target[ids]))
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * step / max(1, steps)))
            net.step(max(cur, lr * 0.01))
            step += 1
        vl = []
        for b in range(0, len(val_idx) - batch + 1, batch):
            ids = val_idx[b:b + batch]
            load(ids)
            vl.append(net.backward(target[ids]))
        hist.append(dict(epoch=ep, train=float(np.mean(losses)), val=float(np.mean(vl)) if vl else None,
                         seconds=time.perf_counter() - t0))
        if log:
            log(json.dumps(hist[-1]))
    params = net.get_params()
    net.close()
    return params, hist


# ------------------------------------------------------------------ use

class Proposal:
    """A trained network used to seed a registration."""

    def __init__(self, params, var_scale=4.0):
        self.net = binding.Cnn(max_batch=1)
        self.net.set_params(params)
        self.var_scale = var_scale

    def propose(self, reg, src_vol, tgt_vol, scale=1.0):
        """Network forward on a (device) pair, then the registration's next
        prior drawn from its prediction (smc_set_proposal_from_network).
        Returns the (mean, logvar) that was set."""
        self.net.input(0, src_vol, tgt_vol, scale)
        return reg.set_proposal_from_network(self.net.forward(1)[0], self.var_scale)

    def close(self):
        self.net.close()


def load_weights(path=WEIGHTS) -> np.ndarray:
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32)


def _events_run(reg, K, events):
    torch = _torch()
    for k in range(K):
        reg.step(1)
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        events.append(e)


def time_to_dice(pair, params, n_plain=4096, n_learned=512, K=40, seed=0, tol=0.005, var_scale=4.0):
    """Time until the estimate's Dice first reaches (plain final Dice - tol),
    for the plain filter (N = n_plain, uniform prior) and for the learned
    proposal (N = n_learned, including downsampling and the network)."""
    torch = _torch()
    src = torch.from_numpy(pair["src"]).cuda()
    tgt = torch.from_numpy(pair["tgt"]).cuda()
    out = {}
    # plain
    prm = default_params("dice", n_plain, K, ROT_DEG, TRANS, seed=seed)
    reg = binding.Registration(src, tgt, prm)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    start.record()
    ev = []
    _events_run(reg, K, ev)
    torch.cuda.synchronize()
    tp = np.array([start.elapsed_time(e) for e in ev])
    trp = reg.trace()["score"]
    reg.close()
    d_star = trp[-1]
    # learned
    prop = Proposal(params, var_scale=var_scale)
    prm_l = default_params("dice", n_learned, K, ROT_DEG, TRANS, seed=seed)
    reg = binding.Registration(src, tgt, prm_l)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    start.record()
    mean, logvar = prop.propose(reg, reg.src, reg.tgt, scale=1.0)
    reg.reset(seed)
    ev = []
    _events_run(reg, K, ev)
    torch.cuda.synchronize()
    tl = np.array([start.elapsed_time(e) for e in ev])
    trl = reg.trace()["score"]
    est = reg.estimate()["params"]
    reg.close()
    prop.close()

    def first(tr, times):
        # trace[k] is the score of the estimate after iteration k (k >= 1)
        for k in range(1, len(tr)):
            if tr[k] >= d_star - tol:
                return float(times[k - 1]), k
        return None, None

    out["d_star"] = float(d_star)
    out["t_plain_ms"], out["k_plain"] = first(trp, tp)
    out["t_learned_ms"], out["k_learned"] = first(trl, tl)
    out["learned_final_dice"] = float(trl[-1])
    out["network_mean"] = [float(v) for v in mean]
    out["learned_est"] = [float(v) for v in est]
    out["gt"] = [float(v) for v in pair["gt"]]
    out["ratio"] = (out["t_plain_ms"] / out["t_learned_ms"]) if out["t_learned_ms"] else None
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="learned proposal: train / eval")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--pairs", type=int, default=20000)
    t.add_argument("--epochs", type=int, default=8)
    t.add_argument("--batch", type=int, default=32)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--workers", type=int, default=16)
    t.add_argument("--out", default=WEIGHTS)
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--pairs", type=int, default=16)
    e.add_argument("--seed0", type=int, default=900000)
    e.add_argument("--var-scale", type=float, default=4.0)
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    if args.cmd == "train":
        t0 = time.perf_counter()
        # the worker pool forks before anything touches the GPU
        data = make_training_set(args.pairs, workers=args.workers, log=log)
        log(f"generated {args.pairs} pairs in {time.perf_counter() - t0:.1f}s")
        _torch().cuda.set_device(0)
        mean, var = label_with_smc(data, log=log)
        log(f"labelled in {time.perf_counter() - t0:.1f}s")
        params, hist = train(data, mean, var, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
        os.makedirs(os.path.dirname(args.out), exist_ok=True)
        np.savez_compressed(args.out, params=params, history=json.dumps(hist))
        log(f"saved {args.out} after {time.perf_counter() - t0:.1f}s")
    else:
        import synth
        _torch().cuda.set_device(0)
        params = load_weights(args.weights)
        rows = []
        for i in range(args.pairs):
            pair = synth.lv_sequence(seed=args.seed0 + i, frames=[0], speckle=False)
            r = time_to_dice(pair, params, seed=i, var_scale=args.var_scale)
            rows.append(r)
            log(json.dumps(r))
        ratios = [r["ratio"] for r in rows if r["ratio"]]
        log(json.dumps(dict(median_ratio=float(np.median(ratios)) if ratios else None, reached=len(ratios),
                            pairs=len(rows))))
    return 0


if __name__ == "__main__":
    sys.exit(main())
