"""Default filter parameters and the named workloads.

The paper keeps the particle-filter parameters of its earlier work
(Implementation Details) and does not restate them; the values here are
readings tuned on the synthetic inputs: a Gaussian likelihood of the score
deficit with width 0.01 (Dice), 0.02 (NCC) or 0.1 (normalised SSD), a random
walk starting at 0.15 x the limits and shrinking by 0.85 per iteration.
"""

from __future__ import annotations

import math

SIGMA_SCORE = {"dice": 0.01, "ncc": 0.02, "ssd": 0.1, "mi": 0.02}


def default_params(score: str, n_particles: int, n_iters: int, rot_limit_deg: float, trans_limit: float,
                   seed: int = 0, pair_id: int = 0, interp: str | None = None, x0=None) -> dict:
    lim = [math.radians(rot_limit_deg)] * 3 + [float(trans_limit)] * 3
    if interp is None:
        interp = "nearest" if score == "dice" else "trilinear"
    return dict(n_particles=int(n_particles), n_iters=int(n_iters), seed=int(seed), pair_id=int(pair_id),
                score=score, interp=interp, x0=list(x0) if x0 is not None else [0.0] * 6, limit=lim,
                sigma_score=SIGMA_SCORE[score], sigma0=[0.15 * v for v in lim], anneal=0.85,
                min_overlap_frac=0.05)


# The workloads: 64^3 shell masks; 160^3 speckle images (the throughput
# workload); full-size 224 x 208 x 176 contracting LV masks.
WORKLOADS = {
    "shell64": dict(kind="mask", side=64, n_particles=256, n_iters=10, score="dice", rot=15.0, trans=8.0,
                    seed=0),
    "speckle160": dict(kind="image", side=160, n_particles=2048, n_iters=30, score="ncc", rot=20.0,
                       trans=12.0, seed=0),
    "lv224": dict(kind="lv", shape=(224, 208, 176), n_particles=4096, n_iters=40, score="dice", rot=15.0,
                  trans=16.0, seed=0),
}


def workload_params(name: str, **over) -> dict:
    w = dict(WORKLOADS[name])
    w.update(over)
    return default_params(w["score"], w["n_particles"], w["n_iters"], w["rot"], w["trans"], seed=w["seed"])
