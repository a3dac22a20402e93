"""Stored expected results of whole registrations at full size, computed by
the CPU oracle alone.

Each run is a complete filter (every iteration, every particle scored over
the whole target grid) on a seeded synthetic pair at the size of a named
workload; it takes from about fifteen minutes (224 x 208 x 176 masks) to
about forty (160^3 trilinear images) on eight cores, far too long to repeat
inside a test, so the results are written once to ``full_runs.json`` beside
this script and the GPU tests compare the HIP library's runs with them.

Only ``oracle`` (and the input generators of ``synth``, which hold none of
the method's arithmetic) are used; the filter parameters are spelled out
below, so the stored values depend on nothing in the product package.  The
input bytes are hashed, so a test can tell when the generators (numpy /
scipy versions) no longer reproduce the inputs the values were computed on.

    python tests/golden/make_full_runs.py [--threads T] [name ...]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "full_runs.json")


def _params(score, n, K, rot_deg, trans, seed, sigma_score):
    lim = [math.radians(rot_deg)] * 3 + [float(trans)] * 3
    interp = "nearest" if score == "dice" else "trilinear"
    return dict(n_particles=n, n_iters=K, seed=seed, pair_id=0, score=score, interp=interp, x0=[0.0] * 6,
                limit=lim, sigma_score=sigma_score, sigma0=[0.15 * v for v in lim], anneal=0.85,
                min_overlap_frac=0.05)


# name -> (input generator arguments, filter parameters)
RUNS = {
    # the 160^3 speckle image workload: NCC over the overlap, trilinear,
    # 60-degree apical-cone source FOV
    "speckle160": (dict(gen="speckle", side=160, seed=2), _params("ncc", 2048, 30, 20.0, 12.0, 0, 0.02)),
    # the full-size mask workload: ED frame of the contracting LV sequence
    "lv224": (dict(gen="lv", seed=3), _params("dice", 4096, 40, 15.0, 16.0, 0, 0.01)),
    # held-out pairs of the learned-proposal comparison (plain filter, N = 4096)
    "lv224_heldout0": (dict(gen="lv", seed=900000), _params("dice", 4096, 40, 15.0, 16.0, 0, 0.01)),
    "lv224_heldout1": (dict(gen="lv", seed=900001), _params("dice", 4096, 40, 15.0, 16.0, 1, 0.01)),
}


def make_inputs(gen: dict) -> dict:
    """The seeded synthetic pair of a run (numpy arrays; src_fov may be None)."""
    if gen["gen"] == "speckle":
        p = synth.speckle_pair(side=gen["side"], seed=gen["seed"])
        return dict(src=p["src"], tgt=p["tgt"], src_fov=p["src_fov"])
    s = synth.lv_sequence(seed=gen["seed"], frames=[0], speckle=False)
    return dict(src=s["src"], tgt=s["tgt"], src_fov=None)


def input_digest(inp: dict) -> str:
    h = hashlib.sha256()
    for k in ("src", "tgt", "src_fov"):
        a = inp[k]
        h.update(k.encode())
        if a is not None:
            h.update(str(a.shape).encode())
            h.update(np.ascontiguousarray(a, np.uint8).tobytes())
    return h.hexdigest()


def ancestors_digest(anc) -> str:
    return hashlib.sha256(np.ascontiguousarray(anc, "<i4").tobytes()).hexdigest()


def run(name: str) -> dict:
    gen, prm = RUNS[name]
    inp = make_inputs(gen)
    src = oracle.Volume(inp["src"], fov=inp["src_fov"])
    tgt = oracle.Volume(inp["tgt"])
    t0 = time.time()
    o = oracle.smc_run(src, tgt, prm)
    dt = time.time() - t0
    anc = o["ancestors"]
    return dict(inputs=gen, params=prm, input_sha256=input_digest(inp),
                est=[float(v) for v in o["est"]],
                trace_score=[float(v) for v in o["trace_score"]],
                trace_ess=[float(v) for v in o["trace_ess"]],
                trace_est=[[float(v) for v in row] for row in o["trace_est"]],
                ancestors_sha256=ancestors_digest(anc), distinct_ancestors=int(len(np.unique(anc))),
                ancestors_head=[int(v) for v in anc[:16]], degenerate=bool(o["degenerate"]),
                oracle_seconds=round(dt, 1), oracle_threads=oracle.num_threads())


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("names", nargs="*", default=list(RUNS))
    ap.add_argument("--threads", type=int, default=0, help="oracle threads (0: all)")
    args = ap.parse_args()
    oracle.set_threads(args.threads)
    stored = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            stored = json.load(fh)
    for name in args.names:
        print(f"{name}: running the oracle ...", flush=True)
        stored[name] = run(name)
        print(f"{name}: {stored[name]['oracle_seconds']} s, final score {stored[name]['trace_score'][-1]:.6f}",
              flush=True)
        with open(OUT + ".tmp", "w") as fh:
            json.dump(stored, fh, indent=1, sort_keys=True)
            fh.write("\n")
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
