"""Whole registrations at full size against stored oracle results.

``tests/golden/full_runs.json`` holds complete oracle runs (every iteration,
every particle scored over the whole target grid) of the full-size workloads
-- the 160^3 speckle images (N = 2048, K = 30, NCC, trilinear, source FOV),
the 224 x 208 x 176 ED LV masks (N = 4096, K = 40, Dice) and two held-out
pairs of the learned-proposal comparison (the plain filter whose final Dice
is the time-to-Dice target) -- written by ``tests/golden/make_full_runs.py``,
which calls only the oracle.  Here the HIP library runs the same
registrations from the same seeds: identical resampling ancestors (digest
over the last resampling and its distinct count), every traced score, ESS
and per-iteration estimate within 1e-9, the final transform within 0.05 mm
and 0.02 deg."""

import importlib.util
import json
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "full_runs.json")
TOL_MM, TOL_DEG = 0.05, 0.02


def _gen_module():
    spec = importlib.util.spec_from_file_location("make_full_runs", os.path.join(HERE, "golden", "make_full_runs.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _stored():
    if not os.path.exists(GOLDEN):
        return {}
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def smc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19930_amd import binding
    binding.lib()
    return binding


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _geodesic_deg(p, q, orc):
    R1, R2 = orc.euler_R(p[:3]), orc.euler_R(q[:3])
    return math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(R1.T @ R2) - 1) / 2))))


@pytest.mark.parametrize("name", ["speckle160", "lv224", "lv224_heldout0", "lv224_heldout1"])
def test_full_run_matches_stored_oracle_run(smc, orc, name):
    stored = _stored()
    if name not in stored:
        pytest.skip(f"no stored oracle run '{name}' (tests/golden/make_full_runs.py {name})")
    g = stored[name]
    gen = _gen_module()
    inp = gen.make_inputs(g["inputs"])
    assert gen.input_digest(inp) == g["input_sha256"], "the input generators no longer reproduce the stored inputs"
    prm = g["params"]
    reg = smc.Registration(_dev(inp["src"]), _dev(inp["tgt"]), prm,
                           src_fov=None if inp["src_fov"] is None else _dev(inp["src_fov"]))
    reg.run()
    part = reg.particles()
    tr = reg.trace()
    est = reg.estimate()
    reg.close()
    K = prm["n_iters"]
    assert gen.ancestors_digest(part["ancestors"]) == g["ancestors_sha256"]
    assert len(np.unique(part["ancestors"])) == g["distinct_ancestors"]
    assert np.allclose(tr["score"], g["trace_score"], rtol=0, atol=1e-9)
    assert np.allclose(tr["ess"], g["trace_ess"], rtol=1e-9, atol=1e-9)
    assert np.allclose(tr["est"], np.array(g["trace_est"]).reshape(K, 6), rtol=0, atol=1e-9)
    assert np.linalg.norm(est["params"][3:] - np.array(g["est"][3:])) <= TOL_MM
    assert _geodesic_deg(est["params"], np.array(g["est"]), orc) <= TOL_DEG
    assert abs(est["score"] - g["trace_score"][-1]) <= 1e-9
