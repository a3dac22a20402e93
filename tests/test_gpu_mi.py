"""GPU parity of the mutual-information score: particle scores equal the
oracle's bit for bit (exact joint-histogram counts, the same logarithm and
summation order on both sides) under every layout, with and without source
FOV and over several frames; whole MI registrations match the oracle."""

import numpy as np
import pytest

import synth
from paper_2504_19930_amd import config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19930_amd import binding
    binding.lib()
    return binding


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _states(n, rot_deg, trans, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([np.deg2rad(rng.uniform(-rot_deg, rot_deg, (n, 3))),
                           rng.uniform(-trans, trans, (n, 3))], axis=1)


@pytest.mark.parametrize("with_fov", [False, True])
def test_mi_scores_bit_exact_every_layout(smc, orc, with_fov):
    pair = synth.speckle_pair(side=37, seed=17, trans=3.0)
    prm = config.default_params("mi", 41, 2, 20.0, 3.0)
    kw = dict(src_fov=dev(pair["src_fov"])) if with_fov else {}
    r = smc.Registration(dev(pair["src"]), dev(pair["tgt"]), prm, **kw)
    x = np.vstack([np.zeros(6), _states(44, 20, 3, 8), [[0.0, 0.0, 0.0, 60.0, 0.0, 0.0]]])
    src = orc.Volume(pair["src"], fov=pair["src_fov"] if with_fov else None)
    want = orc.Problem(src, orc.Volume(pair["tgt"])).score(prm, x)
    assert np.isneginf(want[-1])  # below the minimum overlap
    for layout in ("raw", "pairx", "quadxy", "oct", "octtile", "lerp"):
        for pt in (4, 8):
            r.tune(layout, pt, 32)
            got = r.scores(x)
            assert np.array_equal(got, want), (layout, pt)
    with pytest.raises(smc.SmcError):
        r.evaluate(x)


def test_mi_registration_matches_oracle_and_frames(smc, orc):
    pair = synth.speckle_pair(side=40, seed=9, trans=3.0)
    prm = config.default_params("mi", 192, 5, 20.0, 3.0, seed=4)
    r = smc.Registration(dev(pair["src"]), dev(pair["tgt"]), prm, src_fov=dev(pair["src_fov"]))
    r.run()
    o = orc.smc_run(orc.Volume(pair["src"], fov=pair["src_fov"]), orc.Volume(pair["tgt"]), prm)
    g = r.particles()
    assert np.array_equal(g["ancestors"], o["ancestors"])
    assert np.allclose(g["states"], o["states"], rtol=0, atol=1e-12)
    assert np.array_equal(g["logw"], o["logw"])
    assert np.allclose(r.trace()["score"], o["trace_score"], rtol=0, atol=1e-12)
    assert np.allclose(r.estimate()["params"], o["est"], atol=1e-12)
    # two frames: pooled histograms
    other = synth.speckle_pair(side=40, seed=10, trans=3.0)
    r2 = smc.Registration(dev(pair["src"]), dev(pair["tgt"]), prm, src_fov=dev(pair["src_fov"]))
    r2.set_frames([dict(src=dev(other["src"]), tgt=dev(other["tgt"]), src_fov=dev(other["src_fov"]))])
    x = np.vstack([np.zeros(6), _states(20, 20, 3, 2)])
    frames = orc.Frames([(orc.Volume(pair["src"], fov=pair["src_fov"]), orc.Volume(pair["tgt"])),
                         (orc.Volume(other["src"], fov=other["src_fov"]), orc.Volume(other["tgt"]))])
    assert np.array_equal(r2.scores(x), frames.score(prm, x))
