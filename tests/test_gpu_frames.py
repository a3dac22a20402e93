"""GPU parity of the multi-frame score: pooled sums over several frame
pairs equal the oracle's bit for bit (masks; trilinear NCC with source
FOVs, every layout), whole two-frame registrations match the oracle, and
the entry point's checks."""

import math

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


def _mask_frames():
    gt = np.array([math.radians(6.0), math.radians(-4.0), math.radians(5.0), 2.5, -1.5, 2.0])
    shape, c = (48, 44, 40), (25.5, 22.5, 19.0)
    return [synth.mask_pair(shape, outer=o, inner=None, gt=gt, centre=c)
            for o in ((16.0, 10.0, 8.0), (12.8, 8.0, 6.4), (14.4, 9.0, 7.2))]


def _image_frames():
    return [synth.speckle_pair(side=37, seed=s, trans=3.0) for s in (17, 18)]


def _states(n, rot_deg, trans, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([np.deg2rad(rng.uniform(-rot_deg, rot_deg, (n, 3))),
                           rng.uniform(-trans, trans, (n, 3))], axis=1)


def test_pooled_mask_sums_bit_exact(smc, orc):
    fr = _mask_frames()
    prm = config.default_params("dice", 33, 2, 10.0, 4.0)
    r = smc.Registration(dev(fr[0]["src"]), dev(fr[0]["tgt"]), prm)
    r.set_frames([dict(src=dev(f["src"]), tgt=dev(f["tgt"])) for f in fr[1:]])
    x = np.vstack([np.zeros(6), _states(32, 10, 4, 1)])
    want = orc.Frames([(f["src"], f["tgt"]) for f in fr]).sums(prm, x)
    got = r.evaluate(x)
    assert np.array_equal(got[:, :4], want[:, :4])
    # removing the frames restores the single-pair sums
    r.set_frames([])
    assert np.array_equal(r.evaluate(x)[:, :4], orc.Frames([(fr[0]["src"], fr[0]["tgt"])]).sums(prm, x)[:, :4])


def test_pooled_image_sums_bit_exact_every_layout(smc, orc):
    fr = _image_frames()
    prm = config.default_params("ncc", 41, 2, 20.0, 3.0)
    r = smc.Registration(dev(fr[0]["src"]), dev(fr[0]["tgt"]), prm, src_fov=dev(fr[0]["src_fov"]))
    r.set_frames([dict(src=dev(f["src"]), tgt=dev(f["tgt"]), src_fov=dev(f["src_fov"])) for f in fr[1:]])
    x = np.vstack([np.zeros(6), _states(40, 20, 3, 8)])
    want = orc.Frames([(orc.Volume(f["src"], fov=f["src_fov"]), orc.Volume(f["tgt"])) for f in fr]).sums(prm, x)
    for layout in ("raw", "quadxy", "oct", "octtile", "lerp"):
        r.tune(layout, 4, 32)
        assert np.array_equal(r.evaluate(x), want), layout


def _compare(smc, orc, frames, prm, fov):
    kw = dict(src_fov=dev(frames[0]["src_fov"])) if fov else {}
    r = smc.Registration(dev(frames[0]["src"]), dev(frames[0]["tgt"]), prm, **kw)
    r.set_frames([dict(src=dev(f["src"]), tgt=dev(f["tgt"]), **(dict(src_fov=dev(f["src_fov"])) if fov else {}))
                  for f in frames[1:]])
    r.run()
    V = (lambda f: orc.Volume(f["src"], fov=f["src_fov"])) if fov else (lambda f: orc.Volume(f["src"]))
    o = orc.smc_run(V(frames[0]), orc.Volume(frames[0]["tgt"]), prm,
                    frames=[(V(f), orc.Volume(f["tgt"])) for f in frames[1:]])
    g = r.particles()
    assert np.array_equal(g["ancestors"], o["ancestors"])
    assert np.allclose(g["states"], o["states"], rtol=0, atol=1e-12)
    assert np.allclose(g["logw"], o["logw"], rtol=1e-12, atol=1e-12)
    tr = r.trace()
    assert np.allclose(tr["score"], o["trace_score"], rtol=1e-12, atol=1e-15)
    assert np.allclose(r.estimate()["params"], o["est"], atol=1e-12)
    return r, o


def test_two_and_three_frame_registrations_match_oracle(smc, orc):
    fr = _mask_frames()
    r, o = _compare(smc, orc, fr, config.default_params("dice", 256, 8, 10.0, 4.0, seed=3), fov=False)
    assert o["trace_score"][-1] > 0.9
    _compare(smc, orc, _image_frames(), config.default_params("ncc", 128, 4, 20.0, 3.0, seed=2), fov=True)


def test_set_frames_checks(smc):
    fr = _image_frames()
    src, tgt, fov = dev(fr[0]["src"]), dev(fr[0]["tgt"]), dev(fr[0]["src_fov"])
    other = dict(src=dev(fr[1]["src"]), tgt=dev(fr[1]["tgt"]), src_fov=dev(fr[1]["src_fov"]))
    r = smc.Registration(src, tgt, config.default_params("ssd", 16, 2, 20.0, 3.0), src_fov=fov)
    with pytest.raises(smc.SmcError):
        r.set_frames([other])
    r = smc.Registration(src, tgt, config.default_params("ncc", 16, 2, 20.0, 3.0), src_fov=fov)
    with pytest.raises(smc.SmcError):                      # FOV missing where the first pair has one
        r.set_frames([dict(src=other["src"], tgt=other["tgt"])])
    small = synth.speckle_pair(side=30, seed=3)
    with pytest.raises(smc.SmcError):                      # shape mismatch
        r.set_frames([dict(src=dev(small["src"]), tgt=dev(small["tgt"]), src_fov=dev(small["src_fov"]))])
    r.step(1)
    with pytest.raises(smc.SmcError):                      # after the first iteration
        r.set_frames([other])
    r.reset(3)
    r.set_frames([other])
    r.run()
