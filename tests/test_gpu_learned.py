"""GPU parity of the learned proposal: the MFMA convolution network's
forward and backward against the FP64 oracle (same bfloat16 precision
decisions; relative L2 error <= 2e-2), the downsampler, Adam, and the
proposal-seeded filter against the oracle's."""

import numpy as np
import pytest

import synth
from oracle import cnn as ocnn
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


def rel_l2(a, b):
    a, b = np.asarray(a, float).ravel(), np.asarray(b, float).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _inputs(smc, net, B, seed=0):
    """B pairs into the network's input slots; returns the oracle's view of
    the same input (FP16 storage, bfloat16 on use)."""
    rng = np.random.default_rng(seed)
    xs = []
    keep = []
    for b in range(B):
        if b % 2 == 0:
            pr = synth.proposal_pair(seed=seed * 100 + b)
            s, t, scale = pr["src"], pr["tgt"], 1.0
        else:
            s = rng.integers(0, 256, (40, 50, 60)).astype(np.uint8)
            t = rng.integers(0, 256, (70, 66, 64)).astype(np.uint8)
            scale = 1.0 / 255.0
        ts, tt = dev(s), dev(t)
        keep += [ts, tt]
        net.input(b, smc.volume(ts), smc.volume(tt), scale)
        x = np.stack([ocnn.downsample(s, scale=scale), ocnn.downsample(t, scale=scale)])
        xs.append(x)
    x = np.stack(xs).astype(np.float16).astype(np.float32)
    return ocnn.bf16(x).astype(np.float64), keep


def _oracle_params(p32):
    """The device computes convolutions with bfloat16 weights, the head in FP32."""
    p = p32.astype(np.float32).copy()
    n_conv = sum(int(np.prod(s)) for s in ocnn.param_shapes()[:8])
    p[:n_conv] = ocnn.bf16(p[:n_conv])
    return p.astype(np.float64)


def test_forward_and_backward_match_oracle(smc):
    B = 4
    net = smc.Cnn(max_batch=B)
    p32 = ocnn.init_params(3)
    p32[ocnn.n_params() - 12:] = np.linspace(-0.5, 0.5, 12)  # nonzero head bias
    net.set_params(p32)
    x, keep = _inputs(smc, net, B)
    out = net.forward(B)
    po = _oracle_params(p32)
    ref, acts = ocnn.forward(po, x, bf16_acts=True)
    assert rel_l2(out, ref) <= 2e-2, rel_l2(out, ref)
    rng = np.random.default_rng(1)
    target = np.concatenate([rng.normal(0, 0.5, (B, 6)), rng.uniform(0.01, 0.2, (B, 6))], 1)
    loss, g = net.backward(target, grads=True)
    ref_loss = ocnn.nll(ref, target[:, :6], target[:, 6:])
    assert abs(loss - ref_loss) <= 2e-2 * abs(ref_loss)
    ref_g = ocnn.backward(po, acts, ocnn.nll_grad(ref, target[:, :6], target[:, 6:]))
    offs = np.cumsum([0] + [int(np.prod(s)) for s in ocnn.param_shapes()])
    for q in range(len(offs) - 1):
        e = rel_l2(g[offs[q]:offs[q + 1]], ref_g[offs[q]:offs[q + 1]])
        assert e <= 2e-2, (q, e)
    assert np.array_equal(net.get_params(), p32)
    net.close()


def test_downsample_matches_oracle(smc):
    net = smc.Cnn(max_batch=2)
    rng = np.random.default_rng(4)
    s = rng.integers(0, 256, (37, 81, 50)).astype(np.uint8)
    t = synth.lv_sequence(seed=2, frames=[0], speckle=False)["tgt"]
    ts, tt = dev(s), dev(t)
    net.input(1, smc.volume(ts), smc.volume(tt), 1.0 / 255.0)
    got = net.read_input(1).astype(np.float64)
    for c, v in enumerate((s, t)):
        ref = ocnn.downsample(v, scale=1.0 / 255.0)
        # FP32 arithmetic then one FP16 rounding on the device
        assert np.all(np.abs(got[c] - ref) <= 2.0 ** -10 * np.abs(ref) + 1e-6), c
    net.close()


def test_adam_training_reduces_loss(smc):
    B = 8
    net = smc.Cnn(max_batch=B)
    p32 = ocnn.init_params(7)
    net.set_params(p32)
    x, keep = _inputs(smc, net, B, seed=2)
    rng = np.random.default_rng(2)
    target = np.concatenate([rng.normal(0, 0.3, (B, 6)), rng.uniform(0.01, 0.1, (B, 6))], 1)
    first = net.backward(target)
    for _ in range(30):
        net.backward(target)
        net.step(1e-3)
    last = net.backward(target)
    assert last < 0.5 * first, (first, last)
    net.close()


def test_adam_steps_match_oracle(smc):
    """Five backward + Adam steps on the GPU against the oracle's FP64 Adam fed
    the same read-back gradients: the FP32 master weights agree to FP32
    rounding, and the bfloat16 copies the forward pass uses are the rounded
    master weights (a fresh network given the same weights computes the same
    outputs bit for bit)."""
    B, lr = 4, 2e-3
    net = smc.Cnn(max_batch=B)
    p32 = ocnn.init_params(11)
    net.set_params(p32)
    x, keep = _inputs(smc, net, B, seed=5)
    rng = np.random.default_rng(9)
    target = np.concatenate([rng.normal(0, 0.4, (B, 6)), rng.uniform(0.01, 0.2, (B, 6))], 1)
    p, m, v = p32.astype(np.float64), np.zeros(p32.size), np.zeros(p32.size)
    for t in range(1, 6):
        _, g = net.backward(target, grads=True)
        net.step(lr)
        p, m, v = ocnn.adam(p, g.astype(np.float64), m, v, t, lr)
        got = net.get_params().astype(np.float64)
        err = np.abs(got - p)
        # FP32 storage of the weights (2^-24 relative per step) and FP32 moment
        # arithmetic (a few 1e-7 of the lr-sized update)
        assert np.all(err <= 2.0 ** -24 * t * np.abs(p) + 1e-5 * lr), (t, float(err.max()))
        moved = np.abs(got - p32) > 0
        assert moved.mean() > 0.5, t
    out = net.forward(B)
    fresh = smc.Cnn(max_batch=B)
    fresh.set_params(net.get_params())
    x2, keep2 = _inputs(smc, fresh, B, seed=5)
    assert np.array_equal(fresh.forward(B), out)
    fresh.close()
    net.close()


def test_proposal_changes_only_the_next_prior(smc, orc):
    """smc_set_proposal affects the next prior draw only: set on a context
    whose particles came from the uniform box, the next steps are the plain
    filter's (no importance correction); removed after a proposal draw, the
    drawn set keeps its correction; a caller's particle set never gets one."""
    pair = synth.shell_pair(seed=8, side=36)
    prm = config.default_params("dice", 80, 3, 15.0, 5.0, seed=33)
    mean = np.array([0.02, 0.01, -0.03, 0.6, -0.4, 0.2])
    logvar = 2 * np.log(np.array([0.04, 0.04, 0.04, 0.9, 0.9, 0.9]))
    plain = orc.smc_run(pair["src"], pair["tgt"], prm)
    prop = orc.smc_run(pair["src"], pair["tgt"], dict(prm, proposal=dict(mean=list(mean), logvar=list(logvar))))
    r = smc.Registration(dev(pair["src"]), dev(pair["tgt"]), prm)
    r.set_proposal(mean, logvar)          # uniform prior already drawn
    r.run()
    g = r.particles()
    assert np.array_equal(g["ancestors"], plain["ancestors"])
    assert np.allclose(g["logw"], plain["logw"], rtol=1e-12, atol=1e-12)
    r.reset(33)                           # draws from the proposal
    r.set_proposal(None)                  # the drawn set keeps its correction
    r.run()
    g = r.particles()
    assert np.array_equal(g["ancestors"], prop["ancestors"])
    assert np.allclose(g["states"], prop["states"], rtol=0, atol=1e-12)
    assert np.allclose(r.estimate()["params"], prop["est"], atol=1e-12)
    # a caller's set (here the plain prior) is not corrected, proposal or not
    r.set_proposal(mean, logvar)
    r.set_particles(orc.init_particles(prm), 0)
    r.run()
    g = r.particles()
    assert np.array_equal(g["ancestors"], plain["ancestors"])
    assert np.allclose(r.estimate()["params"], plain["est"], atol=1e-12)
    r.close()


def test_cloud_label_and_network_proposal_match_oracle(smc, orc):
    """The two library calls the learned path is built from: the training
    label (smc_cloud_moments: the final weighted cloud in units of the
    limits) equals the oracle's on the oracle's own run of the same pair, and
    the proposal set from network outputs (smc_set_proposal_from_network)
    equals the oracle's map, down to the prior it draws."""
    pair = synth.shell_pair(seed=12, side=36)
    x0 = [0.01, 0.0, -0.02, 0.5, 0.0, -0.5]
    prm = config.default_params("dice", 150, 4, 15.0, 5.0, seed=3, x0=x0)
    r = smc.Registration(dev(pair["src"]), dev(pair["tgt"]), prm)
    with pytest.raises(smc.SmcError):
        r.cloud_moments()  # no weights before the first iteration
    r.run()
    o = orc.smc_run(pair["src"], pair["tgt"], prm)
    gm, gv = r.cloud_moments(1e-4)
    om, ov = orc.cloud_moments(o["logw"], o["states"], x0, prm["limit"], 1e-4)
    assert np.allclose(gm, om, rtol=1e-10, atol=1e-11)
    assert np.allclose(gv, ov, rtol=1e-8, atol=1e-12)
    out = np.array([0.3, -2.0, 0.1, -0.4, 0.9, 1.5, -3.0, -25.0, 0.5, -1.0, 3.0, -6.0], np.float32)
    m, lv = r.set_proposal_from_network(out, 4.0)
    om, olv = orc.proposal_from_network(out, x0, prm["limit"], 4.0)
    assert np.allclose(m, om, rtol=0, atol=1e-15) and np.allclose(lv, olv, rtol=0, atol=1e-13)
    r.reset(5)
    x, _ = orc.init_proposal(dict(prm, seed=5, proposal=dict(mean=list(om), logvar=list(olv))))
    assert np.allclose(r.particles()["states"], x, rtol=0, atol=1e-13)
    r.close()


def test_proposal_prior_and_filter_match_oracle(smc, orc):
    pair = synth.shell_pair(seed=6, side=40)
    prm = config.default_params("dice", 96, 4, 15.0, 5.0, seed=21)
    mean = np.array([0.05, -0.02, 0.03, 1.0, -0.5, 0.25])
    logvar = 2 * np.log(np.array([0.03, 0.03, 0.03, 0.8, 0.8, 0.8]))
    r = smc.Registration(dev(pair["src"]), dev(pair["tgt"]), prm)
    r.set_proposal(mean, logvar)
    r.reset(21)
    p = dict(prm, proposal=dict(mean=list(mean), logvar=list(logvar)))
    x, lq = orc.init_proposal(p)
    # Box-Muller transcendentals may differ in the last bit between the two libms
    assert np.allclose(r.particles()["states"], x, rtol=0, atol=1e-14)
    r.run()
    o = orc.smc_run(pair["src"], pair["tgt"], p)
    g = r.particles()
    assert np.array_equal(g["ancestors"], o["ancestors"])
    assert np.allclose(g["states"], o["states"], rtol=0, atol=1e-12)
    assert np.allclose(r.estimate()["params"], o["est"], atol=1e-12)
    # without the proposal the context is the plain filter again: same prior,
    # no importance correction, the plain oracle's run
    r.set_proposal(None)
    r.reset(21)
    assert np.array_equal(r.particles()["states"], orc.init_particles(prm))
    r.run()
    o = orc.smc_run(pair["src"], pair["tgt"], prm)
    g = r.particles()
    assert np.array_equal(g["ancestors"], o["ancestors"])
    assert np.allclose(g["states"], o["states"], rtol=0, atol=1e-12)
    assert np.allclose(r.estimate()["params"], o["est"], atol=1e-12)


def test_trained_proposal_reaches_plain_dice_with_less_work(smc):
    """The committed trained network, on held-out pairs (seeds disjoint from
    the training seeds): the proposal-seeded filter with N = 512 reaches the
    plain filter's final Dice (N = 4096, K = 40) within 0.005, and needs at
    least 5x fewer particle x iteration evaluations to get there (the timed
    ratio is measured by bench.py)."""
    import os
    from paper_2504_19930_amd import learned
    if not os.path.exists(learned.WEIGHTS):
        pytest.skip("no trained weights")
    params = learned.load_weights()
    for i in range(2):
        pair = synth.lv_sequence(seed=910000 + i, frames=[0], speckle=False)
        r = learned.time_to_dice(pair, params, seed=i)
        assert r["k_learned"] is not None, r
        assert r["learned_final_dice"] >= r["d_star"] - 0.005, r
        work_plain = 4096 * r["k_plain"]
        work_learned = 512 * r["k_learned"]
        assert work_plain >= 5 * work_learned, r
