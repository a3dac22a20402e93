"""Pins of the learned-proposal oracle (CPU only): forward against
torch.nn.functional.conv3d (a library special case), every gradient against
central finite differences in FP64, the downsampler against scipy, and the
bfloat16 rounding against torch's."""

import numpy as np
import pytest
import torch
from scipy import ndimage

from oracle import cnn


def test_conv_forward_matches_torch():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 8, 6, 10))
    w = rng.normal(size=(4, 3, 3, 3, 3))
    b = rng.normal(size=4)
    y = cnn.conv_fwd(x, w, b)
    ref = torch.nn.functional.conv3d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b), stride=2,
                                     padding=1).numpy()
    assert y.shape == (2, 4, 4, 3, 5)
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_conv_backward_matches_torch_autograd():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 3, 8, 6, 4))
    w = rng.normal(size=(5, 3, 3, 3, 3))
    b = rng.normal(size=5)
    dy = rng.normal(size=(2, 5, 4, 3, 2))
    dx, dw, db = cnn.conv_bwd(x, w, dy)
    tx, tw, tb = (torch.from_numpy(a).requires_grad_() for a in (x, w, b))
    torch.nn.functional.conv3d(tx, tw, tb, stride=2, padding=1).backward(torch.from_numpy(dy))
    assert np.allclose(dx, tx.grad.numpy(), atol=1e-12)
    assert np.allclose(dw, tw.grad.numpy(), atol=1e-11)
    assert np.allclose(db, tb.grad.numpy(), atol=1e-12)


def _fd_check(f, x, g, idx, h=1e-6, rtol=1e-6):
    for i in idx:
        xp, xm = x.copy(), x.copy()
        xp.flat[i] += h
        xm.flat[i] -= h
        fd = (f(xp) - f(xm)) / (2 * h)
        assert abs(fd - g.flat[i]) <= rtol * max(1.0, abs(fd)), (i, fd, g.flat[i])


def test_full_network_gradients_finite_differences(monkeypatch):
    # a reduced network (same code path) so FP64 finite differences stay cheap
    monkeypatch.setattr(cnn, "SIDE", 16)
    monkeypatch.setattr(cnn, "FLAT", 64 * 1 * 1 * 1)
    rng = np.random.default_rng(3)
    shapes = cnn.param_shapes()
    params = np.concatenate([rng.normal(0, 0.08, int(np.prod(s))) for s in shapes])
    x = rng.normal(size=(2, 2, 16, 16, 16))
    xbar = rng.normal(size=(2, 6))
    var = rng.uniform(0.1, 1.0, size=(2, 6))
    loss, g, _ = cnn.loss_and_grad(params, x, xbar, var)
    f = lambda p: cnn.loss_and_grad(p, x, xbar, var)[0]
    offs = np.cumsum([0] + [int(np.prod(s)) for s in shapes])
    idx = [int(rng.integers(offs[i], offs[i + 1])) for i in range(len(shapes))]
    idx += [int(offs[-2]), int(offs[-1] - 1)]
    _fd_check(f, params, g, idx)


def test_nll_gradient_and_minimum():
    rng = np.random.default_rng(4)
    out = rng.normal(size=(3, 12))
    xbar, var = rng.normal(size=(3, 6)), rng.uniform(0.1, 2, (3, 6))
    g = cnn.nll_grad(out, xbar, var)
    _fd_check(lambda o: cnn.nll(o.reshape(3, 12), xbar, var), out.ravel().copy(), g.ravel(), range(36))
    # the minimum sits at mu = xbar, l = log var
    best = np.concatenate([xbar, np.log(var)], axis=1)
    assert np.allclose(cnn.nll_grad(best, xbar, var), 0.0, atol=1e-15)


def test_downsample_vs_scipy_and_invariants():
    rng = np.random.default_rng(5)
    v = rng.integers(0, 256, (20, 30, 40)).astype(np.uint8)
    d = cnn.downsample(v, side=8)
    c = [np.clip((np.arange(8) + 0.5) * n / 8 - 0.5, 0, n - 1) for n in v.shape]
    zz, yy, xx = np.meshgrid(*c, indexing="ij")
    ref = ndimage.map_coordinates(v.astype(float), [zz, yy, xx], order=1)
    assert np.allclose(d, ref, atol=1e-10)
    assert np.allclose(cnn.downsample(np.full((9, 7, 5), 42, np.uint8), side=4), 42.0)
    k, j, i = np.meshgrid(np.arange(32), np.arange(32), np.arange(32), indexing="ij")
    ramp = (2 * i + 3 * j + k).astype(np.uint8)
    dr = cnn.downsample(ramp, side=16)   # factor 2: centres at 2a + 0.5
    a = np.arange(16) * 2 + 0.5
    kk, jj, ii = np.meshgrid(a, a, a, indexing="ij")
    assert np.allclose(dr, 2 * ii + 3 * jj + kk, atol=1e-10)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-8, 8, 1000), [0.0, -0.0, 1.0, 3.0]])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(cnn.bf16(x), ref)


def test_param_count_and_layout():
    assert cnn.n_params() == 229916
    p = cnn.init_params(0)
    assert p.dtype == np.float32 and p.size == cnn.n_params()
    parts = cnn.unflatten(p)
    assert [q.shape for q in parts] == cnn.param_shapes()
    assert np.array_equal(cnn.flatten(parts).astype(np.float32), p)


def test_adam_matches_torch_over_several_steps():
    """Five steps of the oracle's Adam against torch.optim.Adam in FP64
    (beta 0.9 / 0.999, eps 1e-8): parameters and both moment estimates.
    The gradients change from step to step and span magnitudes down to the
    scale of eps, so swapped betas, bias-corrected moments returned in place
    of the raw ones, or eps inside the square root would all show."""
    rng = np.random.default_rng(12)
    n = 64
    p0 = rng.normal(size=n)
    grads = [rng.normal(size=n) * 10.0 ** rng.uniform(-9, 1, n) for _ in range(5)]
    lr = 0.01
    w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    for t, g in enumerate(grads, start=1):
        w.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = cnn.adam(p, g, m, v, t, lr)
        st = opt.state[w]
        assert np.allclose(p, w.detach().numpy(), rtol=1e-13, atol=1e-15), t
        assert np.allclose(m, st["exp_avg"].numpy(), rtol=1e-13, atol=0), t
        assert np.allclose(v, st["exp_avg_sq"].numpy(), rtol=1e-13, atol=0), t


def test_adam_step_direction():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -0.25])
    q, m, v = cnn.adam(p, g, np.zeros(2), np.zeros(2), 1, lr=0.1)
    assert np.allclose(q, p - 0.1 * np.sign(g), atol=1e-6)  # first step: lr * sign(g)
