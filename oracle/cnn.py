"""CPU oracle of the learned proposal network (test infrastructure only).

The paper names a machine-learning approach as future work (Conclusion); the
network itself is specified by the workload: two 64^3 input channels (source
and target downsampled), four 3x3x3 stride-2 convolutions (16, 32, 64, 64
channels, zero padding 1, bias, ReLU), a linear head to 6 means and 6
log-variances, trained with the Gaussian negative log-likelihood of the
particle filter's final weighted cloud.  Plain numpy in FP64; a convolution
is a sum over the 27 kernel offsets of strided slices contracted with
``numpy.einsum`` (a library primitive as a step), the backward pass is the
same sums transposed.

``bf16`` reproduces round-to-nearest-even to bfloat16 so that the oracle can
take the same precision decisions as the device (weights and stored
activations in bfloat16, everything else FP64 here).
"""

from __future__ import annotations

import numpy as np

SIDE = 64
CHANNELS = (2, 16, 32, 64, 64)
FLAT = 64 * 4 * 4 * 4
OUT = 12


def bf16(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (b.astype(np.uint32) << 16).view(np.float32)


def param_shapes():
    shapes = []
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        shapes += [(co, ci, 3, 3, 3), (co,)]
    shapes += [(OUT, FLAT), (OUT,)]
    return shapes


def n_params() -> int:
    return int(sum(np.prod(s) for s in param_shapes()))


def unflatten(flat):
    out, o = [], 0
    for s in param_shapes():
        n = int(np.prod(s))
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def flatten(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def init_params(seed: int) -> np.ndarray:
    """He-uniform convolution weights, small head, zero biases (host-side init
    shared by both sides as an input)."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        lim = np.sqrt(6.0 / (ci * 27))
        parts += [rng.uniform(-lim, lim, (co, ci, 3, 3, 3)), np.zeros(co)]
    parts += [rng.uniform(-1, 1, (OUT, FLAT)) * np.sqrt(1.0 / FLAT), np.zeros(OUT)]
    return flatten(parts).astype(np.float32)


# ------------------------------------------------------------------ downsampling

def _interp_matrix(n: int, m: int) -> np.ndarray:
    """Linear interpolation from n samples to m samples at half-pixel centres:
    output a samples input position (a + 0.5) n / m - 0.5, clamped to [0, n-1]."""
    pos = (np.arange(m) + 0.5) * (n / m) - 0.5
    pos = np.clip(pos, 0.0, n - 1.0)
    i0 = np.floor(pos).astype(int)
    f = pos - i0
    i1 = np.minimum(i0 + 1, n - 1)
    W = np.zeros((m, n))
    W[np.arange(m), i0] += 1.0 - f
    W[np.arange(m), i1] += f
    return W


def downsample(vol_zyx, side: int = SIDE, scale: float = 1.0) -> np.ndarray:
    """Trilinear resampling of a (nz, ny, nx) volume to side^3 at half-pixel
    centres (separable: trilinear weights are products of 1-D weights)."""
    v = np.asarray(vol_zyx, dtype=np.float64)
    nz, ny, nx = v.shape
    v = np.einsum("ax,zyx->zya", _interp_matrix(nx, side), v)
    v = np.einsum("by,zya->zba", _interp_matrix(ny, side), v)
    v = np.einsum("cz,zba->cba", _interp_matrix(nz, side), v)
    return v * scale


# ------------------------------------------------------------------ layers

def conv_fwd(x, w, b):
    """3x3x3 convolution, stride 2, zero padding 1: x [B, Ci, D, H, W] -> [B, Co, D/2, H/2, W/2]."""
    B, Ci, D, H, W = x.shape
    Do, Ho, Wo = D // 2, H // 2, W // 2
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    y = np.zeros((B, w.shape[0], Do, Ho, Wo))
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                xs = xp[:, :, kz:kz + 2 * Do:2, ky:ky + 2 * Ho:2, kx:kx + 2 * Wo:2]
                y += np.einsum("bcdhw,oc->bodhw", xs, w[:, :, kz, ky, kx])
    return y + b[None, :, None, None, None]


def conv_bwd(x, w, dy):
    """Gradients of conv_fwd: (dx, dw, db)."""
    B, Ci, D, H, W = x.shape
    Do, Ho, Wo = D // 2, H // 2, W // 2
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                sl = (slice(None), slice(None), slice(kz, kz + 2 * Do, 2), slice(ky, ky + 2 * Ho, 2),
                      slice(kx, kx + 2 * Wo, 2))
                dw[:, :, kz, ky, kx] = np.einsum("bodhw,bcdhw->oc", dy, xp[sl])
                dxp[sl] += np.einsum("bodhw,oc->bcdhw", dy, w[:, :, kz, ky, kx])
    return dxp[:, :, 1:-1, 1:-1, 1:-1], dw, dy.sum(axis=(0, 2, 3, 4))


def forward(params, x, bf16_acts=False):
    """Network forward.  Returns the 12 outputs per sample and the cache the
    backward pass needs.  With bf16_acts the stored activations (conv
    outputs after ReLU) are rounded to bfloat16, as on the device."""
    P = unflatten(params)
    acts = [np.asarray(x, dtype=np.float64)]
    h = acts[0]
    for L in range(4):
        h = np.maximum(conv_fwd(h, P[2 * L], P[2 * L + 1]), 0.0)
        if bf16_acts:
            h = bf16(h).astype(np.float64)
        acts.append(h)
    flat = h.reshape(h.shape[0], -1)
    out = flat @ P[8].T + P[9]
    return out, acts


def nll(out, xbar, var):
    """Gaussian NLL of the cloud (mean xbar, variance var) under N(mu, exp(l)),
    averaged over the batch: 0.5 sum_d [(var + (xbar - mu)^2) e^-l + l]."""
    mu, l = out[:, :6], out[:, 6:]
    e = np.exp(-l)
    per = 0.5 * np.sum((var + (xbar - mu) ** 2) * e + l, axis=1)
    return float(per.mean())


def nll_grad(out, xbar, var):
    mu, l = out[:, :6], out[:, 6:]
    e = np.exp(-l)
    B = out.shape[0]
    dmu = -(xbar - mu) * e / B
    dl = 0.5 * (1.0 - (var + (xbar - mu) ** 2) * e) / B
    return np.concatenate([dmu, dl], axis=1)


def backward(params, acts, dout):
    """Gradients of all parameters (flat, FP64) given dL/dout."""
    P = unflatten(params)
    grads = [None] * 10
    h = acts[4]
    flat = h.reshape(h.shape[0], -1)
    grads[8] = dout.T @ flat
    grads[9] = dout.sum(axis=0)
    dh = (dout @ P[8]).reshape(h.shape)
    for L in range(3, -1, -1):
        dh = dh * (acts[L + 1] > 0)
        dx, dw, db = conv_bwd(acts[L], P[2 * L], dh)
        grads[2 * L], grads[2 * L + 1] = dw, db
        dh = dx
    return flatten(grads)


def loss_and_grad(params, x, xbar, var, bf16_acts=False):
    out, acts = forward(params, x, bf16_acts)
    return nll(out, xbar, var), backward(params, acts, nll_grad(out, xbar, var)), out


def adam(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), FP64."""
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
