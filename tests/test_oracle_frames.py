"""Pins of the oracle's multi-frame score (several frame pairs under one
transform, sums pooled before the score): repeated frames leave the score
unchanged, pooled Dice and NCC under integer shifts equal their numpy
definitions over the union of the frames, and a two-frame registration
recovers a known transform."""

import math

import numpy as np
import pytest

import synth
from paper_2504_19930_amd import config


def _shift_warp(src, t):
    """Nearest / trilinear warp of a (nz, ny, nx) volume by an integer shift
    t = (tx, ty, tz): target voxel p reads source p + t; outside -> absent."""
    nz, ny, nx = src.shape
    out = np.zeros_like(src)
    inside = np.zeros(src.shape, bool)
    tx, ty, tz = t
    zs, ys, xs = slice(max(0, -tz), min(nz, nz - tz)), slice(max(0, -ty), min(ny, ny - ty)), \
        slice(max(0, -tx), min(nx, nx - tx))
    zd, yd, xd = slice(zs.start + tz, zs.stop + tz), slice(ys.start + ty, ys.stop + ty), \
        slice(xs.start + tx, xs.stop + tx)
    out[zs, ys, xs] = src[zd, yd, xd]
    inside[zs, ys, xs] = True
    return out, inside


def _frames(seed):
    lv = synth.lv_sequence(shape_xyz=(40, 36, 32), n_frames=4, seed=seed, rot_deg=0.0, trans=0.0,
                           speckle=True, frames=[0, 2])
    return lv


def test_repeated_frames_leave_the_score_unchanged(orc):
    lv = _frames(1)
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-0.2, 0.2, (6, 3)), rng.uniform(-3, 3, (6, 3))], 1)
    for score, s, t in (("dice", lv["src_masks"][0], lv["tgt_masks"][0]),
                        ("ncc", lv["src_speckle"][0], lv["tgt_speckle"][0])):
        prm = config.default_params(score, 4, 2, 10.0, 3.0)
        one = orc.Frames([(s, t)]).score(prm, x)
        # doubling every sum scales each term of the formulas by a power of two
        assert np.array_equal(orc.Frames([(s, t)] * 2).score(prm, x), one), score
        assert np.allclose(orc.Frames([(s, t)] * 3).score(prm, x), one, rtol=1e-14, atol=0), score
        assert np.array_equal(orc.Frames([(s, t)] * 3).sums(prm, x), 3 * orc.Frames([(s, t)]).sums(prm, x))


def test_pooled_dice_and_ncc_under_integer_shifts(orc):
    lv = _frames(2)
    ms, mt = lv["src_masks"], lv["tgt_masks"]
    ss, st = lv["src_speckle"], lv["tgt_speckle"]
    for t in ((0, 0, 0), (2, -1, 3), (-4, 2, -1)):
        p = np.array([0.0, 0.0, 0.0, *t], float)
        # Dice: 2 sum |S n T| / (sum |warped S| + sum |T|) over both frames
        inter = on = tot = 0
        for f in range(2):
            w, inside = _shift_warp(ms[f], t)
            inter += int(np.sum((w != 0) & inside & (mt[f] != 0)))
            on += int(np.sum((w != 0) & inside))
            tot += int(np.sum(mt[f] != 0))
        prm = config.default_params("dice", 1, 1, 10.0, 3.0)
        got = orc.Frames([(ms[0], mt[0]), (ms[1], mt[1])]).score(prm, p[None])[0]
        assert got == 2.0 * inter / (on + tot)
        # NCC: squared correlation over the union of the two overlaps
        sv, tv = [], []
        for f in range(2):
            w, inside = _shift_warp(ss[f], t)
            sv.append(w[inside].astype(float))
            tv.append(st[f][inside].astype(float))
        sv, tv = np.concatenate(sv), np.concatenate(tv)
        want = np.corrcoef(sv, tv)[0, 1] ** 2
        prm = config.default_params("ncc", 1, 1, 10.0, 3.0)
        got = orc.Frames([(ss[0], st[0]), (ss[1], st[1])]).score(prm, p[None])[0]
        assert abs(got - want) <= 1e-12 * max(1.0, want)


def test_ssd_is_not_pooled(orc):
    lv = _frames(3)
    prm = config.default_params("ssd", 1, 1, 10.0, 3.0)
    pair = (lv["src_speckle"][0], lv["tgt_speckle"][0])
    assert math.isnan(orc.Frames([pair, pair]).score(prm, np.zeros((1, 6)))[0])


def test_two_frame_registration_recovers_the_transform(orc):
    gt = np.array([math.radians(6.0), math.radians(-4.0), math.radians(5.0), 2.5, -1.5, 2.0])
    shape, c = (48, 44, 40), (25.5, 22.5, 19.0)
    ed = synth.mask_pair(shape, outer=(16.0, 10.0, 8.0), inner=None, gt=gt, centre=c)
    es = synth.mask_pair(shape, outer=(12.8, 8.0, 6.4), inner=None, gt=gt, centre=c)
    prm = config.default_params("dice", 256, 12, 10.0, 4.0, seed=3)
    out = orc.smc_run(ed["src"], ed["tgt"], prm, frames=[(es["src"], es["tgt"])])
    assert np.abs(out["est"][3:] - gt[3:]).max() < 1.0
    assert out["trace_score"][-1] > 0.9
