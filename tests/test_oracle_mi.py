"""Pins of the oracle's mutual-information score: the joint histogram
under integer shifts equals numpy's over the overlap, the symmetric
uncertainty equals scikit-learn's mutual information over scipy's
entropies, identical images score 1, a bijection of the target bins leaves
the score unchanged, independent noise scores near 0, and an MI
registration recovers a known transform."""

import math

import numpy as np
import pytest
from scipy.stats import entropy
from sklearn.metrics import mutual_info_score

import synth
from paper_2504_19930_amd import config


def _shift_pairs(src, tgt, t):
    nz, ny, nx = tgt.shape
    tx, ty, tz = t
    zs, ys, xs = slice(max(0, -tz), min(nz, nz - tz)), slice(max(0, -ty), min(ny, ny - ty)), \
        slice(max(0, -tx), min(nx, nx - tx))
    zd, yd, xd = slice(zs.start + tz, zs.stop + tz), slice(ys.start + ty, ys.stop + ty), \
        slice(xs.start + tx, xs.stop + tx)
    return src[zd, yd, xd].ravel(), tgt[zs, ys, xs].ravel()


def _u_reference(a, b):
    mi = mutual_info_score(a, b)
    hs = entropy(np.bincount(a))
    ht = entropy(np.bincount(b))
    return 2.0 * mi / (hs + ht)


@pytest.mark.parametrize("t", [(0, 0, 0), (3, -2, 1), (-5, 4, -3)])
def test_histogram_and_score_under_integer_shifts(orc, t):
    pair = synth.speckle_pair(side=32, seed=5, trans=3.0)
    src, tgt = pair["src"], pair["tgt"]
    w = orc.recipe_words(np.array([0.0, 0.0, 0.0, *t], float), src, tgt, nn=False)
    h = orc.joint_histogram(src, tgt, w)
    s, tv = _shift_pairs(src, tgt, t)
    ref = np.zeros((32, 32), np.uint64)
    np.add.at(ref, (s >> 3, tv >> 3), 1)
    assert np.array_equal(h, ref)
    got = orc.mi_score(h)
    assert abs(got - _u_reference(s >> 3, tv >> 3)) <= 1e-12


def test_identical_images_score_one_and_bin_bijection_invariance(orc):
    pair = synth.speckle_pair(side=32, seed=6)
    img = pair["tgt"]
    w = orc.recipe_words(np.zeros(6), img, img, nn=False)
    assert orc.mi_score(orc.joint_histogram(img, img, w)) == 1.0
    src = pair["src"]
    h1 = orc.joint_histogram(src, img, orc.recipe_words(np.zeros(6), src, img, nn=False))
    flipped = (255 - img).astype(np.uint8)
    h2 = orc.joint_histogram(src, flipped, orc.recipe_words(np.zeros(6), src, flipped, nn=False))
    assert np.array_equal(h2, h1[:, ::-1])
    assert abs(orc.mi_score(h2) - orc.mi_score(h1)) <= 1e-14


def test_independent_noise_scores_near_zero(orc):
    rng = np.random.default_rng(7)
    a = rng.integers(0, 256, (40, 40, 40)).astype(np.uint8)
    b = rng.integers(0, 256, (40, 40, 40)).astype(np.uint8)
    u = orc.mi_score(orc.joint_histogram(a, b, orc.recipe_words(np.zeros(6), a, b, nn=False)))
    assert 0.0 <= u < 0.03


def test_mi_registration_recovers_transform(orc):
    pair = synth.speckle_pair(side=40, seed=9, trans=3.0)
    prm = config.default_params("mi", 256, 12, 20.0, 3.0, seed=4)
    out = orc.smc_run(orc.Volume(pair["src"], fov=pair["src_fov"]), orc.Volume(pair["tgt"]), prm)
    err = np.abs(out["est"] - pair["gt"])
    assert np.degrees(err[:3]).max() < 2.0 and err[3:].max() < 1.0, (np.degrees(err[:3]), err[3:])


def test_mi_log_matches_the_library_log(orc):
    rng = np.random.default_rng(8)
    xs = np.concatenate([rng.uniform(1e-9, 1.0, 20000), 10.0 ** rng.uniform(-300, 0, 2000),
                         [1.0, 0.5, 2.0 ** -20, 1.0 / 3.0, 0.7071067811865476, 0.70710678118654746]])
    for x in xs:
        want = math.log(x)
        got = orc.mi_log(x)
        assert abs(got - want) <= 4 * np.spacing(abs(want)) + 1e-300, (x, got, want)
    assert orc.mi_log(1.0) == 0.0
