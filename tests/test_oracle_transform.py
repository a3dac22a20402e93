"""Pins of the oracle's random numbers and transform (CPU only).

Philox against the published known-answer vectors and against rocRAND's
implementation of the same generator; the Euler 3D transform of
Implementation Details / Eq. 3 against scipy's rotation (a library special
case), orthonormality, det = +1, composition and the fixed rotation centre.
"""

import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(orc):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert list(orc.philox(ctr, key)) == want


def test_philox_matches_rocrand_engine(orc, tmp_path):
    """The oracle's Philox4x32-10 against rocRAND's implementation of the
    same generator (its header engine built for the host), on the
    published vectors and random counters and keys."""
    import ctypes
    import shutil
    import subprocess
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr) or shutil.which("g++") is None:
        pytest.skip("rocRAND headers or g++ not available")
    so = str(tmp_path / "librr.so")
    shim = os.path.join(os.path.dirname(__file__), "rocrand_philox_shim.cpp")
    subprocess.run(["g++", "-O2", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", shim,
                    "-o", so], check=True, capture_output=True)
    rr = ctypes.CDLL(so)
    rng = np.random.default_rng(5)
    n = 20000
    ctr = rng.integers(0, 2 ** 32, (n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:8] = 0  # small counters, as the filter uses them
    ctr[:8, 0] = np.arange(8)
    key = rng.integers(0, 2 ** 32, (n, 2), dtype=np.uint64).astype(np.uint32)
    key[:4] = 0
    for ctr_k, key_k, _ in _kat():
        ctr = np.vstack([ctr, np.array(ctr_k, np.uint32)])
        key = np.vstack([key, np.array(key_k, np.uint32)])
    ctr, key = np.ascontiguousarray(ctr), np.ascontiguousarray(key)
    out = np.zeros((len(ctr), 4), np.uint32)
    rr.rr_philox_blocks(ctypes.c_ulonglong(len(ctr)), ctr.ctypes.data_as(ctypes.c_void_p),
                        key.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p))
    want = np.array([orc.philox(c, k) for c, k in zip(ctr, key)], np.uint32)
    assert np.array_equal(out, want)


def test_u53_range_and_resolution(orc):
    assert orc.u53(0, 0) == 0.5 * 2.0 ** -53
    assert 0.0 < orc.u53(0, 63) == orc.u53(0, 0)  # low 6 bits of b are dropped
    assert orc.u53(0, 64) == 1.5 * 2.0 ** -53
    assert orc.u53(0xFFFFFFFF, 0xFFFFFFFF) <= 1.0
    assert orc.u53(1 << 31, 0) == 0.5 + 0.5 * 2.0 ** -53


def test_euler_matches_scipy_intrinsic_zxy(orc):
    rng = np.random.default_rng(0)
    for _ in range(50):
        p = rng.uniform(-np.pi, np.pi, 3)
        want = Rotation.from_euler("ZXY", [p[2], p[0], p[1]]).as_matrix()
        assert np.abs(orc.euler_R(p) - want).max() < 1e-14


def test_elementary_axes_right_handed(orc):
    a = 0.3
    ey = np.array([0.0, 1.0, 0.0])
    ez = np.array([0.0, 0.0, 1.0])
    ex = np.array([1.0, 0.0, 0.0])
    # rotation about x carries y toward z, about y carries z toward x, about z carries x toward y
    assert np.allclose(orc.euler_R([a, 0, 0]) @ ey, [0, np.cos(a), np.sin(a)], atol=1e-15)
    assert np.allclose(orc.euler_R([0, a, 0]) @ ez, [np.sin(a), 0, np.cos(a)], atol=1e-15)
    assert np.allclose(orc.euler_R([0, 0, a]) @ ex, [np.cos(a), np.sin(a), 0], atol=1e-15)
    # order: R = Rz Rx Ry
    p = [0.2, -0.4, 0.7]
    Rx, Ry, Rz = orc.euler_R([p[0], 0, 0]), orc.euler_R([0, p[1], 0]), orc.euler_R([0, 0, p[2]])
    assert np.abs(orc.euler_R(p) - Rz @ Rx @ Ry).max() < 1e-15


def test_orthonormal_det_one_and_composition(orc):
    rng = np.random.default_rng(1)
    for _ in range(50):
        R1 = orc.euler_R(rng.uniform(-np.pi, np.pi, 3))
        R2 = orc.euler_R(rng.uniform(-np.pi, np.pi, 3))
        for R in (R1, R2, R1 @ R2, R2 @ R1 @ R1):
            assert np.abs(R @ R.T - np.eye(3)).max() <= 1e-14
            assert abs(np.linalg.det(R) - 1.0) <= 1e-14
        assert np.abs(R1 @ R1.T - np.eye(3)).max() <= 1e-14  # compose with inverse = identity


def test_quarter_turns_are_permutations(orc):
    for p, perm in [([0, 0, np.pi / 2], [[0, -1, 0], [1, 0, 0], [0, 0, 1]]),
                    ([np.pi / 2, 0, 0], [[1, 0, 0], [0, 0, -1], [0, 1, 0]]),
                    ([0, np.pi / 2, 0], [[0, 0, 1], [0, 1, 0], [-1, 0, 0]])]:
        assert np.abs(orc.euler_R(p) - np.array(perm, float)).max() < 1e-15


def test_phys_matrix_fixed_centre_and_scipy(orc):
    import synth
    rng = np.random.default_rng(2)
    for _ in range(20):
        p = np.concatenate([rng.uniform(-0.5, 0.5, 3), rng.uniform(-10, 10, 3)])
        shape = tuple(int(v) for v in rng.integers(8, 90, 3))
        sp = tuple(rng.uniform(0.7, 1.3, 3))
        M = orc.phys_matrix(p, shape, sp)
        c = 0.5 * np.asarray(sp) * (np.asarray(shape) - 1)
        assert np.abs(M[:, :3] @ c + M[:, 3] - (c + p[3:])).max() < 1e-12
        G = synth.gt_matrix(p, shape, sp)
        assert np.abs(M - G[:3]).max() < 1e-12
    M0 = orc.phys_matrix(np.zeros(6), (10, 12, 14))
    assert np.array_equal(M0, np.hstack([np.eye(3), np.zeros((3, 1))]))


def test_recipe_words_identity_and_spacing(orc):
    src = np.zeros((5, 6, 7), np.uint8)
    w_tri = orc.recipe_words(np.zeros(6), src, src, nn=False)
    w_nn = orc.recipe_words(np.zeros(6), src, src, nn=True)
    assert np.array_equal(w_tri, np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32))
    assert np.array_equal(w_nn, np.array([1, 0, 0, .5, 0, 1, 0, .5, 0, 0, 1, .5], np.float32))
    # anisotropic spacing: A = diag(1/s_S) R diag(s_T)
    M = np.hstack([np.eye(3), np.array([[1.0], [2.0], [3.0]])])
    w = orc.recipe_words_from_matrix(M, (0.5, 1.0, 2.0), (1.0, 0.25, 4.0), nn=False).reshape(3, 4)
    assert np.allclose(np.diag(w[:, :3]), [0.5, 4.0, 0.5]) and np.allclose(w[:, 3], [1.0, 8.0, 0.75])
