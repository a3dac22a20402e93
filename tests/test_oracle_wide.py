"""Pins of the wide-rotation mode of the oracle: the quaternion route
against the matrix route and scipy, the angle extraction, the quaternion
mean's invariances and its behaviour across the +-pi seam, the wrapped
prediction, and a registration whose rotation sits at the seam."""

import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation as Rot

import synth
from paper_2504_19930_amd import config

pytestmark = pytest.mark.filterwarnings("ignore")


def _scipy_R(p):
    # R = Rz(rz) Rx(rx) Ry(ry): intrinsic Z, X, Y
    return Rot.from_euler("ZXY", [p[2], p[0], p[1]]).as_matrix()


def _angle_between(Ra, Rb):
    # geodesic angle, accurate for small angles (the trace form is not)
    return float(np.linalg.norm(Rot.from_matrix(Ra.T @ Rb).as_rotvec()))


def test_quaternion_route_matches_matrix_route_and_scipy(orc):
    rng = np.random.default_rng(0)
    for _ in range(200):
        p = np.concatenate([rng.uniform(-math.pi, math.pi, 3), np.zeros(3)])
        q = orc.euler_quat(p)
        assert abs(np.linalg.norm(q) - 1.0) < 1e-15
        assert np.allclose(orc.quat_R(q), orc.euler_R(p), atol=1e-14)
        qs = Rot.from_matrix(_scipy_R(p)).as_quat()  # (x, y, z, w)
        qs = np.array([qs[3], qs[0], qs[1], qs[2]])
        assert min(np.abs(q - qs).max(), np.abs(q + qs).max()) < 1e-12


def test_euler_extraction_round_trip(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        p = np.array([rng.uniform(-1.5, 1.5), rng.uniform(-3.1, 3.1), rng.uniform(-3.1, 3.1)])
        e = orc.R_euler(orc.euler_R(np.concatenate([p, np.zeros(3)])))
        assert np.allclose(e, p, atol=1e-12)
        # scipy's intrinsic ZXY angles are (rz, rx, ry)
        s = Rot.from_matrix(_scipy_R(p)).as_euler("ZXY")
        assert np.allclose([s[1], s[2], s[0]], p, atol=1e-10)


def _particles_from_rotations(Rs, t):
    out = []
    for R in Rs:
        s = Rot.from_matrix(R).as_euler("ZXY")
        out.append([s[1], s[2], s[0], *t])
    return np.array(out)


def test_quaternion_mean_of_symmetric_pairs_is_the_centre(orc):
    rng = np.random.default_rng(2)
    for _ in range(20):
        p0 = rng.uniform(-1.2, 1.2, 3)
        R0 = _scipy_R(p0)
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        d = Rot.from_rotvec(axis * rng.uniform(0.05, 0.6)).as_matrix()
        x = _particles_from_rotations([R0 @ d, R0 @ d.T], [1.0, 2.0, 3.0])
        r = orc.normalise_wide(np.zeros(2), x, np.zeros(6))
        assert _angle_between(orc.euler_R(np.concatenate([r["est"][:3], np.zeros(3)])), R0) < 1e-12
        assert np.allclose(r["est"][3:], [1.0, 2.0, 3.0], atol=1e-15)


def test_quaternion_mean_across_the_seam(orc):
    """Two clusters of the same rotation written with rz near +pi and near
    -pi: the Euler mean lands near rz = 0 (a half-turn away), the quaternion
    mean on the true rotation."""
    true = np.array([0.1, -0.2, math.pi - 0.02])
    rng = np.random.default_rng(3)
    n = 64
    x = np.zeros((n, 6))
    for i in range(n):
        R = _scipy_R(true) @ Rot.from_rotvec(rng.normal(0, 0.01, 3)).as_matrix()
        s = Rot.from_matrix(R).as_euler("ZXY")
        e = np.array([s[1], s[2], s[0]])
        if i % 2:
            e[2] = e[2] - 2 * math.pi if e[2] > 0 else e[2] + 2 * math.pi
        x[i, :3] = e
    lw = rng.normal(0, 0.1, n)
    Rt = _scipy_R(true)
    box = orc.normalise(lw, x)["est"]
    wide = orc.normalise_wide(lw, x, np.zeros(6))["est"]
    assert _angle_between(orc.euler_R(np.concatenate([box[:3], np.zeros(3)])), Rt) > 2.0
    assert _angle_between(orc.euler_R(np.concatenate([wide[:3], np.zeros(3)])), Rt) < 0.01
    assert np.all(np.abs(wide[:3]) <= math.pi)


def test_quaternion_mean_ignores_the_double_cover_and_is_near_the_euler_mean_for_small_spreads(orc):
    rng = np.random.default_rng(4)
    p0 = np.array([0.3, -0.5, 0.8])
    x = np.zeros((32, 6))
    x[:, :3] = p0 + rng.normal(0, 0.01, (32, 3))
    x[:, 3:] = rng.normal(0, 1, (32, 3))
    lw = rng.normal(0, 0.5, 32)
    a = orc.normalise_wide(lw, x, np.zeros(6))
    b = orc.normalise(lw, x)
    assert np.allclose(a["est"], b["est"], atol=5e-4)
    assert np.allclose(a["w"], b["w"], rtol=0, atol=0) and a["ess"] == b["ess"]
    # the same rotations written with the other ZXY angle triple
    y = x.copy()
    y[:, 0] = math.pi - x[:, 0]
    y[:, 1] = x[:, 1] + math.pi
    y[:, 2] = x[:, 2] + math.pi
    for i in range(32):
        assert np.allclose(orc.euler_R(y[i]), orc.euler_R(x[i]), atol=1e-14)
    c = orc.normalise_wide(lw, y, np.zeros(6))
    assert np.allclose(c["est"], a["est"], atol=1e-12)


def test_wide_prediction_wraps_full_circle_axes_only(orc):
    prm = config.default_params("dice", 8, 3, 15.0, 5.0)
    prm["limit"] = [math.pi, 0.3, math.pi, 5.0, 5.0, 5.0]
    prm["x0"] = [0.0, 0.0, 1.0, 0.0, 0.0, 0.0]
    prm["sigma0"] = [0.5, 0.5, 0.5, 1.0, 1.0, 1.0]
    x = np.zeros((8, 6))
    x[:, 0] = math.pi - 1e-3
    x[:, 1] = 0.3 - 1e-3
    x[:, 2] = 1.0 + math.pi - 1e-3
    anc = np.arange(8, dtype=np.int32)
    box = orc.perturb(prm, 1, x, anc)
    wide = orc.perturb(dict(prm, rotation_mode="wide"), 1, x, anc)
    g = np.array([orc.gauss6(prm.get("seed", 0), 0, j, 1) for j in range(8)])
    raw = x + np.asarray(prm["sigma0"]) * g
    for j in range(8):
        for d, c in ((0, 0.0), (2, 1.0)):
            # whole turns only, into [c - pi, c + pi)
            assert c - math.pi <= wide[j, d] < c + math.pi
            turns = (raw[j, d] - wide[j, d]) / (2 * math.pi)
            assert abs(turns - round(turns)) < 1e-12
        # limits below pi still reflect, exactly as the box mode
        assert wide[j, 1] == box[j, 1] and np.array_equal(wide[j, 3:], box[j, 3:])
        assert -0.3 <= wide[j, 1] <= 0.3


def test_wide_registration_at_the_seam(orc):
    """An ellipsoid off the rotation centre (so a half-turn is observable),
    turned by 178 degrees about z and searched over the whole circle in rz:
    the wide mode recovers it."""
    gt = np.array([math.radians(4.0), math.radians(-3.0), math.radians(178.0), 2.0, -1.5, 1.0])
    pair = synth.mask_pair((40, 40, 40), outer=(10.0, 7.0, 5.0), inner=None, gt=gt,
                           centre=(19.5 + 7.0, 19.5 + 3.0, 19.5 + 2.0))
    prm = config.default_params("dice", 512, 15, 10.0, 4.0, seed=5)
    prm["limit"][2] = math.pi
    prm["sigma0"][2] = 0.15 * 0.5
    out = orc.smc_run(pair["src"], pair["tgt"], dict(prm, rotation_mode="wide"))
    est = out["est"]
    err = _angle_between(orc.euler_R(np.concatenate([est[:3], np.zeros(3)])),
                         orc.euler_R(np.concatenate([gt[:3], np.zeros(3)])))
    # a 1.5k-voxel mask pins the rotation to a few degrees
    assert math.degrees(err) < 5.0, (math.degrees(err), est)
    assert np.abs(est[3:] - gt[3:]).max() < 1.0
    assert out["trace_score"][-1] > 0.95
