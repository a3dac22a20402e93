"""Pins of the oracle's warps and scores (CPU only).

Warps (Implementation Details: trilinear at non-grid positions; nearest for
masks) against closed forms -- identity, integer shifts, quarter turns of a
cube -- and against scipy.ndimage (library special cases).  DSC (Eq. 4),
NCC (Eq. 2) and the normalised SSD against closed forms and numpy.
"""

import numpy as np
import pytest
from scipy import ndimage

import synth


def _box(shape_zyx, lo, hi):
    v = np.zeros(shape_zyx, np.uint8)
    v[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = 1
    return v


def _M(t=(0, 0, 0), R=None):
    R = np.eye(3) if R is None else R
    return np.hstack([R, np.asarray(t, float).reshape(3, 1)])


def _shift(v, t):
    """dst[k, j, i] = v[k + tz, j + ty, i + tx] where in range, else 0."""
    out = np.zeros_like(v)
    nz, ny, nx = v.shape
    tx, ty, tz = t
    xs, xd = slice(max(tx, 0), nx + min(tx, 0)), slice(max(-tx, 0), nx + min(-tx, 0))
    ys, yd = slice(max(ty, 0), ny + min(ty, 0)), slice(max(-ty, 0), ny + min(-ty, 0))
    zs, zd = slice(max(tz, 0), nz + min(tz, 0)), slice(max(-tz, 0), nz + min(-tz, 0))
    out[zd, yd, xd] = v[zs, ys, xs]
    return out


@pytest.fixture(scope="module")
def img():
    rng = np.random.default_rng(5)
    return rng.integers(0, 256, (13, 17, 19)).astype(np.uint8)


# ------------------------------------------------------------------ warps

@pytest.mark.parametrize("trilinear", [False, True])
def test_warp_identity_and_integer_shift(orc, img, trilinear):
    shp = img.shape[::-1]
    assert np.array_equal(orc.warp_apply(img, _M(), trilinear, shp), img)
    for t in [(2, -1, 3), (-5, 4, 0), (0, 0, -7)]:
        assert np.array_equal(orc.warp_apply(img, _M(t), trilinear, shp), _shift(img, t))


def test_warp_nearest_quarter_turn_is_rot90(orc):
    rng = np.random.default_rng(6)
    n = 11
    v = rng.integers(0, 256, (n, n, n)).astype(np.uint8)
    M = orc.phys_matrix([0, 0, np.pi / 2, 0, 0, 0], (n, n, n))
    out = orc.warp_apply(v, M, False, (n, n, n))
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    assert np.array_equal(out, v[k, i, n - 1 - j])


def test_warp_nearest_half_voxel_tie_rounds_up(orc, img):
    out = orc.warp_apply(img, _M((0.5, 0, 0)), False, img.shape[::-1])
    assert np.array_equal(out, _shift(img, (1, 0, 0)))
    out = orc.warp_apply(img, _M((-0.5, 0, 0)), False, img.shape[::-1])
    assert np.array_equal(out, img)


def _affine_u(M, shape_xyz):
    nx, ny, nz = shape_xyz
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    p = np.stack([i, j, k], 0).reshape(3, -1).astype(float)
    return (M[:, :3] @ p + M[:, 3:4]).reshape(3, nz, ny, nx)


def test_warp_nearest_vs_scipy_interior(orc, img):
    rng = np.random.default_rng(7)
    shp = img.shape[::-1]
    for _ in range(5):
        p = np.concatenate([rng.uniform(-0.3, 0.3, 3), rng.uniform(-2, 2, 3)])
        M = orc.phys_matrix(p, shp)
        out = orc.warp_apply(img, M, False, shp)
        ref = ndimage.affine_transform(img, M[::-1, :3][:, ::-1], offset=M[::-1, 3], order=0, mode="nearest")
        u = _affine_u(M, shp)
        ok = np.ones(img.shape, bool)
        for d, n in enumerate(shp):
            ok &= (u[d] > 0.6) & (u[d] < n - 1.6) & (np.abs(u[d] - np.floor(u[d]) - 0.5) > 1e-3)
        assert ok.sum() > 200
        assert np.array_equal(out[ok], ref[ok])


def test_warp_trilinear_vs_scipy_interior(orc, img):
    rng = np.random.default_rng(8)
    shp = img.shape[::-1]
    for _ in range(5):
        p = np.concatenate([rng.uniform(-0.3, 0.3, 3), rng.uniform(-2, 2, 3)])
        M = orc.phys_matrix(p, shp)
        out = orc.warp_apply(img, M, True, shp).astype(int)
        u = _affine_u(M, shp)
        val = ndimage.map_coordinates(img.astype(float), u[::-1].reshape(3, -1), order=1,
                                      mode="nearest").reshape(img.shape)
        ok = np.ones(img.shape, bool)
        for d, n in enumerate(shp):
            ok &= (u[d] >= 0) & (u[d] <= n - 1)
        near_tie = np.abs(val - np.floor(val) - 0.5) < 1e-3
        assert ok.sum() > 200
        exact = ok & ~near_tie
        assert np.array_equal(out[exact], np.floor(val[exact] + 0.5).astype(int))
        assert np.all(np.abs(out[ok & near_tie] - val[ok & near_tie]) <= 0.51)
        assert np.all(out[~ok] == 0)


def test_warp_trilinear_vs_torch_grid_sample_interior(orc, img):
    """The same check against PyTorch's grid_sample (trilinear, corners
    aligned: normalised coordinate -1 at voxel 0 and +1 at voxel n - 1), a
    second library implementation of the interpolation."""
    import torch
    rng = np.random.default_rng(18)
    shp = img.shape[::-1]
    vol = torch.from_numpy(img.astype(np.float64))[None, None]
    for _ in range(3):
        p = np.concatenate([rng.uniform(-0.3, 0.3, 3), rng.uniform(-2, 2, 3)])
        M = orc.phys_matrix(p, shp)
        out = orc.warp_apply(img, M, True, shp).astype(int)
        u = _affine_u(M, shp)
        grid = np.stack([2.0 * u[d] / (shp[d] - 1) - 1.0 for d in range(3)], -1)  # (z, y, x, 3) as (x, y, z)
        val = torch.nn.functional.grid_sample(vol, torch.from_numpy(grid)[None], mode="bilinear",
                                              padding_mode="border", align_corners=True)[0, 0].numpy()
        ok = np.ones(img.shape, bool)
        for d, n in enumerate(shp):
            ok &= (u[d] >= 0) & (u[d] <= n - 1)
        near_tie = np.abs(val - np.floor(val) - 0.5) < 1e-3
        exact = ok & ~near_tie
        assert exact.sum() > 200
        assert np.array_equal(out[exact], np.floor(val[exact] + 0.5).astype(int))


def test_trilinear_reproduces_affine_ramp(orc):
    # trilinear interpolation is exact on affine intensity fields
    n = 16
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ramp = (3 * i + 2 * j + 5 * k).astype(np.uint8)  # <= 150
    M = _M((0.25, 0.5, 0.75))
    w = orc.recipe_words_from_matrix(M, (1, 1, 1), (1, 1, 1), nn=False)
    mom = orc.image_moments(ramp, ramp, w, True)
    inside = (i + 0.25 <= n - 1) & (j + 0.5 <= n - 1) & (k + 0.75 <= n - 1)
    s = 3 * (i + 0.25) + 2 * (j + 0.5) + 5 * (k + 0.75)
    assert mom[0] == inside.sum()
    assert mom[1] == int(np.floor(256 * s[inside] + 0.5).sum())


def test_constant_volume_stays_constant(orc):
    v = np.full((9, 10, 11), 77, np.uint8)
    M = orc.phys_matrix([0.1, -0.2, 0.3, 0.4, -0.3, 0.2], (11, 10, 9))
    out = orc.warp_apply(v, M, True, (11, 10, 9))
    assert set(np.unique(out)) <= {0, 77} and (out == 77).sum() > 100


# ------------------------------------------------------------------ mask counts / DSC

def test_dice_identity_is_one_and_disjoint_is_zero(orc):
    pair = synth.shell_pair(seed=3)
    t = pair["tgt"]
    w = orc.recipe_words(np.zeros(6), t, t, nn=True)
    n, a, c, b = orc.mask_counts(t, t, w)
    assert (n, a, c, b) == (t.size, t.sum(), t.sum(), t.sum())
    assert orc.dice(a, c, t.sum()) == 1.0
    w = orc.recipe_words(np.array([0, 0, 0, 70.0, 0, 0]), t, t, nn=True)
    n, a, c, b = orc.mask_counts(t, t, w)
    assert (n, a, c) == (0, 0, 0) and orc.dice(a, c, t.sum()) == 0.0
    assert orc.dice(0, 0, 0) == 0.0


def test_dice_shifted_boxes_closed_form(orc):
    shp = (40, 36, 32)
    lo, hi = (8, 9, 7), (30, 24, 22)
    B = _box(shp[::-1], lo, hi)
    for t in [(3, 0, 0), (-2, 4, 1), (5, -6, 3)]:
        w = orc.recipe_words(np.array([0, 0, 0, *t], float), B, B, nn=True)
        n, a, c, b = orc.mask_counts(B, B, w)
        ov = np.prod([(hi[d] - lo[d]) - abs(t[d]) for d in range(3)])
        assert a == B.sum() and c == ov
        assert orc.dice(a, c, B.sum()) == 2.0 * ov / (2.0 * B.sum())


def test_mask_counts_match_numpy_on_warped_volume(orc):
    pair = synth.shell_pair(seed=4)
    s, t = pair["src"], pair["tgt"]
    shp = t.shape[::-1]
    ones = np.ones_like(s)
    rng = np.random.default_rng(9)
    for _ in range(4):
        p = np.concatenate([rng.uniform(-0.3, 0.3, 3), rng.uniform(-8, 8, 3)])
        M = orc.phys_matrix(p, shp)
        ws = orc.warp_apply(s, M, False, shp)
        inside = orc.warp_apply(ones, M, False, shp)
        n, a, c, b = orc.mask_counts(s, t, orc.recipe_words(p, s, t, nn=True))
        assert n == inside.sum() and a == (ws != 0).sum() and c == ((ws != 0) & (t != 0)).sum()
        assert b == ((inside != 0) & (t != 0)).sum()


def test_mask_fov_excludes_voxels(orc):
    pair = synth.shell_pair(seed=4)
    s, t = pair["src"], pair["tgt"]
    fov = np.zeros_like(s)
    fov[:, :, :32] = 1
    w = orc.recipe_words(np.zeros(6), s, t, nn=True)
    n, a, c, b = orc.mask_counts(orc.Volume(s, fov=fov), t, w)
    assert n == fov.sum() and a == (s[:, :, :32] != 0).sum()


# ------------------------------------------------------------------ image moments / NCC / SSD

def _overlap_moments(src, tgt, t):
    """Exact recipe moments for an integer shift, from numpy."""
    warped = _shift(src.astype(np.int64), t)
    inside = _shift(np.ones_like(src, dtype=np.int64), t).astype(bool)
    s = 256 * warped[inside]
    tt = tgt.astype(np.int64)[inside]
    return np.array([inside.sum(), s.sum(), tt.sum(), (s * s).sum(), (tt * tt).sum(), (s * tt).sum()])


def test_image_moments_integer_shift_exact(orc):
    pair = synth.speckle_pair(side=40, seed=11, cone=False)
    s, t = pair["src"], pair["tgt"]
    for sh in [(0, 0, 0), (3, -2, 1), (-4, 0, 5)]:
        w = orc.recipe_words(np.array([0, 0, 0, *sh], float), s, t, nn=False)
        got = orc.image_moments(s, t, w, True)
        assert np.array_equal(got, _overlap_moments(s, t, sh))
        wn = orc.recipe_words(np.array([0, 0, 0, *sh], float), s, t, nn=True)
        assert np.array_equal(orc.image_moments(s, t, wn, False), got)


def test_ncc_linear_relation_is_one_and_matches_corrcoef(orc):
    pair = synth.speckle_pair(side=40, seed=12, cone=False)
    t = pair["tgt"]
    s_lin = np.clip(2 * (t.astype(int) // 2) + 3, 0, 255).astype(np.uint8)
    t_half = (t // 2).astype(np.uint8)
    m = orc.moments_to_double(orc.image_moments(s_lin, t_half, orc.recipe_words(np.zeros(6), t, t, False)))
    assert abs(orc.ncc(m) - 1.0) < 1e-12
    s = pair["src"]
    for sh in [(2, 1, -1), (0, -3, 2)]:
        mi = orc.image_moments(s, t, orc.recipe_words(np.array([0, 0, 0, *sh], float), s, t, False))
        warped = _shift(s.astype(float), sh)
        inside = _shift(np.ones_like(s), sh).astype(bool)
        r = np.corrcoef(warped[inside], t[inside].astype(float))[0, 1]
        assert abs(orc.ncc(orc.moments_to_double(mi)) - r * r) < 1e-12


def test_ncc_degenerate_cases(orc):
    assert orc.ncc([1, 5, 5, 25, 25, 25]) == 0.0            # one voxel
    assert orc.ncc([4, 8, 10, 16, 30, 20]) == 0.0           # constant s (var 0)
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=200000), rng.normal(size=200000)
    m = [a.size, a.sum(), b.sum(), (a * a).sum(), (b * b).sum(), (a * b).sum()]
    assert orc.ncc(m) < 1e-3                                 # independent noise


def test_ssd_identity_zero_and_numpy(orc):
    pair = synth.speckle_pair(side=40, seed=13, cone=False)
    s, t = pair["src"], pair["tgt"]
    pb = orc.Problem(t, t)
    st = pb.stats
    m = orc.moments_to_double(orc.image_moments(t, t, orc.recipe_words(np.zeros(6), t, t, False)))
    assert abs(orc.msd(m, st["mu_s"], st["sd_s"], st["mu_t"], st["sd_t"])) < 1e-12
    pb = orc.Problem(s, t)
    st = pb.stats
    assert abs(st["mu_s"] - s.mean()) < 1e-9 and abs(st["sd_s"] - s.std()) < 1e-9
    sh = (2, -1, 3)
    m = orc.moments_to_double(orc.image_moments(s, t, orc.recipe_words(np.array([0, 0, 0, *sh], float), s, t, False)))
    warped = _shift(s.astype(float), sh)
    inside = _shift(np.ones_like(s), sh).astype(bool)
    d = (warped[inside] - s.mean()) / s.std() - (t[inside] - t.mean()) / t.std()
    assert abs(orc.msd(m, st["mu_s"], st["sd_s"], st["mu_t"], st["sd_t"]) - np.mean(d * d)) < 1e-10


def test_fp64_trilinear_moments_vs_scipy(orc):
    pair = synth.speckle_pair(side=32, seed=14, cone=False)
    s, t = pair["src"], pair["tgt"]
    shp = t.shape[::-1]
    rng = np.random.default_rng(15)
    for _ in range(3):
        p = np.concatenate([rng.uniform(-0.3, 0.3, 3), rng.uniform(-4, 4, 3)])
        M = orc.phys_matrix(p, shp)
        u = _affine_u(M, shp)
        ok = np.ones(t.shape, bool)
        for d, n in enumerate(shp):
            ok &= (u[d] >= 0) & (u[d] <= n - 1)
        val = ndimage.map_coordinates(s.astype(float), u[::-1].reshape(3, -1), order=1,
                                      mode="nearest").reshape(t.shape)[ok]
        tt = t[ok].astype(float)
        want = np.array([ok.sum(), val.sum(), tt.sum(), (val * val).sum(), (tt * tt).sum(), (val * tt).sum()])
        got = orc.image_moments_fp64(s, t, p, True)
        assert got[0] == want[0]
        assert np.allclose(got[1:], want[1:], rtol=1e-11, atol=0)


def test_recipe_vs_fp64_similarity_within_1e5(orc):
    pair = synth.speckle_pair(side=48, seed=16)
    src = orc.Volume(pair["src"], fov=pair["src_fov"])
    pb = orc.Problem(src, pair["tgt"])
    rng = np.random.default_rng(17)
    x = np.concatenate([rng.uniform(-0.2, 0.2, (24, 3)), rng.uniform(-4, 4, (24, 3))], 1)
    x[0] = pair["gt"]
    for score in ("ncc", "ssd"):
        prm = dict(n_particles=len(x), n_iters=1, score=score, limit=[1] * 6, sigma_score=0.1,
                   sigma0=[0] * 6, min_overlap_frac=0.0)
        zr = pb.score(prm, x)
        zf = pb.score(prm, x, fp64_mode=True)
        assert np.all(np.isfinite(zr))
        # FP32 coordinates move a few voxels across the overlap boundary, so the
        # drift is bounded absolutely everywhere and relatively near the optimum
        assert np.max(np.abs(zr - zf) / np.maximum(np.abs(zf), 1.0)) < 1e-5, score
        good = np.abs(zf) > 0.5 if score == "ncc" else np.ones(len(zf), bool)
        assert good.sum() >= 1
        assert np.max(np.abs(zr - zf)[good] / np.abs(zf)[good]) < 1e-5, score


def test_min_overlap_gives_minus_inf(orc):
    pair = synth.speckle_pair(side=24, seed=18, cone=False)
    pb = orc.Problem(pair["src"], pair["tgt"])
    prm = dict(n_particles=2, n_iters=1, score="ncc", limit=[1] * 6, sigma_score=0.1, sigma0=[0] * 6,
               min_overlap_frac=0.5)
    z = pb.score(prm, np.array([[0, 0, 0, 0, 0, 0], [0, 0, 0, 15.0, 0, 0]]))
    assert np.isfinite(z[0]) and z[1] == -np.inf


def test_scores_do_not_depend_on_thread_count(orc):
    """The oracle's parallel loop over particles gives the same scores on one
    thread as on all of them (the CPU baseline times both)."""
    pair = synth.speckle_pair(side=32, seed=9, trans=3.0)
    prm = dict(n_particles=24, n_iters=1, score="ncc", interp="trilinear", sigma_score=0.02,
               limit=list(np.deg2rad([10.0] * 3)) + [3.0] * 3, sigma0=[0.01] * 6)
    x = orc.init_particles(prm)
    pb = orc.Problem(orc.Volume(pair["src"], fov=pair["src_fov"]), orc.Volume(pair["tgt"]))
    threads = orc.num_threads()
    want = pb.score(prm, x)
    orc.set_threads(1)
    try:
        assert orc.num_threads() == 1
        got = pb.score(prm, x)
    finally:
        orc.set_threads(threads)
    assert orc.num_threads() == threads
    assert np.array_equal(got, want)
