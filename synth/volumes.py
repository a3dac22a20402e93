"""Seeded synthetic volume pairs (see the package docstring).

Conventions shared with every consumer:

* arrays are ``(nz, ny, nx)`` uint8, C order, so x is the fastest axis;
* voxel ``(i, j, k)`` sits at ``s * (i, j, k)`` mm (spacing 1 unless stated);
* the ground truth is ``(rx, ry, rz, tx, ty, tz)`` in radians and mm.  It maps a
  target point p to the source point ``q = R (p - c) + c + t`` with
  ``R = Rz(rz) Rx(rx) Ry(ry)`` and c the target centre, so a perfect
  registration recovers exactly these parameters;
* the source is the target scene seen through the inverse map: a source voxel q
  shows what sits at ``R^T (q - c - t) + c`` in the target scene.
"""

from __future__ import annotations

import numpy as np
from scipy import ndimage
from scipy.spatial.transform import Rotation


def _rot(rx: float, ry: float, rz: float) -> np.ndarray:
    # intrinsic Z, then X, then Y: R = Rz @ Rx @ Ry
    return Rotation.from_euler("ZXY", [rz, rx, ry]).as_matrix()


def gt_matrix(params, shape_xyz, spacing=(1.0, 1.0, 1.0)) -> np.ndarray:
    """4x4 homogeneous target-mm -> source-mm map of the ground truth (the
    matrix form of the paper's Eq. 3, built here with scipy's rotation)."""
    rx, ry, rz, tx, ty, tz = (float(v) for v in params)
    R = _rot(rx, ry, rz)
    c = 0.5 * np.asarray(spacing, float) * (np.asarray(shape_xyz, float) - 1.0)
    M = np.eye(4)
    M[:3, :3] = R
    M[:3, 3] = c + np.array([tx, ty, tz]) - R @ c
    return M


def _sample_gt(rng, rot_deg, trans):
    ang = np.deg2rad(rng.uniform(-rot_deg, rot_deg, 3))
    t = rng.uniform(-trans, trans, 3)
    return np.concatenate([ang, t])


def _centres(shape_xyz, spacing=(1.0, 1.0, 1.0), z_slice=None):
    """Voxel-centre coordinates (mm) as three (nz, ny, nx) arrays."""
    nx, ny, nz = shape_xyz
    zs = np.arange(nz) if z_slice is None else np.arange(nz)[z_slice]
    z, y, x = np.meshgrid(zs * spacing[2], np.arange(ny) * spacing[1],
                          np.arange(nx) * spacing[0], indexing="ij")
    return x, y, z


def _preimage(gt, shape_xyz_src, shape_xyz_tgt, spacing=(1.0, 1.0, 1.0)):
    """For every source voxel centre q, the target-scene point R^T (q - off)."""
    M = gt_matrix(gt, shape_xyz_tgt, spacing)
    R, off = M[:3, :3], M[:3, 3]
    x, y, z = _centres(shape_xyz_src, spacing)
    d = np.stack([x - off[0], y - off[1], z - off[2]], axis=0).reshape(3, -1)
    p = R.T @ d
    return [a.reshape(x.shape) for a in p]


def _ellipsoid_r2(x, y, z, centre, axes):
    return (((x - centre[0]) / axes[0]) ** 2 + ((y - centre[1]) / axes[1]) ** 2
            + ((z - centre[2]) / axes[2]) ** 2)


def _shell(x, y, z, centre, outer, inner):
    inside_outer = _ellipsoid_r2(x, y, z, centre, outer) <= 1.0
    if inner is None:
        return inside_outer
    return inside_outer & (_ellipsoid_r2(x, y, z, centre, inner) > 1.0)


def mask_pair(shape_xyz=(64, 64, 64), outer=(22.0, 16.0, 16.0), inner=(19.0, 13.0, 13.0),
              rot_deg=15.0, trans=8.0, seed=1, gt=None, centre=None) -> dict:
    """Binary LV-like mask pair: an ellipsoidal shell (``inner`` given) or a filled
    ellipsoid (``inner=None``) rasterised at voxel centres in the target, and the
    same analytic shape seen through the inverse ground-truth map in the source."""
    rng = np.random.default_rng(seed)
    if gt is None:
        gt = _sample_gt(rng, rot_deg, trans)
    gt = np.asarray(gt, float)
    c = 0.5 * (np.asarray(shape_xyz, float) - 1.0) if centre is None else np.asarray(centre, float)
    x, y, z = _centres(shape_xyz)
    tgt = _shell(x, y, z, c, outer, inner).astype(np.uint8)
    px, py, pz = _preimage(gt, shape_xyz, shape_xyz)
    src = _shell(px, py, pz, c, outer, inner).astype(np.uint8)
    return dict(kind="mask", src=src, tgt=tgt, gt=gt, spacing=(1.0, 1.0, 1.0),
                shape_xyz=tuple(shape_xyz))


def shell_pair(seed=1, side=64, rot_deg=15.0, trans=8.0) -> dict:
    """The 64^3 thick-shell workload: semi-axes 22/16/16, wall 3 voxels,
    rotations U[-15, 15] deg per axis and translations U[-8, 8] voxels
    (scaled with ``side`` for other sizes)."""
    f = side / 64.0
    return mask_pair((side, side, side), outer=(22 * f, 16 * f, 16 * f),
                     inner=(22 * f - 3, 16 * f - 3, 16 * f - 3),
                     rot_deg=rot_deg, trans=trans * f, seed=seed)


# ----------------------------------------------------------------------------- images

def _sigmoid(v):
    return 1.0 / (1.0 + np.exp(-v))


def _anatomy(x, y, z, centre, side, blobs, lv_axes=None, lv_centre=None):
    """Echo-like intensity scene (float): dark chamber (~20) inside a bright
    myocardium (~180) on tissue (~80), an offset atrium, and seeded tissue blobs
    that break the ellipsoid's rotational symmetry.  Sigmoid edges."""
    if lv_axes is None:
        lv_axes = np.array([0.21, 0.21, 0.30]) * side   # long axis along the beam (z)
    if lv_centre is None:
        lv_centre = np.asarray(centre, float)
    wall = 0.045 * side
    r_in = np.sqrt(_ellipsoid_r2(x, y, z, lv_centre, lv_axes))
    r_out = np.sqrt(_ellipsoid_r2(x, y, z, lv_centre, np.asarray(lv_axes) + wall))
    m_out = _sigmoid((1.0 - r_out) * float(np.mean(lv_axes) + wall) / 1.5)
    m_in = _sigmoid((1.0 - r_in) * float(np.mean(lv_axes)) / 1.5)
    img = 80.0 * (1.0 - m_out) + 180.0 * (m_out - m_in) + 20.0 * m_in
    # atrium: a smaller dark chamber beyond the base, off-axis
    a_c = np.asarray(centre, float) + np.array([0.10, 0.05, 0.36]) * side
    a_ax = np.array([0.13, 0.11, 0.10]) * side
    m_a = _sigmoid((1.0 - np.sqrt(_ellipsoid_r2(x, y, z, a_c, a_ax))) * float(np.mean(a_ax)) / 1.5)
    img = img * (1.0 - m_a) + 30.0 * m_a
    for (bx, by, bz, br, amp) in blobs:
        img = img + amp * np.exp(-(((x - bx) ** 2 + (y - by) ** 2 + (z - bz) ** 2) / (2.0 * br * br)))
    return img


def _blobs(rng, centre, side, n=14):
    out = []
    for _ in range(n):
        pos = np.asarray(centre) + rng.uniform(-0.45, 0.45, 3) * side
        out.append((pos[0], pos[1], pos[2], rng.uniform(0.04, 0.10) * side, rng.uniform(-45, 45)))
    return out


def _to_u8(v):
    return np.clip(np.floor(v + 0.5), 0, 255).astype(np.uint8)


def _cone(shape_xyz, half_angle_deg=30.0, apex_offset=0.30):
    """Apical cone field of view: apex above the z = 0 face, axis +z."""
    nx, ny, nz = shape_xyz
    x, y, z = _centres(shape_xyz)
    ax, ay, az = 0.5 * (nx - 1), 0.5 * (ny - 1), -apex_offset * nz
    r = np.sqrt((x - ax) ** 2 + (y - ay) ** 2)
    return ((z - az) > 0) & (r <= np.tan(np.deg2rad(half_angle_deg)) * (z - az))


def speckle_pair(side=160, rot_deg=20.0, trans=12.0, seed=2, cone=True, speckle_sigma=0.6,
                 blur=1.0, gt=None) -> dict:
    """Speckled intensity pair: anatomy x Rayleigh(speckle_sigma) speckle,
    Gaussian blur (sigma 1 voxel), uint8.  The source is the same scene through
    the inverse ground-truth map (trilinear spline resampling of the speckle
    field by scipy), cropped to a 60 deg apical cone whose mask is returned as
    ``src_fov``."""
    rng = np.random.default_rng(seed)
    if gt is None:
        gt = _sample_gt(rng, rot_deg, trans)
    gt = np.asarray(gt, float)
    shape = (side, side, side)
    c = 0.5 * (np.asarray(shape, float) - 1.0)
    m = max(8, side // 4)
    wshape = (side + 2 * m,) * 3
    wx, wy, wz = _centres(wshape)
    blobs = _blobs(rng, c, side)
    scene = _anatomy(wx - m, wy - m, wz - m, c, side, blobs).astype(np.float32)
    del wx, wy, wz
    scene *= rng.rayleigh(speckle_sigma, size=scene.shape).astype(np.float32)
    scene = ndimage.gaussian_filter(scene, blur, truncate=3.0, mode="nearest")
    tgt = _to_u8(scene[m:m + side, m:m + side, m:m + side])
    px, py, pz = _preimage(gt, shape, shape)
    coords = np.stack([pz + m, py + m, px + m], axis=0)
    del px, py, pz
    src_f = ndimage.map_coordinates(scene, coords, order=1, mode="nearest")
    src = _to_u8(src_f)
    out = dict(kind="image", src=src, tgt=tgt, gt=gt, spacing=(1.0, 1.0, 1.0), shape_xyz=shape)
    if cone:
        fov = _cone(shape).astype(np.uint8)
        src[fov == 0] = 0
        out["src"] = src
        out["src_fov"] = fov
        # fraction of target voxels whose true source position is in the cone
        M = gt_matrix(gt, shape)
        x, y, z = _centres(shape)
        q = np.stack([x, y, z], 0).reshape(3, -1)
        q = M[:3, :3] @ q + M[:3, 3:4]
        qi = np.floor(q + 0.5).astype(np.int64)
        ok = np.all((qi >= 0) & (qi < side), axis=0)
        hit = np.zeros(ok.shape, bool)
        hit[ok] = fov[qi[2, ok], qi[1, ok], qi[0, ok]] != 0
        out["overlap"] = float(hit.mean())
    return out


# ----------------------------------------------------------------------------- sequences

def lv_sequence(shape_xyz=(224, 208, 176), n_frames=20, seed=3, rot_deg=15.0, trans=16.0,
                speckle=True, frames=None, gt=None) -> dict:
    """Contracting LV sequence: a filled ellipsoid (semi-axes ~80/45/40 with
    +-10 % seeded jitter) scaled about a fixed apex so that
    V(f)/V_ED = 1 - 0.55 (1 - cos(2 pi f / F)) / 2 (ED at f = 0, ES at F / 2,
    ratio 0.45).  Returns target/source masks per frame and, with ``speckle``,
    a speckled intensity volume per source frame."""
    rng = np.random.default_rng(seed)
    if gt is None:
        gt = _sample_gt(rng, rot_deg, trans)
    gt = np.asarray(gt, float)
    axes_ed = np.array([80.0, 45.0, 40.0]) * (1.0 + rng.uniform(-0.1, 0.1, 3))
    c = 0.5 * (np.asarray(shape_xyz, float) - 1.0)
    apex = c - np.array([axes_ed[0], 0.0, 0.0])
    frames = range(n_frames) if frames is None else frames
    blobs = _blobs(rng, c, float(min(shape_xyz)))
    x, y, z = _centres(shape_xyz)
    px, py, pz = _preimage(gt, shape_xyz, shape_xyz)
    spk_t = rng.rayleigh(0.6, size=x.shape).astype(np.float32) if speckle else None
    spk_s = None
    if speckle:
        coords = np.stack([pz, py, px], axis=0)
        spk_s = ndimage.map_coordinates(spk_t, coords, order=1, mode="nearest")
        del coords
    tm, sm, ts, ss, ratios = [], [], [], [], []
    for f in frames:
        ratio = 1.0 - 0.55 * (1.0 - np.cos(2.0 * np.pi * f / n_frames)) / 2.0
        s = ratio ** (1.0 / 3.0)
        ax = axes_ed * s
        cen = apex + np.array([ax[0], 0.0, 0.0])
        tm.append(_shell(x, y, z, cen, ax, None).astype(np.uint8))
        sm.append(_shell(px, py, pz, cen, ax, None).astype(np.uint8))
        ratios.append(ratio)
        if speckle:
            side = float(min(shape_xyz))
            a_t = _anatomy(x, y, z, c, side, blobs, lv_axes=ax, lv_centre=cen).astype(np.float32)
            ts.append(_to_u8(ndimage.gaussian_filter(a_t * spk_t, 1.0, truncate=3.0, mode="nearest")))
            a_s = _anatomy(px, py, pz, c, side, blobs, lv_axes=ax, lv_centre=cen).astype(np.float32)
            ss.append(_to_u8(ndimage.gaussian_filter(a_s * spk_s, 1.0, truncate=3.0, mode="nearest")))
    out = dict(kind="mask", gt=gt, spacing=(1.0, 1.0, 1.0), shape_xyz=tuple(shape_xyz),
               tgt_masks=np.stack(tm), src_masks=np.stack(sm), volume_ratio=np.array(ratios),
               src=sm[0], tgt=tm[0])
    if speckle:
        out["tgt_speckle"] = np.stack(ts)
        out["src_speckle"] = np.stack(ss)
    return out


# ----------------------------------------------------------------------------- batches

def batch_pairs(n_pairs=64, seed=4, side_range=(96, 224), n_choices=(1024, 2048, 4096, 8192)):
    """Descriptors of the batched workload: cubic sides U{96..224}, particles
    from ``n_choices``, half mask pairs (scaled shells) and half speckle image
    pairs.  Volumes are produced lazily by ``make``."""
    rng = np.random.default_rng(seed)
    specs = []
    for p in range(n_pairs):
        side = int(rng.integers(side_range[0], side_range[1] + 1))
        n = int(rng.choice(n_choices))
        kind = "mask" if p % 2 == 0 else "image"
        specs.append(dict(pair=p, side=side, n_particles=n, kind=kind, seed=int(rng.integers(1 << 30))))
    return specs


def make_batch_pair(spec) -> dict:
    if spec["kind"] == "mask":
        return shell_pair(seed=spec["seed"], side=spec["side"])
    return speckle_pair(side=spec["side"], seed=spec["seed"])


def proposal_pair(seed, side=64, rot_deg=15.0, trans=8.0) -> dict:
    """Small LV mask pair for proposal-network training: a filled ellipsoid
    with seeded semi-axes (asymmetric, so every rotation is observable) and
    a seeded rigid ground truth."""
    rng = np.random.default_rng(seed)
    f = side / 64.0
    axes = np.array([22.0, 15.0, 11.0]) * f * (1.0 + rng.uniform(-0.1, 0.1, 3))
    gt = _sample_gt(rng, rot_deg, trans * f)
    return mask_pair((side, side, side), outer=tuple(axes), inner=None, gt=gt)


# ----------------------------------------------------------------------------- proposal training

LV_SHAPE = (224, 208, 176)


def lv_train_pair(seed, shape_xyz=LV_SHAPE, side=64, rot_deg=15.0, trans=16.0, supersample=2) -> dict:
    """A contracting-LV ED pair seen at the proposal network's sampling grid:
    side^3 cells over the full shape_xyz volume (cell size s = n / side per
    axis, centres at full-volume voxel coordinates (a + 0.5) s - 0.5), each
    cell's value the fraction of supersample^3 sub-points inside the analytic
    LV (as uint8 0..255), plus the binary masks (fraction >= 0.5) that the
    filter registers with spacing s.  Same LV model and transform ranges as
    lv_sequence at frame 0."""
    rng = np.random.default_rng(seed)
    gt = _sample_gt(rng, rot_deg, trans)
    axes_ed = np.array([80.0, 45.0, 40.0]) * (1.0 + rng.uniform(-0.1, 0.1, 3))
    n = np.asarray(shape_xyz, float)
    c = 0.5 * (n - 1.0)
    s = n / side
    M = gt_matrix(gt, shape_xyz)
    R, off = M[:3, :3], M[:3, 3]
    sub = (np.arange(supersample) + 0.5) / supersample - 0.5
    frac_t = np.zeros((side, side, side))
    frac_s = np.zeros((side, side, side))
    base = [(np.arange(side) + 0.5) * s[d] - 0.5 for d in range(3)]
    for oz in sub:
        for oy in sub:
            for ox in sub:
                z, y, x = np.meshgrid(base[2] + oz * s[2], base[1] + oy * s[1], base[0] + ox * s[0], indexing="ij")
                frac_t += _ellipsoid_r2(x, y, z, c, axes_ed) <= 1.0
                d = np.stack([x - off[0], y - off[1], z - off[2]], 0).reshape(3, -1)
                p = (R.T @ d).reshape(3, *x.shape)
                frac_s += _ellipsoid_r2(p[0], p[1], p[2], c, axes_ed) <= 1.0
    k = float(supersample ** 3)
    tgt = np.floor(frac_t / k * 255.0 + 0.5).astype(np.uint8)
    src = np.floor(frac_s / k * 255.0 + 0.5).astype(np.uint8)
    return dict(src=src, tgt=tgt, src_mask=(src >= 128).astype(np.uint8), tgt_mask=(tgt >= 128).astype(np.uint8),
                gt=gt, spacing=tuple(float(v) for v in s))
