"""CPU oracle for the particle-filter rigid registration (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The product path (``paper_2504_19930_amd``)
never does.  The arithmetic lives in ``smc_oracle.c`` (plain C, FP64, with the
FP32 coordinate recipe where the recipe fixes it); this module only builds the
library with gcc and marshals numpy arrays.

Every function names the passage it follows in ``smc_oracle.c``'s header.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

SCORES = {"dice": 0, "ncc": 1, "ssd": 2, "mi": 3}
# the resampling CDF sums floor(w 2^48) per particle in 64 bits (smc_oracle.c)
MAX_PARTICLES = 65535


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` in-tree with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Vol(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("sx", C.c_double), ("sy", C.c_double), ("sz", C.c_double),
                ("data", C.c_void_p), ("fov", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("n_particles", C.c_uint32), ("n_iters", C.c_uint32), ("seed", C.c_uint64),
                ("pair_id", C.c_uint32), ("score", C.c_int32), ("trilinear", C.c_int32),
                ("fp64_mode", C.c_int32), ("x0", C.c_double * 6), ("limit", C.c_double * 6),
                ("sigma_score", C.c_double), ("sigma0", C.c_double * 6), ("anneal", C.c_double),
                ("min_overlap_frac", C.c_double), ("has_proposal", C.c_int32), ("prop_mu", C.c_double * 6),
                ("prop_sigma", C.c_double * 6), ("wide_rotation", C.c_int32)]


class _Problem(C.Structure):
    _fields_ = [("src", _Vol), ("tgt", _Vol), ("t_on", C.c_uint64), ("t_fov", C.c_uint64),
                ("mu_s", C.c_double), ("sd_s", C.c_double), ("mu_t", C.c_double), ("sd_t", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        d, u8, i32, u64, i64, f32 = (np.ctypeslib.ndpointer(t, flags="C") for t in
                                     (np.float64, np.uint8, np.int32, np.uint64, np.int64, np.float32))
        u32 = np.ctypeslib.ndpointer(np.uint32, flags="C")
        P = C.POINTER
        sig = {
            "or_philox4x32_10": (None, [u32, u32, u32]),
            "or_u53": (C.c_double, [C.c_uint32, C.c_uint32]),
            "or_euler_R": (None, [d, d]),
            "or_phys_matrix": (None, [d, i32, d, d]),
            "or_recipe_words_from_matrix": (None, [d, d, d, C.c_int, f32]),
            "or_recipe_words": (None, [d, P(_Vol), P(_Vol), C.c_int, f32]),
            "or_mask_counts": (None, [P(_Vol), P(_Vol), f32, u64]),
            "or_image_moments": (None, [P(_Vol), P(_Vol), f32, C.c_int, i64]),
            "or_mask_counts_fp64": (None, [P(_Vol), P(_Vol), d, u64]),
            "or_image_moments_fp64": (None, [P(_Vol), P(_Vol), d, C.c_int, d]),
            "or_dice": (C.c_double, [C.c_uint64, C.c_uint64, C.c_uint64]),
            "or_ncc_from_moments": (C.c_double, [d]),
            "or_msd_from_moments": (C.c_double, [d, C.c_double, C.c_double, C.c_double, C.c_double]),
            "or_moments_to_double": (None, [i64, d]),
            "or_problem_init": (None, [P(_Problem), P(_Vol), P(_Vol)]),
            "or_score_particle": (C.c_double, [P(_Problem), P(_Params), d]),
            "or_score_particles": (None, [P(_Problem), P(_Params), C.c_uint32, d, d]),
            "or_loglik": (C.c_double, [C.c_double, C.c_int, C.c_double]),
            "or_normalise": (C.c_int, [C.c_uint32, d, d, d, d, P(C.c_double)]),
            "or_normalise_wide": (C.c_int, [C.c_uint32, d, d, d, d, d, P(C.c_double)]),
            "or_cloud_moments": (None, [C.c_uint32, d, d, d, d, C.c_double, d, d]),
            "or_proposal_from_network": (None, [f32, d, d, C.c_double, d, d]),
            "or_euler_quat": (None, [d, d]),
            "or_quat_R": (None, [d, d]),
            "or_R_euler": (None, [d, d]),
            "or_resample": (C.c_int, [C.c_uint32, d, C.c_uint32, i32]),
            "or_gauss6": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, d]),
            "or_perturb": (None, [P(_Params), C.c_uint32, d, i32, d]),
            "or_init_particles": (None, [P(_Params), d]),
            "or_resample_word": (C.c_uint32, [P(_Params), C.c_uint32]),
            "or_filter_update": (C.c_int, [P(_Params), C.c_uint32, d, d, C.c_void_p, d, d, d, P(C.c_double), i32,
                                           d]),
            "or_init_proposal": (None, [P(_Params), d, d]),
            "or_smc_run": (C.c_int, [P(_Vol), P(_Vol), P(_Params), d, d, d, d, d, d, i32]),
            "or_smc_run_frames": (C.c_int, [P(_Vol), P(_Vol), C.c_uint32, P(_Params), d, d, d, d, d, d, i32]),
            "or_frame_sums": (None, [P(_Problem), C.c_uint32, P(_Params), d, i64]),
            "or_score_particle_frames": (C.c_double, [P(_Problem), C.c_uint32, P(_Params), d]),
            "or_warp_apply": (None, [P(_Vol), d, C.c_int, u8, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_double, C.c_double, C.c_double]),
            "or_num_threads": (C.c_int, []),
            "or_set_threads": (None, [C.c_int]),
            "or_joint_histogram": (None, [P(_Vol), P(_Vol), f32, u64]),
            "or_mi_score": (C.c_double, [u64]),
            "or_mi_log": (C.c_double, [C.c_double]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


# ---------------------------------------------------------------- marshalling

class Volume:
    """A uint8 ``(nz, ny, nx)`` volume with spacing and an optional FOV mask."""

    def __init__(self, data, spacing=(1.0, 1.0, 1.0), fov=None):
        self.data = np.ascontiguousarray(data, dtype=np.uint8)
        assert self.data.ndim == 3
        self.fov = None if fov is None else np.ascontiguousarray(fov, dtype=np.uint8)
        if self.fov is not None:
            assert self.fov.shape == self.data.shape
        self.spacing = tuple(float(s) for s in spacing)

    @property
    def shape_xyz(self):
        nz, ny, nx = self.data.shape
        return (nx, ny, nz)

    def c(self) -> _Vol:
        nz, ny, nx = self.data.shape
        return _Vol(nx, ny, nz, *self.spacing, self.data.ctypes.data,
                    None if self.fov is None else self.fov.ctypes.data)


def _vol(v) -> Volume:
    return v if isinstance(v, Volume) else Volume(v)


def make_params(p: dict, fp64_mode: bool = False) -> _Params:
    score = SCORES[p.get("score", "dice")]
    tri = 1 if p.get("interp", "nearest" if score == 0 else "trilinear") == "trilinear" else 0
    out = _Params()
    out.n_particles = int(p["n_particles"])
    out.n_iters = int(p["n_iters"])
    out.seed = int(p.get("seed", 0))
    out.pair_id = int(p.get("pair_id", 0))
    out.score = score
    out.trilinear = tri
    out.fp64_mode = 1 if fp64_mode else 0
    out.x0[:] = [float(v) for v in p.get("x0", [0.0] * 6)]
    out.limit[:] = [float(v) for v in p["limit"]]
    out.sigma_score = float(p["sigma_score"])
    out.sigma0[:] = [float(v) for v in p["sigma0"]]
    out.anneal = float(p.get("anneal", 0.9))
    out.min_overlap_frac = float(p.get("min_overlap_frac", 0.05))
    out.wide_rotation = 1 if p.get("rotation_mode", "box") == "wide" else 0
    prop = p.get("proposal")
    if prop is not None:
        out.has_proposal = 1
        out.prop_mu[:] = [float(v) for v in prop["mean"]]
        # sigma = exp(logvar / 2), computed the same way on every side
        import math
        out.prop_sigma[:] = [math.exp(0.5 * float(v)) for v in prop["logvar"]]
    return out


# ---------------------------------------------------------------- primitives

def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def u53(a: int, b: int) -> float:
    return lib().or_u53(int(a), int(b))


def euler_R(p) -> np.ndarray:
    q = np.zeros(6)
    q[:3] = np.asarray(p, float)[:3]
    R = np.zeros(9)
    lib().or_euler_R(q, R)
    return R.reshape(3, 3)


def phys_matrix(p, tgt_shape_xyz, tgt_spacing=(1.0, 1.0, 1.0)) -> np.ndarray:
    M = np.zeros(12)
    lib().or_phys_matrix(np.asarray(p, float), np.asarray(tgt_shape_xyz, np.int32),
                         np.asarray(tgt_spacing, float), M)
    return M.reshape(3, 4)


def recipe_words_from_matrix(M, tgt_spacing, src_spacing, nn: bool) -> np.ndarray:
    w = np.zeros(12, np.float32)
    lib().or_recipe_words_from_matrix(np.ascontiguousarray(M, float).reshape(12),
                                      np.asarray(tgt_spacing, float), np.asarray(src_spacing, float),
                                      1 if nn else 0, w)
    return w


def recipe_words(p, src, tgt, nn: bool) -> np.ndarray:
    s, t = _vol(src), _vol(tgt)
    w = np.zeros(12, np.float32)
    lib().or_recipe_words(np.asarray(p, float), C.byref(s.c()), C.byref(t.c()), 1 if nn else 0, w)
    return w


def mask_counts(src, tgt, words) -> np.ndarray:
    s, t = _vol(src), _vol(tgt)
    out = np.zeros(4, np.uint64)
    lib().or_mask_counts(C.byref(s.c()), C.byref(t.c()), np.asarray(words, np.float32), out)
    return out


def mask_counts_fp64(src, tgt, p) -> np.ndarray:
    s, t = _vol(src), _vol(tgt)
    out = np.zeros(4, np.uint64)
    lib().or_mask_counts_fp64(C.byref(s.c()), C.byref(t.c()), np.asarray(p, float), out)
    return out


def image_moments(src, tgt, words, trilinear=True) -> np.ndarray:
    s, t = _vol(src), _vol(tgt)
    out = np.zeros(6, np.int64)
    lib().or_image_moments(C.byref(s.c()), C.byref(t.c()), np.asarray(words, np.float32),
                           1 if trilinear else 0, out)
    return out


def image_moments_fp64(src, tgt, p, trilinear=True) -> np.ndarray:
    s, t = _vol(src), _vol(tgt)
    out = np.zeros(6)
    lib().or_image_moments_fp64(C.byref(s.c()), C.byref(t.c()), np.asarray(p, float),
                                1 if trilinear else 0, out)
    return out


def joint_histogram(src, tgt, words) -> np.ndarray:
    """32 x 32 joint histogram (source bin, target bin) of the trilinear MI score."""
    s, t = _vol(src), _vol(tgt)
    sv, tv = s.c(), t.c()
    h = np.zeros(32 * 32, np.uint64)
    lib().or_joint_histogram(C.byref(sv), C.byref(tv), np.ascontiguousarray(words, np.float32), h)
    return h.reshape(32, 32)


def mi_log(x: float) -> float:
    return lib().or_mi_log(float(x))


def mi_score(hist) -> float:
    return lib().or_mi_score(np.ascontiguousarray(hist, np.uint64).reshape(-1))


def dice(a, c, b) -> float:
    return lib().or_dice(int(a), int(c), int(b))


def moments_to_double(mi) -> np.ndarray:
    out = np.zeros(6)
    lib().or_moments_to_double(np.asarray(mi, np.int64), out)
    return out


def ncc(m) -> float:
    return lib().or_ncc_from_moments(np.asarray(m, float))


def msd(m, mu_s, sd_s, mu_t, sd_t) -> float:
    return lib().or_msd_from_moments(np.asarray(m, float), mu_s, sd_s, mu_t, sd_t)


def loglik(z, score, sigma) -> float:
    return lib().or_loglik(float(z), SCORES[score], float(sigma))


def normalise(lw, x):
    lw = np.ascontiguousarray(lw, float)
    x = np.ascontiguousarray(x, float).reshape(-1, 6)
    w = np.zeros(len(lw))
    est = np.zeros(6)
    ess = C.c_double()
    deg = lib().or_normalise(len(lw), lw, x, w, est, C.byref(ess))
    return dict(w=w, est=est, ess=ess.value, degenerate=bool(deg))


def normalise_wide(lw, x, x0):
    """Normalisation with the quaternion-mean rotation of the wide mode."""
    lw = np.ascontiguousarray(lw, float)
    x = np.ascontiguousarray(x, float).reshape(-1, 6)
    w = np.zeros(len(lw))
    est = np.zeros(6)
    ess = C.c_double()
    deg = lib().or_normalise_wide(len(lw), lw, x, np.ascontiguousarray(x0, float), w, est, C.byref(ess))
    return dict(w=w, est=est, ess=ess.value, degenerate=bool(deg))


def cloud_moments(lw, x, x0, limit, var_floor=0.0):
    """Weighted mean and per-axis variance of a particle cloud in units of
    the limits about x0 (the learned proposal's training label)."""
    lw = np.ascontiguousarray(lw, float)
    x = np.ascontiguousarray(x, float).reshape(-1, 6)
    mean, var = np.zeros(6), np.zeros(6)
    lib().or_cloud_moments(len(lw), lw, x, np.ascontiguousarray(x0, float), np.ascontiguousarray(limit, float),
                           float(var_floor), mean, var)
    return mean, var


def proposal_from_network(out, x0, limit, var_scale):
    """(mean, logvar) of the proposal the network's 12 outputs stand for."""
    mean, logvar = np.zeros(6), np.zeros(6)
    lib().or_proposal_from_network(np.ascontiguousarray(out, np.float32).reshape(12),
                                   np.ascontiguousarray(x0, float), np.ascontiguousarray(limit, float),
                                   float(var_scale), mean, logvar)
    return mean, logvar


def euler_quat(p) -> np.ndarray:
    q = np.zeros(4)
    lib().or_euler_quat(np.ascontiguousarray(np.resize(np.asarray(p, float), 6)), q)
    return q


def quat_R(q) -> np.ndarray:
    R = np.zeros(9)
    lib().or_quat_R(np.ascontiguousarray(q, float), R)
    return R.reshape(3, 3)


def R_euler(R) -> np.ndarray:
    e = np.zeros(3)
    lib().or_R_euler(np.ascontiguousarray(R, float).reshape(9), e)
    return e


def resample(w, u32) -> np.ndarray:
    w = np.ascontiguousarray(w, float)
    anc = np.zeros(len(w), np.int32)
    if lib().or_resample(len(w), w, int(u32), anc) != 0:
        raise ValueError(f"{len(w)} particles: resampling takes 1 .. {MAX_PARTICLES}")
    return anc


def gauss6(seed, pair, j, k) -> np.ndarray:
    g = np.zeros(6)
    lib().or_gauss6(int(seed), int(pair), int(j), int(k), g)
    return g


def init_particles(params: dict) -> np.ndarray:
    pr = make_params(params)
    x = np.zeros((pr.n_particles, 6))
    lib().or_init_particles(C.byref(pr), x)
    return x


def init_proposal(params: dict):
    pr = make_params(params)
    x = np.zeros((pr.n_particles, 6))
    lq = np.zeros(pr.n_particles)
    lib().or_init_proposal(C.byref(pr), x, lq)
    return x, lq


def resample_word(params: dict, k: int) -> int:
    return lib().or_resample_word(C.byref(make_params(params)), int(k))


def perturb(params: dict, k: int, x_old, anc) -> np.ndarray:
    pr = make_params(params)
    xo = np.ascontiguousarray(x_old, float).reshape(-1, 6)
    xn = np.zeros_like(xo)
    lib().or_perturb(C.byref(pr), int(k), xo, np.ascontiguousarray(anc, np.int32), xn)
    return xn


class Problem:
    """Source / target pair with the per-volume statistics the scores need."""

    def __init__(self, src, tgt):
        self.src, self.tgt = _vol(src), _vol(tgt)
        self._c = _Problem()
        self._sv, self._tv = self.src.c(), self.tgt.c()
        lib().or_problem_init(C.byref(self._c), C.byref(self._sv), C.byref(self._tv))

    @property
    def stats(self):
        c = self._c
        return dict(t_on=c.t_on, t_fov=c.t_fov, mu_s=c.mu_s, sd_s=c.sd_s, mu_t=c.mu_t, sd_t=c.sd_t)

    def score(self, params: dict, states, fp64_mode=False) -> np.ndarray:
        x = np.ascontiguousarray(states, float).reshape(-1, 6)
        z = np.zeros(len(x))
        pr = make_params(dict(params, n_particles=max(1, len(x))), fp64_mode)
        lib().or_score_particles(C.byref(self._c), C.byref(pr), len(x), x, z)
        return z


def filter_update(params: dict, k: int, x, z) -> dict:
    pr = make_params(params)
    n = pr.n_particles
    x = np.ascontiguousarray(x, float).reshape(n, 6)
    z = np.ascontiguousarray(z, float)
    lw, w, est = np.zeros(n), np.zeros(n), np.zeros(6)
    anc = np.full(n, -1, np.int32)
    xn = np.zeros_like(x)
    ess = C.c_double()
    deg = lib().or_filter_update(C.byref(pr), int(k), x, z, None, lw, w, est, C.byref(ess), anc, xn)
    if deg < 0:
        raise ValueError(f"{n} particles: the filter takes 1 .. {MAX_PARTICLES}")
    return dict(lw=lw, w=w, est=est, ess=ess.value, anc=anc, x_next=xn, degenerate=bool(deg))


def smc_run(src, tgt, params: dict, fp64_mode=False, frames=None) -> dict:
    """Whole registration; ``frames`` optionally lists further (src, tgt)
    frame pairs scored together with the first (multi-frame score)."""
    pairs = [(_vol(src), _vol(tgt))] + [(_vol(a), _vol(b)) for a, b in (frames or [])]
    pr = make_params(params, fp64_mode)
    n, K = pr.n_particles, pr.n_iters
    est = np.zeros(6)
    ts, te, tx = np.zeros(K + 1), np.zeros(K), np.zeros((K, 6))
    x, lw = np.zeros((n, 6)), np.zeros(n)
    anc = np.zeros(n, np.int32)
    svs = (_Vol * len(pairs))(*[a.c() for a, _ in pairs])
    tvs = (_Vol * len(pairs))(*[b.c() for _, b in pairs])
    deg = lib().or_smc_run_frames(svs, tvs, len(pairs), C.byref(pr), est, ts, te, tx, x, lw, anc)
    if deg < 0:
        raise ValueError(f"{n} particles: the filter takes 1 .. {MAX_PARTICLES}")
    return dict(est=est, trace_score=ts, trace_ess=te, trace_est=tx, states=x, logw=lw, ancestors=anc,
                degenerate=bool(deg))


class Frames:
    """Several (src, tgt) frame pairs scored together under one transform."""

    def __init__(self, pairs):
        self.vols = [(_vol(a), _vol(b)) for a, b in pairs]
        self.pbs = (_Problem * len(self.vols))()
        self._keep = []
        for f, (a, b) in enumerate(self.vols):
            av, bv = a.c(), b.c()
            self._keep += [av, bv]
            lib().or_problem_init(C.byref(self.pbs[f]), C.byref(av), C.byref(bv))

    def sums(self, params: dict, x) -> np.ndarray:
        pr = make_params(params)
        x = np.ascontiguousarray(x, float).reshape(-1, 6)
        out = np.zeros((len(x), 6), np.int64)
        for i in range(len(x)):
            lib().or_frame_sums(self.pbs, len(self.vols), C.byref(pr), x[i], out[i])
        return out

    def score(self, params: dict, x) -> np.ndarray:
        pr = make_params(params)
        x = np.ascontiguousarray(x, float).reshape(-1, 6)
        return np.array([lib().or_score_particle_frames(self.pbs, len(self.vols), C.byref(pr), x[i])
                         for i in range(len(x))])


def warp_apply(src, M, trilinear, out_shape_xyz, out_spacing=(1.0, 1.0, 1.0)) -> np.ndarray:
    s = _vol(src)
    nx, ny, nz = out_shape_xyz
    dst = np.zeros((nz, ny, nx), np.uint8)
    sv = s.c()
    lib().or_warp_apply(C.byref(sv), np.ascontiguousarray(M, float).reshape(12), 1 if trilinear else 0, dst,
                        nx, ny, nz, *[float(v) for v in out_spacing])
    return dst


def num_threads() -> int:
    return lib().or_num_threads()


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (n < 1: all)."""
    lib().or_set_threads(int(n))
