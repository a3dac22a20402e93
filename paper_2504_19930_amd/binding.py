"""ctypes binding of ``libsmc.so`` (declared in ``include/smc.h``).

Argument marshalling only: every step of the registration runs in the HIP
library.  PyTorch supplies device memory (uint8 tensors on a ROCm device) and
the current stream.  The functions keep the C names (``smc_init``,
``smc_step``, ``smc_estimate``, ``warp_apply`` ...); ``Registration`` wraps a
context for convenience.  Importing works without a GPU, but every call that
needs the library raises if it has not been built.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsmc.so")

SMC_OK, SMC_EINVAL, SMC_ENOMEM, SMC_EDEVICE, SMC_ESTATE, SMC_ENOOVERLAP = 0, -1, -2, -3, -4, -5
SCORES = {"dice": 0, "ncc": 1, "ssd": 2, "mi": 3}
INTERPS = {"nearest": 0, "trilinear": 1}
ROTATIONS = {"box": 0, "wide": 1}

# every symbol include/smc.h declares
EXPORTS = ("smc_init", "smc_reset", "smc_step", "smc_estimate", "smc_get_particles", "smc_trace",
           "smc_evaluate", "smc_set_particles", "smc_get_state", "smc_set_state", "smc_destroy",
           "warp_apply", "smc_last_error", "smc_version", "smc_profile", "smc_profile_read", "smc_profile_work",
           "smc_set_tuning", "smc_get_tuning", "smc_batch_init", "smc_batch_set_seeds", "smc_batch_run",
           "smc_batch_pair", "smc_batch_destroy", "smc_cnn_create", "smc_cnn_set_params", "smc_cnn_get_params",
           "smc_cnn_input", "smc_cnn_read_input", "smc_cnn_forward", "smc_cnn_backward", "smc_cnn_step", "smc_cnn_destroy",
           "smc_set_proposal", "smc_exhaustive", "smc_autotune", "smc_batch_autotune", "smc_set_frames",
           "smc_score_particles", "smc_cloud_moments", "smc_set_proposal_from_network",
           "smc_evaluate_noalloc", "smc_gather_probe")


class SmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"smc status {status}: {msg}")
        self.status = status


class SmcVolume(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("sx", C.c_double), ("sy", C.c_double), ("sz", C.c_double),
                ("data", C.c_void_p), ("fov", C.c_void_p)]


class SmcParams(C.Structure):
    _fields_ = [("n_particles", C.c_uint32), ("n_iters", C.c_uint32), ("seed", C.c_uint64),
                ("pair_id", C.c_uint32), ("score", C.c_int32), ("interp", C.c_int32),
                ("x0", C.c_double * 6), ("limit", C.c_double * 6), ("sigma_score", C.c_double),
                ("sigma0", C.c_double * 6), ("anneal", C.c_double), ("min_overlap_frac", C.c_double),
                ("rotation_mode", C.c_int32)]


_lib = None


def lib():
    """Load ``libsmc.so``; raise if it has not been built (no silent fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2504_19930_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, u32, u64, i32, i64, dp = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_int64, C.c_double
        P = C.POINTER
        sig = {
            "smc_init": [P(vp), P(SmcVolume), P(SmcVolume), P(SmcParams), vp],
            "smc_reset": [vp, u64],
            "smc_step": [vp, u32],
            "smc_estimate": [vp, vp, vp, vp, vp],
            "smc_get_particles": [vp, vp, vp, vp],
            "smc_trace": [vp, vp, vp, vp],
            "smc_evaluate": [vp, vp, u32, vp],
            "smc_evaluate_noalloc": [vp, vp, u32, vp],
            "smc_gather_probe": [vp, u32, vp, vp],
            "smc_set_particles": [vp, vp, u32],
            "smc_get_state": [vp, vp, P(C.c_size_t)],
            "smc_set_state": [vp, vp, C.c_size_t],
            "warp_apply": [P(SmcVolume), vp, i32, vp, i32, i32, i32, dp, dp, dp, u32, i64, i64, vp],
            "smc_profile": [vp, i32],
            "smc_profile_read": [vp, vp, vp, vp, vp],
            "smc_profile_work": [vp, vp, vp, vp],
            "smc_set_tuning": [vp, i32, i32, i32],
            "smc_set_frames": [vp, u32, vp, vp],
            "smc_score_particles": [vp, vp, u32, vp],
            "smc_get_tuning": [vp, vp, vp, vp],
            "smc_batch_init": [P(vp), u32, vp, vp, vp, vp],
            "smc_batch_set_seeds": [vp, vp],
            "smc_batch_run": [vp],
            "smc_cnn_create": [P(vp), u32, vp],
            "smc_cnn_set_params": [vp, vp, C.c_size_t],
            "smc_cnn_get_params": [vp, vp, C.c_size_t],
            "smc_cnn_input": [vp, u32, P(SmcVolume), P(SmcVolume), C.c_float],
            "smc_cnn_forward": [vp, u32, vp],
            "smc_cnn_read_input": [vp, u32, vp],
            "smc_cnn_backward": [vp, u32, vp, vp, vp],
            "smc_cnn_step": [vp, C.c_float],
            "smc_set_proposal": [vp, vp, vp],
            "smc_cloud_moments": [vp, dp, vp, vp],
            "smc_set_proposal_from_network": [vp, vp, dp, vp, vp],
            "smc_exhaustive": [vp, vp, vp, vp, vp, vp, vp],
            "smc_autotune": [vp, u32, vp],
            "smc_batch_autotune": [vp, u32],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.smc_destroy.argtypes = [vp]
        L.smc_destroy.restype = None
        L.smc_batch_pair.argtypes = [vp, u32]
        L.smc_batch_pair.restype = vp
        L.smc_batch_destroy.argtypes = [vp]
        L.smc_batch_destroy.restype = None
        L.smc_cnn_destroy.argtypes = [vp]
        L.smc_cnn_destroy.restype = None
        L.smc_last_error.restype = C.c_char_p
        L.smc_version.restype = C.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != SMC_OK:
        raise SmcError(status, lib().smc_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def volume(data, spacing=(1.0, 1.0, 1.0), fov=None) -> SmcVolume:
    """Describe a device uint8 tensor of shape (nz, ny, nx) (C-contiguous)."""
    import torch
    for t in (data,) if fov is None else (data, fov):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.uint8 and t.dim() == 3
                and t.is_contiguous()):
            raise ValueError("volumes must be contiguous 3-D uint8 tensors on the GPU")
    if fov is not None and fov.shape != data.shape:
        raise ValueError("fov must have the volume's shape")
    nz, ny, nx = data.shape
    return SmcVolume(nx, ny, nz, *(float(s) for s in spacing), data.data_ptr(),
                     None if fov is None else fov.data_ptr())


def params(p: dict) -> SmcParams:
    """Build smc_params from a dict (score / interp given by name)."""
    out = SmcParams()
    score = SCORES[p.get("score", "dice")]
    out.n_particles = int(p["n_particles"])
    out.n_iters = int(p["n_iters"])
    out.seed = int(p.get("seed", 0))
    out.pair_id = int(p.get("pair_id", 0))
    out.score = score
    out.interp = INTERPS[p.get("interp", "nearest" if score == 0 else "trilinear")]
    out.x0[:] = [float(v) for v in p.get("x0", [0.0] * 6)]
    out.limit[:] = [float(v) for v in p["limit"]]
    out.sigma_score = float(p["sigma_score"])
    out.sigma0[:] = [float(v) for v in p["sigma0"]]
    out.anneal = float(p.get("anneal", 0.85))
    out.min_overlap_frac = float(p.get("min_overlap_frac", 0.05))
    out.rotation_mode = ROTATIONS[p.get("rotation_mode", "box")]
    return out


# ------------------------------------------------------------------ C names

def smc_init(src: SmcVolume, tgt: SmcVolume, prm: SmcParams, stream=None) -> C.c_void_p:
    ctx = C.c_void_p()
    _check(lib().smc_init(C.byref(ctx), C.byref(src), C.byref(tgt), C.byref(prm), _stream_handle(stream)))
    return ctx


def smc_reset(ctx, seed: int):
    _check(lib().smc_reset(ctx, int(seed)))


def smc_step(ctx, n_iters: int):
    _check(lib().smc_step(ctx, int(n_iters)))


def smc_estimate(ctx) -> dict:
    p, M = np.zeros(6), np.zeros(12)
    score, ess = C.c_double(), C.c_double()
    st = lib().smc_estimate(ctx, _ptr(p), _ptr(M), C.cast(C.byref(score), C.c_void_p),
                            C.cast(C.byref(ess), C.c_void_p))
    if st != SMC_ENOOVERLAP:
        _check(st)
    return dict(params=p, matrix=M.reshape(3, 4), score=score.value, ess=ess.value, no_overlap=st == SMC_ENOOVERLAP)


def smc_get_particles(ctx, n: int) -> dict:
    x, lw, anc = np.zeros((n, 6)), np.zeros(n), np.zeros(n, np.int32)
    _check(lib().smc_get_particles(ctx, _ptr(x), _ptr(lw), _ptr(anc)))
    return dict(states=x, logw=lw, ancestors=anc)


def smc_trace(ctx, n_iters: int) -> dict:
    sc, ess, est = np.zeros(n_iters + 1), np.zeros(n_iters), np.zeros((n_iters, 6))
    _check(lib().smc_trace(ctx, _ptr(sc), _ptr(ess), _ptr(est)))
    return dict(score=sc, ess=ess, est=est)


def smc_evaluate(ctx, states) -> np.ndarray:
    x = np.ascontiguousarray(states, dtype=np.float64).reshape(-1, 6)
    out = np.zeros((len(x), 6), np.int64)
    _check(lib().smc_evaluate(ctx, _ptr(x), len(x), _ptr(out)))
    return out


def smc_gather_probe(ctx, reps: int = 1):
    pm, sm = C.c_double(), C.c_double()
    _check(lib().smc_gather_probe(ctx, int(reps), C.byref(pm), C.byref(sm)))
    return pm.value, sm.value


NOALLOC_MAX_PARTICLES = 65536


def smc_evaluate_noalloc(ctx, states_dev, moments_dev, n: int | None = None):
    """Allocation-free evaluation on device tensors: states_dev (float64,
    n x 6) and moments_dev (int64, n x 6) stay on the GPU; asynchronous on the
    context's stream."""
    n = len(states_dev) if n is None else int(n)
    _check(lib().smc_evaluate_noalloc(ctx, C.c_void_p(states_dev.data_ptr()), n,
                                      C.c_void_p(moments_dev.data_ptr())))


def smc_set_particles(ctx, states, k_done: int):
    x = np.ascontiguousarray(states, dtype=np.float64).reshape(-1, 6)
    _check(lib().smc_set_particles(ctx, _ptr(x), int(k_done)))


def smc_get_state(ctx) -> bytes:
    n = C.c_size_t(0)
    _check(lib().smc_get_state(ctx, None, C.byref(n)))
    buf = C.create_string_buffer(n.value)
    _check(lib().smc_get_state(ctx, C.cast(buf, C.c_void_p), C.byref(n)))
    return buf.raw[: n.value]


def smc_set_state(ctx, blob: bytes):
    buf = C.create_string_buffer(blob, len(blob))
    _check(lib().smc_set_state(ctx, C.cast(buf, C.c_void_p), len(blob)))


def smc_destroy(ctx):
    if ctx:
        lib().smc_destroy(ctx)


def warp_apply(src: SmcVolume, matrix, interp: str, dst, spacing=(1.0, 1.0, 1.0), n_frames: int = 1,
               src_frame_stride: int = 0, dst_frame_stride: int = 0, stream=None):
    """Apply a 3x4 target-mm -> source-mm map to ``n_frames`` source frames,
    writing into the device uint8 tensor ``dst`` of shape ([F,] nz, ny, nx)."""
    M = np.ascontiguousarray(matrix, dtype=np.float64).reshape(12)
    nz, ny, nx = dst.shape[-3:]
    _check(lib().warp_apply(C.byref(src), _ptr(M), INTERPS[interp], C.c_void_p(dst.data_ptr()), nx, ny, nz,
                            *(float(s) for s in spacing), int(n_frames), int(src_frame_stride),
                            int(dst_frame_stride), _stream_handle(stream)))


def smc_profile(ctx, enable: bool):
    _check(lib().smc_profile(ctx, 1 if enable else 0))


def smc_profile_work(ctx) -> dict:
    ev, cov, inr = C.c_uint64(), C.c_uint64(), C.c_uint64()
    _check(lib().smc_profile_work(ctx, C.cast(C.byref(ev), C.c_void_p), C.cast(C.byref(cov), C.c_void_p),
                                  C.cast(C.byref(inr), C.c_void_p)))
    return dict(evaluated=ev.value, covered=cov.value, interior=inr.value)


def smc_profile_read(ctx) -> dict:
    sm, fm = C.c_double(), C.c_double()
    sn, fn = C.c_uint64(), C.c_uint64()
    _check(lib().smc_profile_read(ctx, C.cast(C.byref(sm), C.c_void_p), C.cast(C.byref(sn), C.c_void_p),
                                  C.cast(C.byref(fm), C.c_void_p), C.cast(C.byref(fn), C.c_void_p)))
    return dict(score_ms=sm.value, score_launches=sn.value, filter_ms=fm.value, filter_launches=fn.value)


LAYOUTS = {"raw": 0, "pairx": 1, "quadxy": 2, "oct": 3, "octtile": 4, "lerp": 5}


def smc_exhaustive(ctx, lo, step, count, want_scores=False) -> dict:
    lo_ = np.ascontiguousarray(lo, dtype=np.float64)
    st = np.ascontiguousarray(step, dtype=np.float64)
    cn = np.ascontiguousarray(count, dtype=np.uint32)
    best, score = np.zeros(6), C.c_double()
    scores = np.zeros(int(np.prod(cn.astype(np.int64)))) if want_scores else None
    _check(lib().smc_exhaustive(ctx, _ptr(lo_), _ptr(st), _ptr(cn), _ptr(best), C.cast(C.byref(score), C.c_void_p),
                                None if scores is None else _ptr(scores)))
    return dict(params=best, score=score.value, scores=scores)


def smc_set_proposal(ctx, mean=None, logvar=None):
    if mean is None:
        _check(lib().smc_set_proposal(ctx, None, None))
        return
    m = np.ascontiguousarray(mean, dtype=np.float64)
    lv = np.ascontiguousarray(logvar, dtype=np.float64)
    _check(lib().smc_set_proposal(ctx, _ptr(m), _ptr(lv)))


def smc_cloud_moments(ctx, var_floor=0.0):
    """Weighted mean and variance of the particle cloud in units of the limits."""
    mean, var = np.zeros(6), np.zeros(6)
    _check(lib().smc_cloud_moments(ctx, float(var_floor), _ptr(mean), _ptr(var)))
    return mean, var


def smc_set_proposal_from_network(ctx, out, var_scale):
    """Proposal from the network's 12 outputs; returns the (mean, logvar) set."""
    o = np.ascontiguousarray(out, dtype=np.float32).reshape(12)
    mean, logvar = np.zeros(6), np.zeros(6)
    _check(lib().smc_set_proposal_from_network(ctx, _ptr(o), float(var_scale), _ptr(mean), _ptr(logvar)))
    return mean, logvar


def smc_set_tuning(ctx, layout=None, particles_per_group=None, tile_depth=None):
    lay = -1 if layout is None else (LAYOUTS[layout] if isinstance(layout, str) else int(layout))
    pt = -1 if particles_per_group is None else int(particles_per_group)
    td = -1 if tile_depth is None else int(tile_depth)
    _check(lib().smc_set_tuning(ctx, lay, pt, td))


def smc_score_particles(ctx, states) -> np.ndarray:
    x = np.ascontiguousarray(states, dtype=np.float64).reshape(-1, 6)
    out = np.zeros(len(x))
    _check(lib().smc_score_particles(ctx, _ptr(x), len(x), _ptr(out)))
    return out


def smc_set_frames(ctx, src_frames, tgt_frames):
    """Further frame pairs (lists of SmcVolume) scored with the first."""
    n = len(src_frames)
    if n != len(tgt_frames):
        raise ValueError("src_frames and tgt_frames differ in length")
    srcs = (SmcVolume * max(n, 1))(*src_frames)
    tgts = (SmcVolume * max(n, 1))(*tgt_frames)
    _check(lib().smc_set_frames(ctx, n, C.cast(srcs, C.c_void_p), C.cast(tgts, C.c_void_p)))


def smc_get_tuning(ctx) -> dict:
    lay, pt, td = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().smc_get_tuning(ctx, C.cast(C.byref(lay), C.c_void_p), C.cast(C.byref(pt), C.c_void_p),
                                C.cast(C.byref(td), C.c_void_p)))
    return dict(layout=lay.value, particles_per_group=pt.value, tile_depth=td.value)


def version() -> str:
    return lib().smc_version().decode()


class Registration:
    """One registration pair: owns an smc context on the current device."""

    def __init__(self, src, tgt, prm: dict, spacing=(1.0, 1.0, 1.0), src_fov=None, tgt_fov=None,
                 tgt_spacing=None, stream=None):
        self._keep = (src, tgt, src_fov, tgt_fov)  # device memory must outlive the context
        self.params = dict(prm)
        self.n = int(prm["n_particles"])
        self.K = int(prm["n_iters"])
        self.src = volume(src, spacing, src_fov)
        self.tgt = volume(tgt, spacing if tgt_spacing is None else tgt_spacing, tgt_fov)
        self.ctx = smc_init(self.src, self.tgt, params(prm), stream)

    def step(self, n=1):
        smc_step(self.ctx, n)

    def run(self):
        smc_step(self.ctx, self.K)
        return self.estimate()

    def reset(self, seed):
        smc_reset(self.ctx, seed)

    def estimate(self):
        return smc_estimate(self.ctx)

    def particles(self):
        return smc_get_particles(self.ctx, self.n)

    def trace(self):
        return smc_trace(self.ctx, self.K)

    def evaluate(self, states):
        return smc_evaluate(self.ctx, states)

    def scores(self, states):
        return smc_score_particles(self.ctx, states)

    def set_frames(self, frames, spacing=(1.0, 1.0, 1.0), tgt_spacing=None):
        """Score on further frame pairs too: ``frames`` is a list of dicts with
        device tensors src, tgt and optional src_fov, tgt_fov."""
        ts = spacing if tgt_spacing is None else tgt_spacing
        self._frames = [(q["src"], q["tgt"], q.get("src_fov"), q.get("tgt_fov")) for q in frames]
        smc_set_frames(self.ctx, [volume(q["src"], spacing, q.get("src_fov")) for q in frames],
                       [volume(q["tgt"], ts, q.get("tgt_fov")) for q in frames])

    def set_particles(self, states, k_done):
        smc_set_particles(self.ctx, states, k_done)

    def get_state(self):
        return smc_get_state(self.ctx)

    def set_state(self, blob):
        smc_set_state(self.ctx, blob)

    def exhaustive(self, lo, step, count, want_scores=False):
        return smc_exhaustive(self.ctx, lo, step, count, want_scores)

    def set_proposal(self, mean=None, logvar=None):
        smc_set_proposal(self.ctx, mean, logvar)

    def set_proposal_from_network(self, out, var_scale):
        return smc_set_proposal_from_network(self.ctx, out, var_scale)

    def cloud_moments(self, var_floor=0.0):
        return smc_cloud_moments(self.ctx, var_floor)

    def autotune(self, reps=3):
        ms = C.c_double()
        _check(lib().smc_autotune(self.ctx, int(reps), C.cast(C.byref(ms), C.c_void_p)))
        return dict(self.tuning(), ms=ms.value)

    def tune(self, layout=None, particles_per_group=None, tile_depth=None):
        smc_set_tuning(self.ctx, layout, particles_per_group, tile_depth)

    def tuning(self):
        return smc_get_tuning(self.ctx)

    def profile(self, enable=True):
        smc_profile(self.ctx, enable)

    def profile_read(self):
        return smc_profile_read(self.ctx)

    def profile_work(self):
        """Particle x voxel pairs the culled mask launches evaluated, covered
        and evaluated on interior tiles since the previous call."""
        return smc_profile_work(self.ctx)

    def gather_probe(self, reps=1):
        """(probe ms, production ms) per launch on the current particle set."""
        return smc_gather_probe(self.ctx, reps)

    def close(self):
        if self.ctx:
            smc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many registration pairs run as one graph launch (smc_batch_*).  Each
    pair is a dict with src, tgt (device uint8 tensors), params (dict) and
    optional src_fov, tgt_fov, spacing, tgt_spacing."""

    def __init__(self, pairs, stream=None):
        n = len(pairs)
        self._keep = [(q["src"], q["tgt"], q.get("src_fov"), q.get("tgt_fov")) for q in pairs]
        srcs = (SmcVolume * n)()
        tgts = (SmcVolume * n)()
        prms = (SmcParams * n)()
        for i, q in enumerate(pairs):
            sp = q.get("spacing", (1.0, 1.0, 1.0))
            srcs[i] = volume(q["src"], sp, q.get("src_fov"))
            tgts[i] = volume(q["tgt"], q.get("tgt_spacing", sp), q.get("tgt_fov"))
            prms[i] = params(q["params"])
        self.n_particles = [int(q["params"]["n_particles"]) for q in pairs]
        self.n_iters = [int(q["params"]["n_iters"]) for q in pairs]
        self.b = C.c_void_p()
        _check(lib().smc_batch_init(C.byref(self.b), n, C.cast(srcs, C.c_void_p), C.cast(tgts, C.c_void_p),
                                    C.cast(prms, C.c_void_p), _stream_handle(stream)))
        self.n = n

    def set_seeds(self, seeds):
        a = np.ascontiguousarray(seeds, dtype=np.uint64)
        _check(lib().smc_batch_set_seeds(self.b, _ptr(a)))

    def run(self):
        _check(lib().smc_batch_run(self.b))

    def autotune(self, reps=3):
        _check(lib().smc_batch_autotune(self.b, int(reps)))

    def pair(self, i):
        return C.c_void_p(lib().smc_batch_pair(self.b, int(i)))

    def estimate(self, i):
        return smc_estimate(self.pair(i))

    def particles(self, i):
        return smc_get_particles(self.pair(i), self.n_particles[i])

    def trace(self, i):
        return smc_trace(self.pair(i), self.n_iters[i])

    def close(self):
        if self.b:
            lib().smc_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


CNN_PARAMS = 229916


class Cnn:
    """The learned-proposal network (smc_cnn_*): bfloat16 MFMA convolutions,
    FP32 head, Gaussian-NLL backward and Adam, all on the GPU."""

    def __init__(self, max_batch=32, stream=None):
        self.net = C.c_void_p()
        _check(lib().smc_cnn_create(C.byref(self.net), int(max_batch), _stream_handle(stream)))
        self.max_batch = int(max_batch)

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32)
        _check(lib().smc_cnn_set_params(self.net, _ptr(a), a.size))

    def get_params(self):
        a = np.zeros(CNN_PARAMS, np.float32)
        _check(lib().smc_cnn_get_params(self.net, _ptr(a), a.size))
        return a

    def input(self, slot, src: SmcVolume, tgt: SmcVolume, scale=1.0):
        _check(lib().smc_cnn_input(self.net, int(slot), C.byref(src), C.byref(tgt), float(scale)))

    def read_input(self, slot):
        a = np.zeros((2, 64, 64, 64), np.uint16)
        _check(lib().smc_cnn_read_input(self.net, int(slot), _ptr(a)))
        return a.view(np.float16)

    def forward(self, B):
        out = np.zeros((B, 12), np.float32)
        _check(lib().smc_cnn_forward(self.net, int(B), _ptr(out)))
        return out

    def backward(self, target, grads=False):
        t = np.ascontiguousarray(target, dtype=np.float32).reshape(-1, 12)
        loss = C.c_float()
        g = np.zeros(CNN_PARAMS, np.float32) if grads else None
        _check(lib().smc_cnn_backward(self.net, len(t), _ptr(t), C.cast(C.byref(loss), C.c_void_p),
                                      None if g is None else _ptr(g)))
        return (loss.value, g) if grads else loss.value

    def step(self, lr):
        _check(lib().smc_cnn_step(self.net, float(lr)))

    def close(self):
        if self.net:
            lib().smc_cnn_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
