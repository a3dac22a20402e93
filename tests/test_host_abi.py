"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/smc.h declares, and rejects bad arguments before any
device work."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:smc|warp)_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def smc():
    from paper_2504_19930_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2504_19930_amd import build
        build.build()
    binding.lib()
    return binding


def test_exports_every_declared_symbol(smc):
    names = _declared()
    assert "smc_init" in names and "warp_apply" in names and len(names) >= 13
    for name in names:
        assert hasattr(smc.lib(), name), name
    assert set(names) == set(smc.EXPORTS)
    assert "gfx950" in smc.version()


def _vol(smc, nx=8, ny=8, nz=8, s=1.0, data=0x1000):
    return smc.SmcVolume(nx, ny, nz, s, s, s, data, None)


def _params(smc, **kw):
    from paper_2504_19930_amd import config
    p = config.default_params("dice", 16, 3, 15.0, 8.0)
    p.update(kw)
    return smc.params(p)


def _init_status(smc, src, tgt, prm):
    ctx = C.c_void_p()
    return smc.lib().smc_init(C.byref(ctx), C.byref(src), C.byref(tgt), C.byref(prm), None), ctx


@pytest.mark.parametrize("bad", [
    dict(n_particles=0), dict(n_particles=65536), dict(n_particles=70000), dict(n_iters=0), dict(score="ncc", interp="nearest",
                                                                          sigma_score=-1.0),
    dict(anneal=0.0), dict(anneal=1.5), dict(min_overlap_frac=2.0), dict(limit=[0.1, 0.1, 0.0, 1, 1, 1]),
    dict(sigma0=[-1.0] * 6), dict(x0=[float("nan")] + [0.0] * 5), dict(interp="trilinear"),
])
def test_bad_params_rejected_before_device_work(smc, bad):
    st, ctx = _init_status(smc, _vol(smc), _vol(smc), _params(smc, **bad))
    assert st == smc.SMC_EINVAL and not ctx.value
    assert smc.lib().smc_last_error().decode()


@pytest.mark.parametrize("vol", [dict(nx=0), dict(nz=70000), dict(s=0.0), dict(s=float("inf")), dict(data=None),
                                 dict(nx=2048, ny=2048, nz=1024), dict(nx=4096, ny=4096, nz=1)])
def test_bad_volumes_rejected(smc, vol):
    st, _ = _init_status(smc, _vol(smc, **vol), _vol(smc), _params(smc))
    assert st == smc.SMC_EINVAL
    st, _ = _init_status(smc, _vol(smc), _vol(smc, **vol), _params(smc))
    assert st == smc.SMC_EINVAL


def test_null_arguments(smc):
    L = smc.lib()
    assert L.smc_init(None, None, None, None, None) == smc.SMC_EINVAL
    assert L.smc_step(None, 1) == smc.SMC_EINVAL
    assert L.smc_estimate(None, None, None, None, None) == smc.SMC_EINVAL
    assert L.smc_get_particles(None, None, None, None) == smc.SMC_EINVAL
    assert L.smc_set_frames(None, 0, None, None) == smc.SMC_EINVAL
    L.smc_destroy(None)
    M = np.eye(3, 4)
    src = _vol(smc)
    assert L.warp_apply(C.byref(src), M.ctypes.data_as(C.c_void_p), 0, None, 8, 8, 8, 1.0, 1.0, 1.0, 1, 0, 0,
                        None) == smc.SMC_EINVAL
    M[0, 0] = np.nan
    assert L.warp_apply(C.byref(src), M.ctypes.data_as(C.c_void_p), 0, C.c_void_p(0x1000), 8, 8, 8, 1.0, 1.0,
                        1.0, 1, 0, 0, None) == smc.SMC_EINVAL
    assert L.warp_apply(C.byref(src), np.eye(3, 4).ctypes.data_as(C.c_void_p), 7, C.c_void_p(0x1000), 8, 8, 8,
                        1.0, 1.0, 1.0, 1, 0, 0, None) == smc.SMC_EINVAL


def test_binding_refuses_host_tensors(smc):
    import torch
    with pytest.raises(ValueError):
        smc.volume(torch.zeros((4, 4, 4), dtype=torch.uint8))


def test_struct_layouts_match_the_header(smc, tmp_path):
    """The ctypes mirrors of smc_volume and smc_params have the sizes and
    field offsets the C compiler gives the header's structs."""
    import subprocess
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "smc.h"\n'
                    'int main(void) { printf("%zu %zu %zu %zu %zu\\n", sizeof(smc_volume), sizeof(smc_params), '
                    'offsetof(smc_params, min_overlap_frac), offsetof(smc_params, rotation_mode), '
                    'offsetof(smc_volume, fov)); return 0; }\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [C.sizeof(smc.SmcVolume), C.sizeof(smc.SmcParams), smc.SmcParams.min_overlap_frac.offset,
            smc.SmcParams.rotation_mode.offset, smc.SmcVolume.fov.offset]
    assert got == want


def test_unknown_rotation_mode_rejected(smc):
    prm = _params(smc)
    prm.rotation_mode = 2
    st, _ = _init_status(smc, _vol(smc), _vol(smc), prm)
    assert st == smc.SMC_EINVAL
    assert "rotation_mode" in smc.lib().smc_last_error().decode()
