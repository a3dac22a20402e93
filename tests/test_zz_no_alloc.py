"""The allocation-free evaluation entry point (smc_evaluate_noalloc) against
the allocating one (smc_evaluate) on the same context: identical integer sums
for masks and for trilinear images with a source FOV, on two calls in a row
(the second smaller, so the shared scratch array holds the first call's
words past the second's end), with output rows past n left untouched, and a
clear error above the maximum size."""

import numpy as np
import pytest

import synth
from paper_2504_19930_amd import config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_19930_amd import binding
    binding.lib()
    return binding


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _states(n, rot_deg, trans, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([np.deg2rad(rng.uniform(-rot_deg, rot_deg, (n, 3))),
                           rng.uniform(-trans, trans, (n, 3))], 1)


def _cases():
    shell = synth.shell_pair(seed=1, side=40)
    speckle = synth.speckle_pair(side=48, seed=2)
    return [
        ("mask", dict(src=shell["src"], tgt=shell["tgt"]), None, config.default_params("dice", 64, 3, 15.0, 5.0)),
        ("image", dict(src=speckle["src"], tgt=speckle["tgt"]), speckle["src_fov"],
         config.default_params("ncc", 64, 3, 20.0, 4.0)),
    ]


@pytest.mark.parametrize("case", [0, 1])
def test_noalloc_equals_evaluate_on_two_calls(smc, case):
    import torch
    kind, pair, fov, prm = _cases()[case]
    reg = smc.Registration(_dev(pair["src"]), _dev(pair["tgt"]), prm, src_fov=None if fov is None else _dev(fov))
    rot, trans = (15.0, 5.0) if kind == "mask" else (20.0, 4.0)
    n_cap = 301
    out = torch.full((n_cap, 6), -7, dtype=torch.int64, device="cuda")
    for n, seed in ((n_cap, 11), (37, 12)):
        x = _states(n, rot, trans, seed)
        want = reg.evaluate(x)
        assert want[:, 0].max() > 0  # the particles reach the source
        xd = _dev(x)
        smc.smc_evaluate_noalloc(reg.ctx, xd, out, n)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got[:n], want), (kind, n)
        # rows past n keep what the previous call wrote
        if n < n_cap:
            assert np.array_equal(got[n:], prev[n:]), (kind, n)
        prev = got
    reg.close()


def test_noalloc_rejects_oversize_and_null(smc):
    import torch
    _, pair, _, prm = _cases()[0]
    reg = smc.Registration(_dev(pair["src"]), _dev(pair["tgt"]), prm)
    x = torch.zeros((4, 6), dtype=torch.float64, device="cuda")
    out = torch.zeros((4, 6), dtype=torch.int64, device="cuda")
    with pytest.raises(smc.SmcError) as e:
        smc.smc_evaluate_noalloc(reg.ctx, x, out, smc.NOALLOC_MAX_PARTICLES + 1)
    assert e.value.status == smc.SMC_EINVAL
    assert "allocation-free maximum" in str(e.value)
    import ctypes as C
    st = smc.lib().smc_evaluate_noalloc(reg.ctx, None, 4, C.c_void_p(out.data_ptr()))
    assert st == smc.SMC_EINVAL
    # n = 0 does nothing
    smc.smc_evaluate_noalloc(reg.ctx, x, out, 0)
    # the context still works after the rejected calls
    smc.smc_evaluate_noalloc(reg.ctx, x, out, 4)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), reg.evaluate(np.zeros((4, 6))))
    reg.close()
