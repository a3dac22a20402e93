"""MI355X-native particle-filter (sequential Monte Carlo) rigid registration
of 3D echo volumes, after arXiv 2504.19930.

The hot path is the HIP library ``libsmc.so`` (C ABI in ``include/smc.h``);
``binding`` marshals PyTorch device tensors into it.  Nothing here falls back
to the CPU: without the built library every call raises.
"""

from .binding import (  # noqa: F401
    EXPORTS,
    Batch,
    Cnn,
    Registration,
    SmcError,
    lib,
    params,
    smc_destroy,
    smc_estimate,
    smc_evaluate,
    smc_get_particles,
    smc_get_state,
    smc_init,
    smc_profile,
    smc_profile_read,
    smc_reset,
    smc_set_particles,
    smc_set_state,
    smc_step,
    smc_trace,
    version,
    volume,
    warp_apply,
)
from .config import default_params  # noqa: F401
