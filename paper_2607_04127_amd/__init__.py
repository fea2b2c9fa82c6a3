"""MI355X (gfx950) spherical surfel range-image renderer with its backward pass.

The renderer lives in ``liblgsr.so`` (hand-written HIP kernels behind the C ABI of
include/lgsr.h); :mod:`paper_2607_04127_amd.lgsr` is its ctypes binding.
"""
from . import lgsr  # noqa: F401
from .lgsr import (  # noqa: F401
    Context,
    LgsrError,
    State,
    default_loss_weights,
    default_opts,
    lgsr_backward,
    lgsr_forward,
    lgsr_loss,
    lgsr_profile,
    lgsr_profile_read,
    lgsr_query,
    lgsr_state_free,
    lgsr_sync,
)
