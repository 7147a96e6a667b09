"""MI355X (gfx950) batched pair-potential simulation: HIP library + thin Python binding.

The compute path is the C-ABI library ``libts_mi355x.so`` (``include/ts_api.h``); this package
only marshals torch device buffers into its entry points (``api``) and composes them into the
checkpointed trajectory gradient (``trajectory``).
"""
from .build import LIB_PATH, build  # noqa: F401
