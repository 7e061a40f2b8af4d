"""MI355X (gfx950) implementation of CIDER's masked-diffusion refinement path.

The decoder itself is the HIP library libcider.so (C ABI in include/cider.h);
``abi`` is its ctypes binding.  Build with ``paper_2605_26580_amd.build.build()``.
"""
from . import abi, protocol  # noqa: F401
from .abi import (  # noqa: F401
    CIDER_BF16, CIDER_FP32, CIDER_FP64, CIDER_FP8, CIDER_MASK, CIDER_SCHED_COSINE, CIDER_SCHED_LINEAR,
    CiderError, Code, CodeQ, Server, Weights, cider_code_create_q, cider_decode_q_batch, cider_step_debug_q, cider_amp_evidence, cider_gf64_check_update, cider_code_create, cider_decode, cider_decode_batch, cider_decode_noalloc, cider_evidence,
    cider_last_error, cider_opts_default, cider_profile_read, cider_tuning_read, cider_step_debug, cider_strerror, cider_weights_blob_floats,
    cider_weights_create, cider_workspace_size, make_cfg,
)
from .protocol import decode_frames, serve_frames  # noqa: F401
