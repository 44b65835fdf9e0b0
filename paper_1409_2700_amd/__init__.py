"""MCPT(2) doubles hot path on AMD Instinct MI355X (gfx950).

The compute path is libmcpt.so (HIP, C ABI declared in include/mcpt.h); this
package holds its sources (csrc/), the build step and a thin ctypes binding.
"""
from .mcpt import (  # noqa: F401
    Context, MCPTError, HostProblem, make_options, split_t, load_library, lib, LIB_PATH, EXPORTS,
    mcpt_singles_summary, device_rates,
    MCPT_OK, MCPT_PENDING, MCPT_ERR_INVALID, MCPT_ERR_NOMEM, MCPT_ERR_DEVICE, MCPT_ERR_NOT_CONVERGED,
    MCPT_ERR_DIVERGED, MCPT_ERR_NONFINITE, MCPT_ERR_ADMISSION, MCPT_ERR_UNKNOWN_ID,
    MCPT_FP64, MCPT_FP32, MCPT_BF16, MCPT_HOST, MCPT_DEVICE,
    MCPT_SERVE_BATCH_END, MCPT_SERVE_RETIRE_AT_TICKS, MCPT_SERVE_JOIN_AT_TICKS,
)
