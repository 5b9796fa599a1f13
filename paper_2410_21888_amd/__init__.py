"""MI355X (gfx950) closed-shell RI-MP2 fragment kernel.

The compute path is the HIP library ``librimp2.so`` (C ABI in
``include/rimp2.h``); this package only marshals arguments to it.  PyTorch
provides device memory and streams.
"""
from .rimp2 import (  # noqa: F401
    RIMP2_OK, RIMP2_EINVAL, RIMP2_ENOMEM, RIMP2_EWORKSPACE, RIMP2_EDEVICE, RIMP2_EGAP, RIMP2_ENOTSUP, RIMP2_ENOCONV,
    FP64, SPLIT_INT8, Rimp2Error, Result, Opts, lib, version, workspace_size, fragment, fragment_into,
    read_status, batch_workspace_size, fragment_batch, flops, make_opts, timing_enable, timing_collect, Batch,
    autotune_report, autotune_reset,
)
