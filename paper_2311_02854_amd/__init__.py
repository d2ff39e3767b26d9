"""MI355X two-site DMRG sigma-vector engine (Python side of libdmrg.so).

The computation lives in the HIP library built from csrc/; this package only
loads it and marshals arguments.  There is no CPU fallback: if the library is
missing, loading fails with an error.
"""

from .binding import (BF16X3, FP32, FP64, Context, DmrgError, Ops, load,
                      sigma_batched)

__all__ = ["Context", "Ops", "DmrgError", "load", "sigma_batched", "FP64", "FP32", "BF16X3",
           "gpu_context"]


def gpu_context(device=0):
    """Context on `device` issuing work on torch's current HIP stream."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the DMRG sigma engine runs on the HIP device only")
    torch.cuda.set_device(device)
    return Context(device, torch.cuda.current_stream(device).cuda_stream)
