"""MI355X-native Kalman-filter track building and fitting (arXiv 2002.06295).

The compute path is the HIP library libkfx.so (C ABI in include/kfx.h);
`kfx` is its Python binding and `autograd` wraps the fit and its adjoint as
a torch.autograd.Function.  Nothing here falls back to the CPU: without the
library or a GPU the calls raise.
"""
from .kfx import (MODE_FUSED, MODE_PLAIN, Context, DeviceHits, KfxError, States, load_library,
                  pack_cov, unpack_cov)
from .autograd import FitChi2, fit_chi2

__all__ = ["Context", "DeviceHits", "KfxError", "States", "MODE_PLAIN", "MODE_FUSED", "load_library",
           "pack_cov", "unpack_cov", "FitChi2", "fit_chi2"]
