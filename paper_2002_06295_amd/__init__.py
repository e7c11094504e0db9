"""MI355X-native Kalman-filter track building and fitting (arXiv 2002.06295).

The compute path is the HIP library libkfx.so (C ABI in include/kfx.h);
`kfx` is its Python binding.  Nothing here falls back to the CPU: without
the library or a GPU the calls raise.
"""
from .kfx import (MODE_FUSED, MODE_PLAIN, Context, DeviceHits, KfxError, States, load_library,
                  pack_cov, unpack_cov)

__all__ = ["Context", "DeviceHits", "KfxError", "States", "MODE_PLAIN", "MODE_FUSED", "load_library",
           "pack_cov", "unpack_cov"]
