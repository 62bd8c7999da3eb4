"""Split-CTMRG free energy and gradient of the 3D Ising PEPO / PEPS network on
MI355X (gfx950).

The computation lives in the HIP library ``libctm.so`` (C ABI in
``include/ctm.h``); this package only marshals arguments to it.
"""
from .ctm import (CTM_BF16, CTM_FP32, CTM_FP64, CtmError, SplitCTM, abi_version,
                  library_path, load_library)

__all__ = ["SplitCTM", "CtmError", "load_library", "library_path", "abi_version",
           "CTM_FP64", "CTM_FP32", "CTM_BF16"]
