"""MI355X (gfx950) Monte Carlo evaluation of the lattice functional integral of
Burgers' equation (Honkonen & Honkonen, arXiv:1803.07560).

The computation lives in ``libbfi.so`` (HIP kernels + C ABI, ``include/bfi.h``);
this package is its ctypes binding.  Importing it does not touch the GPU; the
first call loads the library and fails loudly if it is not built.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import (BFI_FP32_SHIFTED, BFI_FP64, BFI_FP64_SHIFTED, EXPORTED, LIB_PATH, BfiError, Subvolumes,  # noqa
                       load, partial_len, split_len)
