"""MI355X-native QRNG post-processing (arXiv 2011.04130): Python binding.

A thin ctypes layer over ``libqrng.so`` (C ABI in ``include/qrng.h``).  It
only marshals arguments: every step of the hashing and of the histogram runs
in the library's HIP kernels on the GPU.  Torch tensors supply device memory
(``data_ptr()``) and the current HIP stream; nothing here falls back to the
CPU.  Importing works without a GPU; creating a ``Context`` needs one and the
built library (``python -m paper_2011_04130_amd.build``), and raises
otherwise.
"""
from __future__ import annotations

import ctypes
import os

from ._lib import (LIB_PATH, QrngError, PATH_AUTO, PATH_DIRECT, PATH_NTT, PATH_MFMA,
                   U_MODEL_ARGMAX, U_BOTH_ARGMAX, U_ALL, MODEL_FIT, MODEL_GIVEN, MODEL_QUANTUM,
                   Block, MeOpts, MeResult, load_library, output_bits, version)
from .api import Context

__all__ = [
    "Context", "QrngError", "output_bits", "version", "load_library", "LIB_PATH",
    "PATH_AUTO", "PATH_DIRECT", "PATH_NTT", "PATH_MFMA",
    "U_MODEL_ARGMAX", "U_BOTH_ARGMAX", "U_ALL", "MODEL_FIT", "MODEL_GIVEN", "MODEL_QUANTUM",
    "Block", "MeOpts", "MeResult",
]
