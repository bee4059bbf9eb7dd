"""LSLU and Hybrid LSLU on MI355X (gfx950).

The solver lives in ``liblslu.so`` (HIP kernels behind the C ABI declared in
``include/lslu.h``); :mod:`paper_2409_05239_amd.capi` is its ctypes binding.
Build with ``python -m paper_2409_05239_amd.build``.
"""

import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblslu.so")
