"""MI355X (gfx950) blockwise 16-point multiplierless approximate DCT.

The transform of Silveira et al. (Section 2: T over {0, +1, -1}, 44-addition
factorisation; Section 3: blockwise 2D coding) as hand-written HIP kernels
behind a C ABI (``include/adct.h``, ``libadct.so``).  ``adct`` is the
ctypes binding.
"""
from . import adct  # noqa: F401

__all__ = ["adct"]
