"""MI355X-native Fourier ADI hot path (GRAPHIC, arXiv:1510.04331).

The computation lives in libgraphic.so (hand-written HIP for gfx950) behind the
C ABI of include/graphic.h; this package only marshals torch tensors to it.
"""

from .ops import (shift, rotate, median, adi_reduce, adi_reduce_batch, workspace_size, resolved_pad,  # noqa: F401
                  median_window, adi_reduce_window, alpha_min_deg, parallactic_angles, register,
                  median_nan, mask_disk, subtract_nearest, badpix_map, badpix_fix, annular_rms,
                  batch_workspace_size, AdiGraph, autotune, tuning_export, tuning_import,
                  timing_enable, timing_read)
from ._abi import LIB_PATH, GraphicError  # noqa: F401
