"""FP64 CPU oracle of the Fourier ADI hot path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library.
"""

from .fourier_adi import *  # noqa: F401,F403
from .fourier_adi import __all__ as _adi_all
from . import registration  # noqa: F401  (Sect. 3.1: parallactic angles, centroid, Moffat fit)
from . import preprocess  # noqa: F401  (Sect. 3.2: master sky, bad pixels)
from . import quality  # noqa: F401  (Sect. 4.1: double shift / rotation residuals in annuli)

__all__ = list(_adi_all) + ["registration", "preprocess", "quality"]
