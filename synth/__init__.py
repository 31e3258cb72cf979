"""Seeded synthetic ADI cubes (inputs only; shared by the oracle tests and the
GPU path, and holding none of the reduction's arithmetic)."""

from .cube import (CubeParams, make_params, make_batch_params, make_arrivals,  # noqa: F401
                   render_host, render_device, companion_positions,
                   STAR_PEAK, SIGMA_PX, FWHM_PX, BASE_SEED)
