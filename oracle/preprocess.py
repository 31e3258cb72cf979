"""FP64 / float32 CPU oracle of the image pre-processing (Sect. 3.2, 3.2.1 and 3.2.2
of Hagelberg et al. 2016, arXiv:1510.04331): master sky and bad pixels.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.  It shares no code
with the HIP library.

Readings (the paper leaves these open; the HIP path follows the same ones):

* Star mask: the pixels within ``radius`` of the star position, (x - x_s)^2 +
  (y - y_s)^2 <= radius^2 with x the column and y the row, are set to NaN
  before the sky median.
* Master sky: the per-pixel median of the frames ignoring NaN values (the
  float32 median of the remaining values, as the PSF median); a pixel with no
  value left is NaN.
* Sky subtraction: every frame subtracts the master sky closest in time (the
  earliest one on a tie).
* Bad pixel map: pixels that are not finite, or whose value differs from the
  frame's median by more than C sigma (median in float32 as above, sigma the
  population standard deviation in float64, both over the finite pixels).
* Bad pixel correction: flagged pixels are set to NaN; then, pass after pass,
  every NaN pixel with at least one non-NaN pixel among its 8 neighbours takes
  the (float32) median of those neighbours, all from the previous pass's
  values, until no NaN is left or no pixel changes (a pixel whose whole frame
  is NaN stays NaN).
"""

import numpy as np

from .fourier_adi import median_f32

__all__ = ["mask_disk", "median_nan_f32", "subtract_nearest", "badpix_map", "badpix_fix"]


def mask_disk(cube, xs, ys, radius):
    """NaN out the disc of ``radius`` around (xs[i], ys[i]) in frame i."""
    out = np.array(cube, dtype=np.float32, copy=True)
    T, n, _ = out.shape
    yy, xx = np.mgrid[0:n, 0:n]
    for i in range(T):
        out[i][(xx - xs[i]) ** 2 + (yy - ys[i]) ** 2 <= radius * radius] = np.nan
    return out


def median_nan_f32(stack):
    """Per-pixel float32 median over axis 0 ignoring NaN (NaN where none is left)."""
    st = np.asarray(stack, dtype=np.float32)
    T, h, w = st.shape
    out = np.full((h, w), np.nan, dtype=np.float32)
    for y in range(h):
        for x in range(w):
            v = st[:, y, x]
            v = v[~np.isnan(v)]
            if v.size:
                out[y, x] = median_f32(v[:, None])[0]
    return out


def subtract_nearest(cube, times, skies, sky_times):
    """frame_i - sky_s with s the closest sky time (earliest on a tie), in float32."""
    cube = np.asarray(cube, dtype=np.float32)
    st = np.asarray(sky_times, dtype=np.float64)
    out = np.empty_like(cube)
    for i, t in enumerate(np.asarray(times, dtype=np.float64)):
        s = int(np.argmin(np.abs(st - t)))        # argmin returns the first minimum
        out[i] = cube[i] - np.asarray(skies[s], dtype=np.float32)
    return out


def badpix_map(frame, c_sigma):
    """Boolean map of the bad pixels of one frame (Sect. 3.2.2)."""
    f = np.asarray(frame, dtype=np.float32)
    fin = np.isfinite(f)
    vals = f[fin]
    med = float(median_f32(vals[:, None])[0])
    sigma = float(np.std(vals.astype(np.float64)))
    return ~fin | (np.abs(f.astype(np.float64) - med) > c_sigma * sigma)


def badpix_fix(cube, bad=None, max_passes=64):
    """Set the flagged pixels to NaN and fill every NaN pixel with the median
    of its non-NaN 8-neighbours, pass after pass (each pass reads the previous
    one).  Returns (cube, passes)."""
    out = np.array(cube, dtype=np.float32, copy=True)
    if bad is not None:
        out[:, np.asarray(bad, bool)] = np.nan
    T, n, _ = out.shape
    passes = 0
    for _ in range(max_passes):
        nan = np.isnan(out)
        if not nan.any():
            break
        prev = out.copy()
        changed = False
        for i, y, x in zip(*np.nonzero(nan)):
            nb = [prev[i, y + dy, x + dx] for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                  if (dy or dx) and 0 <= y + dy < n and 0 <= x + dx < n]
            nb = np.array([v for v in nb if not np.isnan(v)], dtype=np.float32)
            if nb.size:
                out[i, y, x] = median_f32(nb[:, None])[0]
                changed = True
        passes += 1
        if not changed:
            break
    return out, passes
