"""FP64 CPU oracle of the image-quality test of Sect. 4.1 of Hagelberg et al.
2016 (arXiv:1510.04331): an image is shifted (or rotated) and moved back,
the original is subtracted, and the root mean square of the difference is
taken in concentric annuli around the frame centre.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only the test-suite,
the smoke check and the benchmark's reference lines may import it.  It
shares no code with the HIP library.

Readings (the paper leaves these open; the HIP path follows the same ones):

* Annulus k of width w holds the pixels with (k w)^2 <= d^2 < ((k + 1) w)^2,
  d^2 = (x - cx)^2 + (y - cy)^2, x the column and y the row, the centre
  (cx, cy) = (N/2, N/2) unless given; the comparison is made on the squared
  distance in float64, so no square root decides membership.
* The annular RMS is sqrt(sum (a - b)^2 / count) with the sum in float64;
  an empty annulus gives NaN.  Normalising the profile (the paper plots it
  normalised) is left to the caller.
* The interpolation curve of the paper is a third-order spline; here it
  comes from scipy.ndimage (order 3, zero outside the frame), used only as
  the reference the Fourier curve is compared with.
"""

import numpy as np

from .fourier_adi import shift, rotate

__all__ = ["annular_rms", "double_shift", "double_rotate", "spline_double_shift", "spline_double_rotate"]


def annular_rms(a, b=None, width=1.0, n_rings=None, cx=None, cy=None):
    """RMS of a - b (or of a) in annuli of `width` pixels around (cx, cy).
    a, b: [N, N] or [T, N, N].  Returns (rms [T, n_rings], counts [n_rings])."""
    a = np.asarray(a, dtype=np.float64)
    single = a.ndim == 2
    if single:
        a = a[None]
    T, n, m = a.shape
    d = a if b is None else a - np.asarray(b, dtype=np.float64).reshape(a.shape if np.ndim(b) == 3 else (1, n, m))
    cx = n / 2.0 if cx is None else float(cx)
    cy = n / 2.0 if cy is None else float(cy)
    yy, xx = np.mgrid[0:n, 0:m].astype(np.float64)
    d2 = (xx - cx) ** 2 + (yy - cy) ** 2
    if n_rings is None:
        n_rings = int(np.ceil(np.sqrt(d2.max()) / width)) + 1
    ring = np.full(d2.shape, -1, dtype=np.int64)
    for k in range(n_rings):
        inside = ((k * width) ** 2 <= d2) & (d2 < ((k + 1) * width) ** 2)
        ring[inside] = k
    counts = np.array([(ring == k).sum() for k in range(n_rings)], dtype=np.int64)
    rms = np.full((T, n_rings), np.nan)
    for t in range(T):
        sq = d[t] ** 2
        for k in range(n_rings):
            if counts[k]:
                rms[t, k] = np.sqrt(sq[ring == k].sum() / counts[k])
    return (rms[0] if single else rms), counts


def double_shift(img, dx, dy, P=None):
    """Shift by (dx, dy), then by (-dx, -dy), with the Fourier shift."""
    return shift(shift(img, dx, dy, P), -dx, -dy, P)


def double_rotate(img, angle_deg, P=None):
    """Rotate by angle, then by -angle, with the three Fourier shears."""
    return rotate(rotate(img, angle_deg, P), -angle_deg, P)


def spline_double_shift(img, dx, dy):
    """The same with third-order spline interpolation (scipy.ndimage)."""
    from scipy import ndimage
    f = np.asarray(img, dtype=np.float64)
    once = ndimage.shift(f, (dy, dx), order=3, mode="constant", cval=0.0)
    return ndimage.shift(once, (-dy, -dx), order=3, mode="constant", cval=0.0)


def spline_double_rotate(img, angle_deg):
    """The same with third-order spline interpolation (scipy.ndimage)."""
    from scipy import ndimage
    f = np.asarray(img, dtype=np.float64)
    once = ndimage.rotate(f, angle_deg, reshape=False, order=3, mode="constant", cval=0.0)
    return ndimage.rotate(once, -angle_deg, reshape=False, order=3, mode="constant", cval=0.0)
