"""FP64 CPU oracle of the registration step (Sect. 3.1 of Hagelberg et al. 2016,
arXiv:1510.04331): parallactic angles, star centroid and Moffat fit.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only the test-suite,
the smoke check and the CPU-baseline leg of the benchmark may import it.  It
shares no code with the HIP library.

Readings (the paper leaves these open; the HIP path follows the same ones):

* Parallactic angle: the arctangent of Sect. 3.1.1 is taken with its two
  arguments (atan2), which fixes the quadrant; the hour angle is
  h = 15 LST / 3600 - RA in degrees (LST in seconds, RA in degrees).
* Centroid: the patch is the 4-connected set of pixels above the threshold
  that contains the brightest pixel, searched inside a 64 x 64 box centred on
  that pixel; its centre of mass uses the pixel values as weights.  A patch
  whose size falls outside [min_size, max_size] fails, and the brightest
  pixel stands in for the centroid.
* Moffat fit: the model of Sect. 3.1.2 over a (2 half) x (2 half) box around the
  rounded centroid, pixels at or above the saturation level (and non-finite
  ones) masked out, least squares with MINPACK's Levenberg-Marquardt (lmdif,
  the routine the paper names) from the starting point below.
* Starting point: background = mean of the box's unmasked border pixels,
  alpha = 2.5 px, beta = 2.5, centre = centroid, and I0 such that the model
  peak equals the brightest unmasked pixel of the box above the background.
* Pixel (x, y) is column x, row y, both from 0; a star centred on pixel
  (N/2, N/2) needs no recentring, so the shift is (N/2 - x0, N/2 - y0).
"""

import numpy as np

__all__ = ["parallactic_angle", "centroid", "moffat", "moffat_fwhm", "fit_moffat", "register", "BOX"]

BOX = 64          # side of the centroid search box


def parallactic_angle(lst_s, ra_deg, dec_deg, lat_deg):
    """Parallactic angle in degrees (Sect. 3.1.1): hour angle from the local
    sidereal time (seconds) and right ascension (degrees), then
    atan2(cos(phi) sin(h), cos(delta) sin(phi) - sin(delta) cos(phi) cos(h))."""
    h = np.radians(15.0 * np.asarray(lst_s, dtype=np.float64) / 3600.0 - ra_deg)
    d, p = np.radians(dec_deg), np.radians(lat_deg)
    return np.degrees(np.arctan2(np.cos(p) * np.sin(h), np.cos(d) * np.sin(p) - np.sin(d) * np.cos(p) * np.cos(h)))


def _box(n, c, side):
    lo = int(c) - side // 2
    lo = max(0, min(lo, n - side)) if side <= n else 0
    return lo, min(n, lo + side)


def centroid(frame, threshold, min_size, max_size):
    """Centre of mass of the contiguous patch above ``threshold`` holding the
    brightest pixel (Sect. 3.1.2, first stage).  Returns (x, y, ok, size)."""
    from scipy import ndimage
    f = np.asarray(frame, dtype=np.float64)
    n = f.shape[0]
    flat = np.where(np.isfinite(f), f, -np.inf)
    iy, ix = np.unravel_index(int(np.argmax(flat)), f.shape)   # first maximum in row-major order
    y0, y1 = _box(n, iy, BOX)
    x0, x1 = _box(n, ix, BOX)
    sub = flat[y0:y1, x0:x1]
    above = sub > threshold
    if not above[iy - y0, ix - x0]:
        return float(ix), float(iy), False, 0
    lab, _ = ndimage.label(above)                 # 4-connectivity
    patch = lab == lab[iy - y0, ix - x0]
    size = int(patch.sum())
    if size < min_size or size > max_size:
        return float(ix), float(iy), False, size
    w = sub[patch]
    yy, xx = np.nonzero(patch)
    return float((w * (xx + x0)).sum() / w.sum()), float((w * (yy + y0)).sum() / w.sum()), True, size


def moffat(p, x, y):
    """I0 (beta - 1) / (pi alpha^2) (1 + ((x - x0)^2 + (y - y0)^2) / alpha^2)^-beta + Bg
    with p = (I0, x0, y0, alpha, beta, Bg) (Sect. 3.1.2)."""
    i0, xc, yc, a, b, bg = p
    u = 1.0 + ((x - xc) ** 2 + (y - yc) ** 2) / a ** 2
    return i0 * (b - 1.0) / (np.pi * a ** 2) * u ** (-b) + bg


def moffat_fwhm(alpha, beta):
    """FWHM = 2 alpha sqrt(2^(1/beta) - 1) (Sect. 3.1.2)."""
    return 2.0 * alpha * np.sqrt(2.0 ** (1.0 / beta) - 1.0)


def fit_moffat(frame, xc, yc, half=16, saturation=np.inf):
    """Least-squares Moffat fit around (xc, yc) with MINPACK's
    Levenberg-Marquardt.  Returns (params, cost, n_pixels)."""
    from scipy.optimize import least_squares
    f = np.asarray(frame, dtype=np.float64)
    n = f.shape[0]
    y0, y1 = _box(n, int(round(yc)), 2 * half)
    x0, x1 = _box(n, int(round(xc)), 2 * half)
    sub = f[y0:y1, x0:x1]
    yy, xx = np.mgrid[y0:y1, x0:x1]
    ok = np.isfinite(sub) & (sub < saturation)
    border = np.zeros_like(ok)
    border[0, :] = border[-1, :] = border[:, 0] = border[:, -1] = True
    bg = float(sub[ok & border].mean()) if (ok & border).any() else 0.0
    a0, b0 = 2.5, 2.5
    peak = float(sub[ok].max()) - bg
    i0 = peak * np.pi * a0 ** 2 / (b0 - 1.0)
    xs, ys, vs = xx[ok].astype(np.float64), yy[ok].astype(np.float64), sub[ok]
    res = least_squares(lambda p: moffat(p, xs, ys) - vs, np.array([i0, xc, yc, a0, b0, bg]), method="lm",
                        xtol=1e-12, ftol=1e-12, gtol=1e-12, max_nfev=20000)
    return res.x, 0.5 * float(np.sum(res.fun ** 2)), int(ok.sum())


def register(cube, threshold, min_size, max_size, half=16, saturation=np.inf):
    """Per frame: centroid, Moffat fit, and the recentring shift.  Returns a
    dict of float64 arrays (x0, y0, i0, alpha, beta, bg, fwhm, dx, dy) and the
    centroid flags."""
    cube = np.asarray(cube)
    T, n, _ = cube.shape
    out = {k: np.zeros(T) for k in ("cx", "cy", "x0", "y0", "i0", "alpha", "beta", "bg", "fwhm", "dx", "dy")}
    out["centroid_ok"] = np.zeros(T, dtype=bool)
    for i in range(T):
        cx, cy, ok, _ = centroid(cube[i], threshold, min_size, max_size)
        p, _, _ = fit_moffat(cube[i], cx, cy, half, saturation)
        out["cx"][i], out["cy"][i], out["centroid_ok"][i] = cx, cy, ok
        out["i0"][i], out["x0"][i], out["y0"][i], out["alpha"][i], out["beta"][i], out["bg"][i] = p
        out["fwhm"][i] = moffat_fwhm(p[3], p[4])
        out["dx"][i], out["dy"][i] = n / 2.0 - p[1], n / 2.0 - p[2]
    return out
