"""Pins of the registration oracle (Sect. 3.1): parallactic angle against
spherical-trigonometry identities, centroid against symmetric blobs and the
patch rules, Moffat fit against noiseless images of known parameters."""

import numpy as np
import pytest

from oracle import registration as R


def test_parallactic_angle_special_cases():
    # at the pole every hour angle gives 0
    assert np.allclose(R.parallactic_angle(np.array([0.0, 3600.0, 20000.0]), 10.0, 35.0, 90.0), 0.0, atol=1e-12)
    # at transit: 0 south of the zenith (phi > delta), 180 north of it
    lst = 15.0 * 3600 / 15.0 * 2.0          # LST = 2 h = 7200 s -> h = 30 deg - RA
    assert abs(R.parallactic_angle(lst, 30.0, -60.0, -24.6)) < 1e-12
    assert abs(abs(R.parallactic_angle(lst, 30.0, 10.0, -24.6)) - 180.0) < 1e-12
    # on the equator, for a star on the celestial equator: +-90 away from transit
    assert abs(R.parallactic_angle(3600.0, 0.0, 0.0, 0.0) - 90.0) < 1e-12
    assert abs(R.parallactic_angle(-3600.0, 0.0, 0.0, 0.0) + 90.0) < 1e-12


def test_parallactic_angle_sine_rule():
    """Sine rule of the astronomical triangle: sin(q) sin(z) = cos(phi) sin(h),
    with z the zenith distance (cos z = sin phi sin delta + cos phi cos delta cos h)."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        lst, ra = rng.uniform(0, 86400), rng.uniform(0, 360)
        dec, lat = rng.uniform(-80, 80), rng.uniform(-70, 70)
        q = np.radians(R.parallactic_angle(lst, ra, dec, lat))
        h = np.radians(15 * lst / 3600 - ra)
        d, p = np.radians(dec), np.radians(lat)
        cz = np.sin(p) * np.sin(d) + np.cos(p) * np.cos(d) * np.cos(h)
        sz = np.sqrt(1 - cz * cz)
        assert abs(np.sin(q) * sz - np.cos(p) * np.sin(h)) < 1e-9
        # and the cosine relation: cos(q) sin(z) = cos(delta) sin(phi) - sin(delta) cos(phi) cos(h)
        assert abs(np.cos(q) * sz - (np.cos(d) * np.sin(p) - np.sin(d) * np.cos(p) * np.cos(h))) < 1e-9


def _blob(n, xc, yc, s, peak):
    yy, xx = np.mgrid[0:n, 0:n]
    return peak * np.exp(-((xx - xc) ** 2 + (yy - yc) ** 2) / (2 * s * s))


def test_centroid_symmetric_blob_and_rules():
    f = _blob(96, 40.0, 51.0, 2.0, 100.0) + _blob(96, 80.0, 20.0, 2.0, 60.0)   # a fainter second star
    x, y, ok, size = R.centroid(f, 5.0, 5, 500)
    assert ok and abs(x - 40.0) < 1e-12 and abs(y - 51.0) < 1e-12
    assert size == int((_blob(96, 40.0, 51.0, 2.0, 100.0) > 5.0).sum())
    # a patch outside the size range falls back to the brightest pixel
    x, y, ok, _ = R.centroid(f, 5.0, 5, 10)
    assert not ok and (x, y) == (40.0, 51.0)
    # a brightest pixel below the threshold: no patch
    x, y, ok, size = R.centroid(f, 1000.0, 1, 500)
    assert not ok and size == 0


def test_moffat_fwhm_is_half_maximum():
    p = np.array([5000.0, 0.0, 0.0, 2.2, 3.1, 7.0])
    r = R.moffat_fwhm(2.2, 3.1) / 2.0
    top = R.moffat(p, 0.0, 0.0) - 7.0
    assert abs((R.moffat(p, r, 0.0) - 7.0) - top / 2.0) < 1e-12 * top


@pytest.mark.parametrize("sat", [np.inf, 400.0])
def test_moffat_fit_recovers_noiseless_parameters(sat):
    n = 64
    true = np.array([20000.0, 31.3, 29.8, 2.7, 2.9, 12.0])
    yy, xx = np.mgrid[0:n, 0:n]
    f = R.moffat(true, xx, yy)
    f = np.where(f >= sat, sat, f)            # a saturated core, masked by the fit
    cx, cy, ok, _ = R.centroid(f, 30.0, 4, 4000)
    assert ok and abs(cx - 31.3) < 0.5 and abs(cy - 29.8) < 0.5
    p, cost, npx = R.fit_moffat(f, cx, cy, half=16, saturation=sat)
    assert np.allclose(p, true, rtol=1e-7, atol=1e-7), p
    assert cost < 1e-12
    assert npx == 32 * 32 - (int((R.moffat(true, xx, yy)[14:46, 15:47] >= sat).sum()) if np.isfinite(sat) else 0)


def test_register_shift_convention():
    n, T = 64, 3
    cube = np.stack([R.moffat(np.array([9000.0, 32.0 + d, 32.0 - d, 2.5, 2.5, 5.0]), *np.mgrid[0:n, 0:n][::-1])
                     for d in (0.0, 0.4, -1.3)])
    out = R.register(cube, 20.0, 4, 2000)
    assert np.allclose(out["dx"], [0.0, -0.4, 1.3], atol=1e-7)
    assert np.allclose(out["dy"], [0.0, 0.4, -1.3], atol=1e-7)
