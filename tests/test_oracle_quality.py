"""CPU pins of the image-quality oracle (Sect. 4.1: double shift and double
rotation, residual RMS in annuli).  Each test checks the oracle against a fact
from outside it: lattice-point counts of the sum-of-two-squares function,
closed-form ring averages, exact round trips of band-limited blobs, and the
paper's qualitative result against scipy's independent spline interpolation."""

import numpy as np
import pytest

from oracle import quality as Q


def test_ring_counts_are_sums_of_two_square_representations():
    # pixels with k^2 <= x^2 + y^2 < (k + 1)^2 around an integer centre:
    # r2(0) = 1; r2(1) + r2(2) = 8; r2(4) + r2(5) + r2(8) = 16;
    # r2(9) + r2(10) + r2(13) = 20; r2(16) + r2(17) + r2(18) + r2(20) = 24
    _, counts = Q.annular_rms(np.ones((32, 32)), None, 1.0, 5)
    assert counts.tolist() == [1, 8, 16, 20, 24]
    # width 2 merges pairs of unit rings: [0, 4) and [4, 16)
    _, counts2 = Q.annular_rms(np.ones((32, 32)), None, 2.0, 2)
    assert counts2.tolist() == [1 + 8, 16 + 20]


def test_constant_and_self_difference():
    a = np.full((40, 40), -3.25)
    rms, counts = Q.annular_rms(a, None, 1.5, 40)
    full = counts > 0
    assert np.all(np.abs(rms[full] - 3.25) < 1e-15)
    assert np.all(np.isnan(rms[~full]))                  # rings past the corners are empty
    rms0, _ = Q.annular_rms(a, a, 1.5, 10)
    assert np.all(rms0 == 0.0)
    assert counts.sum() == 40 * 40                         # every pixel in exactly one ring


def test_ring_averages_of_closed_forms():
    n = 256
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    phi = np.arctan2(yy - n / 2, xx - n / 2)
    d = np.hypot(xx - n / 2, yy - n / 2)
    rms, _ = Q.annular_rms(np.cos(2 * phi), None, 4.0, 30)
    assert np.all(np.abs(rms[5:30] - np.sqrt(0.5)) < 0.02)    # mean of cos^2 over a circle is 1/2
    rd, _ = Q.annular_rms(d, None, 1.0, 100)
    k = np.arange(100)
    assert np.all((rd >= k) & (rd < k + 1))                   # sqrt(mean d^2) stays inside its ring


def test_round_trips_of_a_band_limited_blob_are_exact():
    n = 64
    yy, xx = np.mgrid[0:n, 0:n]
    g = np.exp(-((xx - 32) ** 2 + (yy - 32) ** 2) / 18.0)
    r1, _ = Q.annular_rms(Q.double_shift(g, 3.5, 2.7), g, 1.0, 24)     # the paper's shift
    r2, _ = Q.annular_rms(Q.double_rotate(g, 11.3), g, 1.0, 24)        # the paper's angle
    assert np.nanmax(r1) < 1e-12 and np.nanmax(r2) < 1e-12


@pytest.mark.parametrize("kind", ["shift", "rotate"])
def test_fourier_residuals_below_spline_residuals(kind):
    """The paper's result: spline interpolation acts as a low-pass filter, so
    its round-trip residual is far larger than the Fourier one."""
    n = 64
    yy, xx = np.mgrid[0:n, 0:n]
    rng = np.random.default_rng(11)
    img = 1000.0 * np.exp(-((xx - 32) ** 2 + (yy - 32) ** 2) / 18.0) + rng.normal(0.0, 1.0, (n, n))
    if kind == "shift":
        f, s = Q.double_shift(img, 3.5, 2.7), Q.spline_double_shift(img, 3.5, 2.7)
    else:
        f, s = Q.double_rotate(img, 11.3), Q.spline_double_rotate(img, 11.3)
    rf, _ = Q.annular_rms(f, img, 2.0, 12)
    rs, _ = Q.annular_rms(s, img, 2.0, 12)
    assert np.all(rf[1:12] * 3.0 < rs[1:12])
