"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the plausible oracle mistake it would catch.  None of them
re-types an oracle formula: they compare against an explicit DFT matrix, exact
permutations, closed forms, brute-force sorting or invariants.
"""

import math

import numpy as np
import pytest

import oracle as O
import synth


def _blobs(n, centres, sigma=3.0, amps=None):
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    f = np.zeros((n, n))
    amps = amps or [1.0] * len(centres)
    for (x0, y0), a in zip(centres, amps):
        f += a * np.exp(-((xx - x0) ** 2 + (yy - y0) ** 2) / (2 * sigma ** 2))
    return f


# --- transform convention ---------------------------------------------------

@pytest.mark.parametrize("P", [8, 16])
def test_fft2_equals_direct_dft(P):
    """np.fft follows exp(-2 pi i k n / P) (sign or scaling slip in the FFT
    convention)."""
    g = np.random.default_rng(P).normal(size=(P, P))
    F = np.exp(-2j * np.pi * np.outer(np.arange(P), np.arange(P)) / P)
    direct = F @ g @ F.T
    np.testing.assert_allclose(np.fft.fft2(g), direct, atol=1e-11 * P * P)


# --- Fourier shift -----------------------------------------------------------

@pytest.mark.parametrize("dx,dy", [(1, 0), (0, 1), (3, -2), (-5, 7), (0, 0)])
def test_integer_shift_is_exact_roll(dx, dy):
    """Integer shift = exact circular roll of the padded frame, content moving
    toward +index (shift sign, axis order)."""
    f = np.random.default_rng(1).normal(size=(12, 12))
    P = 32
    out = O.shift(f, dx, dy, P=P, keep_padded=True)
    ref = np.roll(np.pad(f, ((10, 10), (10, 10))), (dy, dx), axis=(0, 1))
    np.testing.assert_allclose(out, ref, atol=1e-12)


def _dirichlet(u, P):
    """Closed form D_P(u) = sin(pi u) / (P tan(pi u / P)), D_P(0) = 1, written
    independently of the oracle's helper."""
    u = np.asarray(u, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        v = np.sin(np.pi * u) / (P * np.tan(np.pi * u / P))
    return np.where(np.abs(u) < 1e-15, 1.0, v)


def test_gibbs_single_pixel_closed_form(golden):
    """The paper's Gibbs example: one pixel shifted by (0.3, 1.5) becomes the
    separable periodic sinc D_P(x - x0 - 0.3) D_P(y - y0 - 1.5) (Nyquist
    convention, shift sign, transposed axes)."""
    ex = golden["gibbs_single_pixel_shift"]
    n, P = 16, 32
    f = np.zeros((n, n))
    x0, y0 = 5, 9
    f[y0, x0] = 1.0
    out = O.shift(f, ex["dx"], ex["dy"], P=P, keep_padded=True)
    o = (P - n) // 2
    xs = np.arange(P)
    ref = np.outer(_dirichlet(xs - (y0 + o) - ex["dy"], P), _dirichlet(xs - (x0 + o) - ex["dx"], P))
    np.testing.assert_allclose(out, ref, atol=1e-13)
    # The oracle's own kernel helper agrees with the closed form too.
    np.testing.assert_allclose(O.dirichlet_kernel(xs - 3.7, P), _dirichlet(xs - 3.7, P), atol=1e-14)


@pytest.mark.parametrize("fx,fy,dx,dy", [(3, 1, 0.25, -0.6), (-5, 7, 1.7, 2.2), (0, 4, -3.3, 0.5)])
def test_band_limited_sinusoid_shift(fx, fy, dx, dy):
    """With no padding (P = N) a sinusoid of integer frequency |f| < N/2 shifts
    to its closed form cos(2 pi (fx (x - dx) + fy (y - dy)) / N + phi)."""
    n = 32
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    phi = 0.4
    f = np.cos(2 * np.pi * (fx * xx + fy * yy) / n + phi)
    out = O.shift(f, dx, dy, P=n)
    ref = np.cos(2 * np.pi * (fx * (xx - dx) + fy * (yy - dy)) / n + phi)
    np.testing.assert_allclose(out, ref, atol=1e-12)


def test_shift_identity_and_inverse(golden):
    """shift(0) is the identity; shift(-s) after shift(s) recovers a
    band-limited frame (the paper's double-shift test with (3.5, 2.7))."""
    ex = golden["double_shift"]
    n = 64
    f = _blobs(n, [(30.0, 33.0), (36.5, 28.0), (25.0, 38.0)], sigma=3.0, amps=[1.0, -0.5, 0.3])
    np.testing.assert_allclose(O.shift(f, 0.0, 0.0), f, atol=1e-13)
    back = O.shift(O.shift(f, ex["dx"], ex["dy"]), -ex["dx"], -ex["dy"])
    np.testing.assert_allclose(back, f, atol=1e-11)
    # and the forward shift moves the blob where the closed form says
    fwd = O.shift(f, ex["dx"], ex["dy"])
    ref = _blobs(n, [(30.0 + 3.5, 33.0 + 2.7), (36.5 + 3.5, 28.0 + 2.7), (25.0 + 3.5, 38.0 + 2.7)],
                 sigma=3.0, amps=[1.0, -0.5, 0.3])
    np.testing.assert_allclose(fwd, ref, atol=1e-10)


def test_shear_rows_delta_closed_form():
    """Row y of a sheared delta column is D_P(x - x0 - s[y]) (per-row shift,
    row/column transposition)."""
    P = 32
    g = np.zeros((P, P))
    x0 = 11
    g[:, x0] = np.arange(1, P + 1)
    s = np.linspace(-4.3, 5.1, P)
    out = O.shear_rows(g, s)
    xs = np.arange(P)
    ref = np.stack([(y + 1) * _dirichlet(xs - x0 - s[y], P) for y in range(P)])
    np.testing.assert_allclose(out, ref, atol=1e-12)
    out_c = O.shear_cols(g.T, s)
    np.testing.assert_allclose(out_c, ref.T, atol=1e-12)


# --- three-shear rotation ----------------------------------------------------

def test_rotate_zero_is_identity():
    f = np.random.default_rng(2).normal(size=(20, 20))
    np.testing.assert_allclose(O.rotate(f, 0.0), f, atol=1e-13)


def test_rotate_90_is_exact_permutation():
    """theta = 90 deg: content at c + (ux, uy) lands exactly at c + (-uy, ux)
    (rotation sense, shear factors tan(45) = sin(90) = 1)."""
    n, P = 16, 32
    f = np.random.default_rng(3).normal(size=(n, n))
    out = O.rotate(f, 90.0, P=P, keep_padded=True)
    g = np.pad(f, ((8, 8), (8, 8)))
    c = P // 2
    ref = np.zeros_like(g)
    for y in range(P):
        for x in range(P):
            ux, uy = x - c, y - c
            ref[(c + ux) % P, (c - uy) % P] = g[y, x]
    np.testing.assert_allclose(out, ref, atol=1e-12)


@pytest.mark.parametrize("theta", [180.0, -180.0])
def test_rotate_half_turn_is_point_reflection(theta):
    n, P = 10, 32
    f = np.random.default_rng(4).normal(size=(n, n))
    out = O.rotate(f, theta, P=P, keep_padded=True)
    g = np.pad(f, ((11, 11), (11, 11)))
    c = P // 2
    ref = np.zeros_like(g)
    for y in range(P):
        for x in range(P):
            ref[(2 * c - y) % P, (2 * c - x) % P] = g[y, x]
    np.testing.assert_allclose(out, ref, atol=1e-12)


@pytest.mark.parametrize("theta", [30.0, -45.0, 60.0, 120.0, -150.0, 350.0, -300.0, 420.0, 710.0])
def test_rotated_gaussian_closed_form(theta):
    """A Gaussian at c + p0 ends at c + R_theta p0, counter-clockwise in the
    (x right, y up) frame (rotation sign, shear order, centre)."""
    n = 64
    c = n // 2
    p0 = (9.0, -5.0)
    f = _blobs(n, [(c + p0[0], c + p0[1])], sigma=3.0)
    out = O.rotate(f, theta)
    a = math.radians(theta)
    q = (math.cos(a) * p0[0] - math.sin(a) * p0[1], math.sin(a) * p0[0] + math.cos(a) * p0[1])
    ref = _blobs(n, [(c + q[0], c + q[1])], sigma=3.0)
    np.testing.assert_allclose(out, ref, atol=1e-9)


@pytest.mark.parametrize("theta", [0.0, 11.3, -30.0, 135.0, -170.0, 89.0])
def test_rotation_is_periodic_in_360_degrees(theta):
    """R_theta has period 360 deg, so theta + 360 k turns the frame like theta
    (a missing angle reduction sends tan(theta/2) toward infinity and wraps
    the shears round the padded frame)."""
    f = _blobs(48, [(30.0, 20.0), (18.0, 27.0)], sigma=3.0, amps=[1.0, -0.5])
    ref = O.rotate(f, theta)
    for k in (1, -1, 2, -3):
        np.testing.assert_allclose(O.rotate(f, theta + 360.0 * k), ref, atol=1e-10)


def test_full_turn_is_identity():
    """theta = 360 deg and -720 deg leave the frame as it is."""
    f = np.random.default_rng(12).normal(size=(20, 20))
    np.testing.assert_allclose(O.rotate(f, 360.0), f, atol=1e-13)
    np.testing.assert_allclose(O.rotate(f, -720.0), f, atol=1e-13)


def test_double_rotation_recovers_input(golden):
    """The paper's double-rotation test: rotate by 11.3 deg and back; a
    band-limited frame inside the inscribed disc is recovered."""
    th = golden["double_rotation"]["theta_deg"]
    n = 64
    f = _blobs(n, [(30.0, 34.0), (40.0, 25.0), (22.0, 30.0)], sigma=3.0, amps=[1.0, 0.7, -0.4])
    back = O.rotate(O.rotate(f, th), -th)
    np.testing.assert_allclose(back, f, atol=1e-9)


def test_double_rotation_white_noise_residual_is_high_frequency(golden):
    """On white noise the double rotation loses only content near the band
    edge: the residual has (almost) no power at low spatial frequency."""
    th = golden["double_rotation"]["theta_deg"]
    n = 64
    f = np.zeros((n, n))
    f[16:48, 16:48] = np.random.default_rng(5).normal(size=(32, 32))
    res = O.rotate(O.rotate(f, th), -th) - f
    R = np.abs(np.fft.fft2(res))
    F = np.abs(np.fft.fft2(f))
    k = np.hypot(*np.meshgrid(np.fft.fftfreq(n), np.fft.fftfreq(n)))
    low = k < 0.2
    assert R[low].sum() < 0.05 * F[low].sum()


# --- flux and energy ---------------------------------------------------------

def test_flux_and_energy():
    """The padded sum is invariant (each line keeps its DC term); the energy
    does not grow (|phasor| <= 1)."""
    rng = np.random.default_rng(6)
    f = rng.normal(size=(24, 24)) + 3.0
    P = 64
    g = O.pad(f, P)
    for out in (O.shift(f, 0.37, -1.8, P=P, keep_padded=True),
                O.rotate(f, 23.0, P=P, keep_padded=True),
                O.rotate(f, -71.0, P=P, keep_padded=True)):
        assert abs(out.sum() - g.sum()) < 1e-10 * np.abs(g).sum()
        assert np.linalg.norm(out) <= np.linalg.norm(g) * (1 + 1e-12)


def test_flip180_involution():
    g = np.random.default_rng(7).normal(size=(16, 16))
    np.testing.assert_array_equal(O.flip180(O.flip180(g)), g)
    assert O.flip180(g)[8 + 3, 8 - 2] == g[8 - 3, 8 + 2]


# --- median ------------------------------------------------------------------

def _brute_median(vals):
    s = sorted((float(v) for v in vals), key=lambda v: (v, math.copysign(1.0, v)))
    T = len(s)
    lo, hi = np.float32(s[(T - 1) // 2]), np.float32(s[T // 2])
    return np.float32((lo + hi) * np.float32(0.5))


@pytest.mark.parametrize("T", [1, 2, 3, 16, 17, 1024])
def test_median_f32_brute_force(T):
    """Exact order statistics, even-T midpoint in float32, ties and signed
    zeros in totalOrder (off-by-one rank, wrong midpoint, float64 midpoint)."""
    rng = np.random.default_rng(T)
    st = rng.normal(size=(T, 5, 7)).astype(np.float32)
    st[:, 0, 0] = 0.0
    st[: T // 2, 0, 0] = -0.0
    st[:, 1, :] = np.round(st[:, 1, :] * 2) / 2          # many ties
    st[:, 2, 0] = np.float32(1e30)
    st[:, 2, 1] = rng.choice([np.float32(1.0000001), np.float32(1.0)], size=T)
    med = O.median_f32(st)
    for y in range(5):
        for x in range(7):
            b = _brute_median(st[:, y, x])
            assert med[y, x].tobytes() == b.tobytes(), (T, y, x)


def test_median_f64_matches_numpy():
    st = np.random.default_rng(8).normal(size=(10, 4, 4))
    np.testing.assert_array_equal(O.median_f64(st), np.median(st, axis=0))
    np.testing.assert_array_equal(O.median_f64(st[:9]), np.median(st[:9], axis=0))


# --- end-to-end ADI ----------------------------------------------------------

def test_adi_identical_frames_give_zero():
    f = np.random.default_rng(9).normal(size=(16, 16))
    cube = np.stack([f] * 5)
    z = np.zeros(5)
    res = O.adi_reduce(cube, z + 0.3, z - 0.2, z)
    assert np.all(res["final"] == 0.0)


def test_adi_recovers_companion_position():
    """Static PSF + companion that follows the field rotation: the final
    image peaks within 0.5 px of the injected position (derotation sign)."""
    n, T = 48, 9
    c = n // 2
    ang = np.linspace(0.0, 160.0, T)      # wide enough that the median PSF
    p0 = np.array([13.0, 6.0])            # does not absorb the companion
    rng = np.random.default_rng(10)
    off = rng.uniform(-0.5, 0.5, size=(T, 2))
    cube = []
    for i in range(T):
        a = math.radians(ang[i])
        q = (math.cos(a) * p0[0] - math.sin(a) * p0[1], math.sin(a) * p0[0] + math.cos(a) * p0[1])
        cube.append(_blobs(n, [(c + off[i, 0], c + off[i, 1]),
                               (c + off[i, 0] + q[0], c + off[i, 1] + q[1])],
                           sigma=3.0, amps=[100.0, 1.0]))
    res = O.adi_reduce(np.stack(cube), -off[:, 0], -off[:, 1], ang)
    fin = res["final"]
    yy, xx = np.mgrid[0:n, 0:n]
    y, x = np.unravel_index(np.argmax(fin), fin.shape)
    w = np.clip(fin, 0, None) * (np.hypot(xx - x, yy - y) < 3)
    cx, cy = (w * xx).sum() / w.sum(), (w * yy).sum() / w.sum()
    assert math.hypot(cx - (c + p0[0]), cy - (c + p0[1])) < 0.5


# ---------------------------------------------------------------------------
# Per-frame PSF selection (Sect. 3.3: time separation below t_max, field
# rotation above alpha_min)
# ---------------------------------------------------------------------------

def test_alpha_min_chord_angle():
    # a point at radius 10 px moving 2 x 4 px along its arc: chord 8 px -> 2 arcsin(0.4)
    assert abs(O.alpha_min_deg(2, 4.0, 10.0) - 47.15635696) < 1e-6
    assert O.alpha_min_deg(0, 4.0, 10.0) == 0.0
    # small-angle limit: the arc length n FWHM / r_min radians
    assert abs(O.alpha_min_deg(1, 0.01, 100.0) - np.degrees(1e-4)) < 1e-10


def test_select_frames_by_hand():
    # frames every 1 s, 2 degrees apart: frame i takes k with |k - i| < 3.5 and 2|k - i| > 3
    t = np.arange(8.0)
    a = 2.0 * np.arange(8.0)
    sel = O.select_frames(t, a, 3.5, 3.0)
    for i in range(8):
        want = {k for k in range(8) if 2 <= abs(k - i) <= 3}
        assert set(np.flatnonzero(sel[i])) == want, i
    # nothing rotates enough: every frame falls back to all frames
    sel = O.select_frames(t, np.zeros(8), 10.0, 1.0)
    assert sel.all()


def test_select_row_by_hand():
    # the same frames one row at a time
    t = np.arange(8.0)
    a = 2.0 * np.arange(8.0)
    for i in range(8):
        want = {k for k in range(8) if 2 <= abs(k - i) <= 3}
        assert set(np.flatnonzero(O.select_row(t, a, 3.5, 3.0, i))) == want, i
        assert O.select_row(t, np.zeros(8), 10.0, 1.0, i).all()
    # a frame alone in time falls back while its neighbours select each other
    t2 = np.array([0.0, 1.0, 2.0, 100.0])
    a2 = np.array([0.0, 5.0, 10.0, 0.0])
    assert list(O.select_row(t2, a2, 3.0, 4.0, 3)) == [True] * 4
    assert list(O.select_row(t2, a2, 3.0, 4.0, 0)) == [False, True, True, False]


def test_window_median_brute_force():
    rng = np.random.default_rng(12)
    st = rng.normal(size=(11, 3, 4)).astype(np.float32)
    st[:, 0, 0] = 1.0                                   # ties
    sel = rng.random((11, 11)) < 0.5
    sel[3] = False
    sel[3, 5] = True                                    # a single frame
    got = O.median_window_f32(st, sel)
    for i in range(11):
        vals = np.sort(st[sel[i]].astype(np.float64), axis=0)
        K = vals.shape[0]
        want = ((vals[(K - 1) // 2] + vals[K // 2]) * 0.5).astype(np.float32)
        assert np.array_equal(got[i], want)
    assert np.array_equal(got[3], st[5])


def test_window_reduces_to_classical_adi():
    """With no time limit and a negative minimum rotation every frame selects
    all frames, and the reduction is the classical one."""
    p = synth.make_params(1, T=8, N=32)
    cube = synth.render_host(p)
    t = np.arange(p.T, dtype=np.float64)
    a = O.adi_reduce(cube, p.dx, p.dy, p.parang)
    b = O.adi_reduce_window(cube, p.dx, p.dy, p.parang, t, np.inf, -1.0)
    assert np.array_equal(b["psf"][3], a["psf"])
    assert np.allclose(b["final"], a["final"], rtol=0, atol=1e-12 * np.abs(a["psf"]).max())


def test_window_adi_keeps_more_companion_flux():
    """The selection keeps frames where the companion sits at the same place
    out of its PSF, so less of it is subtracted than with the all-frames PSF
    (the motivation of the per-frame PSF in Sect. 3.3)."""
    T, N = 24, 48
    ang = np.linspace(0.0, 120.0, T)
    yy, xx = np.mgrid[0:N, 0:N]
    c = N / 2.0
    cube = np.zeros((T, N, N))
    for i in range(T):
        cube[i] += 100.0 * np.exp(-((xx - c) ** 2 + (yy - c) ** 2) / (2 * 3.0 ** 2))
        th = np.radians(ang[i])
        px, py = c + 10.0 * np.cos(th), c + 10.0 * np.sin(th)
        cube[i] += 5.0 * np.exp(-((xx - px) ** 2 + (yy - py) ** 2) / (2 * 1.5 ** 2))
    z = np.zeros(T)
    t = np.arange(T, dtype=np.float64)
    amin = O.alpha_min_deg(1.5, 3.5, 10.0)
    w = O.adi_reduce_window(cube.astype(np.float32), z, z, ang, t, 100.0, amin)
    a = O.adi_reduce(cube.astype(np.float32), z, z, ang)
    ref = (int(round(c)), int(round(c + 10)))              # companion at angle 0 after derotation
    assert w["final"][ref[0], ref[1]] > a["final"][ref[0], ref[1]]
    assert w["final"][ref[0], ref[1]] > 0.6 * 5.0
