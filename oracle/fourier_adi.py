"""Plain FP64 CPU oracle of the GRAPHIC Fourier ADI hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import this
module.  The product path (the HIP library and its Python binding) never
imports, calls or links it, and it shares no code, table or helper with that
path.

Source: Hagelberg, Segransan, Udry & Wildi, "The Geneva Reduction and Analysis
Pipeline for High-contrast Imaging of planetary Companions", MNRAS 2016
(arXiv:1510.04331).  Every function names the passage it follows.

Everything is evaluated in float64 with NumPy's FFT (pocketfft).  Nothing is
blocked, fused or reordered beyond what the cited definitions state, so the code
can be checked against the paper by eye.

Conventions (the paper leaves these open; the readings are fixed here once):

* Frames are ``[row][column]`` arrays; ``x`` is the column index and ``y`` the
  row index, both increasing; positive angles turn the content
  counter-clockwise in that (x right, y up) frame.
* ``pad`` places an N x N frame at offset ``(P - N) // 2`` of a P x P zero
  array, so the rotation and recentring centre ``c = P // 2`` is pixel
  ``(N // 2, N // 2)`` of the frame.  ``P`` defaults to the smallest power of
  two that is at least 2N (Sect. 3.3.1: the frames are zero-padded to at least
  double size).
* A shift ``s`` moves content toward larger index: ``out[n] = in[n - s]``.
* The Nyquist bin of an even-length transform gets the real, symmetric phasor
  ``cos(pi s)``.  With it every one-dimensional shift maps real lines to real
  lines and an integer shift is an exact circular roll.
"""

import math

import numpy as np

__all__ = [
    "padded_size", "pad", "crop", "signed_freq", "phasor", "shift",
    "shear_rows", "shear_cols", "flip180", "reduce_angle", "rotate",
    "median_f32", "median_f64", "adi_reduce", "dirichlet_kernel",
    "alpha_min_deg", "select_frames", "select_row", "median_window_f32", "adi_reduce_window",
]


# ---------------------------------------------------------------------------
# Geometry of the zero-padded working frame (Sect. 3.3.1, last paragraph, and
# Sect. 3.4, last paragraph: operations run on at least double-sized frames).
# ---------------------------------------------------------------------------

def padded_size(n):
    """Smallest power of two P with P >= 2 n (the default working size)."""
    p = 1
    while p < 2 * n:
        p *= 2
    return p


def _offset(n, P):
    return (P - n) // 2


def pad(f, P):
    """Place the N x N frame ``f`` at offset (P-N)//2 of a P x P zero frame."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    if f.shape != (n, n) or P < n:
        raise ValueError("pad expects a square frame no larger than P")
    g = np.zeros((P, P), dtype=np.float64)
    o = _offset(n, P)
    g[o:o + n, o:o + n] = f
    return g


def crop(g, n):
    """Inverse of :func:`pad`: the N x N window at offset (P-N)//2."""
    P = g.shape[0]
    o = _offset(n, P)
    return g[o:o + n, o:o + n].copy()


# ---------------------------------------------------------------------------
# The translation phasor (Sect. 3.3.1: a shift multiplies the transform by a
# linear phase; Fourier transform defined with exp(-i 2 pi nu x)).
# ---------------------------------------------------------------------------

def signed_freq(P):
    """Signed frequency index of DFT bin k: k for k < P/2, k - P above."""
    k = np.arange(P)
    return np.where(k < P // 2, k, k - P)


def phasor(P, s):
    """Phasor that delays a length-P periodic line by ``s`` samples.

    ``phi[k] = exp(-2 pi i kt s / P)`` with ``kt`` the signed frequency; for
    even P the Nyquist bin ``k = P/2`` is ``cos(pi s)``, the mean of the two
    exponentials at +P/2 and -P/2.
    """
    kt = signed_freq(P).astype(np.float64)
    phi = np.exp(-2j * np.pi * kt * float(s) / P)
    if P % 2 == 0:
        phi[P // 2] = np.cos(np.pi * float(s))
    return phi


def dirichlet_kernel(u, P):
    """Periodic band-limited interpolation kernel of the shift.

    A length-P line shifted by ``s`` with :func:`phasor` equals the circular
    convolution of the line with ``D_P(n - s)``, where
    ``D_P(u) = sin(pi u) / (P tan(pi u / P))`` and ``D_P(0) = 1``.  Used as a
    closed form in the tests; the shift itself never calls it.
    """
    u = np.asarray(u, dtype=np.float64)
    out = np.ones_like(u)
    nz = np.abs(np.sin(np.pi * u / P)) > 1e-300
    out[nz] = np.sin(np.pi * u[nz]) / (P * np.tan(np.pi * u[nz] / P))
    return out


# ---------------------------------------------------------------------------
# Fourier shift (Sect. 3.3.1, 2-D shift equation): FT, multiply by the phasor
# exp(-i 2 pi (nu_x a + nu_y b)), inverse FT, on the zero-padded frame.
# ---------------------------------------------------------------------------

def _real_part(z, what):
    # With the symmetric Nyquist phasor the product spectrum is Hermitian, so
    # the exact inverse is real; what is left is float64 rounding of the
    # transforms (about 1e-15 of the peak).  The guard sits at 1e-9 of the
    # peak so that it only trips on a broken phasor, never on rounding.
    re = z.real
    scale = max(np.max(np.abs(re)), 1e-300)
    if np.max(np.abs(z.imag)) > 1e-9 * scale:
        raise AssertionError(what + ": imaginary residue above rounding level")
    return re


def shift(f, dx, dy, P=None, keep_padded=False):
    """Move the content of frame ``f`` by ``(dx, dy)`` pixels.

    Pads to P x P, takes the 2-D FFT, multiplies by the separable phasor
    ``phasor(P, dy)[:, None] * phasor(P, dx)[None, :]`` and inverts.  Returns
    the N x N window, or the whole P x P frame when ``keep_padded``.
    """
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    P = padded_size(n) if P is None else int(P)
    g = pad(f, P)
    G = np.fft.fft2(g)
    G = G * phasor(P, dy)[:, None] * phasor(P, dx)[None, :]
    out = _real_part(np.fft.ifft2(G), "shift")
    return out if keep_padded else crop(out, n)


# ---------------------------------------------------------------------------
# Three-shear rotation (Sect. 3.4): R_theta = S_x(-tan(theta/2)) S_y(sin theta)
# S_x(-tan(theta/2)); each shear is a one-dimensional FT along one axis, a
# phase ramp proportional to the other coordinate, and an inverse FT.
# ---------------------------------------------------------------------------

def shear_rows(g, s):
    """Shift row y of the P x P frame ``g`` along x by ``s[y]``."""
    g = np.asarray(g, dtype=np.float64)
    P = g.shape[1]
    F = np.fft.fft(g, axis=1)
    F = F * np.stack([phasor(P, sy) for sy in s])
    return _real_part(np.fft.ifft(F, axis=1), "shear_rows")


def shear_cols(g, s):
    """Shift column x of the P x P frame ``g`` along y by ``s[x]``."""
    return shear_rows(np.asarray(g).T, s).T


def flip180(g):
    """Exact half-turn about the centre c = P//2: g'[c + u] = g[c - u mod P]."""
    P = g.shape[0]
    idx = (-np.arange(P)) % P          # c + u -> c - u with c = P/2, mod P
    return g[idx][:, idx]


def reduce_angle(theta_deg):
    """The angle in [-180, 180] degrees with the same rotation matrix.

    R_theta (Sect. 3.4) is periodic in theta with period 360 degrees, while
    tan(theta/2) of the shear factors is not bounded on a period: the angle is
    first brought to the period around zero (IEEE remainder, exact in float64).
    """
    return math.remainder(float(theta_deg), 360.0)


def rotate(f, theta_deg, P=None, keep_padded=False, padded_input=False):
    """Turn the content of ``f`` counter-clockwise by ``theta_deg`` about c.

    Content at ``c + u`` ends at ``c + R_theta u``.  The angle is first
    reduced to [-180, 180] degrees (:func:`reduce_angle`).  The three shears
    act in the order x, y, x: rows move by ``-tan(theta/2) (y - c)``, then
    columns by ``sin(theta) (x - c)``, then rows again by
    ``-tan(theta/2) (y - c)`` (Sect. 3.4, shear equations).  For |theta| > 90
    degrees an exact half-turn is applied first and theta is reduced by 180
    degrees, so tan(theta/2) stays bounded.
    """
    f = np.asarray(f, dtype=np.float64)
    if padded_input:
        g = f.copy()
        P = g.shape[0]
        n = None
    else:
        n = f.shape[0]
        P = padded_size(n) if P is None else int(P)
        g = pad(f, P)
    th = reduce_angle(theta_deg)
    if abs(th) > 90.0:
        g = flip180(g)
        th = th - 180.0 * np.sign(th)
    rad = np.deg2rad(th)
    t = np.tan(rad / 2.0)
    s = np.sin(rad)
    u = np.arange(P, dtype=np.float64) - P // 2
    g = shear_rows(g, -t * u)
    g = shear_cols(g, s * u)
    g = shear_rows(g, -t * u)
    if keep_padded or n is None:
        return g
    return crop(g, n)


# ---------------------------------------------------------------------------
# Per-pixel median (Sect. 3.3: the classical ADI reference PSF is the median
# of the recentred frames; Sect. 3.4: the derotated frames are merged).
# ---------------------------------------------------------------------------

def _total_order_key(a32):
    """Map float32 values to uint32 keys whose unsigned order is IEEE totalOrder."""
    b = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32)
    return np.where(b & np.uint32(0x80000000), ~b, b | np.uint32(0x80000000))


def _from_total_order_key(k):
    k = np.asarray(k, dtype=np.uint32)
    b = np.where(k & np.uint32(0x80000000), k & np.uint32(0x7FFFFFFF), ~k)
    return b.astype(np.uint32).view(np.float32)


def median_f32(stack):
    """Exact float32 median over axis 0 of a NaN-free float32 stack.

    Values are ordered by IEEE totalOrder (-0 before +0).  With T values,
    ``lo`` is the element of rank (T-1)//2 and ``hi`` the one of rank T//2;
    the result is ``(lo + hi) * 0.5`` evaluated in float32 with
    round-to-nearest-even, which is ``lo`` itself when T is odd.
    """
    st = np.asarray(stack, dtype=np.float32)
    T = st.shape[0]
    if T < 1:
        raise ValueError("median of an empty stack")
    keys = np.sort(_total_order_key(st), axis=0)
    lo = _from_total_order_key(keys[(T - 1) // 2])
    hi = _from_total_order_key(keys[T // 2])
    with np.errstate(over="ignore"):       # |lo + hi| may round to inf in float32
        return ((lo + hi) * np.float32(0.5)).astype(np.float32)


def median_f64(stack):
    """Float64 median over axis 0: mean of the two middle order statistics."""
    st = np.sort(np.asarray(stack, dtype=np.float64), axis=0)
    T = st.shape[0]
    if T < 1:
        raise ValueError("median of an empty stack")
    return 0.5 * (st[(T - 1) // 2] + st[T // 2])


# ---------------------------------------------------------------------------
# Classical ADI reduction in the paper's order (Sect. 3: registration, then
# PSF subtraction with the Fourier recentring shift, then derotation and
# merge).  The reference PSF here is the median of all recentred frames.
# ---------------------------------------------------------------------------

def _shift_job(a):
    return shift(*a)


def _rotate_job(a):
    return rotate(*a)


def adi_reduce(cube, dx, dy, parang_deg, P=None, map_fn=map):
    """Classical ADI (Sect. 3.3 and 3.4): shift every frame, take the median
    PSF, subtract it, derotate by -parang, median combine.

    ``map_fn`` maps the per-frame operations (the built-in ``map`` by default;
    a process pool's ``map`` spreads the frames over cores, as the paper's
    frame-parallel scheme does).  Returns a dict with ``final`` (N x N),
    ``psf`` (N x N), ``shifted`` and ``derotated`` (T x N x N), all float64.
    """
    cube = np.asarray(cube, dtype=np.float64)
    T, n, _ = cube.shape
    shifted = np.stack(list(map_fn(_shift_job, [(cube[i], float(dx[i]), float(dy[i]), P) for i in range(T)])))
    psf = median_f64(shifted)
    derot = np.stack(list(map_fn(_rotate_job, [(shifted[i] - psf, -float(parang_deg[i]), P) for i in range(T)])))
    final = median_f64(derot)
    return {"final": final, "psf": psf, "shifted": shifted, "derotated": derot}


# ---------------------------------------------------------------------------
# Per-frame reference PSF with the paper's frame selection (Sect. 3.3, the
# two conditions on time separation and field rotation): frame i gets its own
# PSF from the frames k with |t_k - t_i| < t_max and |alpha_k - alpha_i| >
# alpha_min, combined without coefficients (here by the median, as for the
# classical PSF).
#
# Readings: the minimum rotation is printed as 2 sin(n FWHM / (2 r_min)); the
# angle at which a point at radius r_min moves by n FWHM along its arc is the
# chord angle 2 arcsin(n FWHM / (2 r_min)), which is taken here.  When no frame
# meets both conditions (the paper is silent), the frame falls back to the
# classical PSF, the median of all frames.
# ---------------------------------------------------------------------------

def alpha_min_deg(n_fwhm, fwhm, r_min):
    """Minimum field rotation in degrees: 2 arcsin(n_fwhm * fwhm / (2 r_min))."""
    x = n_fwhm * fwhm / (2.0 * r_min)
    if not 0.0 <= x <= 1.0:
        raise ValueError("n_fwhm * fwhm must lie in [0, 2 r_min]")
    return float(np.degrees(2.0 * np.arcsin(x)))


def select_frames(times, parang_deg, t_max, alpha_min):
    """Boolean [T, T] matrix: row i marks the frames that build frame i's PSF
    (Sect. 3.3 selection), with the classical all-frames fallback."""
    t = np.asarray(times, dtype=np.float64)
    a = np.asarray(parang_deg, dtype=np.float64)
    sel = (np.abs(t[None, :] - t[:, None]) < t_max) & (np.abs(a[None, :] - a[:, None]) > alpha_min)
    empty = ~sel.any(axis=1)
    sel[empty, :] = True
    return sel


def select_row(times, parang_deg, t_max, alpha_min, i):
    """Row i of ``select_frames`` alone (Sect. 3.3 selection with the
    all-frames fallback), in O(T): for sequences too long for the T x T
    matrix."""
    t = np.asarray(times, dtype=np.float64)
    a = np.asarray(parang_deg, dtype=np.float64)
    row = (np.abs(t - t[i]) < t_max) & (np.abs(a - a[i]) > alpha_min)
    if not row.any():
        row[:] = True
    return row


def median_window_f32(stack, sel):
    """Float32 per-frame medians: out[i] = median_f32(stack[sel[i]])."""
    st = np.asarray(stack, dtype=np.float32)
    return np.stack([median_f32(st[np.asarray(sel[i], bool)]) for i in range(st.shape[0])])


def adi_reduce_window(cube, dx, dy, parang_deg, times, t_max, alpha_min, P=None, map_fn=map):
    """ADI with a per-frame PSF (Sect. 3.3): shift every frame, subtract from
    frame i the median of its selected frames, derotate by -parang, median
    combine.  Returns ``final``, ``psf`` (T x N x N), ``shifted``,
    ``derotated`` and the selection ``sel``, all float64 except ``sel``."""
    cube = np.asarray(cube, dtype=np.float64)
    T, n, _ = cube.shape
    sel = select_frames(times, parang_deg, t_max, alpha_min)
    shifted = np.stack(list(map_fn(_shift_job, [(cube[i], float(dx[i]), float(dy[i]), P) for i in range(T)])))
    psf = np.stack([median_f64(shifted[sel[i]]) for i in range(T)])
    derot = np.stack(list(map_fn(_rotate_job, [(shifted[i] - psf[i], -float(parang_deg[i]), P)
                                               for i in range(T)])))
    final = median_f64(derot)
    return {"final": final, "psf": psf, "shifted": shifted, "derotated": derot, "sel": sel}

