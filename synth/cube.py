"""Seeded synthetic ADI cubes shaped like the paper's NACO / SPHERE stacks.

This module only models the *input*: a star image (Gaussian core plus a speckle
halo from a random-phase pupil), faint companions that follow the field
rotation, and photon / read noise.  It holds none of the reduction's own
arithmetic (no recentring shift, no shear, no median) and is the one piece of
code that both the oracle-based tests and the GPU path read from.

Recipe (stands in for the paper's real VLT/NACO, Gemini/NICI and VLT/SPHERE
sequences, which are not available):

* frame i holds the star at pixel (N/2, N/2) + o_i, where o_i are sub-pixel
  offsets; the recentring shift that undoes them is (dx, dy) = -o_i;
* star core: Gaussian of FWHM 4 px and peak 1e4 ADU;
* speckle halo: |FFT(pupil * phi)|^2 on a 2N grid, pupil = disc of diameter
  2N/4 (so lambda/D = 4 px), phi = zero-mean Gaussian random phase screen with
  an f^(-11/3) spectrum and 0.3 rad rms inside the pupil; scaled so that its
  azimuthal mean 10 px from the star is 1e-2 of the core peak.  The halo is
  fixed in the pupil frame: it follows the star offset (a tilt of the pupil
  field) but not the field rotation;
* companions: the same Gaussian, peak = contrast x 1e4, at
  (N/2, N/2) + o_i + R(parang_i) p_j (fake-companion injection that follows the
  field rotation, Sect. 4 and 4.2 of the paper);
* noise: Poisson (gain 1) on the non-negative image plus N(0, 5 ADU) read
  noise, except for the noiseless small configuration.

Random numbers come from NumPy ``Generator(PCG64(1510043310 + k))`` for
configuration k (host) and a seeded ``torch.Generator`` (device rendering).
"""

from dataclasses import dataclass, field
import math

import numpy as np

BASE_SEED = 1510043310
FWHM_PX = 4.0
SIGMA_PX = FWHM_PX / (2.0 * math.sqrt(2.0 * math.log(2.0)))
STAR_PEAK = 1.0e4
READ_NOISE = 5.0


def _next_pow2(v):
    p = 1
    while p < v:
        p *= 2
    return p


@dataclass
class CubeParams:
    """Per-cube parameters; ``dx, dy`` are the recentring shifts (-offsets)."""
    name: str
    T: int
    N: int
    P: int
    dx: np.ndarray
    dy: np.ndarray
    parang: np.ndarray                       # degrees
    companions: list = field(default_factory=list)   # (sep_px, pa_deg, contrast)
    noise: bool = True
    seed: int = BASE_SEED
    screen: np.ndarray = None                # phase screen on the 2N grid

    @property
    def nbytes(self):
        return self.T * self.N * self.N * 4


# ---------------------------------------------------------------------------
# Parameters of the named configurations
# ---------------------------------------------------------------------------

def _phase_screen(rng, M, rms=0.3):
    """Gaussian random phase with an f^(-11/3) power spectrum on an M x M grid,
    zero mean and ``rms`` radians inside the pupil disc of diameter M/4."""
    fx = np.fft.fftfreq(M)
    f2 = fx[None, :] ** 2 + fx[:, None] ** 2
    f2[0, 0] = np.inf
    amp = f2 ** (-11.0 / 12.0)
    noise = rng.normal(size=(M, M)) + 1j * rng.normal(size=(M, M))
    scr = np.fft.ifft2(noise * amp).real
    pupil = _pupil(M)
    scr = scr - scr[pupil].mean()
    scr = scr * (rms / scr[pupil].std())
    return scr


def _pupil(M):
    yy, xx = np.mgrid[0:M, 0:M]
    r = np.hypot(xx - M / 2.0, yy - M / 2.0)
    return r < M / 8.0


def make_params(config, seed=None, T=None, N=None, with_screen=True):
    """Parameters of configuration 1, 2 or 3 (optionally resized).

    1: 16 frames 128 x 128, offsets U(+-0.5), angles i.i.d. U(0, 30) deg sorted,
       one companion at 20 px, contrast 1e-3, noiseless.
    2: 1024 frames 512 x 512, offsets U(+-1), angles linear -30..+30 deg,
       companions 10 / 25 / 50 px at 1e-3 / 1e-4 / 1e-5, noise.
    3: 4096 frames 1024 x 1024, otherwise as 2.
    """
    config = int(config)
    if config not in (1, 2, 3):
        raise ValueError("configurations 1..3 are single cubes")
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + config if seed is None else seed))
    dT, dN = {1: (16, 128), 2: (1024, 512), 3: (4096, 1024)}[config]
    T = dT if T is None else int(T)
    N = dN if N is None else int(N)
    if config == 1:
        off = rng.uniform(-0.5, 0.5, size=(T, 2))
        ang = np.sort(rng.uniform(0.0, 30.0, size=T))
        comps = [(20.0, 0.0, 1e-3)]
        noise = False
    else:
        off = rng.uniform(-1.0, 1.0, size=(T, 2))
        ang = np.linspace(-30.0, 30.0, T)
        comps = [(10.0, 0.0, 1e-3), (25.0, 120.0, 1e-4), (50.0, 240.0, 1e-5)]
        noise = True
    seed_used = BASE_SEED + config if seed is None else seed
    screen = _phase_screen(rng, 2 * N) if with_screen else None
    return CubeParams(name="config%d" % config, T=T, N=N, P=_next_pow2(2 * N),
                      dx=-off[:, 0].copy(), dy=-off[:, 1].copy(), parang=ang,
                      companions=comps, noise=noise, seed=seed_used, screen=screen)


def make_batch_params(n_cubes=64, seed=None, sizes=(256, 512, 1024, 2048),
                      t_range=(32, 2048), with_screen=True):
    """Configuration 4: uneven cubes, T_j = round(exp U(ln 32, ln 2048)),
    N_j uniform over ``sizes``, otherwise generated as configuration 2."""
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + 4 if seed is None else seed))
    out = []
    for j in range(n_cubes):
        T = int(round(math.exp(rng.uniform(math.log(t_range[0]), math.log(t_range[1])))))
        N = int(sizes[rng.integers(len(sizes))])
        sub_seed = int(rng.integers(1 << 31))
        p = make_params(2, seed=sub_seed, T=T, N=N, with_screen=with_screen)
        p.name = "batch%d" % j
        out.append(p)
    return out


def make_arrivals(n_requests=1000, rate=20.0, seed=None):
    """Configuration 5: Poisson arrival times (seconds) at ``rate`` per second."""
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + 5 if seed is None else seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n_requests))


# ---------------------------------------------------------------------------
# Rendering
# ---------------------------------------------------------------------------

def _rot(deg):
    a = math.radians(deg)
    return math.cos(a), math.sin(a)


def companion_positions(p, i):
    """Frame-pixel (x, y) of every companion in frame i."""
    cx = p.N / 2.0 - p.dx[i]
    cy = p.N / 2.0 - p.dy[i]
    out = []
    for sep, pa, _ in p.companions:
        px, py = sep * math.cos(math.radians(pa)), sep * math.sin(math.radians(pa))
        c, s = _rot(p.parang[i])
        out.append((cx + c * px - s * py, cy + s * px + c * py))
    return out


def _halo_field(p):
    M = 2 * p.N
    pup = _pupil(M)
    return np.where(pup, np.exp(1j * p.screen) - 1.0, 0.0)


def _halo_scale(halo0, N):
    yy, xx = np.mgrid[0:N, 0:N]
    r = np.hypot(xx - N / 2.0, yy - N / 2.0)
    ring = (r > 9.5) & (r < 10.5)
    return 1e-2 * STAR_PEAK / max(halo0[ring].mean(), 1e-30)


def _halo_host(field_, N, ox, oy):
    M = field_.shape[0]
    u = np.fft.fftfreq(M) * M                       # integer pupil coordinates
    tilt = np.exp(2j * np.pi * (u[None, :] * ox + u[:, None] * oy) / M)
    img = np.abs(np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(field_) * tilt))) ** 2
    lo = M // 2 - N // 2
    return img[lo:lo + N, lo:lo + N]


def _gauss(N, x0, y0, peak):
    yy, xx = np.mgrid[0:N, 0:N]
    return peak * np.exp(-((xx - x0) ** 2 + (yy - y0) ** 2) / (2.0 * SIGMA_PX ** 2))


def render_host(p, frames=None, noise_seed=None):
    """Render frames on the host as a float32 array ``[len(frames), N, N]``."""
    idx = range(p.T) if frames is None else list(frames)
    N = p.N
    fld = _halo_field(p) if p.screen is not None else None
    scale = _halo_scale(_halo_host(fld, N, 0.0, 0.0), N) if fld is not None else 0.0
    rng = np.random.Generator(np.random.PCG64((p.seed if noise_seed is None else noise_seed) + 7))
    out = np.empty((len(idx), N, N), dtype=np.float32)
    for j, i in enumerate(idx):
        ox, oy = -p.dx[i], -p.dy[i]
        img = _gauss(N, N / 2.0 + ox, N / 2.0 + oy, STAR_PEAK)
        if fld is not None:
            img = img + scale * _halo_host(fld, N, ox, oy)
        for (x, y), (_, _, con) in zip(companion_positions(p, i), p.companions):
            img = img + _gauss(N, x, y, con * STAR_PEAK)
        if p.noise:
            img = rng.poisson(np.clip(img, 0.0, None)).astype(np.float64)
            img = img + rng.normal(0.0, READ_NOISE, size=img.shape)
        out[j] = img.astype(np.float32)
    return out


def render_device(p, device="cuda", chunk=16, out=None, noise_seed=None):
    """Render the whole cube on a torch device (harness-side generation for the
    large configurations).  Returns a float32 tensor ``[T, N, N]``."""
    import torch
    N, T, M = p.N, p.T, 2 * p.N
    if out is None:
        out = torch.empty((T, N, N), dtype=torch.float32, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed((p.seed if noise_seed is None else noise_seed) + 11)
    fld = torch.from_numpy(np.fft.ifftshift(_halo_field(p))).to(device=device, dtype=torch.complex64)
    scale = _halo_scale(_halo_host(_halo_field(p), N, 0.0, 0.0), N)
    u = torch.from_numpy(np.fft.fftfreq(M) * M).to(device=device, dtype=torch.float64)
    ar = torch.arange(N, device=device, dtype=torch.float64)
    lo = M // 2 - N // 2
    for s in range(0, T, chunk):
        e = min(T, s + chunk)
        ox = torch.from_numpy(-p.dx[s:e]).to(device)
        oy = torch.from_numpy(-p.dy[s:e]).to(device)
        ph = (u[None, None, :] * ox[:, None, None] + u[None, :, None] * oy[:, None, None]) * (2 * math.pi / M)
        tilt = torch.polar(torch.ones_like(ph), ph).to(torch.complex64)
        img = torch.fft.fftshift(torch.fft.fft2(fld[None] * tilt), dim=(-2, -1)).abs() ** 2
        img = (img[:, lo:lo + N, lo:lo + N] * scale).to(torch.float64)
        xx = ar[None, None, :]
        yy = ar[None, :, None]

        def g(x0, y0, peak):
            return peak * torch.exp(-((xx - x0[:, None, None]) ** 2 + (yy - y0[:, None, None]) ** 2)
                                    / (2.0 * SIGMA_PX ** 2))
        img = img + g(N / 2.0 + ox, N / 2.0 + oy, STAR_PEAK)
        for j, (_, _, con) in enumerate(p.companions):
            pos = np.array([companion_positions(p, i)[j] for i in range(s, e)])
            img = img + g(torch.from_numpy(pos[:, 0]).to(device), torch.from_numpy(pos[:, 1]).to(device),
                          con * STAR_PEAK)
        if p.noise:
            img = torch.poisson(img.clamp_min(0.0), generator=gen)
            img = img + READ_NOISE * torch.randn(img.shape, generator=gen, device=device, dtype=torch.float64)
        out[s:e] = img.to(torch.float32)
    return out
