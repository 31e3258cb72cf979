"""GPU: stacks deeper than 4096 frames (the paper's sequences run to about
100,000 frames).  Their per-pixel medians take the streaming radix select;
the bar is the same as for shallow stacks: bit-exact against the oracle's
float32 median (IEEE totalOrder, ties, signed zeros, subnormals, even and odd
T), and the ADI reduction within 1e-5 of the oracle's PSF norm."""

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_04331_amd  # noqa: F401
    return torch, torch.device("cuda:0")


def _stack(T, N, seed):
    rng = np.random.default_rng(seed)
    st = (rng.normal(size=(T, N, N)) * 3 + 50).astype(np.float32)
    st[:, 0, 0] = 5.0                                        # all equal
    st[:, 0, 1] = 5.0
    st[T // 3, 0, 1] = 7.0                                   # all but one equal
    st[:, 0, 2] = np.where(np.arange(T) % 2 == 0, -1.5, 2.5).astype(np.float32)   # two alternating values
    st[:, 0, 3] = np.float32(1e-40)                          # subnormals of both signs
    st[::3, 0, 3] = np.float32(-1e-40)
    st[:, 1, 0] = 0.0
    st[: T // 2, 1, 0] = -0.0                                # signed zeros
    st[:, 1, 1] = rng.choice(np.array([1.0, 1.0000001, -3e38, 3e38], np.float32), size=T)
    st[:, 1, 2] = np.round(st[:, 1, 2])                      # many ties
    return st


@pytest.mark.parametrize("T,N", [(4097, 9), (8192, 12), (8193, 8), (20000, 6)])
def test_deep_median_bit_exact(torch_dev, T, N):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("deep median T=%d N=%d" % (T, N), flush=True)
    st = _stack(T, N, seed=T)
    got = G.median(torch.from_numpy(st).to(dev)).cpu().numpy()
    ref = O.median_f32(st)
    assert got.tobytes() == ref.tobytes()


def test_deep_median_many_pixels(torch_dev):
    """Several pixel blocks and a ragged last block."""
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    T, N = 6000, 50
    st = _stack(T, N, seed=3)
    got = G.median(torch.from_numpy(st).to(dev)).cpu().numpy()
    assert got.tobytes() == O.median_f32(st).tobytes()


def test_deep_adi_against_oracle(torch_dev):
    """Classical ADI of 4100 small frames: both medians take the streaming
    select (the PSF one also rewrites the stack as residuals)."""
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("deep adi 4100 x 16^2", flush=True)
    T, N = 4100, 16
    rng = np.random.default_rng(17)
    yy, xx = np.mgrid[0:N, 0:N]
    star = 1e3 * np.exp(-((xx - 8.0) ** 2 + (yy - 8.0) ** 2) / (2 * 1.7 ** 2))
    cube = (star[None] + rng.normal(0.0, 5.0, (T, N, N))).astype(np.float32)
    dx, dy = rng.uniform(-0.5, 0.5, T), rng.uniform(-0.5, 0.5, T)
    pa = np.linspace(-30.0, 30.0, T)
    fin, psf, res = G.adi_reduce(torch.from_numpy(cube).to(dev), dx, dy, pa, psf=True, residuals=True)
    ref = O.adi_reduce(cube, dx, dy, pa)
    scale = np.linalg.norm(ref["psf"])
    assert np.linalg.norm(psf.cpu().numpy() - ref["psf"]) / scale <= 1e-5
    assert np.linalg.norm(fin.cpu().numpy() - ref["final"]) / scale <= 1e-5
    r = res.cpu().numpy()
    for t in (0, 1, 2047, 4099):
        assert np.linalg.norm(r[t] - ref["derotated"][t]) / scale <= 1e-5


def test_deep_batch_equals_single(torch_dev):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    rng = np.random.default_rng(5)
    cubes, dx, dy, pa = [], [], [], []
    for T, N in ((5000, 32), (300, 32), (4500, 64)):
        cubes.append(torch.from_numpy(rng.normal(100.0, 5.0, (T, N, N)).astype(np.float32)).to(dev))
        dx.append(rng.uniform(-1, 1, T))
        dy.append(rng.uniform(-1, 1, T))
        pa.append(np.linspace(-40.0, 40.0, T))
    fins = G.adi_reduce_batch(cubes, dx, dy, pa)
    for i, c in enumerate(cubes):
        one = G.adi_reduce(c, dx[i], dy[i], pa[i])
        assert fins[i].cpu().numpy().tobytes() == one.cpu().numpy().tobytes()
