"""GPU: the persistent x-shear kernels (P = 2048, twiddle tables in LDS).

At 1024 x 1024 (P = 2048) both x-shears run as persistent blocks of 16 waves
that walk (frame, job) slots; half-turned frames are skipped there and taken
by the general path.  These cases check the rotation per frame against the
FP64 oracle (Sect. 3.4) where that kernel's bookkeeping could slip: fewer
slots than one block holds (T = 1), a ragged frame count, half-turned
frames between ordinary ones, and angles beyond a full turn.  Bar: relative
L2 <= 1e-5 and |sum_gpu - sum_oracle| / sum |x_in| <= 1e-6.
"""

import multiprocessing as mp
import os

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5
FLUX = 1e-6
ANGLES = [-30.0, 135.0, 11.3, -170.0, 89.9, 180.0, 350.0, -95.0, 0.0]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_04331_amd  # noqa: F401
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def pool():
    workers = max(1, min(8, os.cpu_count() or 1))
    with mp.get_context("spawn").Pool(workers) as p:
        yield p


def _oracle_rotate(a):
    f, th = a
    return O.rotate(f, th, P=2048)


def _cube(T, seed):
    rng = np.random.default_rng(seed)
    N = 1024
    c = rng.normal(0.0, 5.0, size=(T, N, N)).astype(np.float32)
    yy, xx = np.mgrid[0:N, 0:N]
    for t in range(T):
        x0, y0 = rng.uniform(300, 700, size=2)
        c[t] += (2e3 * np.exp(-((xx - x0) ** 2 + (yy - y0) ** 2) / (2 * 2.5 ** 2))).astype(np.float32)
    return c


@pytest.mark.parametrize("T", [1, 37])
def test_rotate_1024_against_oracle(torch_dev, pool, T):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("persistent x-shears: rotate T=%d at 1024^2" % T, flush=True)
    cube = _cube(T, seed=100 + T)
    ang = [ANGLES[t % len(ANGLES)] + (360.0 if t >= len(ANGLES) else 0.0) for t in range(T)]
    out, fl = G.rotate(torch.from_numpy(cube).to(dev), ang, flux=True)
    got = out.cpu().numpy()
    refs = pool.map(_oracle_rotate, [(cube[t], ang[t]) for t in range(T)], chunksize=1)
    for t in range(T):
        rel = float(np.linalg.norm(got[t].astype(np.float64) - refs[t]) / np.linalg.norm(refs[t]))
        assert rel <= REL_L2, (t, ang[t], rel)
        assert abs(got[t].astype(np.float64).sum() - refs[t].sum()) <= FLUX * np.abs(cube[t]).sum(), (t, ang[t])


def test_rotate_1024_frames_are_independent(torch_dev):
    """A frame's result does not depend on which other frames share the
    launch or on its slot: frames rotated alone equal the same frames rotated
    inside a larger ragged cube, bit for bit."""
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    T = 23
    cube = _cube(T, seed=7)
    ang = [ANGLES[t % len(ANGLES)] for t in range(T)]
    x = torch.from_numpy(cube).to(dev)
    whole = G.rotate(x, ang).cpu().numpy()
    for t in (0, 5, 22):
        one = G.rotate(x[t:t + 1].contiguous(), [ang[t]]).cpu().numpy()
        assert one[0].tobytes() == whole[t].tobytes(), t
