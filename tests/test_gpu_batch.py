"""GPU: batched ADI reduction of uneven cubes equals one reduction per cube,
bit for bit (every frame and pixel is computed by the same kernel code)."""

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_04331_amd  # noqa: F401
    return torch, torch.device("cuda:0")


def _cubes(shapes, seed):
    out = []
    for j, (T, N) in enumerate(shapes):
        p = synth.make_params(2, seed=seed + j, T=T, N=N, with_screen=False)
        p.noise = True
        if j % 2 == 1:      # half-turned frames (|angle| > 90 deg) in every other cube
            p.parang = np.linspace(-175.0, 175.0, T)
        c = synth.render_host(p)
        out.append((c, p))
    return out


def _single(G, torch, dev, cube, p):
    x = torch.from_numpy(cube).to(dev)
    return [t.cpu().numpy() for t in G.adi_reduce(x, p.dx, p.dy, p.parang, psf=True, residuals=True)]


SHAPES = [(7, 64), (33, 128), (5, 64), (20, 32), (3, 128), (12, 64)]


def test_batch_equals_single(torch_dev):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("batch equals single", flush=True)
    data = _cubes(SHAPES, 40)
    xs = [torch.from_numpy(c).to(dev) for c, _ in data]
    fins, psfs, res = G.adi_reduce_batch(xs, [p.dx for _, p in data], [p.dy for _, p in data],
                                         [p.parang for _, p in data], psf=True, residuals=True)
    for j, (c, p) in enumerate(data):
        f1, ps1, r1 = _single(G, torch, dev, c, p)
        assert fins[j].cpu().numpy().tobytes() == f1.tobytes(), j
        assert psfs[j].cpu().numpy().tobytes() == ps1.tobytes(), j
        assert res[j].cpu().numpy().tobytes() == r1.tobytes(), j


def test_batch_inplace_and_small_workspace(torch_dev):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("batch inplace, small workspace", flush=True)
    data = _cubes(SHAPES, 41)
    xs = [torch.from_numpy(c).to(dev) for c, _ in data]
    # workspace for the PSFs plus three working frames: rotation chunks span cubes
    need = G.batch_workspace_size(xs, inplace=True)
    # (PSFs, per-frame parameters, then 4 scratch frames of the N=128 class)
    small = sum(((N * N * 4 + 255) // 256) * 256 for _, N in SHAPES) + 4 * 128 * 256 * 4 + 64 * 1024
    ws = torch.empty(min(need, small), dtype=torch.uint8, device=dev)
    fins = G.adi_reduce_batch(xs, [p.dx for _, p in data], [p.dy for _, p in data],
                              [p.parang for _, p in data], inplace=True, workspace=ws)
    for j, (c, p) in enumerate(data):
        f1, _, r1 = _single(G, torch, dev, c, p)
        assert fins[j].cpu().numpy().tobytes() == f1.tobytes(), j
        assert xs[j].cpu().numpy().tobytes() == r1.tobytes(), j    # the cube now holds its residuals


def test_batch_more_cubes_than_one_launch(torch_dev):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("batch of 20 cubes", flush=True)
    shapes = [(3 + (j % 5), 16) for j in range(20)]
    data = _cubes(shapes, 42)
    xs = [torch.from_numpy(c).to(dev) for c, _ in data]
    fins = G.adi_reduce_batch(xs, [p.dx for _, p in data], [p.dy for _, p in data], [p.parang for _, p in data])
    for j, (c, p) in enumerate(data):
        f1, _, _ = _single(G, torch, dev, c, p)
        assert fins[j].cpu().numpy().tobytes() == f1.tobytes(), j


def test_batch_against_oracle(torch_dev):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("batch vs oracle", flush=True)
    data = _cubes([(9, 32), (6, 48)], 43)
    xs = [torch.from_numpy(c).to(dev) for c, _ in data]
    fins, psfs = G.adi_reduce_batch(xs, [p.dx for _, p in data], [p.dy for _, p in data],
                                    [p.parang for _, p in data], psf=True)
    for j, (c, p) in enumerate(data):
        ref = O.adi_reduce(c, p.dx, p.dy, p.parang)
        scale = np.linalg.norm(ref["psf"])
        assert np.linalg.norm(fins[j].cpu().numpy() - ref["final"]) / scale <= 1e-5
        assert np.linalg.norm(psfs[j].cpu().numpy() - ref["psf"]) / scale <= 1e-5


def test_batch_on_side_stream(torch_dev):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("batch on a side stream", flush=True)
    data = _cubes(SHAPES[:3], 44)
    xs = [torch.from_numpy(c).to(dev) for c, _ in data]
    args = ([p.dx for _, p in data], [p.dy for _, p in data], [p.parang for _, p in data])
    ref = G.adi_reduce_batch(xs, *args)
    s = torch.cuda.Stream(dev)
    got = G.adi_reduce_batch(xs, *args, stream=s)
    torch.cuda.current_stream(dev).wait_stream(s)
    for a, b in zip(ref, got):
        assert a.cpu().numpy().tobytes() == b.cpu().numpy().tobytes()
