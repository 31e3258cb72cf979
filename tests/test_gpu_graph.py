"""GPU: a captured reduction (HIP graph) replays to the same results as the
eager batched call, replay after replay, with new data written into the
bound buffers and eager work and synchronisations between the replays."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

SHAPES = [(9, 64), (21, 128), (5, 64), (12, 32)]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_04331_amd  # noqa: F401
    return torch, torch.device("cuda:0")


def _data(torch, dev, seed):
    out = []
    for j, (T, N) in enumerate(SHAPES):
        p = synth.make_params(2, seed=seed + j, T=T, N=N, with_screen=False)
        if j == 1:
            p.parang = np.linspace(-170.0, 170.0, T)
        out.append((torch.from_numpy(synth.render_host(p)).to(dev), p))
    return out


@pytest.mark.parametrize("inplace", [False, True])
def test_graph_replays_equal_eager(torch_dev, inplace):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("graph replays inplace=%s" % inplace, flush=True)
    first = _data(torch, dev, 500)
    cubes = [c.clone() for c, _ in first]
    ps = [p for _, p in first]
    g = G.AdiGraph(cubes, [p.dx for p in ps], [p.dy for p in ps], [p.parang for p in ps], inplace=inplace,
                   psf=True, residuals=not inplace)
    for rep in range(4):
        data = first if rep == 0 else _data(torch, dev, 600 + 10 * rep)
        for c, (src, _) in zip(cubes, data):
            c.copy_(src)
        # new angles and shifts go into the bound parameter tensors
        for k, (_, p) in enumerate(data):
            g.dx[k].copy_(torch.from_numpy(p.dx))
            g.dy[k].copy_(torch.from_numpy(p.dy))
            g.parang[k].copy_(torch.from_numpy(p.parang))
        g.launch()
        torch.cuda.synchronize()
        ref = G.adi_reduce_batch([src.clone() for src, _ in data], [p.dx for _, p in data],
                                 [p.dy for _, p in data], [p.parang for _, p in data], psf=True, residuals=True)
        torch.cuda.synchronize()
        for k in range(len(SHAPES)):
            assert g.finals[k].cpu().numpy().tobytes() == ref[0][k].cpu().numpy().tobytes(), (rep, k)
            assert g.psfs[k].cpu().numpy().tobytes() == ref[1][k].cpu().numpy().tobytes(), (rep, k)
            got_res = cubes[k] if inplace else g.residuals[k]
            assert got_res.cpu().numpy().tobytes() == ref[2][k].cpu().numpy().tobytes(), (rep, k)
    g.close()


def test_graph_on_side_stream(torch_dev):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("graph on a side stream", flush=True)
    data = _data(torch, dev, 700)
    cubes = [c for c, _ in data]
    ps = [p for _, p in data]
    args = ([p.dx for p in ps], [p.dy for p in ps], [p.parang for p in ps])
    ref = G.adi_reduce_batch(cubes, *args)
    g = G.AdiGraph(cubes, *args)
    s = torch.cuda.Stream(dev)
    for _ in range(3):
        g.launch(stream=s)
        torch.cuda.current_stream(dev).wait_stream(s)
        torch.cuda.synchronize()
        for a, b in zip(ref, g.finals):
            assert a.cpu().numpy().tobytes() == b.cpu().numpy().tobytes()
    g.close()
