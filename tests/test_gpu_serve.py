"""GPU: the request loop.  Every request's final image is the same whether it
is reduced alone or admitted in the mix with others (bitwise: the same kernels
compute every pixel the same way), and the loop keeps to its HBM budget while
overlapping requests on several streams."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _pool(torch, dev, sizes, frames=24):
    pool = {}
    for k, N in enumerate(sizes):
        p = synth.make_params(2, seed=900 + k, T=frames, N=N, with_screen=False)
        pool[N] = torch.from_numpy(synth.render_host(p)).to(dev)
    torch.cuda.synchronize()
    return pool


def _filler(pool, N, offset):
    src = pool[N]

    def fill(cube, stream):
        T, F = cube.shape[0], src.shape[0]
        for s in range(0, T, F):
            n = min(F, T - s)
            cube[s:s + n].copy_(src[(offset + np.arange(n)) % F] if offset else src[:n])
    return fill


def test_served_equals_alone():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_04331_amd as G
    from paper_1510_04331_amd import serve
    print("served requests vs alone", flush=True)
    dev = torch.device("cuda:0")
    sizes = (32, 64, 128)
    pool = _pool(torch, dev, sizes)
    rng = np.random.default_rng(11)
    arrivals = np.cumsum(rng.exponential(1.0 / 400.0, size=18))
    reqs = []
    for i, a in enumerate(arrivals):
        N = int(sizes[i % 3])
        T = int(rng.integers(5, 60))
        reqs.append(serve.Request(rid=i, arrival=float(a), T=T, N=N, dx=rng.uniform(-1, 1, T),
                                  dy=rng.uniform(-1, 1, T), parang=np.sort(rng.uniform(-120, 120, T)),
                                  fill=_filler(pool, N, i)))
    ex = serve.TorchExecutor(dev, slots=3)
    biggest = max(ex.group_bytes([r]) for r in reqs)
    adm = serve.Admission(budget_bytes=3 * biggest, slots=3, max_batch=3, group_bytes=ex.group_bytes)
    st = serve.run(reqs, ex, adm)
    torch.cuda.synchronize()
    assert st.max_used_bytes <= 3 * biggest
    assert st.max_inflight >= 2
    for r in reqs:
        cube = torch.empty((r.T, r.N, r.N), dtype=torch.float32, device=dev)
        r.fill(cube, None)
        alone = G.adi_reduce(cube, r.dx, r.dy, r.parang)
        assert r.final.cpu().numpy().tobytes() == alone.cpu().numpy().tobytes(), r.rid
