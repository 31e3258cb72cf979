"""GPU: autotuning picks among launch shapes that compute identical results;
forcing either variant of every tuned kernel leaves results bit-identical,
and tuning text round-trips through export / import."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_04331_amd  # noqa: F401
    return torch, torch.device("cuda:0")


def _reduce(G, cube, p):
    fin, psf, res = G.adi_reduce(cube, p.dx, p.dy, p.parang, psf=True, residuals=True)
    return [t.cpu().numpy().tobytes() for t in (fin, psf, res)]


@pytest.mark.parametrize("T,N", [(70, 256), (33, 512), (12, 2048)])
def test_variants_bit_identical(torch_dev, T, N):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("tuning variants T=%d N=%d" % (T, N), flush=True)
    p = synth.make_params(2, seed=300 + N, T=T, N=N, with_screen=False)
    p.parang = np.linspace(-140.0, 140.0, T)
    cube = torch.from_numpy(synth.render_host(p)).to(dev)
    M = N                                   # P = 2N
    cls = int(np.ceil(np.log2(max(1, -(-T // 64)))))
    results = []
    for v in (0, 1):
        G.tuning_import("col %d 0 %d\ncol %d 1 %d\nmed %d %d\n" % (M, v, M, v, cls, v))
        results.append(_reduce(G, cube, p))
    assert results[0] == results[1]
    text = G.autotune(T, N)
    assert text.count("col %d" % M) == 2 and ("med %d" % cls) in text
    assert _reduce(G, cube, p) == results[0]
    G.tuning_import(text)
    assert G.tuning_export() == text


def test_tuning_import_rejects_bad_text(torch_dev):
    import paper_1510_04331_amd as G
    before = G.tuning_export()
    for bad in ("col 1000 0 1\n", "col 512 2 0\n", "med 9 0\n", "tmm 8 1\n", "tmm 3 2\n", "col 512 0 3\n", "foo 1 2 3\n", "col 512 0 1 x\n"):
        with pytest.raises(G.GraphicError):
            G.tuning_import(bad)
    assert G.tuning_export() == before
