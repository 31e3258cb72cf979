"""Tile-major workspace stacks of the ADI reduction (frames of 1024 x 1024
pixels, P = 2N; other sizes keep the frame-major stack, which the 2048 cases
check through the same comparison: the workspace stack against the caller's
residual array, with small rotation chunks).

When the caller asks for no residuals and the cube is not overwritten, the
reduction keeps its stack in the workspace in the tile-major layout (the
values of 16 neighbouring pixels over all frames are one contiguous run);
with residuals it works in the caller's frame-major array instead.  The
arithmetic is identical, so both give the same bits.  The cases cover ragged
frame counts (the tile-major median gives each thread ceil(T/64) consecutive
frames, rounded up to a power of two: at T = 130 and T = 2500 the last
threads hold a few frames or none), half-turned frames, rotation chunks that
start inside a cube and batches of two cubes in one launch, and one reduction
is checked against the oracle.
"""

import multiprocessing as mp
import os

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1510_04331_amd  # noqa: F401
    return torch, torch.device("cuda:0")


def _params(N, T, seed, wide):
    q = synth.make_params(2, seed=synth.BASE_SEED + 300 + seed, T=T, N=N)
    if wide:
        q.parang = np.linspace(-150.0, 150.0, T)       # half-turned frames too
    return q


def _small_ws(torch, dev, bytes_default, N, F, chunk):
    """A workspace that leaves room for about `chunk` frames per rotation chunk."""
    per_frame = N * 2 * N * 4
    default_cf = min(F, (4 << 30) // per_frame)
    return torch.empty(bytes_default - (default_cf - chunk) * per_frame, dtype=torch.uint8, device=dev)


@pytest.mark.parametrize("N,T,wide,chunk", [(1024, 37, True, None), (1024, 70, False, 6), (1024, 1, True, None),
                                             (1024, 64, True, 5), (1024, 32, True, None), (1024, 130, True, None),
                                             (1024, 2500, False, None),
                                             (2048, 19, True, 4), (2048, 70, False, None), (2048, 33, True, 7)])
def test_tile_major_equals_frame_major(torch_dev, N, T, wide, chunk):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    from paper_1510_04331_amd import _abi
    print("tile-major vs frame-major N=%d T=%d wide=%s chunk=%s" % (N, T, wide, chunk), flush=True)
    q = _params(N, T, N + T, wide)
    cube = synth.render_device(q, dev)
    fin_fm, psf_fm, res = G.adi_reduce(cube, q.dx, q.dy, q.parang, psf=True, residuals=True)
    del res
    ws = None
    if chunk:
        ws = _small_ws(torch, dev, G.workspace_size(_abi.OP_ADI, T, N), N, T, chunk)
    fin_tm, psf_tm = G.adi_reduce(cube, q.dx, q.dy, q.parang, psf=True, workspace=ws)
    torch.cuda.synchronize()
    assert psf_tm.cpu().numpy().tobytes() == psf_fm.cpu().numpy().tobytes()
    assert fin_tm.cpu().numpy().tobytes() == fin_fm.cpu().numpy().tobytes()


def test_tile_major_batch_with_split_chunks(torch_dev):
    """Two cubes in the same launches, rotation chunks of about 16 frames, so
    one chunk starts in the first cube and ends in the second."""
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("tile-major batch 37 + 70 frames of 1024^2", flush=True)
    qs = [_params(1024, 37, 1, True), _params(1024, 70, 2, False)]
    cubes = [synth.render_device(q, dev) for q in qs]
    n = G.batch_workspace_size(cubes)
    ws = _small_ws(torch, dev, n, 1024, 107, 16)
    fins = G.adi_reduce_batch(cubes, [q.dx for q in qs], [q.dy for q in qs], [q.parang for q in qs], workspace=ws)
    torch.cuda.synchronize()
    for c, q, f in zip(cubes, qs, fins):
        one, _ = G.adi_reduce(c, q.dx, q.dy, q.parang, residuals=True)
        assert f.cpu().numpy().tobytes() == one.cpu().numpy().tobytes()


def test_tile_major_against_oracle(torch_dev):
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("tile-major ADI 12 x 1024^2 against the oracle", flush=True)
    q = _params(1024, 12, 3, True)
    cube = synth.render_device(q, dev)
    fin, psf = G.adi_reduce(cube, q.dx, q.dy, q.parang, psf=True)
    host = cube.cpu().numpy()
    workers = max(1, min(12, os.cpu_count() or 1))
    with mp.get_context("spawn").Pool(workers) as pool:
        ref = O.adi_reduce(host, q.dx, q.dy, q.parang, map_fn=lambda f, a: pool.map(f, a, chunksize=1))
    scale = np.linalg.norm(ref["psf"])
    assert np.linalg.norm(psf.cpu().numpy() - ref["psf"]) / scale <= REL_L2
    assert np.linalg.norm(fin.cpu().numpy() - ref["final"]) / scale <= REL_L2


def test_workspace_stack_2048_against_oracle(torch_dev):
    """The 2048^2 reduction with its stack in the workspace (two-wave line
    passes, no residuals requested) against the oracle."""
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("workspace-stack ADI 5 x 2048^2 against the oracle", flush=True)
    q = _params(2048, 5, 5, True)
    cube = synth.render_device(q, dev)
    fin, psf = G.adi_reduce(cube, q.dx, q.dy, q.parang, psf=True)
    host = cube.cpu().numpy()
    workers = max(1, min(5, os.cpu_count() or 1))
    with mp.get_context("spawn").Pool(workers) as pool:
        ref = O.adi_reduce(host, q.dx, q.dy, q.parang, map_fn=lambda f, a: pool.map(f, a, chunksize=1))
    scale = np.linalg.norm(ref["psf"])
    assert np.linalg.norm(psf.cpu().numpy() - ref["psf"]) / scale <= REL_L2
    assert np.linalg.norm(fin.cpu().numpy() - ref["final"]) / scale <= REL_L2


def test_tile_major_variants_bit_identical(torch_dev):
    """Both tile widths of the staged column pass and both pixel tiles of the
    tile-major median give the frame-major result; the autotuner picks among
    them and reports its choice for the tile-major median."""
    torch, dev = torch_dev
    import paper_1510_04331_amd as G
    print("tile-major variants T=70 N=1024", flush=True)
    T, N = 70, 1024
    q = _params(N, T, 4, True)
    cube = synth.render_device(q, dev)
    ref, _ = G.adi_reduce(cube, q.dx, q.dy, q.parang, residuals=True)
    ref = ref.cpu().numpy().tobytes()
    cls = int(np.ceil(np.log2(max(1, -(-T // 64)))))
    before = G.tuning_export()
    try:
        for v in (0, 1):
            G.tuning_import("col %d 0 %d\ncol %d 1 %d\ntmm %d %d\n" % (N, v, N, v, cls, v))
            assert G.adi_reduce(cube, q.dx, q.dy, q.parang).cpu().numpy().tobytes() == ref
        text = G.autotune(T, N)
        assert ("tmm %d" % cls) in text
        assert G.adi_reduce(cube, q.dx, q.dy, q.parang).cpu().numpy().tobytes() == ref
    finally:
        G.tuning_import(before)
