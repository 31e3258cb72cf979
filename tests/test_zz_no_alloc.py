"""GPU: graphic_rotate_noalloc (no workspace, static scratch) against
graphic_rotate with a workspace, through the C ABI.

The two run the same passes, only the chunking of frames differs (the
static scratch holds fewer frames per chunk than the default workspace), and
every frame is computed independently, so the results must agree bit for bit
(stronger than the 1e-5 relative-L2 bar).  Two calls in a row, the second on a
smaller input, check that the shared scratch keeps nothing that matters from
one call to the next.
"""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_04331_amd import _abi, ops
    return torch, torch.device("cuda:0"), _abi, _abi.load(), ops.context(0)


def _p(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _frames(torch, dev, T, N, seed):
    rng = np.random.default_rng(seed)
    c = rng.normal(0.0, 5.0, size=(T, N, N)).astype(np.float32)
    c[:, N // 3:N // 3 + 4, N // 2:N // 2 + 3] += 1e3
    return torch.from_numpy(c).to(dev)


def _both(env, x, ang, flags=0):
    torch, dev, _abi, lib, ctx = env
    T, N = x.shape[0], x.shape[1]
    g = _abi.Geom(T, N, 0, flags)
    P = lib.graphic_resolved_pad(ctypes.byref(g))
    No = P if flags & _abi.KEEP_PADDED else N
    th = torch.tensor(ang, dtype=torch.float64, device=dev)
    ref = torch.empty((T, No, No), dtype=torch.float32, device=dev)
    got = torch.full((T, No, No), float("nan"), dtype=torch.float32, device=dev)
    fr = torch.empty((T, 2), dtype=torch.float64, device=dev)
    fg = torch.empty((T, 2), dtype=torch.float64, device=dev)
    nws = ctypes.c_size_t()
    _abi.check(lib.graphic_workspace_size(ctx, _abi.OP_ROTATE, ctypes.byref(g), ctypes.byref(nws)), "ws size")
    ws = torch.empty(max(nws.value, 256), dtype=torch.uint8, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _abi.check(lib.graphic_rotate(ctx, ctypes.byref(g), _p(x), _p(ref), _p(th), _p(fr), _p(ws), nws.value, st),
               "graphic_rotate")
    _abi.check(lib.graphic_rotate_noalloc(ctx, ctypes.byref(g), _p(x), _p(got), _p(th), _p(fg), st),
               "graphic_rotate_noalloc")
    torch.cuda.synchronize()
    return ref, got, fr, fg


def test_noalloc_equals_workspace_call_twice(env):
    torch, dev, _abi, lib, ctx = env
    print("noalloc: 40 x 1024^2 then 5 x 128^2", flush=True)
    # 40 frames of 1024^2: 8 MiB of scratch per frame, so several chunks
    x = _frames(torch, dev, 40, 1024, 1)
    ang = list(np.linspace(-170.0, 170.0, 40))
    ref, got, fr, fg = _both(env, x, ang)
    assert torch.equal(got, ref)
    assert torch.equal(fg, fr)
    # a smaller second call: nothing left behind in the scratch matters
    y = _frames(torch, dev, 5, 128, 2)
    ref2, got2, fr2, fg2 = _both(env, y, [11.3, -30.0, 135.0, 350.0, 0.0])
    assert torch.equal(got2, ref2)
    assert torch.equal(fg2, fr2)


def test_noalloc_keep_padded(env):
    torch, dev, _abi, lib, ctx = env
    x = _frames(torch, dev, 6, 256, 3)
    ref, got, _, _ = _both(env, x, [5.0, -95.0, 30.0, 180.0, -12.5, 89.0], flags=_abi.KEEP_PADDED)
    assert torch.equal(got, ref)


def test_noalloc_rejects_oversized_geometry(env):
    """The static scratch holds the parameters of T frames and one N x P
    frame; beyond that the call fails before doing anything."""
    torch, dev, _abi, lib, ctx = env
    g = _abi.Geom(4_000_000, 4096, 4096, 0)
    assert lib.graphic_rotate_noalloc(ctx, ctypes.byref(g), None, None, None, None, None) == _abi.ERR_UNSUPPORTED
    g = _abi.Geom(3, 64, 0, _abi.CHECK_FINITE)
    x = torch.zeros((3, 64, 64), device=dev)
    d = torch.zeros(3, dtype=torch.float64, device=dev)
    assert lib.graphic_rotate_noalloc(ctx, ctypes.byref(g), _p(x), _p(x), _p(d), None, None) == _abi.ERR_ARG
    torch.cuda.synchronize()
