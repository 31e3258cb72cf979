"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and its host-only queries validate geometry (no GPU needed)."""

import ctypes
import math
import os
import re

import pytest

from paper_1510_04331_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "graphic.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(graphic_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return _abi.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(names) == sorted(_abi.EXPORTS)


def test_status_strings_and_version(lib):
    for s in range(7):
        assert lib.graphic_status_string(s).startswith(b"GRAPHIC")
    assert b"NONFINITE" in lib.graphic_status_string(_abi.ERR_NONFINITE)
    assert b"gfx950" in lib.graphic_version()


@pytest.mark.parametrize("n,pad,expect", [
    (128, 0, 256), (100, 0, 256), (6, 0, 16), (64, 64, 64), (48, 256, 256),
    (1024, 0, 2048), (2048, 0, 4096),
    (7, 0, -1), (0, 0, -1), (4, 8, -1), (64, 96, -1), (64, 32, -1), (4096, 0, -1), (64, 8192, -1),
])
def test_resolved_pad(lib, n, pad, expect):
    g = _abi.Geom(3, n, pad, 0)
    assert lib.graphic_resolved_pad(ctypes.byref(g)) == expect


def test_workspace_sizes(lib):
    sz = ctypes.c_size_t()
    g = _abi.Geom(16, 128, 0, 0)
    assert lib.graphic_workspace_size(None, _abi.OP_SHIFT, ctypes.byref(g), ctypes.byref(sz)) == _abi.OK
    assert sz.value == 0
    assert lib.graphic_workspace_size(None, _abi.OP_ROTATE, ctypes.byref(g), ctypes.byref(sz)) == _abi.OK
    assert sz.value >= 16 * 128 * 256 * 4
    assert lib.graphic_workspace_size(None, _abi.OP_ADI, ctypes.byref(g), ctypes.byref(sz)) == _abi.OK
    assert sz.value >= 16 * 128 * 128 * 4 + 16 * 128 * 256 * 4
    deep = _abi.Geom(100_000, 64, 0, 0)        # a night of frames: the streaming select
    assert lib.graphic_workspace_size(None, _abi.OP_MEDIAN, ctypes.byref(deep), ctypes.byref(sz)) == _abi.OK
    g_big = _abi.Geom((1 << 24) + 1, 64, 0, 0)
    assert lib.graphic_workspace_size(None, _abi.OP_MEDIAN, ctypes.byref(g_big), ctypes.byref(sz)) == \
        _abi.ERR_UNSUPPORTED
    bad = _abi.Geom(16, 7, 0, 0)
    assert lib.graphic_workspace_size(None, _abi.OP_SHIFT, ctypes.byref(bad), ctypes.byref(sz)) == _abi.ERR_ARG
    for fl in (_abi.KEEP_PADDED, _abi.CHECK_FINITE, _abi.KEEP_PADDED | _abi.CHECK_FINITE):
        flags = _abi.Geom(16, 8, 0, fl)
        assert lib.graphic_workspace_size(None, _abi.OP_SHIFT, ctypes.byref(flags), ctypes.byref(sz)) == _abi.OK
    unknown = _abi.Geom(16, 8, 0, 4)
    assert lib.graphic_workspace_size(None, _abi.OP_SHIFT, ctypes.byref(unknown), ctypes.byref(sz)) == _abi.ERR_ARG
    assert lib.graphic_workspace_size(None, 99, ctypes.byref(g), ctypes.byref(sz)) == _abi.ERR_ARG


def test_entry_points_reject_null_context(lib):
    g = _abi.Geom(1, 8, 0, 0)
    assert lib.graphic_shift(None, ctypes.byref(g), None, None, None, None, None, None, 0, None) == _abi.ERR_ARG
    assert lib.graphic_rotate(None, ctypes.byref(g), None, None, None, None, None, 0, None) == _abi.ERR_ARG
    assert lib.graphic_adi_reduce(None, ctypes.byref(g), None, None, None, None, None, None, None, None, 0,
                                  None) == _abi.ERR_ARG
    assert lib.graphic_median(None, ctypes.byref(g), None, None, None, 0, None) == _abi.ERR_ARG
    assert lib.graphic_median_window(None, ctypes.byref(g), None, None, None, 1.0, 1.0, None, None, None, 0,
                                     None) == _abi.ERR_ARG
    assert lib.graphic_adi_reduce_window(None, ctypes.byref(g), None, None, None, None, None, 1.0, 1.0, None, None,
                                         None, None, 0, None) == _abi.ERR_ARG
    assert lib.graphic_autotune(None, ctypes.byref(g), None, 0, None) == _abi.ERR_ARG
    assert lib.graphic_tuning_import(None, b"") == _abi.ERR_ARG
    assert lib.graphic_graph_launch(None, None) == _abi.ERR_ARG


def test_window_workspace_sizes(lib):
    sz = ctypes.c_size_t()
    g = _abi.Geom(100, 64, 0, 0)
    assert lib.graphic_workspace_size(None, _abi.OP_MEDIAN_WINDOW, ctypes.byref(g), ctypes.byref(sz)) == _abi.OK
    assert sz.value >= 100 * 64 * 8 + 100 * 4
    assert lib.graphic_workspace_size(None, _abi.OP_ADI_WINDOW, ctypes.byref(g), ctypes.byref(sz)) == _abi.OK
    assert sz.value >= 100 * 64 * 64 * 4 + 100 * 64 * 8 + 64 * 128 * 4
    # longer sequences run in groups of 256 rows: the plan (2048 frame indices
    # and two ints per group, a flag word), one image for the rows that select
    # nothing and a ring of 9 x 256 PSF frames
    small = ctypes.c_size_t()
    lib.graphic_workspace_size(None, _abi.OP_MEDIAN_WINDOW, ctypes.byref(_abi.Geom(2048, 64, 0, 0)),
                               ctypes.byref(small))
    long_ = _abi.Geom(2049, 64, 0, 0)
    assert lib.graphic_workspace_size(None, _abi.OP_MEDIAN_WINDOW, ctypes.byref(long_), ctypes.byref(sz)) == _abi.OK
    groups = 9
    assert sz.value >= small.value + groups * 2048 * 4 + 64 * 64 * 4 + 9 * 256 * 64 * 64 * 4
    assert sz.value <= small.value + groups * 2048 * 4 + 64 * 64 * 4 + 9 * 256 * 64 * 64 * 4 + 16 * 256
    top = _abi.Geom(1 << 18, 64, 0, 0)
    big = _abi.Geom((1 << 18) + 1, 64, 0, 0)    # the plan compares all pairs of frames
    for op in (_abi.OP_MEDIAN_WINDOW, _abi.OP_ADI_WINDOW):
        assert lib.graphic_workspace_size(None, op, ctypes.byref(top), ctypes.byref(sz)) == _abi.OK
        assert lib.graphic_workspace_size(None, op, ctypes.byref(big), ctypes.byref(sz)) == _abi.ERR_UNSUPPORTED


def test_preprocess_and_register_reject_bad_arguments(lib):
    g = _abi.Geom(2, 8, 0, 0)
    assert lib.graphic_median_nan(None, ctypes.byref(g), None, None, None) == _abi.ERR_ARG
    assert lib.graphic_mask_disk(None, ctypes.byref(g), None, None, None, 1.0, None) == _abi.ERR_ARG
    assert lib.graphic_subtract_nearest(None, ctypes.byref(g), None, None, None, None, 1, None) == _abi.ERR_ARG
    assert lib.graphic_badpix_map(None, 8, None, 5.0, None, None, None, 0, None) == _abi.ERR_ARG
    assert lib.graphic_badpix_fix(None, ctypes.byref(g), None, None, 4, None, None, 0, None) == _abi.ERR_ARG
    prm = _abi.RegisterParams(1.0, 1, 10, 16, 50, float("inf"))
    assert lib.graphic_register(None, ctypes.byref(g), None, ctypes.byref(prm), None, None, None) == _abi.ERR_ARG
    assert lib.graphic_parallactic_angles(None, None, 1, 0.0, 0.0, 0.0, None, None) == _abi.ERR_ARG
    sz = ctypes.c_size_t()
    assert lib.graphic_workspace_size(None, _abi.OP_BADPIX_MAP, ctypes.byref(g), ctypes.byref(sz)) == _abi.OK
    assert sz.value >= 256 * 256 * 4
    assert lib.graphic_workspace_size(None, _abi.OP_BADPIX_FIX, ctypes.byref(g), ctypes.byref(sz)) == _abi.OK
    assert sz.value >= 2 * 8 * 8 * 4


@pytest.mark.parametrize("n_fwhm,fwhm,r_min", [(1.0, 4.0, 10.0), (1.5, 4.0, 25.0), (0.0, 4.0, 3.0), (2.0, 5.0, 5.0)])
def test_alpha_min_chord_angle(lib, n_fwhm, fwhm, r_min):
    """graphic_alpha_min_deg: the chord of the arc that a point at radius
    r_min sweeps through alpha_min has length n_fwhm * fwhm."""
    out = ctypes.c_double()
    assert lib.graphic_alpha_min_deg(n_fwhm, fwhm, r_min, ctypes.byref(out)) == _abi.OK
    chord = 2.0 * r_min * math.sin(math.radians(out.value) / 2.0)
    assert abs(chord - n_fwhm * fwhm) <= 1e-12 * max(1.0, n_fwhm * fwhm)
    assert 0.0 <= out.value <= 180.0


def test_alpha_min_rejects_impossible_chords(lib):
    out = ctypes.c_double()
    for args in ((3.0, 4.0, 5.0), (-1.0, 4.0, 10.0), (1.0, 4.0, 0.0), (1.0, float("nan"), 10.0),
                 (1.0, float("inf"), 10.0)):
        assert lib.graphic_alpha_min_deg(*args, ctypes.byref(out)) == _abi.ERR_ARG
    assert lib.graphic_alpha_min_deg(1.0, 4.0, 10.0, None) == _abi.ERR_ARG


def test_output_tensor_checks():
    """Caller-supplied outputs must match the result exactly (shape, dtype,
    contiguity, device) before any pointer reaches the library."""
    import torch
    from paper_1510_04331_amd import ops
    dev = torch.device("cpu")
    good = torch.empty((3, 8, 8), dtype=torch.float32)
    assert ops._check_out(good, (3, 8, 8), dev) is good
    for bad in (torch.empty((2, 8, 8)), torch.empty((3, 8, 6)), torch.empty((3, 8, 8), dtype=torch.float64),
                torch.empty((3, 8, 16))[:, :, ::2], torch.empty(192)):
        with pytest.raises(ValueError):
            ops._check_out(bad, (3, 8, 8), dev)
    with pytest.raises(ValueError):
        ops._check_out(good, (3, 8, 8), torch.device("cuda", 0))
    with pytest.raises(ValueError):
        ops._check_out(torch.empty((8, 8)), (3, 8, 8), dev)
    with pytest.raises(ValueError):
        ops._check_out(None, (8, 8), dev)
