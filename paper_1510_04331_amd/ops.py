"""Python entry points over the C ABI (torch tensors in, torch tensors out).

PyTorch supplies device memory and the current stream; the computation is the
HIP library's.  Names follow the C ABI: shift, rotate, median, adi_reduce.
"""

import ctypes

from . import _abi

_contexts = {}


def context(device_index):
    """The library context of one HIP device (created on first use)."""
    ctx = _contexts.get(device_index)
    if ctx is None:
        lib = _abi.load()
        h = ctypes.c_void_p()
        _abi.check(lib.graphic_create(ctypes.byref(h), int(device_index)), "graphic_create")
        ctx = h
        _contexts[device_index] = ctx
    return ctx


def _geom(T, N, pad, flags=0):
    return _abi.Geom(int(T), int(N), int(pad or 0), int(flags))


def _stream(dev):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _on_stream(stream, dev, tensors):
    """Stream handle for a call; a side stream first waits for the current
    stream (which produced the arguments) and keeps the tensors alive."""
    import torch
    if stream is None:
        return _stream(dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    for t in tensors:
        if t is not None:
            t.record_stream(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _check_cube(x, name="cube"):
    import torch
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)
    if x.dtype != torch.float32 or x.dim() != 3 or x.shape[1] != x.shape[2] or not x.is_contiguous():
        raise ValueError("%s must be a contiguous float32 [T, N, N] tensor" % name)
    return x.shape[0], x.shape[1]


def _check_out(out, shape, device, name="out"):
    """A caller-supplied output must be a contiguous float32 tensor of exactly
    the result's shape on the input's device (the kernels write that many
    values through its pointer)."""
    import torch
    if not isinstance(out, torch.Tensor):
        raise ValueError("%s must be a tensor" % name)
    if out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("%s must be a contiguous float32 tensor" % name)
    if tuple(out.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, not %s" % (name, tuple(shape), tuple(out.shape)))
    if out.device != device:
        raise ValueError("%s must be on %s, not %s" % (name, device, out.device))
    return out


def _flags(keep_padded=False, check_finite=False):
    return (_abi.KEEP_PADDED if keep_padded else 0) | (_abi.CHECK_FINITE if check_finite else 0)


def resolved_pad(N, pad=None):
    """Working size P of an N x N frame (pad, or the default next_pow2(2N))."""
    P = _abi.load().graphic_resolved_pad(ctypes.byref(_geom(1, N, pad)))
    if P < 0:
        raise ValueError("unsupported frame size N=%d pad=%s" % (N, pad))
    return P


def _f64(v, T, dev, name):
    import torch
    t = torch.as_tensor(v, dtype=torch.float64, device=dev).contiguous()
    if t.shape != (T,):
        raise ValueError("%s must have shape [T]" % name)
    return t


def workspace_size(op, T, N, pad=None, device_index=0):
    lib = _abi.load()
    out = ctypes.c_size_t()
    g = _geom(T, N, pad)
    _abi.check(lib.graphic_workspace_size(context(device_index), op, ctypes.byref(g), ctypes.byref(out)),
               "graphic_workspace_size")
    return out.value


def _workspace(op, T, N, pad, dev):
    import torch
    n = workspace_size(op, T, N, pad, dev.index or 0)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=dev), n


def shift(cube, dx, dy, pad=None, out=None, flux=False, keep_padded=False, check_finite=False):
    """Fourier shift of every frame by (dx[i], dy[i]) pixels (content moves
    toward +x, +y).  Returns ``out`` (and a [T, 2] float64 flux tensor).
    With ``keep_padded`` the result is the whole zero-padded [T, P, P] frame;
    with ``check_finite`` non-finite inputs raise GraphicError."""
    import torch
    T, N = _check_cube(cube)
    dev = cube.device
    dx, dy = _f64(dx, T, dev, "dx"), _f64(dy, T, dev, "dy")
    No = resolved_pad(N, pad) if keep_padded else N
    if out is None:
        out = torch.empty((T, No, No), dtype=torch.float32, device=dev)
    _check_out(out, (T, No, No), dev)
    fl = torch.empty((T, 2), dtype=torch.float64, device=dev) if flux else None
    ws, n = _workspace(_abi.OP_SHIFT, T, N, pad, dev)
    g = _geom(T, N, pad, _flags(keep_padded, check_finite))
    lib = _abi.load()
    _abi.check(lib.graphic_shift(context(dev.index or 0), ctypes.byref(g), _ptr(cube), _ptr(out), _ptr(dx),
                                 _ptr(dy), _ptr(fl), _ptr(ws), n, _stream(dev)), "graphic_shift")
    return (out, fl) if flux else out


def rotate(cube, theta_deg, pad=None, out=None, flux=False, keep_padded=False, check_finite=False):
    """Three-shear Fourier rotation of every frame by theta_deg[i] degrees
    (counter-clockwise, centre at pixel (N/2, N/2)).  ``keep_padded`` and
    ``check_finite`` as for :func:`shift`."""
    import torch
    T, N = _check_cube(cube)
    dev = cube.device
    th = _f64(theta_deg, T, dev, "theta_deg")
    No = resolved_pad(N, pad) if keep_padded else N
    if out is None:
        out = torch.empty((T, No, No), dtype=torch.float32, device=dev)
    _check_out(out, (T, No, No), dev)
    fl = torch.empty((T, 2), dtype=torch.float64, device=dev) if flux else None
    ws, n = _workspace(_abi.OP_ROTATE, T, N, pad, dev)
    g = _geom(T, N, pad, _flags(keep_padded, check_finite))
    lib = _abi.load()
    _abi.check(lib.graphic_rotate(context(dev.index or 0), ctypes.byref(g), _ptr(cube), _ptr(out), _ptr(th),
                                  _ptr(fl), _ptr(ws), n, _stream(dev)), "graphic_rotate")
    return (out, fl) if flux else out


def median(stack, out=None, check_finite=False):
    """Exact per-pixel float32 median over axis 0 of a [T, N, N] stack."""
    import torch
    T, N = _check_cube(stack, "stack")
    out = torch.empty((N, N), dtype=torch.float32, device=stack.device) if out is None else out
    _check_out(out, (N, N), stack.device)
    g = _geom(T, N, 0, _flags(False, check_finite))
    lib = _abi.load()
    _abi.check(lib.graphic_median(context(stack.device.index or 0), ctypes.byref(g), _ptr(stack), _ptr(out),
                                  None, 0, _stream(stack.device)), "graphic_median")
    return out


def adi_reduce(cube, dx, dy, parang_deg, pad=None, psf=False, residuals=False, workspace=None, stream=None,
               check_finite=False):
    """Classical ADI: recentre, median PSF, subtract, derotate by -parang,
    median combine.  Returns the final image, plus the PSF and the derotated
    residual cube when asked."""
    import torch
    T, N = _check_cube(cube)
    dev = cube.device
    dx, dy = _f64(dx, T, dev, "dx"), _f64(dy, T, dev, "dy")
    pa = _f64(parang_deg, T, dev, "parang_deg")
    final = torch.empty((N, N), dtype=torch.float32, device=dev)
    psf_t = torch.empty((N, N), dtype=torch.float32, device=dev) if psf else None
    res_t = torch.empty_like(cube) if residuals else None
    if workspace is None:
        ws, n = _workspace(_abi.OP_ADI, T, N, pad, dev)
    else:
        ws, n = workspace, workspace.numel()
    g = _geom(T, N, pad, _flags(False, check_finite))
    lib = _abi.load()
    st = _on_stream(stream, dev, [cube, dx, dy, pa, final, psf_t, res_t, ws])
    _abi.check(lib.graphic_adi_reduce(context(dev.index or 0), ctypes.byref(g), _ptr(cube), _ptr(dx), _ptr(dy),
                                      _ptr(pa), _ptr(final), _ptr(psf_t), _ptr(res_t), _ptr(ws), n, st),
               "graphic_adi_reduce")
    out = [final]
    if psf:
        out.append(psf_t)
    if residuals:
        out.append(res_t)
    return out[0] if len(out) == 1 else tuple(out)


def alpha_min_deg(n_fwhm, fwhm, r_min):
    """Minimum field rotation (degrees) of the per-frame PSF selection, from
    the library (graphic_alpha_min_deg: the chord angle at which a point at
    radius r_min has moved by n_fwhm FWHM)."""
    out = ctypes.c_double()
    st = _abi.load().graphic_alpha_min_deg(float(n_fwhm), float(fwhm), float(r_min), ctypes.byref(out))
    if st != _abi.OK:
        raise ValueError("alpha_min_deg: n_fwhm * fwhm must lie in [0, 2 r_min] with r_min > 0 (%s)"
                         % _abi.status_string(st))
    return out.value


def median_window(stack, times, parang_deg, t_max, alpha_min, psf=True, resid=False, inplace=False):
    """Per-frame medians over the frames selected for each frame (time
    separation below t_max, rotation above alpha_min degrees).  Returns the
    PSF cube and/or the residual cube stack - PSF (written into ``stack``
    when ``inplace``)."""
    import torch
    T, N = _check_cube(stack, "stack")
    dev = stack.device
    t = _f64(times, T, dev, "times")
    pa = _f64(parang_deg, T, dev, "parang_deg")
    psf_t = torch.empty_like(stack) if psf else None
    res_t = stack if inplace else (torch.empty_like(stack) if resid else None)
    ws, n = _workspace(_abi.OP_MEDIAN_WINDOW, T, N, None, dev)
    g = _geom(T, N, None)
    _abi.check(_abi.load().graphic_median_window(context(dev.index or 0), ctypes.byref(g), _ptr(stack), _ptr(t),
                                                 _ptr(pa), float(t_max), float(alpha_min), _ptr(psf_t),
                                                 _ptr(res_t), _ptr(ws), n, _stream(dev)), "graphic_median_window")
    out = [x for x in (psf_t, res_t) if x is not None]
    return out[0] if len(out) == 1 else tuple(out)


def adi_reduce_window(cube, dx, dy, parang_deg, times, t_max, alpha_min, pad=None, psf=False, residuals=False,
                      workspace=None, stream=None):
    """ADI with the per-frame PSF of the paper's frame selection.  Returns the
    final image, plus the PSF cube and the derotated residual cube when
    asked."""
    import torch
    T, N = _check_cube(cube)
    dev = cube.device
    dx, dy = _f64(dx, T, dev, "dx"), _f64(dy, T, dev, "dy")
    pa = _f64(parang_deg, T, dev, "parang_deg")
    t = _f64(times, T, dev, "times")
    final = torch.empty((N, N), dtype=torch.float32, device=dev)
    psf_t = torch.empty_like(cube) if psf else None
    res_t = torch.empty_like(cube) if residuals else None
    if workspace is None:
        ws, n = _workspace(_abi.OP_ADI_WINDOW, T, N, pad, dev)
    else:
        ws, n = workspace, workspace.numel()
    g = _geom(T, N, pad)
    st = _on_stream(stream, dev, [cube, dx, dy, pa, t, final, psf_t, res_t, ws])
    _abi.check(_abi.load().graphic_adi_reduce_window(context(dev.index or 0), ctypes.byref(g), _ptr(cube), _ptr(dx),
                                                     _ptr(dy), _ptr(pa), _ptr(t), float(t_max), float(alpha_min),
                                                     _ptr(final), _ptr(psf_t), _ptr(res_t), _ptr(ws), n, st),
               "graphic_adi_reduce_window")
    out = [final] + [x for x in (psf_t, res_t) if x is not None]
    return out[0] if len(out) == 1 else tuple(out)


def parallactic_angles(lst_s, ra_deg, dec_deg, lat_deg, device=None):
    """Per-frame parallactic angles (degrees) from local sidereal times in
    seconds (a float64 tensor or array)."""
    import torch
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    lst = torch.as_tensor(lst_s, dtype=torch.float64, device=dev).contiguous().reshape(-1)
    out = torch.empty_like(lst)
    _abi.check(_abi.load().graphic_parallactic_angles(context(dev.index or 0), _ptr(lst), lst.numel(), float(ra_deg),
                                                      float(dec_deg), float(lat_deg), _ptr(out), _stream(dev)),
               "graphic_parallactic_angles")
    return out


REGISTER_COLUMNS = ("cx", "cy", "x0", "y0", "i0", "alpha", "beta", "bg", "cost", "fwhm", "dx", "dy")


def register(cube, threshold, min_size, max_size, half=16, saturation=float("inf"), max_iter=200):
    """Star centroid and Moffat fit of every frame.  Returns a dict of float64
    [T] tensors (REGISTER_COLUMNS: centroid, fit parameters, final cost, FWHM
    and recentring shift, all computed by the library) and int32 flags."""
    import torch
    T, N = _check_cube(cube)
    dev = cube.device
    out = torch.empty((T, len(REGISTER_COLUMNS)), dtype=torch.float64, device=dev)
    flags = torch.empty(T, dtype=torch.int32, device=dev)
    prm = _abi.RegisterParams(float(threshold), int(min_size), int(max_size), int(half), int(max_iter),
                              float(saturation))
    g = _geom(T, N, None)
    _abi.check(_abi.load().graphic_register(context(dev.index or 0), ctypes.byref(g), _ptr(cube), ctypes.byref(prm),
                                            _ptr(out), _ptr(flags), _stream(dev)), "graphic_register")
    res = {k: out[:, i] for i, k in enumerate(REGISTER_COLUMNS)}
    res["flags"] = flags
    return res


def median_nan(stack, out=None):
    """Per-pixel median over axis 0 ignoring NaN (NaN where none is left)."""
    import torch
    T, N = _check_cube(stack, "stack")
    out = torch.empty((N, N), dtype=torch.float32, device=stack.device) if out is None else out
    _check_out(out, (N, N), stack.device)
    g = _geom(T, N, 0)
    _abi.check(_abi.load().graphic_median_nan(context(stack.device.index or 0), ctypes.byref(g), _ptr(stack),
                                              _ptr(out), _stream(stack.device)), "graphic_median_nan")
    return out


def mask_disk(cube, xs, ys, radius):
    """NaN out, in place, the disc of ``radius`` around (xs[i], ys[i]) in frame i."""
    T, N = _check_cube(cube)
    dev = cube.device
    x, y = _f64(xs, T, dev, "xs"), _f64(ys, T, dev, "ys")
    g = _geom(T, N, 0)
    _abi.check(_abi.load().graphic_mask_disk(context(dev.index or 0), ctypes.byref(g), _ptr(cube), _ptr(x), _ptr(y),
                                             float(radius), _stream(dev)), "graphic_mask_disk")
    return cube


def subtract_nearest(cube, times, skies, sky_times):
    """In place: every frame minus the sky closest to it in time."""
    T, N = _check_cube(cube)
    S, Ns = _check_cube(skies, "skies")
    if Ns != N:
        raise ValueError("skies must have the frames' size")
    dev = cube.device
    t, st_ = _f64(times, T, dev, "times"), _f64(sky_times, S, dev, "sky_times")
    g = _geom(T, N, 0)
    _abi.check(_abi.load().graphic_subtract_nearest(context(dev.index or 0), ctypes.byref(g), _ptr(cube), _ptr(t),
                                                    _ptr(skies), _ptr(st_), S, _stream(dev)),
               "graphic_subtract_nearest")
    return cube


def badpix_map(frame, c_sigma):
    """Bad pixel map of one N x N frame and its (median, mean, sigma)."""
    import torch
    if frame.dim() != 2 or frame.shape[0] != frame.shape[1] or frame.dtype != torch.float32 or not frame.is_contiguous():
        raise ValueError("frame must be a contiguous float32 [N, N] tensor")
    N = frame.shape[0]
    dev = frame.device
    m = torch.empty((N, N), dtype=torch.uint8, device=dev)
    stats = torch.empty(3, dtype=torch.float64, device=dev)
    ws, n = _workspace(_abi.OP_BADPIX_MAP, 1, 8, 0, dev)
    _abi.check(_abi.load().graphic_badpix_map(context(dev.index or 0), N, _ptr(frame), float(c_sigma), _ptr(m),
                                              _ptr(stats), _ptr(ws), n, _stream(dev)), "graphic_badpix_map")
    return m, stats


def badpix_fix(cube, bad_map=None, max_passes=64):
    """In place: flagged pixels to NaN, then neighbour-median repair passes.
    Returns the number of passes that met a NaN."""
    T, N = _check_cube(cube)
    dev = cube.device
    ws, n = _workspace(_abi.OP_BADPIX_FIX, T, N, 0, dev)
    passes = ctypes.c_int32()
    g = _geom(T, N, 0)
    _abi.check(_abi.load().graphic_badpix_fix(context(dev.index or 0), ctypes.byref(g), _ptr(cube), _ptr(bad_map),
                                              int(max_passes), ctypes.byref(passes), _ptr(ws), n, _stream(dev)),
               "graphic_badpix_fix")
    return passes.value


def annular_rms(a, b=None, width=1.0, n_rings=None, centre=None):
    """RMS of a - b (or of a) in annuli of `width` px around `centre` (x, y;
    default (N/2, N/2)) for every frame of a [T, N, N] (or [N, N]) tensor,
    the image-quality measure of Sect. 4.1.  Returns (rms [T, n_rings] or
    [n_rings] float64, counts [n_rings] int64), both on the device; n_rings
    defaults to the annuli that reach the frame corners."""
    import math
    import torch
    single = a.dim() == 2
    a3 = a.unsqueeze(0) if single else a
    T, N = _check_cube(a3, "a")
    b3 = None
    if b is not None:
        b3 = b.unsqueeze(0) if b.dim() == 2 else b
        _check_cube(b3, "b")
        if b3.shape != a3.shape or b3.device != a3.device:
            raise ValueError("b must have the shape and device of a")
    cx, cy = (N / 2.0, N / 2.0) if centre is None else (float(centre[0]), float(centre[1]))
    if n_rings is None:
        far = max(math.hypot(x - cx, y - cy) for x in (0, N - 1) for y in (0, N - 1))
        n_rings = int(far // width) + 1
    dev = a3.device
    rms = torch.empty((T, int(n_rings)), dtype=torch.float64, device=dev)
    counts = torch.empty(int(n_rings), dtype=torch.int64, device=dev)
    g = _geom(T, N, 0)
    _abi.check(_abi.load().graphic_annular_rms(context(dev.index or 0), ctypes.byref(g), _ptr(a3), _ptr(b3), cx, cy,
                                               float(width), int(n_rings), _ptr(rms), _ptr(counts), _stream(dev)),
               "graphic_annular_rms")
    return (rms[0] if single else rms), counts


def _batch_descs(cubes, dx, dy, parang, pad, psf, residuals):
    import torch
    n = len(cubes)
    if not (len(dx) == len(dy) == len(parang) == n) or n < 1:
        raise ValueError("one dx, dy and parang array per cube")
    keep = []                      # tensors that must outlive the call
    descs = (_abi.CubeDesc * n)()
    finals, psfs, resids = [], [], []
    dev = cubes[0].device
    for i, c in enumerate(cubes):
        T, N = _check_cube(c, "cubes[%d]" % i)
        if c.device != dev:
            raise ValueError("all cubes must be on one device")
        a, b, p = _f64(dx[i], T, dev, "dx"), _f64(dy[i], T, dev, "dy"), _f64(parang[i], T, dev, "parang")
        f = torch.empty((N, N), dtype=torch.float32, device=dev)
        ps = torch.empty((N, N), dtype=torch.float32, device=dev) if psf else None
        rs = torch.empty_like(c) if residuals else None
        keep += [a, b, p]
        finals.append(f)
        psfs.append(ps)
        resids.append(rs)
        descs[i] = _abi.CubeDesc(c.data_ptr(), T, N, int(pad or 0), a.data_ptr(), b.data_ptr(), p.data_ptr(),
                                 f.data_ptr(), 0 if ps is None else ps.data_ptr(),
                                 0 if rs is None else rs.data_ptr())
    return descs, keep, finals, psfs, resids


def batch_workspace_size(cubes, pad=None, inplace=False, device_index=0):
    """Workspace bytes of adi_reduce_batch for these cubes (shapes only)."""
    import torch
    n = len(cubes)
    descs = (_abi.CubeDesc * n)()
    for i, c in enumerate(cubes):
        T, N = c.shape[0], c.shape[1]
        descs[i] = _abi.CubeDesc(256, T, N, int(pad or 0), 256, 256, 256, 256, 0, 0)
    out = ctypes.c_size_t()
    flags = _abi.BATCH_INPLACE if inplace else 0
    _abi.check(_abi.load().graphic_batch_workspace_size(context(device_index), descs, n, flags,
                                                        ctypes.byref(out)), "graphic_batch_workspace_size")
    return out.value


def adi_reduce_batch(cubes, dx, dy, parang_deg, pad=None, inplace=False, psf=False, residuals=False,
                     workspace=None, stream=None):
    """ADI reduction of several cubes (uneven frame counts and sizes) in
    batched launches.  Returns the list of final images (and PSFs /
    residual cubes when asked).  With ``inplace`` every input cube is
    overwritten with its derotated residuals."""
    import torch
    dev = cubes[0].device
    descs, keep, finals, psfs, resids = _batch_descs(cubes, dx, dy, parang_deg, pad, psf, residuals)
    flags = _abi.BATCH_INPLACE if inplace else 0
    if workspace is None:
        n = ctypes.c_size_t()
        _abi.check(_abi.load().graphic_batch_workspace_size(context(dev.index or 0), descs, len(cubes), flags,
                                                            ctypes.byref(n)), "graphic_batch_workspace_size")
        workspace = torch.empty(max(n.value, 256), dtype=torch.uint8, device=dev)
    st = _on_stream(stream, dev, list(cubes) + keep + finals + psfs + resids + [workspace])
    _abi.check(_abi.load().graphic_adi_reduce_batch(context(dev.index or 0), descs, len(cubes), flags,
                                                    _ptr(workspace), workspace.numel(), st),
               "graphic_adi_reduce_batch")
    out = [finals]
    if psf:
        out.append(psfs)
    if residuals:
        out.append(resids)
    return out[0] if len(out) == 1 else tuple(out)


class AdiGraph:
    """A captured batched reduction (HIP graph) over fixed buffers.

    ``cubes``, the parameter tensors, ``finals`` (and ``psfs`` /
    ``residuals``) and the workspace are bound at capture; ``launch()``
    replays the whole reduction on the current (or a given) stream with the
    buffers' current contents.  Write new frames into the same cube tensors
    (``cube.copy_(...)``) between launches.
    """

    def __init__(self, cubes, dx, dy, parang_deg, pad=None, inplace=False, psf=False, residuals=False,
                 workspace=None):
        import torch
        self.device = cubes[0].device
        self.cubes = list(cubes)
        descs, keep, finals, psfs, resids = _batch_descs(self.cubes, dx, dy, parang_deg, pad, psf, residuals)
        self._keep = keep
        self.dx, self.dy, self.parang = keep[0::3], keep[1::3], keep[2::3]
        self.finals, self.psfs, self.residuals = finals, psfs, resids
        flags = _abi.BATCH_INPLACE if inplace else 0
        lib = _abi.load()
        ctx = context(self.device.index or 0)
        if workspace is None:
            n = ctypes.c_size_t()
            _abi.check(lib.graphic_batch_workspace_size(ctx, descs, len(self.cubes), flags, ctypes.byref(n)),
                       "graphic_batch_workspace_size")
            workspace = torch.empty(max(n.value, 256), dtype=torch.uint8, device=self.device)
        self.workspace = workspace
        torch.cuda.synchronize(self.device)     # parameter uploads done before capture
        h = ctypes.c_void_p()
        _abi.check(lib.graphic_adi_graph_create(ctx, descs, len(self.cubes), flags, _ptr(workspace),
                                                workspace.numel(), ctypes.byref(h)), "graphic_adi_graph_create")
        self._h = h

    def launch(self, stream=None):
        tensors = self.cubes + self._keep + self.finals + self.psfs + self.residuals + [self.workspace]
        st = _on_stream(stream, self.device, tensors)
        _abi.check(_abi.load().graphic_graph_launch(self._h, st), "graphic_graph_launch")

    def close(self):
        if getattr(self, "_h", None):
            _abi.load().graphic_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:   # interpreter shutdown
            pass


def autotune(T, N, pad=None, device_index=0, workspace=None):
    """Time the alternative launch shapes for this geometry and keep the
    fastest in the device's context (returns the tuning text)."""
    import torch
    dev = torch.device("cuda", device_index)
    P = _abi.load().graphic_resolved_pad(ctypes.byref(_geom(T, N, pad)))
    if P < 0:
        raise ValueError("unsupported geometry T=%d N=%d pad=%s" % (T, N, pad))
    if workspace is None:
        workspace = torch.empty(max(workspace_size(_abi.OP_ADI, T, N, pad, device_index), 256),
                                dtype=torch.uint8, device=dev)
    g = _geom(T, N, pad)
    _abi.check(_abi.load().graphic_autotune(context(device_index), ctypes.byref(g), _ptr(workspace),
                                            workspace.numel(), _stream(dev)), "graphic_autotune")
    return tuning_export(device_index)


def tuning_export(device_index=0):
    lib = _abi.load()
    need = ctypes.c_size_t()
    _abi.check(lib.graphic_tuning_export(context(device_index), None, 0, ctypes.byref(need)),
               "graphic_tuning_export")
    buf = ctypes.create_string_buffer(need.value)
    _abi.check(lib.graphic_tuning_export(context(device_index), buf, need.value, ctypes.byref(need)),
               "graphic_tuning_export")
    return buf.value.decode()


def tuning_import(text, device_index=0):
    _abi.check(_abi.load().graphic_tuning_import(context(device_index), text.encode()), "graphic_tuning_import")


def timing_enable(enable=True, device_index=0):
    _abi.check(_abi.load().graphic_timing_enable(context(device_index), int(bool(enable))), "graphic_timing_enable")


def timing_read(family, device_index=0):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _abi.check(_abi.load().graphic_timing_read(context(device_index), family.encode(), ctypes.byref(ms),
                                               ctypes.byref(n)), "graphic_timing_read")
    return ms.value, n.value
