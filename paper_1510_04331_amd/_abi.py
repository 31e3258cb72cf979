"""ctypes declarations of libgraphic.so (include/graphic.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgraphic.so")

# status codes (graphic_status)
OK, ERR_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP, ERR_NOMEM, ERR_NONFINITE = range(7)
# graphic_geom.flags
KEEP_PADDED, CHECK_FINITE = 1, 2
(OP_SHIFT, OP_ROTATE, OP_ADI, OP_MEDIAN, OP_MEDIAN_WINDOW, OP_ADI_WINDOW, OP_BADPIX_MAP,
 OP_BADPIX_FIX) = range(8)

# every symbol that include/graphic.h declares
EXPORTS = (
    "graphic_create", "graphic_destroy", "graphic_status_string", "graphic_version",
    "graphic_resolved_pad", "graphic_workspace_size", "graphic_shift", "graphic_rotate", "graphic_rotate_noalloc",
    "graphic_median", "graphic_adi_reduce", "graphic_median_window", "graphic_alpha_min_deg",
    "graphic_adi_reduce_window",
    "graphic_parallactic_angles", "graphic_register", "graphic_median_nan", "graphic_mask_disk",
    "graphic_subtract_nearest", "graphic_badpix_map", "graphic_badpix_fix", "graphic_annular_rms",
    "graphic_batch_workspace_size", "graphic_adi_reduce_batch",
    "graphic_adi_graph_create", "graphic_graph_launch", "graphic_graph_destroy",
    "graphic_autotune", "graphic_tuning_export", "graphic_tuning_import",
    "graphic_timing_enable", "graphic_timing_read",
)
BATCH_INPLACE = 1


class Geom(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int64), ("n", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class CubeDesc(ctypes.Structure):
    _fields_ = [("cube", ctypes.c_void_p), ("n_frames", ctypes.c_int64), ("n", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("dx", ctypes.c_void_p), ("dy", ctypes.c_void_p),
                ("parang_deg", ctypes.c_void_p), ("final_img", ctypes.c_void_p), ("psf", ctypes.c_void_p),
                ("residuals", ctypes.c_void_p)]


class RegisterParams(ctypes.Structure):
    _fields_ = [("threshold", ctypes.c_double), ("min_size", ctypes.c_int32), ("max_size", ctypes.c_int32),
                ("half", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("saturation", ctypes.c_double)]


class GraphicError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s" % (where, status_string(status)))


_lib = None


def load():
    """Load libgraphic.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libgraphic.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    g = ctypes.POINTER(Geom)
    st = ctypes.c_int
    lib.graphic_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.graphic_create.restype = st
    lib.graphic_destroy.argtypes = [vp]
    lib.graphic_destroy.restype = None
    lib.graphic_status_string.argtypes = [st]
    lib.graphic_status_string.restype = ctypes.c_char_p
    lib.graphic_version.argtypes = []
    lib.graphic_version.restype = ctypes.c_char_p
    lib.graphic_resolved_pad.argtypes = [g]
    lib.graphic_resolved_pad.restype = i32
    lib.graphic_workspace_size.argtypes = [vp, ctypes.c_int, g, ctypes.POINTER(sz)]
    lib.graphic_workspace_size.restype = st
    lib.graphic_shift.argtypes = [vp, g, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.graphic_shift.restype = st
    lib.graphic_rotate.argtypes = [vp, g, vp, vp, vp, vp, vp, sz, vp]
    lib.graphic_rotate.restype = st
    lib.graphic_rotate_noalloc.argtypes = [vp, g, vp, vp, vp, vp, vp]
    lib.graphic_rotate_noalloc.restype = st
    lib.graphic_median.argtypes = [vp, g, vp, vp, vp, sz, vp]
    lib.graphic_median.restype = st
    lib.graphic_adi_reduce.argtypes = [vp, g, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.graphic_adi_reduce.restype = st
    f64 = ctypes.c_double
    lib.graphic_median_window.argtypes = [vp, g, vp, vp, vp, f64, f64, vp, vp, vp, sz, vp]
    lib.graphic_median_window.restype = st
    lib.graphic_alpha_min_deg.argtypes = [f64, f64, f64, ctypes.POINTER(f64)]
    lib.graphic_alpha_min_deg.restype = st
    lib.graphic_adi_reduce_window.argtypes = [vp, g, vp, vp, vp, vp, vp, f64, f64, vp, vp, vp, vp, sz, vp]
    lib.graphic_adi_reduce_window.restype = st
    lib.graphic_parallactic_angles.argtypes = [vp, vp, i64, f64, f64, f64, vp, vp]
    lib.graphic_parallactic_angles.restype = st
    lib.graphic_register.argtypes = [vp, g, vp, ctypes.POINTER(RegisterParams), vp, vp, vp]
    lib.graphic_register.restype = st
    lib.graphic_median_nan.argtypes = [vp, g, vp, vp, vp]
    lib.graphic_median_nan.restype = st
    lib.graphic_mask_disk.argtypes = [vp, g, vp, vp, vp, f64, vp]
    lib.graphic_mask_disk.restype = st
    lib.graphic_subtract_nearest.argtypes = [vp, g, vp, vp, vp, vp, i32, vp]
    lib.graphic_subtract_nearest.restype = st
    lib.graphic_badpix_map.argtypes = [vp, i32, vp, f64, vp, vp, vp, sz, vp]
    lib.graphic_badpix_map.restype = st
    lib.graphic_badpix_fix.argtypes = [vp, g, vp, vp, i32, ctypes.POINTER(i32), vp, sz, vp]
    lib.graphic_badpix_fix.restype = st
    lib.graphic_annular_rms.argtypes = [vp, g, vp, vp, f64, f64, f64, i32, vp, vp, vp]
    lib.graphic_annular_rms.restype = st
    cd = ctypes.POINTER(CubeDesc)
    lib.graphic_batch_workspace_size.argtypes = [vp, cd, ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(sz)]
    lib.graphic_batch_workspace_size.restype = st
    lib.graphic_adi_reduce_batch.argtypes = [vp, cd, ctypes.c_int, ctypes.c_uint32, vp, sz, vp]
    lib.graphic_adi_reduce_batch.restype = st
    lib.graphic_adi_graph_create.argtypes = [vp, cd, ctypes.c_int, ctypes.c_uint32, vp, sz, ctypes.POINTER(vp)]
    lib.graphic_adi_graph_create.restype = st
    lib.graphic_graph_launch.argtypes = [vp, vp]
    lib.graphic_graph_launch.restype = st
    lib.graphic_graph_destroy.argtypes = [vp]
    lib.graphic_graph_destroy.restype = None
    lib.graphic_autotune.argtypes = [vp, g, vp, sz, vp]
    lib.graphic_autotune.restype = st
    lib.graphic_tuning_export.argtypes = [vp, ctypes.c_char_p, sz, ctypes.POINTER(sz)]
    lib.graphic_tuning_export.restype = st
    lib.graphic_tuning_import.argtypes = [vp, ctypes.c_char_p]
    lib.graphic_tuning_import.restype = st
    lib.graphic_timing_enable.argtypes = [vp, ctypes.c_int]
    lib.graphic_timing_enable.restype = st
    lib.graphic_timing_read.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(i64)]
    lib.graphic_timing_read.restype = st
    _lib = lib
    return lib


def status_string(s):
    try:
        return load().graphic_status_string(int(s)).decode()
    except Exception:  # pragma: no cover - only when the library is absent
        return "status %d" % int(s)


def check(status, where):
    if status != OK:
        raise GraphicError(status, where)
