"""ctypes declarations of the C ABI in include/gsr.h (libgsr.so, built in-tree).

Loading fails loudly when the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgsr.so")

GSR_OK = 0
GSR_ERR_INVALID_ARG = 1
GSR_ERR_WORKSPACE_TOO_SMALL = 2
GSR_ERR_DEVICE = 3
GSR_ERR_UNSUPPORTED = 4
GSR_FP32 = 0
GSR_FP16_BLEND = 1
GSR_FP16_BLEND_T = 2
GSR_FAULT_NONE = 0
GSR_FAULT_ABORT_BEFORE_SORT = 1
GSR_FAULT_WITHHOLD_STATUS = 2
GSR_TILE = 16
GSR_CLUSTER = 128
GSR_MAX_VIEWS = 64
GSR_MAX_BATCH = 16
GSR_NOALLOC_MAX_TILES = 262144

STATUS_NAMES = {0: "GSR_OK", 1: "GSR_ERR_INVALID_ARG", 2: "GSR_ERR_WORKSPACE_TOO_SMALL", 3: "GSR_ERR_DEVICE",
                4: "GSR_ERR_UNSUPPORTED"}

c_int32, c_int64, c_float, c_void_p, c_size_t = (ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p,
                                                 ctypes.c_size_t)


class GsrScene(ctypes.Structure):
    _fields_ = [("n", c_int64), ("sh_degree", c_int32), ("means", c_void_p), ("log_scales", c_void_p),
                ("quats", c_void_p), ("opacity_logits", c_void_p), ("sh", c_void_p)]


class GsrCamera(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("R", c_float * 9), ("t", c_float * 3), ("near_plane", c_float),
                ("bg", c_float * 3)]


class GsrOptions(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("cluster_cull", c_int32), ("stats", c_int32), ("deterministic", c_int32),
                ("radius_mode", c_int32), ("half_reduction", c_int32), ("tile_width", c_int32)]


class GsrGrads(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p), ("opacity_logits", c_void_p),
                ("sh", c_void_p)]


class GsrAdamOptions(ctypes.Structure):
    _fields_ = [("lr_means", c_float), ("lr_log_scales", c_float), ("lr_quats", c_float), ("lr_opacity", c_float),
                ("lr_sh_dc", c_float), ("lr_sh_rest", c_float), ("beta1", c_float), ("beta2", c_float),
                ("eps", c_float), ("reserved", c_int32), ("step", c_int64)]


class GsrDensifyOptions(ctypes.Structure):
    _fields_ = [("threshold", c_float), ("split_log_scale", c_float), ("split_factor", c_float),
                ("prune_logit", c_float), ("max_candidates", c_int64)]


class GsrStats(ctypes.Structure):
    _fields_ = [("S", c_void_p), ("M", c_void_p), ("C", c_void_p)]


class GsrFrameInfo(ctypes.Structure):
    _fields_ = [("n", c_int64), ("n_visible_slots", c_int64), ("instances", c_int64), ("tiles", c_int64),
                ("pixels", c_int64), ("views", c_int32), ("clusters", c_int32), ("visible_clusters", c_int32),
                ("split_tiles", c_int32), ("split_tiles_bwd", c_int32), ("reserved", c_int32)]


class GsrFrameBuffers(ctypes.Structure):
    _fields_ = [("record", c_void_p), ("depth_key", c_void_p), ("tiles", c_void_p), ("rect", c_void_p),
                ("compact2full", c_void_p), ("inst_tile", c_void_p), ("inst_record", c_void_p),
                ("ranges", c_void_p), ("pixel_T", c_void_p), ("pixel_last", c_void_p),
                ("grad2d", c_void_p), ("cluster_bounds", c_void_p), ("cluster_visible", c_void_p),
                ("pixel_base", c_int64 * GSR_MAX_VIEWS), ("tile_base", c_int64 * GSR_MAX_VIEWS),
                ("fwd_items", c_void_p), ("bwd_items", c_void_p)]


EXPORTS = {
    "gsr_context_create": (c_int32, [c_int32, ctypes.POINTER(c_void_p)]),
    "gsr_context_destroy": (None, [c_void_p]),
    "gsr_last_error": (ctypes.c_char_p, [c_void_p]),
    "gsr_required_workspace": (c_size_t, [c_void_p]),
    "gsr_workspace_size": (c_int32, [c_void_p, ctypes.POINTER(GsrScene), ctypes.POINTER(GsrCamera), c_int32,
                                     ctypes.POINTER(GsrOptions), c_int64, ctypes.POINTER(c_size_t)]),
    "gsr_forward": (c_int32, [c_void_p, ctypes.POINTER(GsrScene), ctypes.POINTER(GsrCamera), c_int32,
                              ctypes.POINTER(GsrOptions), c_void_p, c_size_t, ctypes.POINTER(c_void_p), c_void_p]),
    "gsr_backward": (c_int32, [c_void_p, ctypes.POINTER(GsrScene), ctypes.POINTER(GsrCamera), c_int32,
                               ctypes.POINTER(GsrOptions), c_void_p, c_size_t, ctypes.POINTER(c_void_p),
                               ctypes.POINTER(GsrGrads), ctypes.POINTER(GsrStats), c_void_p]),
    "gsr_frame_inspect": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(GsrFrameInfo),
                                    ctypes.POINTER(GsrFrameBuffers)]),
    "gsr_frame_release": (c_int32, [c_void_p, c_void_p]),
    "gsr_prepare": (c_int32, [c_void_p, ctypes.POINTER(GsrScene), ctypes.POINTER(GsrCamera), c_int32,
                              ctypes.POINTER(GsrOptions), c_void_p, c_size_t, c_void_p]),
    "gsr_raster_batch_workspace_size": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p),
                                                  ctypes.POINTER(c_size_t)]),
    "gsr_raster_batch": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p), ctypes.POINTER(ctypes.POINTER(c_void_p)),
                                   c_int32, c_void_p, c_size_t, c_void_p]),
    "gsr_raster_batch_noalloc": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p),
                                           ctypes.POINTER(ctypes.POINTER(c_void_p)), c_int32, c_void_p]),
    "gsr_variance": (c_int32, [c_void_p, ctypes.POINTER(GsrStats), c_int64, c_void_p, c_void_p]),
    "gsr_morton_workspace_size": (c_int32, [c_void_p, c_int64, ctypes.POINTER(c_size_t)]),
    "gsr_morton_order": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_size_t, c_void_p, c_void_p, c_void_p]),
    "gsr_sort_workspace_size": (c_int32, [c_void_p, c_int64, c_int32, ctypes.POINTER(c_size_t)]),
    "gsr_sort_u32": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_size_t,
                               c_void_p]),
    "gsr_apply_permutation": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, ctypes.POINTER(c_void_p),
                                        ctypes.POINTER(c_void_p), ctypes.POINTER(c_int32), c_void_p]),
    "gsr_l1_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p]),
    "gsr_sparse_adam": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, ctypes.POINTER(GsrGrads),
                                  ctypes.POINTER(GsrGrads), ctypes.POINTER(GsrGrads), ctypes.POINTER(GsrGrads),
                                  ctypes.POINTER(GsrAdamOptions), c_void_p]),
    "gsr_backward_adam": (c_int32, [c_void_p, ctypes.POINTER(GsrScene), ctypes.POINTER(GsrCamera), c_int32,
                                    ctypes.POINTER(GsrOptions), c_void_p, c_size_t, ctypes.POINTER(c_void_p),
                                    ctypes.POINTER(GsrGrads), ctypes.POINTER(GsrGrads),
                                    ctypes.POINTER(GsrAdamOptions), ctypes.POINTER(GsrStats), c_void_p]),
    "gsr_densify_workspace_size": (c_int32, [c_void_p, c_int64, c_int64, ctypes.POINTER(c_size_t)]),
    "gsr_densify": (c_int32, [c_void_p, ctypes.POINTER(GsrScene), c_void_p, c_void_p,
                              ctypes.POINTER(GsrDensifyOptions), ctypes.POINTER(GsrGrads), c_int64, c_int32,
                              ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), ctypes.POINTER(c_int32), c_void_p,
                              c_size_t, c_void_p, c_void_p]),
    "gsr_opacity_decay": (c_int32, [c_void_p, c_void_p, c_int64, c_float, c_void_p]),
    "gsr_set_raster_split": (c_int32, [c_void_p, ctypes.c_uint32, ctypes.c_uint32]),
    "gsr_set_profiling": (c_int32, [c_void_p, c_int32]),
    "gsr_set_fault_injection": (c_int32, [c_void_p, c_int32]),
    "gsr_stage_times": (c_int32, [c_void_p, ctypes.POINTER(c_float)]),
}

STAGES = ["cluster", "preprocess", "depth_sort", "offsets", "emit", "tile_sort", "ranges", "raster_fwd",
          "zero_grad", "raster_bwd", "preprocess_bwd"]

_lib = None


class GsrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status


def load(path: str | None = None):
    """Loads libgsr.so (raises if it has not been built: python -m paper_2503_01199_amd.build)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError("libgsr.so is not built (%s); run `python -m paper_2503_01199_amd.build`" % p)
    lib = ctypes.CDLL(p)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib
