"""ctypes view of include/bgs.h.  Loading fails loudly when the HIP library
has not been built: there is no fallback path."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbgs.so")

OK, ERR_INVALID_ARG, ERR_WORKSPACE, ERR_CAPACITY, ERR_HIP, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
BOX_LEFT, BOX_RIGHT, BOX_TOP, BOX_BOTTOM, BOX_CENTER = 0, 1, 2, 3, 4
CLS_WARPED, CLS_HOLE, CLS_GAP, CLS_ROI, CLS_ROWFILL = 0, 1, 2, 3, 4
REPROJECT_NOALLOC_MAX_PIXELS = 1 << 23


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("R", C.c_double * 9), ("t", C.c_double * 3),
                ("z_near", C.c_double), ("z_far", C.c_double)]


class Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("reserved", C.c_int32), ("pos", C.c_void_p),
                ("quat", C.c_void_p), ("scale", C.c_void_p), ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class RasterParams(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("lowpass", C.c_int32), ("bg", C.c_float * 3), ("reserved", C.c_int32)]


class RoiParams(C.Structure):
    _fields_ = [("margin", C.c_int32), ("tile", C.c_int32), ("edge_samples", C.c_int32),
                ("gap_passes", C.c_int32), ("center_roi", C.c_int32), ("a_min", C.c_float),
                ("edge_bounds", C.c_int32), ("view_colour", C.c_int32)]


class Box(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("x1", C.c_int32), ("y1", C.c_int32),
                ("kind", C.c_int32), ("label", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_keys_dom", C.c_int64), ("n_keys_roi", C.c_int64), ("n_holes", C.c_int32),
                ("n_gap", C.c_int32), ("n_center", C.c_int32), ("n_rowfill", C.c_int32),
                ("n_boxes", C.c_int32), ("n_roi_tiles", C.c_int32), ("overflow", C.c_int32),
                ("reserved", C.c_int32), ("pairs_eval_dom", C.c_int64), ("pairs_used_dom", C.c_int64),
                ("pairs_eval_roi", C.c_int64), ("pairs_used_roi", C.c_int64),
                ("blend_work_dom", C.c_int64 * 4), ("blend_work_roi", C.c_int64 * 4)]


class BatchPair(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("cam_dom", Camera), ("cam_aff", Camera), ("roi", RoiParams),
                ("box_capacity", C.c_int32), ("ws", C.c_void_p), ("ws_bytes", C.c_size_t),
                ("rgb_dom", C.c_void_p), ("depth_raw_dom", C.c_void_p), ("alpha_dom", C.c_void_p),
                ("rgb_aff", C.c_void_p), ("z_aff", C.c_void_p), ("alpha_aff", C.c_void_p),
                ("cls_aff", C.c_void_p), ("labels", C.c_void_p), ("boxes", C.c_void_p), ("n_boxes", C.c_void_p),
                ("tile_mask", C.c_void_p)]


STAGES = ["preprocess_dom", "depth_sort_dom", "emit_dom", "tile_sort_dom", "ranges_dom", "blend_dom",
          "reproject", "classify", "preprocess_roi", "depth_sort_roi", "emit_roi", "tile_sort_roi", "ranges_roi",
          "blend_roi"]


EXPORTS = [
    "bgs_ctx_create", "bgs_ctx_destroy", "bgs_ctx_set_stream", "bgs_ctx_set_sync", "bgs_last_error",
    "bgs_workspace_size", "bgs_poll_status", "bgs_render_dominant", "bgs_reproject", "bgs_reproject_noalloc",
    "bgs_classify_holes",
    "bgs_patch_rois", "bgs_render_stereo", "bgs_sort_workspace_size", "bgs_sort_pairs",
    "bgs_label_components", "bgs_preprocess_debug", "bgs_tile_lists_debug", "bgs_ctx_set_count_pairs",
    "bgs_ctx_set_timing", "bgs_timing_collect", "bgs_blend_trace", "bgs_ctx_set_blend_split",
    "bgs_batch_workspace_size", "bgs_render_stereo_batch", "bgs_batch_graph_capture", "bgs_graph_launch",
    "bgs_graph_destroy",
    # include/bgs_repair.h
    "bgs_repair_num_params", "bgs_repair_workspace_size", "bgs_repair_forward", "bgs_repair_grad",
    "bgs_repair_adam", "bgs_repair_hole_error", "bgs_repair_set_block_shape",
]

_lib = None


def load():
    """Load libbgs.so and declare every entry point's signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2609_30741_amd.build`")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    sig = {
        "bgs_ctx_create": [C.POINTER(P), P],
        "bgs_ctx_destroy": [P],
        "bgs_ctx_set_stream": [P, P],
        "bgs_ctx_set_sync": [P, I32],
        "bgs_ctx_set_count_pairs": [P, I32],
        "bgs_ctx_set_timing": [P, I32],
        "bgs_ctx_set_blend_split": [P, I32, I32, I32, I32, I32],
        "bgs_timing_collect": [P, P, P],
        "bgs_workspace_size": [I64, I32, I32, I64, C.POINTER(SZ)],
        "bgs_poll_status": [P, P, SZ, C.POINTER(Stats)],
        "bgs_render_dominant": [P, C.POINTER(Scene), C.POINTER(Camera), C.POINTER(RasterParams), P, SZ, P, P, P,
                                C.POINTER(I64)],
        "bgs_reproject": [P, C.POINTER(Camera), C.POINTER(Camera), C.POINTER(RoiParams), P, P, P, P, SZ, P, P, P, P,
                          P],
        "bgs_reproject_noalloc": [P, C.POINTER(Camera), C.POINTER(Camera), C.POINTER(RoiParams), P, P, P, P, P, P,
                                  P, P],
        "bgs_classify_holes": [P, C.POINTER(Camera), C.POINTER(Camera), C.POINTER(RoiParams),
                               C.POINTER(RasterParams), P, P, SZ, P, P, P, P, P, P, I32, P, P],
        "bgs_patch_rois": [P, C.POINTER(Scene), C.POINTER(Camera), C.POINTER(RasterParams), C.POINTER(RoiParams), P,
                           P, SZ, P, P, P, P, C.POINTER(I64)],
        "bgs_render_stereo": [P, C.POINTER(Scene), C.POINTER(Camera), C.POINTER(Camera), C.POINTER(RasterParams),
                              C.POINTER(RoiParams), P, SZ, P, P, P, P, P, P, P, P, P, I32, P, P, C.POINTER(Stats)],
        "bgs_batch_workspace_size": [I32, C.POINTER(SZ)],
        "bgs_render_stereo_batch": [P, I32, C.POINTER(BatchPair), C.POINTER(RasterParams), P, SZ],
        "bgs_batch_graph_capture": [P, I32, C.POINTER(BatchPair), C.POINTER(RasterParams), P, SZ, C.POINTER(P)],
        "bgs_graph_launch": [P, P],
        "bgs_graph_destroy": [P],
        "bgs_sort_workspace_size": [I64, C.POINTER(SZ)],
        "bgs_blend_trace": [P, I64, I32, I32, P, SZ, P],
        "bgs_sort_pairs": [P, P, P, I64, I32, P, SZ],
        "bgs_label_components": [P, P, I32, I32, I32, P],
        "bgs_preprocess_debug": [P, C.POINTER(Scene), C.POINTER(Camera), C.POINTER(RasterParams), P, SZ, P, P, P],
        "bgs_tile_lists_debug": [P, C.POINTER(Scene), C.POINTER(Camera), C.POINTER(RasterParams), P, SZ, P, P, I64,
                                 C.POINTER(I64)],
        "bgs_repair_num_params": [C.POINTER(I64)],
        "bgs_repair_workspace_size": [I32, I32, I32, I32, C.POINTER(SZ)],
        "bgs_repair_forward": [P, I32, I32, I32, P, P, P, P, P, P, SZ, P],
        "bgs_repair_grad": [P, I32, I32, I32, P, P, P, P, P, P, P, P, SZ, P],
        "bgs_repair_adam": [P, P, P, P, I64, I32, C.c_float, C.c_float, C.c_float, C.c_float, P],
        "bgs_repair_hole_error": [P, P, I32, I32, I32, P, P, P],
        "bgs_repair_set_block_shape": [I32, I32],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = I32
    L.bgs_last_error.argtypes = [P]
    L.bgs_last_error.restype = C.c_char_p
    _lib = L
    return L
