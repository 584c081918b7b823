"""Python binding of the binocular 2DGS frame path.

Argument marshalling only: tensors are handed to the C ABI (libbgs.so) as
device pointers with the current torch stream; every stage runs in the HIP
kernels.  Function names follow the C calls: render_dominant, reproject,
classify_holes, patch_rois, render_stereo (Sec. 3.1 Stages 1-4), plus the
stage-level exports used by the tests.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math

import numpy as np
import torch

from . import _abi
from ._abi import (BOX_BOTTOM, BOX_CENTER, BOX_LEFT, BOX_RIGHT, BOX_TOP, CLS_GAP, CLS_HOLE, CLS_ROI,  # noqa: F401
                   CLS_ROWFILL, CLS_WARPED)


class BgsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bgs error {code}: {msg}")
        self.code = code


@dataclasses.dataclass
class Raster:
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    lowpass: bool = True
    bg: tuple = (0.0, 0.0, 0.0)

    def c(self):
        r = _abi.RasterParams()
        r.alpha_min, r.alpha_max, r.t_min = self.alpha_min, self.alpha_max, self.t_min
        r.lowpass = int(bool(self.lowpass))
        for i in range(3):
            r.bg[i] = float(self.bg[i])
        return r


@dataclasses.dataclass
class Roi:
    margin: int = 32
    tile: int = 16
    edge_samples: int = 64
    gap_passes: int = 2
    center_roi: bool = True
    a_min: float = 0.5
    edge_bounds: int = 0  # 0: Eq. 6 over all edge samples; 1: each side's own edge, worst case
    view_colour: int = 0  # 1: reproject the colours seen from the affiliated eye (outside the paper's method)

    def c(self):
        r = _abi.RoiParams()
        r.margin, r.tile, r.edge_samples, r.gap_passes = self.margin, self.tile, self.edge_samples, self.gap_passes
        r.center_roi = int(bool(self.center_roi))
        r.a_min = self.a_min
        r.edge_bounds = int(self.edge_bounds)
        r.view_colour = int(self.view_colour)
        return r


def camera(cam) -> _abi.Camera:
    c = _abi.Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, np.float64).reshape(9)
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.t[i] = float(cam.t[i])
    c.z_near, c.z_far = float(cam.z_near), float(cam.z_far)
    return c


def _stats_dict(st):
    d = {}
    for f, _ in _abi.Stats._fields_:
        v = getattr(st, f)
        d[f] = [int(x) for x in v] if hasattr(v, "__len__") else int(v)
    return d


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def check_tensor(name, t, shape, dtype, device=None):
    """Raise ValueError unless t is a contiguous tensor of exactly this
    shape and dtype (and on this device, when given): the library writes
    through raw pointers sized from the camera, so a smaller or differently
    typed buffer would be overrun."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a tensor, got {type(t).__name__}")
    if tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(int(x) for x in shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if device is not None:
        dev = torch.device(device)
        if t.device.type != dev.type or (dev.index is not None and t.device.index != dev.index):
            raise ValueError(f"{name}: on {t.device}, expected {dev}")


def check_boxes(boxes, box_capacity, device):
    """A box list with room for at least box_capacity boxes of 6 int32."""
    if box_capacity < 0:
        raise ValueError("box_capacity must be >= 0")
    rows = boxes.shape[0] if isinstance(boxes, torch.Tensor) and boxes.dim() == 2 else -1
    check_tensor("boxes", boxes, (max(rows, 0), 6), torch.int32, device)
    if rows < max(box_capacity, 1):
        raise ValueError(f"boxes: room for {rows} boxes, box_capacity is {box_capacity}")


def _dev(device):
    """The concrete device the library's calls run on."""
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        return torch.device("cuda", torch.cuda.current_device())
    return d


def check_render_out(out, H, W, device):
    """Outputs of a full render of an H x W camera."""
    check_tensor("rgb", out["rgb"], (3, H, W), torch.float32, device)
    check_tensor("depth_raw", out["depth_raw"], (H, W), torch.float32, device)
    check_tensor("alpha", out["alpha"], (H, W), torch.float32, device)


def check_stereo_out(out, cam_dom, cam_aff, box_capacity, tile, device):
    """Outputs of a stereo frame: dominant-eye images at its size, the
    affiliated eye's images and class maps at its own size."""
    Hd, Wd, Ha, Wa = int(cam_dom.height), int(cam_dom.width), int(cam_aff.height), int(cam_aff.width)
    f32, u8, i32 = torch.float32, torch.uint8, torch.int32
    check_tensor("rgb_dom", out["rgb_dom"], (3, Hd, Wd), f32, device)
    check_tensor("depth_raw_dom", out["depth_raw_dom"], (Hd, Wd), f32, device)
    check_tensor("alpha_dom", out["alpha_dom"], (Hd, Wd), f32, device)
    check_tensor("rgb_aff", out["rgb_aff"], (3, Ha, Wa), f32, device)
    check_tensor("z_aff", out["z_aff"], (Ha, Wa), f32, device)
    check_tensor("alpha_aff", out["alpha_aff"], (Ha, Wa), f32, device)
    check_tensor("cls_aff", out["cls_aff"], (Ha, Wa), u8, device)
    check_tensor("labels", out["labels"], (Ha, Wa), i32, device)
    check_boxes(out["boxes"], box_capacity, device)
    check_tensor("n_boxes", out["n_boxes"], (1,), i32, device)
    check_tensor("tile_mask", out["tile_mask"], ((Ha + tile - 1) // tile, (Wa + tile - 1) // tile), u8, device)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class DeviceScene:
    """A scene resident in device memory (fp32 structure of arrays)."""

    def __init__(self, scene, device="cuda"):
        self.n = int(scene.n)
        self.sh_degree = int(scene.sh_degree)
        self.t = {k: torch.from_numpy(np.ascontiguousarray(getattr(scene, k), np.float32)).to(device)
                  for k in ("pos", "quat", "scale", "opacity", "sh")}
        s = _abi.Scene()
        s.n, s.sh_degree, s.reserved = self.n, self.sh_degree, 0
        s.pos, s.quat, s.scale, s.opacity, s.sh = [t.data_ptr() if t.numel() else None
                                                   for t in (self.t[k] for k in ("pos", "quat", "scale",
                                                                                 "opacity", "sh"))]
        self.c = s


class Context:
    """A library context bound to the current torch stream, with a workspace
    that grows when a frame needs more tile keys than it holds."""

    def __init__(self, sync: bool = True, device="cuda"):
        self.L = _abi.load()
        self.device = device
        h = C.c_void_p()
        self._check(self.L.bgs_ctx_create(C.byref(h), _stream()))
        self.h = h
        self.L.bgs_ctx_set_sync(self.h, int(bool(sync)))
        self.sync = bool(sync)
        self.ws = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.L.bgs_ctx_destroy(self.h)
        except Exception:
            pass

    def set_sync(self, sync: bool):
        self.sync = bool(sync)
        self.L.bgs_ctx_set_sync(self.h, int(bool(sync)))

    def set_count_pairs(self, on: bool):
        self._check(self.L.bgs_ctx_set_count_pairs(self.h, int(bool(on))))

    def set_blend_split(self, cap_dom: int = 1024, cap_roi: int = 32, seg_len: int = 32, far_dom: int = 0,
                        far_roi: int = 256):
        """Records a tile composites before the rest of its list may be split
        into segments (dominant / full renders, ROI patch; 0 = never), the
        segment length, and the extrapolated walk a pixel must still have for
        its tile to be split (dominant, ROI)."""
        self._check(self.L.bgs_ctx_set_blend_split(self.h, int(cap_dom), int(cap_roi), int(seg_len), int(far_dom),
                                                   int(far_roi)))

    def set_timing(self, on, stages=None):
        """Per-stage HIP-event timing on this context's stream (clears the
        totals).  on: True times every stage, False none; stages: names from
        _abi.STAGES to time instead of all of them."""
        mask = 0
        if on:
            mask = -1 if stages is None else sum(1 << _abi.STAGES.index(n) for n in stages)
        self._check(self.L.bgs_ctx_set_timing(self.h, mask))

    def timing_collect(self):
        """Accumulate the stages recorded since the last call (the stream must
        have been waited for) and return {stage: (total_ms, count)}."""
        n = len(_abi.STAGES)
        tot = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        self._check(self.L.bgs_timing_collect(self.h, tot, cnt))
        return {name: (tot[i], cnt[i]) for i, name in enumerate(_abi.STAGES)}

    def blend_trace(self, n, W, H):
        """Per-tile trace of the last counting-mode dominant blend:
        (tile, list length, longest wave walk, CU, start, end) rows."""
        nt = ((W + 15) // 16) * ((H + 15) // 16)
        out = np.zeros((nt, 6), np.int64)
        self._check(self.L.bgs_blend_trace(self.h, int(n), int(W), int(H), _ptr(self.ws), self.ws.numel(),
                                           out.ctypes.data_as(C.c_void_p)))
        return out

    def poll_status(self):
        st = _abi.Stats()
        self._check(self.L.bgs_poll_status(self.h, _ptr(self.ws), self.ws.numel(), C.byref(st)))
        return _stats_dict(st)

    def _check(self, rc):
        if rc != 0:
            msg = self.L.bgs_last_error(getattr(self, "h", None)) if hasattr(self, "h") else b""
            raise BgsError(rc, (msg or b"").decode())

    def bind_stream(self):
        self.L.bgs_ctx_set_stream(self.h, _stream())

    def workspace(self, n, W, H, key_capacity):
        need = C.c_size_t()
        self._check(self.L.bgs_workspace_size(int(n), int(W), int(H), int(key_capacity), C.byref(need)))
        if self.ws is None or self.ws.numel() < need.value:
            self.ws = torch.empty(int(need.value), dtype=torch.uint8, device=self.device)
        return self.ws

    def reserve(self, n, W, H, key_capacity):
        """Make the workspace hold at least key_capacity keys for this size."""
        return self.workspace(n, W, H, key_capacity)

    # -- Stage 1 -------------------------------------------------------------
    def render_dominant(self, scene: DeviceScene, cam, raster: Raster = Raster(), out=None):
        self.bind_stream()
        W, H = int(cam.width), int(cam.height)
        if out is None:
            out = dict(rgb=torch.empty((3, H, W), device=self.device), depth_raw=torch.empty((H, W), device=self.device),
                       alpha=torch.empty((H, W), device=self.device))
        check_render_out(out, H, W, _dev(self.device))
        if self.ws is None:
            self.workspace(scene.n, W, H, max(1 << 16, 8 * scene.n))
        nk = C.c_int64(0)
        for _ in range(4):
            rc = self.L.bgs_render_dominant(self.h, C.byref(scene.c), C.byref(camera(cam)), C.byref(raster.c()),
                                            _ptr(self.ws), self.ws.numel(), _ptr(out["rgb"]), _ptr(out["depth_raw"]),
                                            _ptr(out["alpha"]), C.byref(nk))
            if rc != _abi.ERR_CAPACITY and rc != _abi.ERR_WORKSPACE:
                break
            self.workspace(scene.n, W, H, int(max(nk.value, 1) * 1.25) + 1024)
        self._check(rc)
        out["n_keys"] = int(nk.value)
        return out

    # -- Stage 2 -------------------------------------------------------------
    def reproject(self, src, dst, rgb, depth_raw, alpha, roi: Roi = Roi(), out=None):
        self.bind_stream()
        W, H = int(dst.width), int(dst.height)
        if out is None:
            out = dict(rgb=torch.empty((3, H, W), device=self.device), z=torch.empty((H, W), device=self.device),
                       alpha=torch.empty((H, W), device=self.device),
                       hole=torch.empty((H, W), dtype=torch.uint8, device=self.device),
                       depth_range=torch.empty(2, device=self.device))
        dev = _dev(self.device)
        Hs, Ws = int(src.height), int(src.width)
        check_tensor("rgb_src", rgb, (3, Hs, Ws), torch.float32, dev)
        check_tensor("depth_raw_src", depth_raw, (Hs, Ws), torch.float32, dev)
        check_tensor("alpha_src", alpha, (Hs, Ws), torch.float32, dev)
        check_tensor("rgb", out["rgb"], (3, H, W), torch.float32, dev)
        check_tensor("z", out["z"], (H, W), torch.float32, dev)
        check_tensor("alpha", out["alpha"], (H, W), torch.float32, dev)
        check_tensor("hole", out["hole"], (H, W), torch.uint8, dev)
        check_tensor("depth_range", out["depth_range"], (2,), torch.float32, dev)
        ws = self.ws if self.ws is not None else self.workspace(0, W, H, 0)
        if ws.numel() < self._ws_bytes(0, W, H, 0):
            ws = self.workspace(0, W, H, 0)
        self._check(self.L.bgs_reproject(self.h, C.byref(camera(src)), C.byref(camera(dst)), C.byref(roi.c()),
                                         _ptr(rgb), _ptr(depth_raw), _ptr(alpha), _ptr(ws), ws.numel(),
                                         _ptr(out["rgb"]), _ptr(out["z"]), _ptr(out["alpha"]), _ptr(out["hole"]),
                                         _ptr(out["depth_range"])))
        return out

    def reproject_noalloc(self, src, dst, rgb, depth_raw, alpha, roi: Roi = Roi(), out=None):
        """Stage 2 through bgs_reproject_noalloc: the library's static scratch
        instead of a workspace (nothing allocated by the call itself; pass
        `out` to allocate nothing here either)."""
        self.bind_stream()
        W, H = int(dst.width), int(dst.height)
        if out is None:
            out = dict(rgb=torch.empty((3, H, W), device=self.device), z=torch.empty((H, W), device=self.device),
                       alpha=torch.empty((H, W), device=self.device),
                       hole=torch.empty((H, W), dtype=torch.uint8, device=self.device),
                       depth_range=torch.empty(2, device=self.device))
        dev = _dev(self.device)
        Hs, Ws = int(src.height), int(src.width)
        check_tensor("rgb_src", rgb, (3, Hs, Ws), torch.float32, dev)
        check_tensor("depth_raw_src", depth_raw, (Hs, Ws), torch.float32, dev)
        check_tensor("alpha_src", alpha, (Hs, Ws), torch.float32, dev)
        check_tensor("rgb", out["rgb"], (3, H, W), torch.float32, dev)
        check_tensor("z", out["z"], (H, W), torch.float32, dev)
        check_tensor("alpha", out["alpha"], (H, W), torch.float32, dev)
        check_tensor("hole", out["hole"], (H, W), torch.uint8, dev)
        check_tensor("depth_range", out["depth_range"], (2,), torch.float32, dev)
        self._check(self.L.bgs_reproject_noalloc(self.h, C.byref(camera(src)), C.byref(camera(dst)),
                                                 C.byref(roi.c()), _ptr(rgb), _ptr(depth_raw), _ptr(alpha),
                                                 _ptr(out["rgb"]), _ptr(out["z"]), _ptr(out["alpha"]),
                                                 _ptr(out["hole"]), _ptr(out["depth_range"])))
        return out

    def _ws_bytes(self, n, W, H, k):
        need = C.c_size_t()
        self._check(self.L.bgs_workspace_size(int(n), int(W), int(H), int(k), C.byref(need)))
        return need.value

    # -- Stage 3 -------------------------------------------------------------
    def classify_holes(self, src, dst, depth_range, rgb, z, alpha, cls, roi: Roi = Roi(), raster: Raster = Raster(),
                       box_capacity: int = 4096, out=None):
        """rgb, z, alpha and cls are updated in place (cls enters as the hole mask)."""
        self.bind_stream()
        W, H = int(dst.width), int(dst.height)
        T = roi.tile
        if out is None:
            out = dict(labels=torch.empty((H, W), dtype=torch.int32, device=self.device),
                       boxes=torch.empty((max(box_capacity, 1), 6), dtype=torch.int32, device=self.device),
                       n_boxes=torch.empty(1, dtype=torch.int32, device=self.device),
                       tile_mask=torch.empty(((H + T - 1) // T, (W + T - 1) // T), dtype=torch.uint8,
                                             device=self.device))
        dev = _dev(self.device)
        check_tensor("depth_range", depth_range, (2,), torch.float32, dev)
        check_tensor("rgb", rgb, (3, H, W), torch.float32, dev)
        check_tensor("z", z, (H, W), torch.float32, dev)
        check_tensor("alpha", alpha, (H, W), torch.float32, dev)
        check_tensor("cls", cls, (H, W), torch.uint8, dev)
        check_tensor("labels", out["labels"], (H, W), torch.int32, dev)
        check_boxes(out["boxes"], box_capacity, dev)
        check_tensor("n_boxes", out["n_boxes"], (1,), torch.int32, dev)
        check_tensor("tile_mask", out["tile_mask"], ((H + T - 1) // T, (W + T - 1) // T), torch.uint8, dev)
        ws = self.ws if self.ws is not None else self.workspace(0, W, H, 0)
        if ws.numel() < self._ws_bytes(0, W, H, 0):
            ws = self.workspace(0, W, H, 0)
        self._check(self.L.bgs_classify_holes(self.h, C.byref(camera(src)), C.byref(camera(dst)), C.byref(roi.c()),
                                              C.byref(raster.c()), _ptr(depth_range), _ptr(ws), ws.numel(),
                                              _ptr(rgb), _ptr(z), _ptr(alpha), _ptr(cls), _ptr(out["labels"]),
                                              _ptr(out["boxes"]), int(box_capacity), _ptr(out["n_boxes"]),
                                              _ptr(out["tile_mask"])))
        return out

    # -- Stage 4 -------------------------------------------------------------
    def patch_rois(self, scene: DeviceScene, dst, tile_mask, rgb, z, alpha, cls, raster: Raster = Raster(),
                   roi: Roi = Roi()):
        self.bind_stream()
        W, H = int(dst.width), int(dst.height)
        T = roi.tile
        dev = _dev(self.device)
        check_tensor("tile_mask", tile_mask, ((H + T - 1) // T, (W + T - 1) // T), torch.uint8, dev)
        check_tensor("rgb", rgb, (3, H, W), torch.float32, dev)
        check_tensor("z", z, (H, W), torch.float32, dev)
        check_tensor("alpha", alpha, (H, W), torch.float32, dev)
        check_tensor("cls", cls, (H, W), torch.uint8, dev)
        if self.ws is None:
            self.workspace(scene.n, W, H, max(1 << 16, 4 * scene.n))
        nk = C.c_int64(0)
        for _ in range(4):
            rc = self.L.bgs_patch_rois(self.h, C.byref(scene.c), C.byref(camera(dst)), C.byref(raster.c()),
                                       C.byref(roi.c()), _ptr(tile_mask), _ptr(self.ws), self.ws.numel(), _ptr(rgb),
                                       _ptr(z), _ptr(alpha), _ptr(cls), C.byref(nk))
            if rc != _abi.ERR_CAPACITY and rc != _abi.ERR_WORKSPACE:
                break
            self.workspace(scene.n, W, H, int(max(nk.value, 1) * 1.25) + 1024)
        self._check(rc)
        return int(nk.value)

    # -- Stages 1-4 ----------------------------------------------------------
    def render_stereo(self, scene: DeviceScene, cam_dom, cam_aff, raster: Raster = Raster(), roi: Roi = Roi(),
                      box_capacity: int = 4096, out=None):
        self.bind_stream()
        W, H = max(cam_dom.width, cam_aff.width), max(cam_dom.height, cam_aff.height)
        T = roi.tile
        d = self.device
        if out is None:
            out = dict(
                rgb_dom=torch.empty((3, cam_dom.height, cam_dom.width), device=d),
                depth_raw_dom=torch.empty((cam_dom.height, cam_dom.width), device=d),
                alpha_dom=torch.empty((cam_dom.height, cam_dom.width), device=d),
                rgb_aff=torch.empty((3, cam_aff.height, cam_aff.width), device=d),
                z_aff=torch.empty((cam_aff.height, cam_aff.width), device=d),
                alpha_aff=torch.empty((cam_aff.height, cam_aff.width), device=d),
                cls_aff=torch.empty((cam_aff.height, cam_aff.width), dtype=torch.uint8, device=d),
                labels=torch.empty((cam_aff.height, cam_aff.width), dtype=torch.int32, device=d),
                boxes=torch.empty((max(box_capacity, 1), 6), dtype=torch.int32, device=d),
                n_boxes=torch.empty(1, dtype=torch.int32, device=d),
                tile_mask=torch.empty(((cam_aff.height + T - 1) // T, (cam_aff.width + T - 1) // T),
                                      dtype=torch.uint8, device=d))
        check_stereo_out(out, cam_dom, cam_aff, box_capacity, T, _dev(d))
        if self.ws is None:
            self.workspace(scene.n, W, H, max(1 << 16, 8 * scene.n))
        st = _abi.Stats()
        st_arg = C.byref(st) if self.sync else None
        for _ in range(4):
            rc = self.L.bgs_render_stereo(self.h, C.byref(scene.c), C.byref(camera(cam_dom)), C.byref(camera(cam_aff)),
                                          C.byref(raster.c()), C.byref(roi.c()), _ptr(self.ws), self.ws.numel(),
                                          _ptr(out["rgb_dom"]), _ptr(out["depth_raw_dom"]), _ptr(out["alpha_dom"]),
                                          _ptr(out["rgb_aff"]), _ptr(out["z_aff"]), _ptr(out["alpha_aff"]),
                                          _ptr(out["cls_aff"]), _ptr(out["labels"]), _ptr(out["boxes"]),
                                          int(box_capacity), _ptr(out["n_boxes"]), _ptr(out["tile_mask"]),
                                          st_arg)
            if rc != _abi.ERR_CAPACITY and rc != _abi.ERR_WORKSPACE:
                break
            need = max(st.n_keys_dom, st.n_keys_roi, 1)
            self.workspace(scene.n, W, H, int(need * 1.25) + 1024)
        self._check(rc)
        if self.sync:
            out["stats"] = _stats_dict(st)
        return out

    # -- stage-level exports ------------------------------------------------
    def sort_pairs(self, keys, values, key_bits):
        """Stable in-place radix sort of uint32 (as int32 tensors) pairs."""
        self.bind_stream()
        n = keys.numel()
        check_tensor("keys", keys, (n,), torch.int32, _dev(self.device))
        check_tensor("values", values, (n,), torch.int32, _dev(self.device))
        need = C.c_size_t()
        self._check(self.L.bgs_sort_workspace_size(n, C.byref(need)))
        ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=self.device)
        self._check(self.L.bgs_sort_pairs(self.h, _ptr(keys), _ptr(values), n, int(key_bits), _ptr(ws), ws.numel()))
        return keys, values

    def label_components(self, mask, conn=8):
        self.bind_stream()
        H, W = mask.shape
        check_tensor("mask", mask, (H, W), torch.uint8, _dev(self.device))
        labels = torch.empty((H, W), dtype=torch.int32, device=self.device)
        self._check(self.L.bgs_label_components(self.h, _ptr(mask), int(W), int(H), int(conn), _ptr(labels)))
        return labels

    def preprocess_debug(self, scene: DeviceScene, cam, raster: Raster = Raster()):
        self.bind_stream()
        n = scene.n
        ws = self.workspace(n, cam.width, cam.height, 0)
        zkey = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        rects = torch.empty((max(n, 1), 4), dtype=torch.int32, device=self.device)
        counts = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        self._check(self.L.bgs_preprocess_debug(self.h, C.byref(scene.c), C.byref(camera(cam)), C.byref(raster.c()),
                                                _ptr(ws), ws.numel(), _ptr(zkey), _ptr(rects), _ptr(counts)))
        return zkey[:n], rects[:n], counts[:n]

    def tile_lists_debug(self, scene: DeviceScene, cam, raster: Raster = Raster(), capacity=None):
        self.bind_stream()
        T = 16
        n_tiles = ((cam.width + T - 1) // T) * ((cam.height + T - 1) // T)
        cap = capacity or max(1 << 16, 8 * scene.n)
        ws = self.workspace(scene.n, cam.width, cam.height, cap)
        ranges = torch.empty((n_tiles, 2), dtype=torch.int32, device=self.device)
        vals = torch.empty(cap, dtype=torch.int32, device=self.device)
        nk = C.c_int64(0)
        self._check(self.L.bgs_tile_lists_debug(self.h, C.byref(scene.c), C.byref(camera(cam)), C.byref(raster.c()),
                                                _ptr(ws), ws.numel(), _ptr(ranges), _ptr(vals), cap, C.byref(nk)))
        return ranges, vals[:int(nk.value)], int(nk.value)


def psnr(a: torch.Tensor, b: torch.Tensor) -> float:
    """PSNR of two images with values in [0, 1] (both clamped first)."""
    mse = torch.mean((a.clamp(0, 1).double() - b.clamp(0, 1).double()) ** 2).item()
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)
