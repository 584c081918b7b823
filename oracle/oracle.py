"""ctypes front end of the CPU oracle (``bgs_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it; the product path never does.
It shares no code with the HIP library; cameras and scenes are read by
attribute (the synthetic input generator produces them).

``render_stereo`` composes the stages in the order of the paper's
pipeline (Sec. 3.1): full dominant render with the depth proxy, forward
reprojection, hole categorisation with interpolation, ROI re-rendering.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bgs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CLS_WARPED, CLS_HOLE, CLS_GAP, CLS_ROI, CLS_ROWFILL = 0, 1, 2, 3, 4
BOX_LEFT, BOX_RIGHT, BOX_TOP, BOX_BOTTOM, BOX_CENTER = 0, 1, 2, 3, 4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: fp64, OpenMP, no floating-point
    contraction (the reprojection recipe is evaluated op by op)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Cam(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("R", C.c_double * 9), ("t", C.c_double * 3),
                ("z_near", C.c_double), ("z_far", C.c_double)]


class _Raster(C.Structure):
    _fields_ = [("alpha_min", C.c_double), ("alpha_max", C.c_double), ("t_min", C.c_double),
                ("lowpass", C.c_int32), ("pad", C.c_int32), ("bg", C.c_double * 3)]


class _Roi(C.Structure):
    _fields_ = [("margin", C.c_int32), ("tile", C.c_int32), ("edge_samples", C.c_int32),
                ("gap_passes", C.c_int32), ("center_roi", C.c_int32), ("edge_bounds", C.c_int32),
                ("a_min", C.c_double)]


class _Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("pos", C.c_void_p), ("quat", C.c_void_p),
                ("scale", C.c_void_p), ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class _ClsStats(C.Structure):
    _fields_ = [("n_holes", C.c_int64), ("n_gap", C.c_int64), ("n_center", C.c_int64),
                ("n_boxes", C.c_int64), ("n_roi_tiles", C.c_int64), ("n_rowfill", C.c_int64)]


@dataclasses.dataclass
class Raster:
    """Compositing constants of the 3DGS/2DGS rasteriser family the paper
    builds on (Sec. 2.2, Sec. 3.2): alpha clamp, skip and early-stop
    thresholds, the screen-space low-pass term and the background."""
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    lowpass: bool = True
    bg: tuple = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class Roi:
    """ROI generator settings (Sec. 3.5): margin m = 32, 16x16 tiles, N
    edge samples, interpolation passes, center-ROI switch, and the weight
    below which a pixel counts as empty background."""
    margin: int = 32
    tile: int = 16
    edge_samples: int = 64
    gap_passes: int = 2
    center_roi: bool = True
    a_min: float = 0.5
    edge_bounds: int = 0  # 0: Eq. 6 extrema over all edge samples; 1: per-side worst case of its own edge


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        _lib.orc_render.argtypes = [P, P, P, P, C.c_int64, C.c_int32, C.c_int32, P, P, P, P]
        _lib.orc_render.restype = C.c_int
        _lib.orc_render_eye.argtypes = [P, P, P, P, P, C.c_int64, C.c_int32, C.c_int32, P, P, P, P]
        _lib.orc_render_eye.restype = C.c_int
        _lib.orc_composite_order.argtypes = [P, P, P, P]
        _lib.orc_composite_order.restype = C.c_int64
        _lib.orc_pair.argtypes = [P, P, P, C.c_int64, C.c_double, C.c_double, P]
        _lib.orc_pair.restype = C.c_int
        _lib.orc_coverage_boxes.argtypes = [P, P, P, C.c_int32, P]
        _lib.orc_center_zkeys.argtypes = [P, P, P]
        _lib.orc_center_zkeys.restype = None
        _lib.orc_sh_basis.argtypes = [C.c_int32, P, C.c_int64, P]
        _lib.orc_sh_basis.restype = None
        _lib.orc_reproject.argtypes = [P, P, C.c_double, P, P, P, P, P, P, P, P, P]
        _lib.orc_reproject.restype = None
        _lib.orc_edge_rois.argtypes = [P, P, P, P, P, P]
        _lib.orc_edge_rois.restype = C.c_int
        _lib.orc_label_components.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P]
        _lib.orc_classify.argtypes = [P, P, P, P, P, P, P, P, P, P, P, C.c_int32, P, P, P]
        _lib.orc_patch.argtypes = [P, P, P, C.c_double, C.c_int32, P, C.c_int32, P, P, P, P, P]
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _cam(c) -> _Cam:
    s = _Cam()
    s.width, s.height = int(c.width), int(c.height)
    s.fx, s.fy, s.cx, s.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
    R = np.asarray(c.R, np.float64).reshape(9)
    for i in range(9):
        s.R[i] = R[i]
    for i in range(3):
        s.t[i] = float(c.t[i])
    s.z_near, s.z_far = float(c.z_near), float(c.z_far)
    return s


def _raster(r: Raster) -> _Raster:
    s = _Raster()
    s.alpha_min, s.alpha_max, s.t_min = r.alpha_min, r.alpha_max, r.t_min
    s.lowpass = int(bool(r.lowpass))
    for i in range(3):
        s.bg[i] = float(r.bg[i])
    return s


def _roi(r: Roi) -> _Roi:
    s = _Roi()
    s.margin, s.tile, s.edge_samples, s.gap_passes = r.margin, r.tile, r.edge_samples, r.gap_passes
    s.center_roi = int(bool(r.center_roi))
    s.edge_bounds = int(r.edge_bounds)
    s.a_min = r.a_min
    return s


class _SceneRef:
    """Keeps the contiguous fp32 arrays alive while the C struct points at them."""

    def __init__(self, sc):
        self.arrs = [np.ascontiguousarray(getattr(sc, k), np.float32)
                     for k in ("pos", "quat", "scale", "opacity", "sh")]
        self.s = _Scene()
        self.s.n = int(sc.n)
        self.s.sh_degree = int(sc.sh_degree)
        self.s.pos, self.s.quat, self.s.scale, self.s.opacity, self.s.sh = [
            a.ctypes.data if a.size else None for a in self.arrs]


def render(scene, cam, raster: Raster = Raster(), pixels=None, prefilter=True, nthreads=0, eye=None):
    """Per-pixel exact render (fp64).  pixels: None (full image) or an
    (npx, 2) int array of (i, j).  Returns rgb (3, H, W) or (3, npx),
    depth_raw, alpha and the per-pixel ambiguity flags.  eye (a world
    point, default the camera's centre) is where every surfel's colour is
    seen from: with another eye's centre, rgb composites that eye's colours
    with this camera's weights (depth and alpha are unchanged)."""
    L = lib()
    sr = _SceneRef(scene)
    cs, rs = _cam(cam), _raster(raster)
    if pixels is None:
        npx = int(cam.width) * int(cam.height)
        pix = None
        shape = (int(cam.height), int(cam.width))
    else:
        pix = np.ascontiguousarray(pixels, np.int32).reshape(-1, 2)
        npx = pix.shape[0]
        shape = (npx,)
    rgb = np.zeros((3, npx))
    dr = np.zeros(npx)
    al = np.zeros(npx)
    amb = np.zeros(npx, np.uint8)
    eye_arr = None if eye is None else np.ascontiguousarray(np.asarray(eye, np.float64).reshape(3))
    rc = L.orc_render_eye(C.byref(sr.s), C.byref(cs), _ptr(eye_arr) if eye_arr is not None else None, C.byref(rs),
                          _ptr(pix) if pix is not None else None, npx, int(bool(prefilter)), int(nthreads),
                          _ptr(rgb), _ptr(dr), _ptr(al), _ptr(amb))
    if rc != 0:
        raise RuntimeError("oracle render failed")
    return dict(rgb=rgb.reshape((3,) + shape), depth_raw=dr.reshape(shape), alpha=al.reshape(shape),
                amb=amb.reshape(shape))


def composite_order(scene, cam, raster: Raster = Raster()):
    sr = _SceneRef(scene)
    out = np.zeros(max(int(scene.n), 1), np.int64)
    m = lib().orc_composite_order(C.byref(sr.s), C.byref(_cam(cam)), C.byref(_raster(raster)), _ptr(out))
    return out[:m]


def pair(scene, cam, k, i, j, raster: Raster = Raster()):
    sr = _SceneRef(scene)
    out = np.zeros(11)
    rc = lib().orc_pair(C.byref(sr.s), C.byref(_cam(cam)), C.byref(_raster(raster)), int(k), float(i),
                        float(j), _ptr(out))
    if rc == 1:
        return None
    keys = ["alpha", "G3", "G2", "lambda", "u", "v", "depth", "valid3"]
    d = {k_: out[q] for q, k_ in enumerate(keys)}
    d["color"] = out[8:11].copy()
    return d


def coverage_boxes(scene, cam, raster: Raster = Raster(), nthreads=0):
    sr = _SceneRef(scene)
    out = np.zeros((max(int(scene.n), 1), 4), np.int32)
    lib().orc_coverage_boxes(C.byref(sr.s), C.byref(_cam(cam)), C.byref(_raster(raster)), int(nthreads),
                             _ptr(out))
    return out[:int(scene.n)]


def center_zkeys(scene, cam):
    sr = _SceneRef(scene)
    out = np.zeros(max(int(scene.n), 1), np.float32)
    lib().orc_center_zkeys(C.byref(sr.s), C.byref(_cam(cam)), _ptr(out))
    return out[:int(scene.n)]


def sh_basis(deg, dirs):
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    nc = (deg + 1) ** 2
    out = np.zeros((dirs.shape[0], nc))
    lib().orc_sh_basis(int(deg), _ptr(dirs), dirs.shape[0], _ptr(out))
    return out


def reproject(src, dst, rgb, depth_raw, alpha, a_min=0.5):
    """Forward reprojection with the z-test (Eq. 3-5).  Inputs are fp32
    images of the source eye; returns the warped fp32 image, its depth,
    alpha, hole mask, the z-buffer and the depth range."""
    rgb = np.ascontiguousarray(rgb, np.float32)
    depth_raw = np.ascontiguousarray(depth_raw, np.float32)
    alpha = np.ascontiguousarray(alpha, np.float32)
    H, W = int(dst.height), int(dst.width)
    out = dict(rgb=np.zeros((3, H, W), np.float32), z=np.zeros((H, W), np.float32),
               alpha=np.zeros((H, W), np.float32), hole=np.zeros((H, W), np.uint8),
               zbuf=np.zeros((H, W), np.uint64), depth_range=np.zeros(2, np.float32))
    lib().orc_reproject(C.byref(_cam(src)), C.byref(_cam(dst)), float(a_min), _ptr(rgb), _ptr(depth_raw),
                        _ptr(alpha), _ptr(out["rgb"]), _ptr(out["z"]), _ptr(out["alpha"]), _ptr(out["hole"]),
                        _ptr(out["zbuf"]), _ptr(out["depth_range"]))
    return out


def edge_rois(src, dst, roi: Roi, depth_range):
    dr = np.ascontiguousarray(depth_range, np.float32)
    widths = np.zeros(4, np.int32)
    boxes = np.zeros((4, 6), np.int32)
    nb = lib().orc_edge_rois(C.byref(_cam(src)), C.byref(_cam(dst)), C.byref(_roi(roi)), _ptr(dr),
                             _ptr(widths), _ptr(boxes))
    return widths, boxes[:nb].copy()


def label_components(mask, conn=8):
    mask = np.ascontiguousarray(mask, np.uint8)
    H, W = mask.shape
    lab = np.zeros((H, W), np.int32)
    lib().orc_label_components(_ptr(mask), W, H, int(conn), _ptr(lab))
    return lab


def classify(src, dst, roi: Roi, depth_range, rgb, z, alpha, hole, bg=(0.0, 0.0, 0.0), box_cap=1 << 16):
    """Hole categorisation, interpolation and ROI tiles (Sec. 3.1 Stage 3-4,
    Sec. 3.5).  Returns new arrays; inputs are not modified."""
    H, W = int(dst.height), int(dst.width)
    T = roi.tile
    rgb = np.array(rgb, np.float32, copy=True, order="C")
    z = np.array(z, np.float32, copy=True, order="C")
    alpha = np.array(alpha, np.float32, copy=True, order="C")
    cls = np.array(hole, np.uint8, copy=True, order="C")
    labels = np.zeros((H, W), np.int32)
    boxes = np.zeros((max(box_cap, 1), 6), np.int32)
    nb = np.zeros(1, np.int32)
    tm = np.zeros(((H + T - 1) // T, (W + T - 1) // T), np.uint8)
    st = _ClsStats()
    bgv = np.asarray(bg, np.float32)
    dr = np.ascontiguousarray(depth_range, np.float32)
    rc = lib().orc_classify(C.byref(_cam(src)), C.byref(_cam(dst)), C.byref(_roi(roi)), _ptr(dr), _ptr(bgv),
                            _ptr(rgb), _ptr(z), _ptr(alpha), _ptr(cls), _ptr(labels), _ptr(boxes),
                            int(box_cap), _ptr(nb), _ptr(tm), C.byref(st))
    if rc != 0:
        raise RuntimeError("oracle classify failed")
    n_boxes = int(nb[0])
    stats = {f: int(getattr(st, f)) for f, _ in _ClsStats._fields_}
    return dict(rgb=rgb, z=z, alpha=alpha, cls=cls, labels=labels, boxes=boxes[:min(n_boxes, box_cap)].copy(),
                n_boxes=n_boxes, tile_mask=tm, stats=stats)


def patch(scene, cam, tile_mask, rgb, z, alpha, cls, raster: Raster = Raster(), a_min=0.5, tile=16,
          nthreads=0):
    """Re-render every pixel of the masked tiles at `cam` (Stage 4)."""
    sr = _SceneRef(scene)
    rgb = np.array(rgb, np.float32, copy=True, order="C")
    z = np.array(z, np.float32, copy=True, order="C")
    alpha = np.array(alpha, np.float32, copy=True, order="C")
    cls = np.array(cls, np.uint8, copy=True, order="C")
    tm = np.ascontiguousarray(tile_mask, np.uint8)
    amb = np.zeros(cls.shape, np.uint8)
    rc = lib().orc_patch(C.byref(sr.s), C.byref(_cam(cam)), C.byref(_raster(raster)), float(a_min), int(tile),
                         _ptr(tm), int(nthreads), _ptr(rgb), _ptr(z), _ptr(alpha), _ptr(cls), _ptr(amb))
    if rc != 0:
        raise RuntimeError("oracle patch failed")
    return dict(rgb=rgb, z=z, alpha=alpha, cls=cls, amb=amb)


def render_stereo(scene, cam_dom, cam_aff, raster: Raster = Raster(), roi: Roi = Roi(), nthreads=0,
                  view_colour=False):
    """The full binocular frame (Sec. 3.1): dominant render with depth proxy
    -> reprojection -> classification and interpolation -> ROI patch.  The
    dominant render is rounded to fp32 before it is reprojected, as a
    renderer that stores fp32 images would.  view_colour (not part of the
    paper's method): the colour that is reprojected composites every
    surfel's colour seen from the affiliated eye's centre with the dominant
    eye's weights, instead of the dominant image itself."""
    dom = render(scene, cam_dom, raster, nthreads=nthreads)
    rgb32 = dom["rgb"].astype(np.float32)
    if view_colour:
        dom["rgb_view"] = render(scene, cam_dom, raster, nthreads=nthreads, eye=np.asarray(cam_aff.t))["rgb"]
        rgb32 = dom["rgb_view"].astype(np.float32)
    dr32 = dom["depth_raw"].astype(np.float32)
    a32 = dom["alpha"].astype(np.float32)
    rep = reproject(cam_dom, cam_aff, rgb32, dr32, a32, roi.a_min)
    cl = classify(cam_dom, cam_aff, roi, rep["depth_range"], rep["rgb"], rep["z"], rep["alpha"], rep["hole"],
                  raster.bg)
    pt = patch(scene, cam_aff, cl["tile_mask"], cl["rgb"], cl["z"], cl["alpha"], cl["cls"], raster, roi.a_min,
               roi.tile, nthreads)
    return dict(dom=dom, rep=rep, cls=cl, aff=pt)
