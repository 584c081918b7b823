"""The C ABI on the CPU: every symbol include/*.h declares is exported,
and argument validation returns the documented status codes before any
GPU work is launched (no device is touched by these calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2609_30741_amd import _abi, api, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2609_30741_amd import build
        build.build()
    return _abi.load()


def declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"BGS_API\s+[\w\s\*]+?\b(bgs_\w+)\s*\(", text))
    return sorted(names)


def test_header_symbols_exported(L):
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_abi.EXPORTS) == names


def test_struct_sizes():
    assert C.sizeof(_abi.Camera) == 152
    assert C.sizeof(_abi.Scene) == 56
    assert C.sizeof(_abi.RasterParams) == 32
    assert C.sizeof(_abi.RoiParams) == 32
    assert C.sizeof(_abi.Box) == 24
    assert C.sizeof(_abi.Stats) == 144
    # bgs_batch_pair: 456 bytes, box_capacity at 344 and tile_mask at 448
    # (include/bgs.h compiled by the host compiler agrees).
    assert C.sizeof(_abi.BatchPair) == 456
    assert _abi.BatchPair.box_capacity.offset == 344 and _abi.BatchPair.tile_mask.offset == 448


@pytest.fixture
def ctx(L):
    h = C.c_void_p()
    assert L.bgs_ctx_create(C.byref(h), None) == 0
    yield h
    L.bgs_ctx_destroy(h)


def test_workspace_size(L):
    sizes = []
    for k in (0, 1, 1000, 10 ** 6):
        b = C.c_size_t()
        assert L.bgs_workspace_size(1000, 64, 48, k, C.byref(b)) == 0
        sizes.append(b.value)
    assert sizes == sorted(sizes) and sizes[-1] - sizes[0] >= 16 * 10 ** 6
    b = C.c_size_t()
    assert L.bgs_workspace_size(-1, 64, 48, 0, C.byref(b)) == _abi.ERR_INVALID_ARG
    assert L.bgs_workspace_size(10, 0, 48, 0, C.byref(b)) == _abi.ERR_INVALID_ARG
    assert L.bgs_workspace_size(10, 64, 20000, 0, C.byref(b)) == _abi.ERR_INVALID_ARG


FAKE = C.c_void_p(0x1000)  # never dereferenced: validation fails first


def _scene(n=10, deg=0):
    s = _abi.Scene()
    s.n, s.sh_degree = n, deg
    s.pos = s.quat = s.scale = s.opacity = s.sh = 0x1000
    return s


def _cam(**kw):
    cam = synth.look_at((0, -4, 0), (0, 0, 0), (0, 0, 1), 64, 48, 80.0)
    c = api.camera(cam)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _render(L, ctx, scene=None, cam=None, raster=None, ws_bytes=1 << 30):
    scene = scene or _scene()
    cam = cam or _cam()
    raster = raster or api.Raster().c()
    return L.bgs_render_dominant(ctx, C.byref(scene), C.byref(cam), C.byref(raster), FAKE, ws_bytes, FAKE, FAKE,
                                 FAKE, None)


def test_render_validation(L, ctx):
    assert _render(L, ctx, scene=_scene(deg=4)) == _abi.ERR_INVALID_ARG
    assert b"sh_degree" in L.bgs_last_error(ctx)
    assert _render(L, ctx, scene=_scene(n=-1)) == _abi.ERR_INVALID_ARG
    bad = _scene()
    bad.pos = None
    assert _render(L, ctx, scene=bad) == _abi.ERR_INVALID_ARG
    assert _render(L, ctx, cam=_cam(width=0)) == _abi.ERR_INVALID_ARG
    assert _render(L, ctx, cam=_cam(fx=-1.0)) == _abi.ERR_INVALID_ARG
    assert _render(L, ctx, cam=_cam(z_near=0.0)) == _abi.ERR_INVALID_ARG
    c = _cam()
    c.R[0] = 2.0
    assert _render(L, ctx, cam=c) == _abi.ERR_INVALID_ARG and b"orthonormal" in L.bgs_last_error(ctx)
    r = api.Raster(alpha_min=0.0).c()
    assert _render(L, ctx, raster=r) == _abi.ERR_INVALID_ARG
    assert _render(L, ctx, ws_bytes=100) == _abi.ERR_WORKSPACE
    assert L.bgs_render_dominant(ctx, C.byref(_scene()), C.byref(_cam()), C.byref(api.Raster().c()), FAKE, 1 << 30,
                                 None, FAKE, FAKE, None) == _abi.ERR_INVALID_ARG


def test_stage_validation(L, ctx):
    cam = _cam()
    roi = api.Roi(tile=24).c()  # ROI tiles are 8, 16 or 32 pixels
    rc = L.bgs_reproject(ctx, C.byref(cam), C.byref(cam), C.byref(roi), FAKE, FAKE, FAKE, FAKE, 1 << 30, FAKE, FAKE,
                         FAKE, FAKE, FAKE)
    assert rc == _abi.ERR_UNSUPPORTED
    roi = api.Roi(edge_samples=0).c()
    rc = L.bgs_reproject(ctx, C.byref(cam), C.byref(cam), C.byref(roi), FAKE, FAKE, FAKE, FAKE, 1 << 30, FAKE, FAKE,
                         FAKE, FAKE, FAKE)
    assert rc == _abi.ERR_INVALID_ARG
    roi = api.Roi(edge_bounds=2).c()
    rc = L.bgs_reproject(ctx, C.byref(cam), C.byref(cam), C.byref(roi), FAKE, FAKE, FAKE, FAKE, 1 << 30, FAKE, FAKE,
                         FAKE, FAKE, FAKE)
    assert rc == _abi.ERR_INVALID_ARG
    roi = api.Roi(view_colour=2).c()
    rc = L.bgs_reproject(ctx, C.byref(cam), C.byref(cam), C.byref(roi), FAKE, FAKE, FAKE, FAKE, 1 << 30, FAKE, FAKE,
                         FAKE, FAKE, FAKE)
    assert rc == _abi.ERR_INVALID_ARG
    roi = api.Roi().c()
    rc = L.bgs_reproject(ctx, C.byref(cam), C.byref(cam), C.byref(roi), FAKE, FAKE, FAKE, FAKE, 64, FAKE, FAKE,
                         FAKE, FAKE, FAKE)
    assert rc == _abi.ERR_WORKSPACE
    rc = L.bgs_classify_holes(ctx, C.byref(cam), C.byref(cam), C.byref(roi), C.byref(api.Raster().c()), FAKE, FAKE,
                              1 << 30, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, -1, FAKE, FAKE)
    assert rc == _abi.ERR_INVALID_ARG
    rc = L.bgs_patch_rois(ctx, C.byref(_scene()), C.byref(cam), C.byref(api.Raster().c()), C.byref(roi), None, FAKE,
                          1 << 30, FAKE, FAKE, FAKE, FAKE, None)
    assert rc == _abi.ERR_INVALID_ARG
    rc = L.bgs_render_stereo(ctx, C.byref(_scene()), C.byref(cam), C.byref(_cam(height=20000)),
                             C.byref(api.Raster().c()), C.byref(roi), FAKE, 1 << 30, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE,
                             FAKE, FAKE, FAKE, 16, FAKE, FAKE, None)
    assert rc == _abi.ERR_INVALID_ARG


def test_sort_and_label_validation(L, ctx):
    assert L.bgs_sort_pairs(ctx, FAKE, FAKE, 0, 8, None, 0) == 0  # empty: nothing to do
    assert L.bgs_sort_pairs(ctx, FAKE, FAKE, 10, 0, FAKE, 1 << 20) == _abi.ERR_INVALID_ARG
    assert L.bgs_sort_pairs(ctx, FAKE, FAKE, 10, 33, FAKE, 1 << 20) == _abi.ERR_INVALID_ARG
    assert L.bgs_sort_pairs(ctx, FAKE, FAKE, 1000, 8, FAKE, 16) == _abi.ERR_WORKSPACE
    assert L.bgs_label_components(ctx, FAKE, 10, 10, 6, FAKE) == _abi.ERR_INVALID_ARG
    assert L.bgs_label_components(ctx, FAKE, 0, 10, 8, FAKE) == _abi.ERR_INVALID_ARG
    assert L.bgs_ctx_set_sync(None, 1) == _abi.ERR_INVALID_ARG


def test_repair_parameter_count_and_argument_checks(L):
    # bgs_repair_* validate on the host before any launch.
    from oracle import repair_oracle as R
    n = C.c_int64()
    assert L.bgs_repair_num_params(C.byref(n)) == 0
    assert n.value == R.num_params()
    b = C.c_size_t()
    assert L.bgs_repair_workspace_size(2, 16, 24, 1, C.byref(b)) == 0
    train = b.value
    assert L.bgs_repair_workspace_size(2, 16, 24, 0, C.byref(b)) == 0
    assert 0 < b.value < train
    for B, H, W in ((0, 16, 16), (1, 10, 16), (1, 16, 18), (1001, 16, 16), (1, 8200, 16)):
        assert L.bgs_repair_workspace_size(B, H, W, 0, C.byref(b)) == _abi.ERR_INVALID_ARG
    assert L.bgs_repair_workspace_size(1, 16, 16, 2, C.byref(b)) == _abi.ERR_INVALID_ARG
    fake = C.c_void_p(0x100000)
    assert L.bgs_repair_forward(None, 1, 16, 16, fake, fake, fake, fake, None, fake, 1 << 30,
                                None) == _abi.ERR_INVALID_ARG
    assert L.bgs_repair_forward(fake, 1, 16, 16, fake, fake, fake, fake, None, fake, 16, None) == _abi.ERR_WORKSPACE
    assert L.bgs_repair_grad(fake, 1, 16, 16, fake, fake, fake, fake, fake, fake, None, fake, 16,
                             None) == _abi.ERR_WORKSPACE
    assert L.bgs_repair_adam(fake, fake, fake, fake, 0, 1, 1e-3, 0.9, 0.999, 1e-8, None) == _abi.ERR_INVALID_ARG
    assert L.bgs_repair_adam(fake, fake, fake, fake, 10, 0, 1e-3, 0.9, 0.999, 1e-8, None) == _abi.ERR_INVALID_ARG
    assert L.bgs_repair_adam(fake, fake, fake, fake, 10, 1, 1e-3, 1.0, 0.999, 1e-8, None) == _abi.ERR_INVALID_ARG


def test_repair_block_shape_validation(L):
    # Rows 0 (automatic), 2, 4 or 8; tiles 0 (automatic) to 4.  The call only
    # records the choice, so it runs without a device.
    for rows, tiles in [(1, 0), (3, 0), (6, 0), (16, 0), (-2, 0), (0, -1), (0, 5)]:
        assert L.bgs_repair_set_block_shape(rows, tiles) == _abi.ERR_INVALID_ARG, (rows, tiles)
    for rows, tiles in [(2, 1), (4, 3), (8, 2), (0, 4), (0, 0)]:
        assert L.bgs_repair_set_block_shape(rows, tiles) == _abi.OK, (rows, tiles)
