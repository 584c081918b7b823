"""Batched stereo frames over resident scenes (include/bgs.h, batched form).

A batch holds many stereo pairs, each with its own scene, image size,
cameras and ROI settings, its own workspace and outputs.  One call issues
every pair's binning, then ONE persistent blend launch for the dominant-eye
tiles of all pairs, then every pair's reprojection, classification and ROI
binning, then one persistent launch for all ROI tiles
(`bgs_render_stereo_batch`).  The whole batch can be captured once into a
HIP graph and replayed (`bgs_batch_graph_capture`, `bgs_graph_launch`).
This module allocates the tensors and marshals arguments; every step runs
in the library's kernels.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _abi, api


class StereoBatch:
    """pairs: a list of (DeviceScene, cam_dom, cam_aff, Roi).  Each pair's
    workspace is sized from one synchronous frame of that pair alone, with
    `headroom` over its key counts."""

    def __init__(self, ctx: api.Context, pairs, raster: api.Raster = api.Raster(), headroom: float = 1.25,
                 box_capacity: int = 1024, device="cuda"):
        self.ctx = ctx
        self.L = ctx.L
        self.raster = raster
        self.pairs = list(pairs)
        self.device = device
        self.graph = None
        sizer = api.Context(sync=True)
        self.ws, self.outs, self.keys = [], [], []
        n = len(self.pairs)
        arr = (_abi.BatchPair * n)()
        self._keep = []
        for i, (ds, cd, ca, roi) in enumerate(self.pairs):
            o = sizer.render_stereo(ds, cd, ca, raster, roi, box_capacity=box_capacity)
            k = max(o["stats"]["n_keys_dom"], o["stats"]["n_keys_roi"], 1)
            self.keys.append(k)
            W, H = max(cd.width, ca.width), max(cd.height, ca.height)
            need = C.c_size_t()
            ctx._check(self.L.bgs_workspace_size(int(ds.n), int(W), int(H), int(k * headroom) + 4096, C.byref(need)))
            ws = torch.empty(int(need.value), dtype=torch.uint8, device=device)
            o.pop("stats", None)
            self.ws.append(ws)
            self.outs.append(o)
            q = arr[i]
            q.scene = C.addressof(ds.c)
            q.cam_dom = api.camera(cd)
            q.cam_aff = api.camera(ca)
            q.roi = roi.c()
            q.box_capacity = int(box_capacity)
            q.ws = ws.data_ptr()
            q.ws_bytes = ws.numel()
            for f in ("rgb_dom", "depth_raw_dom", "alpha_dom", "rgb_aff", "z_aff", "alpha_aff", "cls_aff", "labels",
                      "boxes", "n_boxes", "tile_mask"):
                setattr(q, f, o[f].data_ptr())
            self._keep.append(ds)
        del sizer
        self.arr = arr
        need = C.c_size_t()
        ctx._check(self.L.bgs_batch_workspace_size(n, C.byref(need)))
        self.bws = torch.empty(int(need.value), dtype=torch.uint8, device=device)
        self.rc = raster.c()

    def __len__(self):
        return len(self.pairs)

    def render(self):
        """Issue the whole batch on the current stream (asynchronous)."""
        self.ctx.bind_stream()
        self.ctx._check(self.L.bgs_render_stereo_batch(self.ctx.h, len(self.pairs), self.arr, C.byref(self.rc),
                                                       api._ptr(self.bws), self.bws.numel()))

    def capture(self):
        """Capture the batch into a HIP graph on the current stream, which
        must not be the default stream.  The batch is rendered once eagerly
        first, so every pair's status block is initialised outside the graph."""
        self.render()
        torch.cuda.current_stream().synchronize()
        self.ctx.bind_stream()
        g = C.c_void_p()
        self.ctx._check(self.L.bgs_batch_graph_capture(self.ctx.h, len(self.pairs), self.arr, C.byref(self.rc),
                                                       api._ptr(self.bws), self.bws.numel(), C.byref(g)))
        self.graph = g
        return g

    def replay(self):
        self.ctx.bind_stream()
        self.ctx._check(self.L.bgs_graph_launch(self.ctx.h, self.graph))

    def poll(self):
        """Per-pair status: key counts and overflow bits since the last poll."""
        res = []
        for ws in self.ws:
            st = _abi.Stats()
            self.ctx._check(self.L.bgs_poll_status(self.ctx.h, api._ptr(ws), ws.numel(), C.byref(st)))
            res.append(api._stats_dict(st))
        return res

    def close(self):
        if self.graph is not None:
            self.L.bgs_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
