"""Autotuner of the batched form's ROI settings.

For each group of stereo pairs that share a scene and an image size, it
chooses the ROI tile size T in {8, 16, 32} (the alignment of the ROI boxes
and the granularity of the patch; the paper fixes 16, the rasteriser's
tile, Sec. 3.5) and the ROI margin m (the dilation of every box; the paper
fixes 32) by measuring, on the group's calibration pairs, the frame time
of each candidate (GPU events, median of a few frames, long lists unsplit
as in the batch) and the affiliated eye's PSNR against its full render.
The fastest candidate whose mean PSNR is within `tol_db` of the paper's
setting (T = 16, m = 32) wins: equal accuracy, less work.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import api

CANDIDATES = tuple((T, m) for T in (8, 16, 32) for m in (16, 32))
PLAIN = (16, 32)


def _psnr(a, b):
    mse = float(((a.clamp(0, 1).double() - b.clamp(0, 1).double()) ** 2).mean())
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def measure(ctx, pairs, T, m, raster, reps=3, full=None):
    """Mean frame time (ms) and mean affiliated-eye PSNR against the full
    render of the candidate (T, m) over the pairs (DeviceScene, cam_dom,
    cam_aff); full: the pairs' full affiliated renders (computed if None)."""
    roi = api.Roi(tile=T, margin=m)
    times, ps = [], []
    out = None
    for i, (ds, cd, ca) in enumerate(pairs):
        if out is not None and tuple(out["rgb_aff"].shape[1:]) != (ca.height, ca.width):
            out = None
        ctx.set_sync(True)
        out = ctx.render_stereo(ds, cd, ca, raster, roi, box_capacity=1024, out=out)
        ps.append(_psnr(out["rgb_aff"], full[i]))
        ctx.set_sync(False)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record()
            ctx.render_stereo(ds, cd, ca, raster, roi, box_capacity=1024, out=out)
            e1.record()
        torch.cuda.synchronize()
        times.append(float(np.median([e0.elapsed_time(e1) for e0, e1 in ev])))
    st = ctx.poll_status()
    ctx.set_sync(True)  # later renders size the workspace again (a synchronous call grows it on overflow)
    if st["overflow"]:
        raise RuntimeError("key capacity exceeded while tuning")
    return float(np.mean(times)), float(np.mean(ps))


def tune(groups, raster: api.Raster = api.Raster(), reps: int = 3, tol_db: float = 0.05, candidates=CANDIDATES):
    """groups: {key: [(DeviceScene, cam_dom, cam_aff), ...]} calibration
    pairs.  Returns {key: {"tile", "margin", "ms", "psnr", "plain_ms",
    "plain_psnr", "table"}}."""
    ctx = api.Context(sync=True)
    ctx.set_blend_split(0, 0, 64, 0, 0)
    res = {}
    for key, pairs in groups.items():
        # Synchronous: the full renders grow the workspace to this group's
        # scene and image size if they need more keys than it holds.
        ctx.set_sync(True)
        full = [ctx.render_dominant(ds, ca, raster)["rgb"].clone() for ds, _, ca in pairs]
        table = {}
        for T, m in candidates:
            table[(T, m)] = measure(ctx, pairs, T, m, raster, reps, full)
        p_ms, p_psnr = table[PLAIN]
        ok = [(ms, (T, m)) for (T, m), (ms, ps) in table.items() if ps >= p_psnr - tol_db]
        ms, (T, m) = min(ok)
        res[key] = {"tile": T, "margin": m, "ms": round(ms, 4), "psnr": round(table[(T, m)][1], 3),
                    "plain_ms": round(p_ms, 4), "plain_psnr": round(p_psnr, 3),
                    "table": {f"T{t}_m{mm}": [round(a, 4), round(b, 3)] for (t, mm), (a, b) in table.items()}}
    return res
