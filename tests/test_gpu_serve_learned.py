"""The serving loop's learned mode through the C ABI: dominant render,
reprojection, the repair network and its mean predicted error at the
holes; above the threshold the request falls back to the method's
interpolation plus ROI re-rendering.  Each branch gives exactly what the
library's calls give when run one by one, the decisions follow the
predicted error, and results alone equal results in the mix."""
import math

import numpy as np
import pytest
import torch

from paper_2609_30741_amd import api, repair, serve, synth

pytestmark = pytest.mark.gpu


def setup():
    sc = synth.scene_uniform_cube(12, 8_000)
    cams = [synth.look_at((4.0 * math.cos(t), 4.0 * math.sin(t), 0.3), (0, 0, 0), (0, 0, 1), 192, 160, 220.0)
            for t in np.linspace(0.0, 2.0, 6)]
    return sc, cams, [synth.affiliated(c, 0.064) for c in cams]


def run(sc, cams, affs, params, slots, threshold):
    ex = serve.GpuExecutor({"s": sc}, slots, mode="learned", key_capacity=1 << 18, keep_outputs=True,
                           repair_params=params, threshold=threshold)
    reqs = [serve.Request(i, "s", cams[i], affs[i], 0.0) for i in range(len(cams))]
    serve.serve(reqs, ex, slots, 1e12)
    torch.cuda.synchronize()
    return reqs


def stages(sc, r, net):
    ctx = api.Context()
    ds = api.DeviceScene(sc)
    d = ctx.render_dominant(ds, r.cam_dom)
    w = ctx.reproject(r.cam_dom, r.cam_aff, d["rgb"], d["depth_raw"], d["alpha"])
    err = torch.empty((1,) + tuple(w["hole"].shape), device=w["rgb"].device)
    x = net.forward(w["rgb"][None].contiguous(), w["z"][None].contiguous(), w["hole"][None].contiguous(),
                    err=err)[0].clone()
    m = w["hole"].bool()
    mean_err = float(err[0][m].double().mean()) if bool(m.any()) else 0.0
    c = ctx.classify_holes(r.cam_dom, r.cam_aff, w["depth_range"], w["rgb"], w["z"], w["alpha"], w["hole"])
    ctx.patch_rois(ds, r.cam_aff, c["tile_mask"], w["rgb"], w["z"], w["alpha"], w["hole"])
    torch.cuda.synchronize()
    return d["rgb"], x, w["rgb"], mean_err


def test_learned_mode_branches_and_mix():
    sc, cams, affs = setup()
    params = repair.init_params(3)
    net = repair.Repair(params=params)
    always = run(sc, cams, affs, params, 2, -1.0)
    never = run(sc, cams, affs, params, 2, math.inf)
    for a, b in zip(always, never):
        dom, x, method, mean_err = stages(sc, a, net)
        assert a.fallback is True and b.fallback is False
        assert torch.equal(a.out["rgb_dom"], dom) and torch.equal(b.out["rgb_dom"], dom)
        assert torch.equal(a.out["rgb_aff"], method)  # fallback: interpolation + ROI re-rendering
        assert torch.equal(b.out["rgb_aff"], x)       # the network's repair
        # The decision's input is the mean of the error channel over the
        # holes (untrained weights may make it negative: it is a plain
        # regression output).
        assert a.pred_err == b.pred_err and math.isfinite(a.pred_err)
        assert abs(a.pred_err - mean_err) <= 1e-5 * max(1.0, abs(mean_err))
    # A threshold between the requests' predicted errors: each decision
    # follows its own error, and the same requests alone and in a
    # three-slot mix give the same decisions and images.
    errs = sorted(r.pred_err for r in never)
    thr = 0.5 * (errs[2] + errs[3])
    alone = run(sc, cams, affs, params, 1, thr)
    mix = run(sc, cams, affs, params, 3, thr)
    for a, b, n in zip(alone, mix, never):
        assert a.fallback == (n.pred_err > thr) == b.fallback
        for k in ("rgb_dom", "rgb_aff"):
            assert torch.equal(a.out[k], b.out[k])
    assert any(r.fallback for r in mix) and not all(r.fallback for r in mix)
