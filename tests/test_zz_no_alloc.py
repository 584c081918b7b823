"""bgs_reproject_noalloc, the reprojection entry point that allocates
nothing (its scratch is the library's static per-GPU array), against
bgs_reproject with a caller workspace: the same bits on two calls in a
row, the second with a smaller image, on a rig that keeps rows (row-local
z-buffer) and on a turned eye (the scratch's global z-buffer)."""
import sys

import numpy as np
import pytest
import torch

from paper_2609_30741_amd import _abi, api, synth

pytestmark = pytest.mark.gpu


def to_np(t):
    return t.detach().cpu().numpy()


def rig(W, H, turn):
    dom = synth.look_at((0.0, -4.0, 0.0), (0, 0, 0), (0, 0, 1), W, H, 1.2 * W)
    aff = synth.affiliated(dom, 0.064)
    if turn:
        aff = synth.look_at(aff.t, (turn, 0.0, 0.3 * turn), (0, 0, 1), W, H, 1.2 * W)
    return dom, aff


@pytest.mark.parametrize("turn", [0.0, 0.08])
def test_noalloc_reproject_matches_workspace_form(turn):
    assert torch.cuda.is_available()
    ctx = api.Context()
    for call, (W, H, seed) in enumerate([(800, 600, 1), (256, 192, 2)]):  # second call smaller
        print(f"noalloc call {call}: {W}x{H} turn {turn}", file=sys.stderr, flush=True)
        dom, aff = rig(W, H, turn)
        rgb, dr, a = (torch.from_numpy(x).cuda() for x in synth.stage_images(W, H, seed))
        want = ctx.reproject(dom, aff, rgb, dr, a)
        got = ctx.reproject_noalloc(dom, aff, rgb, dr, a)
        torch.cuda.synchronize()
        for k in ("hole", "rgb", "z", "alpha", "depth_range"):
            assert np.array_equal(to_np(got[k]), to_np(want[k])), (call, k)
        assert 0 < int(to_np(got["hole"]).sum()) < W * H


def test_noalloc_rejects_images_beyond_its_scratch():
    ctx = api.Context()
    W, H = 4096, 2049  # one row more than the largest image the scratch holds
    assert W * H > _abi.REPROJECT_NOALLOC_MAX_PIXELS
    dom = synth.look_at((0.0, -4.0, 0.0), (0, 0, 0), (0, 0, 1), 8, 8, 10.0)
    aff = synth.look_at((0.0, -4.0, 0.0), (0, 0, 0), (0, 0, 1), W, H, 10.0)
    x = torch.zeros((3, 8, 8), device="cuda")
    out = dict(rgb=torch.empty((3, H, W), device="cuda"), z=torch.empty((H, W), device="cuda"),
               alpha=torch.empty((H, W), device="cuda"), hole=torch.empty((H, W), dtype=torch.uint8, device="cuda"),
               depth_range=torch.empty(2, device="cuda"))
    with pytest.raises(api.BgsError, match="static scratch"):
        ctx.reproject_noalloc(dom, aff, x, x[0].contiguous(), x[0].contiguous(), out=out)
