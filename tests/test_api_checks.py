"""The Python binding's buffer checks (CPU only): every output and input
tensor must match the camera's size, dtype and device before a raw pointer
reaches the library, because the kernels size their writes from the camera."""
import numpy as np
import pytest
import torch

from paper_2609_30741_amd import api, synth

CPU = torch.device("cpu")


def stereo_out(Hd, Wd, Ha, Wa, cap=16, T=16):
    f = lambda *s: torch.zeros(s, dtype=torch.float32)
    return dict(rgb_dom=f(3, Hd, Wd), depth_raw_dom=f(Hd, Wd), alpha_dom=f(Hd, Wd), rgb_aff=f(3, Ha, Wa),
                z_aff=f(Ha, Wa), alpha_aff=f(Ha, Wa), cls_aff=torch.zeros((Ha, Wa), dtype=torch.uint8),
                labels=torch.zeros((Ha, Wa), dtype=torch.int32), boxes=torch.zeros((cap, 6), dtype=torch.int32),
                n_boxes=torch.zeros(1, dtype=torch.int32),
                tile_mask=torch.zeros(((Ha + T - 1) // T, (Wa + T - 1) // T), dtype=torch.uint8))


def test_render_out_checks():
    out = dict(rgb=torch.zeros(3, 20, 30), depth_raw=torch.zeros(20, 30), alpha=torch.zeros(20, 30))
    api.check_render_out(out, 20, 30, CPU)
    with pytest.raises(ValueError, match="rgb: shape"):
        api.check_render_out(out, 40, 30, CPU)  # a larger camera than the buffers
    bad = dict(out, alpha=torch.zeros(20, 30, dtype=torch.float16))
    with pytest.raises(ValueError, match="alpha: dtype"):
        api.check_render_out(bad, 20, 30, CPU)
    bad = dict(out, depth_raw=torch.zeros(30, 20).t())
    with pytest.raises(ValueError, match="contiguous"):
        api.check_render_out(bad, 20, 30, CPU)
    with pytest.raises(ValueError, match="expected meta"):
        api.check_render_out(out, 20, 30, torch.device("meta"))


def test_stereo_out_checks_every_buffer():
    dom = synth.look_at((0.0, -4.0, 0.0), (0, 0, 0), (0, 0, 1), 48, 32, 60.0)
    aff = synth.affiliated(dom, 0.064)
    out = stereo_out(32, 48, 32, 48)
    api.check_stereo_out(out, dom, aff, 16, 16, CPU)
    # A dominant-eye buffer from a smaller frame is caught, not only the
    # affiliated one.
    for key in out:
        o = dict(out)
        t = o[key]
        o[key] = t[..., :-1].contiguous() if t.dim() > 1 else torch.zeros(2, dtype=t.dtype)
        with pytest.raises(ValueError, match=key):
            api.check_stereo_out(o, dom, aff, 16, 16, CPU)
    with pytest.raises(ValueError, match="box_capacity"):
        api.check_stereo_out(out, dom, aff, 17, 16, CPU)
    big = synth.look_at((0.0, -4.0, 0.0), (0, 0, 0), (0, 0, 1), 64, 48, 60.0)
    with pytest.raises(ValueError):
        api.check_stereo_out(out, big, synth.affiliated(big, 0.064), 16, 16, CPU)


def test_check_tensor_rejects_non_tensors():
    with pytest.raises(ValueError, match="expected a tensor"):
        api.check_tensor("x", np.zeros(3), (3,), torch.float32)


def test_repair_image_checks():
    from paper_2609_30741_amd.repair import Repair
    B, H, W = 2, 8, 12
    rgb = torch.zeros(B, 3, H, W)
    z = torch.zeros(B, H, W)
    hole = torch.zeros(B, H, W, dtype=torch.uint8)
    assert Repair.check_images(rgb, z, hole, out=torch.zeros_like(rgb), err=torch.zeros(B, H, W)) == (B, H, W)
    with pytest.raises(ValueError, match="err: shape"):
        Repair.check_images(rgb, z, hole, err=torch.zeros(H, W))  # [H, W] with B > 1
    with pytest.raises(ValueError, match="err: dtype"):
        Repair.check_images(rgb, z, hole, err=torch.zeros(B, H, W, dtype=torch.float16))
    with pytest.raises(ValueError, match="hole: dtype"):
        Repair.check_images(rgb, z, hole.bool())
    with pytest.raises(ValueError, match="target: shape"):
        Repair.check_images(rgb, z, hole, target=torch.zeros(B, 3, H, W + 4))
    with pytest.raises(ValueError, match="z: shape"):
        Repair.check_images(rgb, z[:1], hole)
