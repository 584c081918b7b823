"""Learned gap/edge repair of the affiliated eye (include/bgs_repair.h).

A three-level convolutional U-Net fills the holes the forward reprojection
leaves, from the warped RGB, the hole mask and inverse depth; only hole
pixels change.  It is trained on pairs the method itself produces: the
dominant render reprojected to the affiliated camera (input) and the full
render of the affiliated camera (target).  Every step runs in the
library's kernels (bf16 MFMA convolutions, fp32 Adam); this module only
allocates tensors and marshals arguments.

    python -m paper_2609_30741_amd.repair [--steps 600] [--batch 8] [--crop 128]

trains on sphere800 poses, then reports, on held-out poses at full frame
size, the hole pixels' PSNR for the network, for the method's gap
interpolation with row fill, and for the full method (interpolation plus
ROI re-rendering), and the time of one inference pass.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import sys
import time

import numpy as np
import torch

from . import _abi, api

# (cin, cout) per layer, in the parameter layout's order.
LAYERS = [(5, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (48, 16), (16, 4)]


def _check(rc, what):
    if rc != _abi.OK:
        raise api.BgsError(rc, f"{what} failed with status {rc}")


def num_params() -> int:
    L = _abi.load()
    n = C.c_int64()
    _check(L.bgs_repair_num_params(C.byref(n)), "bgs_repair_num_params")
    return int(n.value)


def set_block_shape(rows: int = 0, tiles: int = 0) -> None:
    """Fix the convolutions' output rows (2, 4 or 8) and 16-channel output
    tiles (1-4) per block for later calls; 0 restores the library's own
    choice (bgs_repair_set_block_shape)."""
    _check(_abi.load().bgs_repair_set_block_shape(int(rows), int(tiles)), "bgs_repair_set_block_shape")


# Pixel count of each layer's level relative to the full image.
LEVEL_SCALE = [1.0, 1.0, 0.25, 0.25, 1.0 / 16, 1.0 / 16, 0.25, 1.0, 1.0]


def flops_per_pixel() -> float:
    """Multiply-adds (x2) of the nine 3x3 convolutions per full-size pixel."""
    return sum(2.0 * 9 * ci * co * s for (ci, co), s in zip(LAYERS, LEVEL_SCALE))


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / (9 cin))), zero biases; the last
    layer starts at a tenth of that so the first residuals are small."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, (ci, co) in enumerate(LAYERS):
        std = math.sqrt(2.0 / (9 * ci)) * (0.1 if i == len(LAYERS) - 1 else 1.0)
        parts.append(rng.normal(0.0, std, size=co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


class Repair:
    """Parameters, Adam state and workspaces on the device."""

    def __init__(self, params=None, seed: int = 0, device="cuda"):
        self.L = _abi.load()
        self.device = device
        p = init_params(seed) if params is None else np.asarray(params, np.float32)
        if p.size != num_params():
            raise ValueError(f"expected {num_params()} parameters, got {p.size}")
        self.params = torch.from_numpy(p.copy()).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, device=device)
        self.step_count = 0
        self._ws = {}

    def _workspace(self, B, H, W, train):
        key = (B, H, W, train)
        if key not in self._ws:
            n = C.c_size_t()
            _check(self.L.bgs_repair_workspace_size(B, H, W, int(train), C.byref(n)), "bgs_repair_workspace_size")
            self._ws[key] = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        return self._ws[key]

    @staticmethod
    def _shape(rgb):
        if not isinstance(rgb, torch.Tensor) or rgb.dim() != 4 or rgb.shape[1] != 3:
            raise ValueError("rgb must be [B, 3, H, W]")
        return int(rgb.shape[0]), int(rgb.shape[2]), int(rgb.shape[3])

    @staticmethod
    def check_images(rgb, z, hole, out=None, err=None, target=None, device=None):
        """Every image buffer against the batch's shape: rgb, out and target
        [B,3,H,W] fp32, z and err [B,H,W] fp32, hole [B,H,W] uint8, all
        contiguous on rgb's device (the kernels write err and out through
        raw pointers sized from rgb).  Returns (B, H, W)."""
        B, H, W = Repair._shape(rgb)
        dev = rgb.device if device is None else device
        api.check_tensor("rgb", rgb, (B, 3, H, W), torch.float32, dev)
        api.check_tensor("z", z, (B, H, W), torch.float32, dev)
        api.check_tensor("hole", hole, (B, H, W), torch.uint8, dev)
        for name, t in (("out", out), ("target", target)):
            if t is not None:
                api.check_tensor(name, t, (B, 3, H, W), torch.float32, dev)
        if err is not None:
            api.check_tensor("err", err, (B, H, W), torch.float32, dev)
        return B, H, W

    def forward(self, rgb, z, hole, out=None, err=None):
        """Repaired rgb [B,3,H,W]; err ([B,H,W], optional) receives the
        predicted squared error at holes."""
        out = torch.empty_like(rgb) if out is None else out
        B, H, W = self.check_images(rgb, z, hole, out=out, err=err)
        ws = self._workspace(B, H, W, False)
        P = _abi_ptr
        _check(self.L.bgs_repair_forward(P(self.params), B, H, W, P(rgb), P(z), P(hole), P(out), P(err), P(ws),
                                         ws.numel(), api._stream()), "bgs_repair_forward")
        return out

    def hole_error(self, err, hole, out=None, scratch=None):
        """Mean predicted squared error over each image's holes ([B]
        device floats), the fallback policy's measure."""
        B, H, W = (int(x) for x in hole.shape)
        api.check_tensor("err", err, (B, H, W), torch.float32, err.device)
        api.check_tensor("hole", hole, (B, H, W), torch.uint8, err.device)
        out = torch.empty(B, device=err.device) if out is None else out
        api.check_tensor("out", out, (B,), torch.float32, err.device)
        scratch = torch.empty(512 * B, device=err.device) if scratch is None else scratch
        api.check_tensor("scratch", scratch, (512 * B,), torch.float32, err.device)
        P = _abi_ptr
        _check(self.L.bgs_repair_hole_error(P(err), P(hole), B, H, W, P(out), P(scratch), api._stream()),
               "bgs_repair_hole_error")
        return out

    def grad_step(self, rgb, z, hole, target, rgb_out=None):
        """Loss and gradient into self.loss / self.grad (asynchronous)."""
        B, H, W = self.check_images(rgb, z, hole, out=rgb_out, target=target)
        ws = self._workspace(B, H, W, True)
        P = _abi_ptr
        _check(self.L.bgs_repair_grad(P(self.params), B, H, W, P(rgb), P(z), P(hole), P(target), P(self.grad),
                                      P(self.loss), P(rgb_out), P(ws), ws.numel(), api._stream()),
               "bgs_repair_grad")
        return self.loss

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        P = _abi_ptr
        _check(self.L.bgs_repair_adam(P(self.params), P(self.grad), P(self.m), P(self.v), self.params.numel(),
                                      self.step_count, lr, beta1, beta2, eps, api._stream()), "bgs_repair_adam")

    def train_step(self, rgb, z, hole, target, lr=1e-3):
        loss = self.grad_step(rgb, z, hole, target)
        self.adam(lr)
        return loss


def _abi_ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device tensors must be contiguous CUDA tensors")
    return C.c_void_p(t.data_ptr())


def make_pairs(scene, cams_dom, cams_aff, roi: api.Roi = api.Roi()):
    """Per pose: the dominant render reprojected to the affiliated camera
    (rgb [3,H,W], z, hole) and the full affiliated render (target)."""
    ctx = api.Context()
    ds = api.DeviceScene(scene)
    out = []
    for cd, ca in zip(cams_dom, cams_aff):
        d = ctx.render_dominant(ds, cd)
        w = ctx.reproject(cd, ca, d["rgb"], d["depth_raw"], d["alpha"], roi)
        t = ctx.render_dominant(ds, ca)
        out.append(dict(rgb=w["rgb"].clone(), z=w["z"].clone(), hole=w["hole"].clone(), alpha=w["alpha"].clone(),
                        depth_range=w["depth_range"].clone(), target=t["rgb"].clone()))
    torch.cuda.synchronize()
    return out


def config_pairs(seed=0):
    """Training and held-out pairs from the three plain configurations'
    scenes: the 10k cube seen from 12 azimuths at distance 4 (256x256), the
    300k shell's 16 orbit poses (800x600) and the 1M unbounded scene's 32
    forward poses (1600x1064); every fourth pose (and the cube's last three)
    is held out.  Returns {config: (train, test, cams_dom_test, cams_aff_test,
    scene)}."""
    from . import synth
    out = {}
    sc = synth.scene_uniform_cube(seed, 10_000)
    cams = [synth.look_at((4.0 * math.sin(t), -4.0 * math.cos(t), 0.8), (0, 0, 0), (0, 0, 1), 256, 256, 300.0)
            for t in np.linspace(0.0, 2.0 * np.pi, 12, endpoint=False)]
    held = [9, 10, 11]
    out["cube256"] = (sc, cams, held, synth.BASELINE_IPD)
    sc, cams, b = synth.WORKLOADS["sphere800"](seed)
    out["sphere800"] = (sc, cams, [0, 5, 10, 15], b)
    sc, cams, b = synth.WORKLOADS["unbounded1600"](seed)
    out["unbounded1600"] = (sc, cams, list(range(3, 32, 4)), b)
    res = {}
    for name, (sc, cams, held, b) in out.items():
        affs = [synth.affiliated(c, b) for c in cams]
        tr = [i for i in range(len(cams)) if i not in held]
        res[name] = (make_pairs(sc, [cams[i] for i in tr], [affs[i] for i in tr]),
                     make_pairs(sc, [cams[i] for i in held], [affs[i] for i in held]),
                     [cams[i] for i in held], [affs[i] for i in held], sc)
    return res


def crops(pairs, batch, size, rng, min_holes=16):
    """A batch of size x size crops, each centred on a random hole pixel."""
    rgb, z, hole, tgt = [], [], [], []
    while len(rgb) < batch:
        p = pairs[int(rng.integers(len(pairs)))]
        H, W = p["hole"].shape
        hy, hx = p["_holes"]
        if hy.size == 0:
            continue
        k = int(rng.integers(hy.size))
        y0 = int(np.clip(hy[k] - size // 2, 0, H - size))
        x0 = int(np.clip(hx[k] - size // 2, 0, W - size))
        h = p["hole"][y0:y0 + size, x0:x0 + size]
        if int(h.sum()) < min_holes:
            continue
        rgb.append(p["rgb"][:, y0:y0 + size, x0:x0 + size])
        z.append(p["z"][y0:y0 + size, x0:x0 + size])
        hole.append(h)
        tgt.append(p["target"][:, y0:y0 + size, x0:x0 + size])
    return (torch.stack(rgb).contiguous(), torch.stack(z).contiguous(), torch.stack(hole).contiguous(),
            torch.stack(tgt).contiguous())


def index_holes(pairs):
    for p in pairs:
        hy, hx = np.nonzero(p["hole"].cpu().numpy())
        p["_holes"] = (hy, hx)
    return pairs


def train(net: Repair, pairs, steps, batch=8, size=128, lr=1e-3, seed=0, log=None):
    rng = np.random.default_rng(seed)
    index_holes(pairs)
    losses = []
    for i in range(steps):
        rgb, z, hole, tgt = crops(pairs, batch, size, rng)
        loss = net.train_step(rgb, z, hole, tgt, lr=lr)
        if log and (i % log == 0 or i == steps - 1):
            losses.append((i, float(loss.item())))
    return losses


def interpolation_fill(pair, cam_dom, cam_aff, roi: api.Roi = api.Roi(center_roi=0)):
    """The method's plain fill of the same holes: gap interpolation, and with
    Step 2 off a row fill of what remains (edge ROIs are left to
    re-rendering and marked in the class map)."""
    ctx = api.Context()
    rgb = pair["rgb"].clone()
    z = pair["z"].clone()
    alpha = pair["alpha"].clone()
    cls = pair["hole"].clone()
    ctx.classify_holes(cam_dom, cam_aff, pair["depth_range"], rgb, z, alpha, cls, roi)
    torch.cuda.synchronize()
    return rgb, cls


def error_correlation(x, target, hole, err):
    """Pearson correlation, over hole pixels, of the predicted squared error
    with the actual one (mean over channels of (x - target)^2)."""
    m = hole.bool()
    actual = ((x.clamp(0, 1) - target.clamp(0, 1)) ** 2).mean(0)[m].double()
    pred = err[m].double()
    if actual.numel() < 2:
        return float("nan")
    return float(torch.corrcoef(torch.stack([pred, actual]))[0, 1])


def hole_psnr(a, b, mask):
    m = mask.bool()
    if int(m.sum()) == 0:
        return float("inf")
    d = (a.clamp(0, 1) - b.clamp(0, 1))[:, m]
    mse = float((d * d).mean())
    return 10.0 * math.log10(1.0 / max(mse, 1e-12))


def evaluate(net, ctx, name, test, cams_dom, cams_aff, scene, reps=20):
    """Held-out poses of one configuration: hole-pixel PSNR of the network,
    of the plain interpolation fill and of the full method (interpolation
    plus ROI re-rendering), the error channel's correlation, and the time of
    the network's pass against the full method's affiliated-eye work."""
    ds = api.DeviceScene(scene)
    rows = []
    for p, cd, ca in zip(test, cams_dom, cams_aff):
        err = torch.empty((1,) + tuple(p["hole"].shape), device=p["rgb"].device)
        x = net.forward(p["rgb"][None].contiguous(), p["z"][None].contiguous(), p["hole"][None].contiguous(),
                        err=err)[0]
        interp, cls = interpolation_fill(p, cd, ca)
        filled = (p["hole"] > 0) & ((cls == _abi.CLS_GAP) | (cls == _abi.CLS_ROWFILL))
        full = ctx.render_stereo(ds, cd, ca)["rgb_aff"]
        rows.append(dict(psnr_net=hole_psnr(x, p["target"], filled), psnr_interp=hole_psnr(interp, p["target"], filled),
                         psnr_net_all=hole_psnr(x, p["target"], p["hole"]),
                         psnr_method_all=hole_psnr(full, p["target"], p["hole"]),
                         corr=error_correlation(x, p["target"], p["hole"], err[0]),
                         pred_err=float(net.hole_error(err, p["hole"][None])[0])))
    # Times at this configuration's frame size: the network's pass, and the
    # method's affiliated-eye work after reprojection (classification and
    # ROI patch).
    p, cd, ca = test[0], cams_dom[0], cams_aff[0]
    a = (p["rgb"][None].contiguous(), p["z"][None].contiguous(), p["hole"][None].contiguous())
    o = torch.empty_like(a[0])

    def timeit(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    net_ms = timeit(lambda: net.forward(*a, out=o))
    rgb, z, al, hole = p["rgb"].clone(), p["z"].clone(), p["alpha"].clone(), p["hole"].clone()
    roi = api.Roi()

    def method():
        rgb.copy_(p["rgb"])
        z.copy_(p["z"])
        al.copy_(p["alpha"])
        hole.copy_(p["hole"])
        c = ctx.classify_holes(cd, ca, p["depth_range"], rgb, z, al, hole, roi)
        ctx.patch_rois(ds, ca, c["tile_mask"], rgb, z, al, hole)

    ctx.set_sync(True)
    method()  # sizes the workspace
    ctx.set_sync(False)
    method_ms = timeit(method)
    ctx.set_sync(True)
    m = lambda k: round(float(np.mean([r[k] for r in rows])), 3)
    H, W = p["hole"].shape
    return {"config": name, "width": int(W), "height": int(H), "held_out_poses": len(rows),
            "hole_psnr_net": m("psnr_net"), "hole_psnr_interp": m("psnr_interp"),
            "hole_psnr_net_all_holes": m("psnr_net_all"), "hole_psnr_method_all_holes": m("psnr_method_all"),
            "err_corr": m("corr"), "pred_err_mean": float(np.mean([r["pred_err"] for r in rows])),
            "net_ms": round(net_ms, 4), "method_aff_ms": round(method_ms, 4)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--configs", action="store_true",
                    help="train on crops from the three configurations' scenes (cube, shell, unbounded) and report "
                         "each configuration's held-out poses")
    ap.add_argument("--save", default="", help="write the trained parameters here (.npy)")
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--crop", type=int, default=128)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    from . import synth
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 3
    if args.configs:
        t0 = time.perf_counter()
        sets = config_pairs(args.seed)
        pairs = [q for tr, *_ in sets.values() for q in tr]
        t_data = time.perf_counter() - t0
        net = Repair(seed=args.seed)
        t0 = time.perf_counter()
        losses = train(net, pairs, args.steps, args.batch, args.crop, args.lr, args.seed, log=250)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        if args.save:
            np.save(args.save, net.params.cpu().numpy())
        ctx = api.Context()
        rows = [evaluate(net, ctx, name, te, cd, ca, sc) for name, (_, te, cd, ca, sc) in sets.items()]
        print(json.dumps({"train_pairs": args.steps * args.batch, "crop": args.crop, "source_frames": len(pairs),
                          "data_s": round(t_data, 2), "train_s": round(t_train, 2), "losses": losses,
                          "configs": rows}), flush=True)
        return 0
    scene, cams, b = synth.WORKLOADS["sphere800"](args.seed)
    affs = [synth.affiliated(c, b) for c in cams]
    held = [0, 5, 10, 15]
    tr = [i for i in range(len(cams)) if i not in held]
    pairs = make_pairs(scene, [cams[i] for i in tr], [affs[i] for i in tr])
    test = make_pairs(scene, [cams[i] for i in held], [affs[i] for i in held])
    net = Repair(seed=args.seed)
    t0 = time.perf_counter()
    losses = train(net, pairs, args.steps, args.batch, args.crop, args.lr, args.seed, log=50)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res = []
    ctx = api.Context()
    ds = api.DeviceScene(scene)
    for i, p in zip(held, test):
        err = torch.empty((1,) + tuple(p["hole"].shape), device=p["rgb"].device)
        x = net.forward(p["rgb"][None].contiguous(), p["z"][None].contiguous(), p["hole"][None].contiguous(),
                        err=err)[0]
        interp, cls = interpolation_fill(p, cams[i], affs[i])
        filled = (p["hole"] > 0) & ((cls == _abi.CLS_GAP) | (cls == _abi.CLS_ROWFILL))
        # The full method: interpolation plus ROI re-rendering (render_stereo).
        full = ctx.render_stereo(ds, cams[i], affs[i])["rgb_aff"]
        res.append(dict(pose=i, holes=int(p["hole"].sum()), compared=int(filled.sum()),
                        psnr_net=round(hole_psnr(x, p["target"], filled), 3),
                        psnr_interp=round(hole_psnr(interp, p["target"], filled), 3),
                        psnr_net_all_holes=round(hole_psnr(x, p["target"], p["hole"]), 3),
                        psnr_method_all_holes=round(hole_psnr(full, p["target"], p["hole"]), 3),
                        err_corr=round(error_correlation(x, p["target"], p["hole"], err[0]), 3)))
    # Inference time at full frame size.
    p = test[0]
    args_t = (p["rgb"][None].contiguous(), p["z"][None].contiguous(), p["hole"][None].contiguous())
    out = torch.empty_like(args_t[0])
    for _ in range(5):
        net.forward(*args_t, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(50):
        net.forward(*args_t, out=out)
    e1.record()
    torch.cuda.synchronize()
    H, W = p["hole"].shape
    ms = e0.elapsed_time(e1) / 50
    tflops = flops_per_pixel() * H * W / (ms * 1e-3) / 1e12
    print(json.dumps({"workload": "sphere800", "width": int(W), "height": int(H), "train_steps": args.steps,
                      "batch": args.batch, "crop": args.crop, "train_s": round(t_train, 2), "losses": losses,
                      "held_out": res, "infer_ms": round(ms, 4),
                      "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": 2500.0, "unit": "TFLOP/s",
                                   "frac": round(tflops / 2500.0, 5),
                                   "flops_per_pixel": flops_per_pixel()}}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
