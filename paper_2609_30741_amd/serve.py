"""Serving loop for stereo-frame requests over resident scenes.

Requests (a scene key, a dominant and an affiliated camera) arrive over time.
The scheduler admits a request when a slot is free and the memory it needs
(workspace and output images) fits in what the in-flight requests leave of
the budget; its frame is then issued at once on the slot's own stream, so
requests that arrive while others run join the work already on the GPU
(continuous batching: no batch boundaries, frames overlap on the device).
Scenes stay resident on the device for the server's lifetime.  Latency is
completion minus arrival; completion is read from GPU events, so the host's
polling interval does not enter it.

The scheduler (`serve`) is plain Python over an executor with six calls
(need_bytes, held_bytes, trim, issue, poll, release), so its admission
logic is testable without a GPU; `GpuExecutor` runs each frame through the
library (`Context.render_stereo`, or two `render_dominant` calls for the
two-pass baseline), one context and one default-priority stream per slot.

Memory is accounted by what the slots actually hold, not by what the
requests in flight asked for: a slot keeps its workspace and output images
after its frame (so the next frame of the same size allocates nothing),
and those bytes stay charged to the budget until the slot is trimmed.  A
request is admitted into a free slot when the bytes every other slot holds
plus its own need fit in the budget; idle slots are trimmed (their buffers
freed) to make room before the request waits.  The bytes held by all slots
together therefore never exceed the budget.

    python -m paper_2609_30741_amd.serve [--workload serve2064] [--rate 90]
        [--requests 300] [--slots 4] [--mode stereo|two_pass]

prints one JSON line with p50/p99 latency, throughput and queueing.
"""
from __future__ import annotations

import argparse
import collections
import dataclasses
import json
import math
import sys
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    scene: str
    cam_dom: object
    cam_aff: object
    arrival: float  # seconds after the start of the run
    slot: int = -1
    admitted: float = math.nan  # host time of issue, seconds after the start
    done: float = math.nan  # completion on the GPU clock, seconds after the start
    out: Optional[dict] = None
    phase: int = 0  # learned mode: 1 after the network pass, 2 after a fallback pass
    pred_err: float = math.nan  # learned mode: the network's mean predicted squared error at the holes
    fallback: Optional[bool] = None  # learned mode: interpolation + ROI re-rendering replaced the network

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def poisson_arrivals(rate: float, n: int, seed: int = 0) -> np.ndarray:
    """n arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def serve(requests: List[Request], executor, n_slots: int, mem_budget: float,
          clock: Callable[[], float] = time.perf_counter, idle: Callable[[], None] = lambda: None) -> List[Request]:
    """Run the requests (sorted by arrival) to completion and return them with
    slot, admission and completion times filled in.  First come, first
    admitted: a request waits for the one ahead of it, so none is starved by
    later, smaller ones."""
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    queue: collections.deque = collections.deque()
    busy: Dict[int, Request] = {}
    free = list(range(n_slots))
    executor.start()  # the GPU clock's zero, then the host's
    t0 = clock()
    while pending or queue or busy:
        progressed = False
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            queue.append(pending.popleft())
            progressed = True
        for s, r in list(busy.items()):
            t = executor.poll(s, r)
            if t is not None:
                r.done = t
                executor.release(s, r)
                del busy[s]
                free.append(s)
                progressed = True
        while queue and free:
            r = queue[0]
            need = executor.need_bytes(r)
            if need > mem_budget:
                raise ValueError(f"request {r.rid} needs {need:.3g} B, more than the whole budget {mem_budget:.3g} B")
            # Prefer a free slot that already holds buffers of this size.
            s = next((q for q in free if executor.held_bytes(q) == need), free[0])
            others = sum(executor.held_bytes(q) for q in range(n_slots) if q != s)
            for q in free:
                if others + need <= mem_budget:
                    break
                if q != s and executor.held_bytes(q) > 0:
                    others -= executor.held_bytes(q)
                    executor.trim(q)
            if others + need > mem_budget:
                break  # waits for memory held by running frames, not only for a slot
            queue.popleft()
            free.remove(s)
            r.slot = s
            r.admitted = clock() - t0
            executor.issue(s, r)
            busy[s] = r
            progressed = True
        if not progressed:
            idle()
    return requests


def summary(reqs: List[Request]) -> dict:
    lat = np.array([r.latency for r in reqs]) * 1e3
    wait = np.array([r.admitted - r.arrival for r in reqs]) * 1e3
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return {"requests": len(reqs), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
            "max_ms": round(float(lat.max()), 3), "queue_p99_ms": round(float(np.percentile(wait, 99)), 3),
            "throughput": round(len(reqs) / span, 2), "span_s": round(span, 4)}


class GpuExecutor:
    """Frames through the library: one context, stream and workspace per slot;
    scenes resident; completion from an event recorded after each frame."""

    def __init__(self, scenes: dict, n_slots: int, raster=None, roi=None, mode: str = "stereo",
                 key_capacity: int = 0, keep_outputs: bool = False, repair_params=None, threshold: float = math.inf):
        import torch
        from . import api
        self.torch, self.api = torch, api
        if mode not in ("stereo", "two_pass", "learned"):
            raise ValueError(f"unknown mode {mode}")
        self.mode = mode
        self.threshold = float(threshold)
        self.nets = []
        if mode == "learned":
            from . import repair
            if repair_params is None:
                raise ValueError("the learned mode needs the repair network's parameters")
            # One network object per slot: the parameters are copied, and each
            # slot's forward passes get a workspace of their own.
            self.nets = [repair.Repair(params=repair_params) for _ in range(n_slots)]
        self.raster = raster or api.Raster()
        self.roi = roi or api.Roi()
        self.keep = keep_outputs
        self.box_capacity = 4096
        self.scenes = {k: api.DeviceScene(s) for k, s in scenes.items()}
        self.key_capacity = key_capacity
        self.streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(n_slots - 1)]
        self.ctxs, self.outs, self.events = [], [], [None] * n_slots
        for s in range(n_slots):
            with torch.cuda.stream(self.streams[s]):
                c = api.Context(sync=False)
                self.ctxs.append(c)
                self.outs.append(None)
        self.start_ev = torch.cuda.Event(enable_timing=True)

    def _sizes(self, r: Request):
        sc = self.scenes[r.scene]
        W = max(r.cam_dom.width, r.cam_aff.width)
        H = max(r.cam_dom.height, r.cam_aff.height)
        return sc.n, W, H

    def _out_bytes(self, r: Request) -> int:
        """Bytes of the output images a frame of this request writes."""
        pd = int(r.cam_dom.width) * int(r.cam_dom.height)
        pa = int(r.cam_aff.width) * int(r.cam_aff.height)
        if self.mode == "two_pass":
            return 20 * (pd + pa)  # rgb, depth, alpha per eye
        if self.mode == "learned":
            import ctypes as C
            rw = C.c_size_t()
            self.nets[0].L.bgs_repair_workspace_size(1, int(r.cam_aff.height), int(r.cam_aff.width), 0, C.byref(rw))
            T = self.roi.tile
            tiles = ((int(r.cam_aff.width) + T - 1) // T) * ((int(r.cam_aff.height) + T - 1) // T)
            # dominant rgb/depth/alpha; warped rgb/z/alpha, class map, labels,
            # network rgb and error; boxes, counts, tile mask, the network's
            # workspace and the error reduction's scratch
            return (20 * pd + 41 * pa + 6 * 4 * self.box_capacity + tiles + 4 + 8 + 4 + 4 * 512 + int(rw.value))
        T = self.roi.tile
        tiles = ((int(r.cam_aff.width) + T - 1) // T) * ((int(r.cam_aff.height) + T - 1) // T)
        # dominant rgb/depth/alpha; affiliated rgb/z/alpha, class map, labels; boxes, count, tile mask
        return 20 * pd + 25 * pa + 6 * 4 * self.box_capacity + 4 + tiles

    def need_bytes(self, r: Request) -> float:
        n, W, H = self._sizes(r)
        return float(self.ctxs[0]._ws_bytes(n, W, H, self.key_capacity) + self._out_bytes(r))

    def held_bytes(self, s: int) -> float:
        ws = self.ctxs[s].ws
        held = 0 if ws is None else ws.numel()
        o = self.outs[s]
        if o is not None:
            ts = []
            for v in o.values():
                if isinstance(v, dict):
                    ts += [t for t in v.values() if isinstance(t, self.torch.Tensor)]
                elif isinstance(v, self.torch.Tensor) and not v.is_pinned():
                    ts.append(v)
            held += sum(t.numel() * t.element_size() for t in ts)
        if self.nets:
            held += sum(w.numel() for w in self.nets[s]._ws.values())
        return float(held)

    def trim(self, s: int):
        """Free an idle slot's workspace and output images."""
        self.ctxs[s].ws = None
        self.outs[s] = None
        if self.nets:
            self.nets[s]._ws.clear()

    def start(self):
        torch = self.torch
        torch.cuda.synchronize()
        self.start_ev.record(self.streams[0])
        torch.cuda.synchronize()

    def issue(self, s: int, r: Request):
        torch = self.torch
        sc = self.scenes[r.scene]
        n, W, H = self._sizes(r)
        ctx = self.ctxs[s]
        with torch.cuda.stream(self.streams[s]):
            # The slot's buffers are replaced unless they are exactly this
            # request's: it then holds what need_bytes charged for it.
            ws_need = ctx._ws_bytes(n, W, H, self.key_capacity)
            if ctx.ws is not None and ctx.ws.numel() != ws_need:
                ctx.ws = None
            ctx.reserve(n, W, H, self.key_capacity)
            o = self.outs[s]
            if o is not None and self.held_bytes(s) != self.need_bytes(r):
                o = None
            if self.mode == "learned":
                self._issue_learned(s, r, ctx, sc, o)
                return
            if self.mode == "stereo":
                if o is not None and not self._stereo_fits(o, r):
                    o = None
                o = ctx.render_stereo(sc, r.cam_dom, r.cam_aff, self.raster, self.roi,
                                      box_capacity=self.box_capacity, out=o)
                self.outs[s] = o
                keys = ("rgb_dom", "depth_raw_dom", "alpha_dom", "rgb_aff", "z_aff", "alpha_aff", "cls_aff")
            else:
                o = o or {}
                fits = lambda d, c: d is not None and tuple(d["rgb"].shape[1:]) == (c.height, c.width)
                a = ctx.render_dominant(sc, r.cam_dom, self.raster,
                                        out=o.get("dom") if fits(o.get("dom"), r.cam_dom) else None)
                b = ctx.render_dominant(sc, r.cam_aff, self.raster,
                                        out=o.get("aff") if fits(o.get("aff"), r.cam_aff) else None)
                o = {"dom": a, "aff": b}
                self.outs[s] = o
                keys = ()
            if self.keep:
                # Copied in stream order, before the slot's next frame reuses the buffers.
                r.out = {k: o[k].clone() for k in keys} if keys else {
                    "rgb_dom": o["dom"]["rgb"].clone(), "rgb_aff": o["aff"]["rgb"].clone()}
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(self.streams[s])
            self.events[s] = ev

    def _issue_learned(self, s: int, r: Request, ctx, sc, o):
        """First phase of a learned-mode frame on slot s's stream: dominant
        render, reprojection into the affiliated buffers, the repair network
        over the warped image, and its mean predicted error at the holes,
        copied to pinned host memory for the fallback decision."""
        torch = self.torch
        cd, ca = r.cam_dom, r.cam_aff
        Hd, Wd, H, W = int(cd.height), int(cd.width), int(ca.height), int(ca.width)
        if o is None or tuple(o["dom"]["rgb"].shape[1:]) != (Hd, Wd) or tuple(o["warp"]["rgb"].shape[1:]) != (H, W):
            dev = "cuda"
            T = self.roi.tile
            o = {"dom": None,
                 "warp": dict(rgb=torch.empty((3, H, W), device=dev), z=torch.empty((H, W), device=dev),
                              alpha=torch.empty((H, W), device=dev),
                              hole=torch.empty((H, W), dtype=torch.uint8, device=dev),
                              depth_range=torch.empty(2, device=dev)),
                 "cls": dict(labels=torch.empty((H, W), dtype=torch.int32, device=dev),
                             boxes=torch.empty((self.box_capacity, 6), dtype=torch.int32, device=dev),
                             n_boxes=torch.empty(1, dtype=torch.int32, device=dev),
                             tile_mask=torch.empty(((H + T - 1) // T, (W + T - 1) // T), dtype=torch.uint8,
                                                   device=dev)),
                 "net": torch.empty((1, 3, H, W), device=dev), "err": torch.empty((1, H, W), device=dev),
                 "stat": torch.empty(1, device=dev), "scratch": torch.empty(512, device=dev),
                 "stat_host": torch.empty(1, pin_memory=True)}
        o["dom"] = ctx.render_dominant(sc, cd, self.raster, out=o["dom"])
        d, w = o["dom"], o["warp"]
        ctx.reproject(cd, ca, d["rgb"], d["depth_raw"], d["alpha"], self.roi, out=w)
        net = self.nets[s]
        net.forward(w["rgb"][None], w["z"][None], w["hole"][None], out=o["net"], err=o["err"])
        net.hole_error(o["err"], w["hole"][None], out=o["stat"], scratch=o["scratch"])
        o["stat_host"].copy_(o["stat"], non_blocking=True)
        self.outs[s] = o
        r.phase = 1
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(self.streams[s])
        self.events[s] = ev

    def _finish_learned(self, s: int, r: Request) -> bool:
        """After the first phase: decide from the predicted error; above the
        threshold, issue the fallback (gap interpolation, Step 2 and ROI
        re-rendering over the warped image) and return False (not done)."""
        torch = self.torch
        o = self.outs[s]
        r.pred_err = float(o["stat_host"][0])
        sc = self.scenes[r.scene]
        if r.phase == 1 and r.pred_err > self.threshold:
            r.fallback = True
            ctx = self.ctxs[s]
            w, c = o["warp"], o["cls"]
            with torch.cuda.stream(self.streams[s]):
                ctx.classify_holes(r.cam_dom, r.cam_aff, w["depth_range"], w["rgb"], w["z"], w["alpha"], w["hole"],
                                   self.roi, self.raster, box_capacity=self.box_capacity, out=c)
                ctx.patch_rois(sc, r.cam_aff, c["tile_mask"], w["rgb"], w["z"], w["alpha"], w["hole"], self.raster,
                               self.roi)
                r.phase = 2
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(self.streams[s])
                self.events[s] = ev
            return False
        if r.fallback is None:
            r.fallback = False
        if self.keep:
            with torch.cuda.stream(self.streams[s]):
                r.out = {"rgb_dom": o["dom"]["rgb"].clone(),
                         "rgb_aff": (o["warp"]["rgb"] if r.fallback else o["net"][0]).clone()}
        return True

    def _stereo_fits(self, o, r: Request) -> bool:
        """Whether a slot's stereo outputs have exactly this request's sizes
        (both eyes): the library writes through them at the cameras' sizes."""
        try:
            self.api.check_stereo_out(o, r.cam_dom, r.cam_aff, self.box_capacity, self.roi.tile,
                                      o["rgb_dom"].device)
            return True
        except ValueError:
            return False

    def poll(self, s: int, r: Optional[Request] = None) -> Optional[float]:
        ev = self.events[s]
        if ev is None or not ev.query():
            return None
        if self.mode == "learned" and r is not None and not self._finish_learned(s, r):
            return None  # the fallback pass is running
        return self.start_ev.elapsed_time(self.events[s]) * 1e-3

    def release(self, s: int, r: Request):
        st = self.ctxs[s].poll_status()
        if st["overflow"]:
            raise RuntimeError(f"request {r.rid}: key capacity {self.key_capacity} exceeded; raise --key-capacity")
        self.events[s] = None


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="serve2064")
    ap.add_argument("--rate", type=float, default=90.0, help="Poisson arrival rate, stereo frames/s")
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--mem-gb", type=float, default=64.0, help="memory budget of the in-flight requests")
    ap.add_argument("--mode", choices=("stereo", "two_pass", "learned"), default="stereo",
                    help="stereo: the method (interpolation + ROI re-rendering); two_pass: two full renders; "
                         "learned: the repair network, with the method as fallback above --threshold")
    ap.add_argument("--params", default="", help="learned mode: trained repair parameters (.npy)")
    ap.add_argument("--threshold", type=float, default=0.01,
                    help="learned mode: fall back when the network's mean predicted squared error at the holes "
                         "exceeds this")
    ap.add_argument("--quality", type=int, default=8,
                    help="affiliated-eye PSNR against the full render over this many poses (after the run)")
    ap.add_argument("--key-capacity", type=int, default=0, help="keys per pass (0: sized on the first poses)")
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)

    import torch
    from . import api, synth
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 3
    scene, cams, b = synth.WORKLOADS[args.workload](args.seed)
    affs = [synth.affiliated(c, b) for c in cams]
    kc = args.key_capacity
    if kc <= 0:
        # Size the key capacity on the poses (a synchronous context reads the
        # key counts back), with headroom.
        ctx = api.Context(sync=True)
        ds = api.DeviceScene(scene)
        out, mx = None, 0
        for cd, ca in zip(cams, affs):
            out = ctx.render_stereo(ds, cd, ca, out=out)
            mx = max(mx, out["stats"]["n_keys_dom"], out["stats"]["n_keys_roi"])
        kc = int(mx * 1.25) + 4096
        del ctx, ds, out
        torch.cuda.synchronize()
    params = np.load(args.params) if args.params else None
    ex = GpuExecutor({"s": scene}, args.slots, mode=args.mode, key_capacity=kc, repair_params=params,
                     threshold=args.threshold)
    n_poses = len(cams)

    def reqs(n, rate, seed):
        t = poisson_arrivals(rate, n, seed)
        return [Request(i, "s", cams[i % n_poses], affs[i % n_poses], float(t[i])) for i in range(n)]

    serve(reqs(args.warmup, args.rate, args.seed + 1), ex, args.slots, args.mem_gb * 1e9)
    done = serve(reqs(args.requests, args.rate, args.seed + 2), ex, args.slots, args.mem_gb * 1e9)
    s = summary(done)
    s.update({"workload": args.workload, "mode": args.mode, "rate": args.rate, "slots": args.slots,
              "width": int(cams[0].width), "height": int(cams[0].height), "surfels": int(scene.n),
              "key_capacity": kc})
    if args.mode == "learned":
        s["threshold"] = args.threshold
        s["fallback_frac"] = round(float(np.mean([bool(r.fallback) for r in done])), 4)
        s["pred_err_p50"] = float(np.percentile([r.pred_err for r in done], 50))
    if args.quality > 0:
        # Quality on a few poses, each request alone through the same
        # executor (outputs kept), against the full render of its eye.
        ex.keep = True
        q = [Request(i, "s", cams[i % n_poses], affs[i % n_poses], 0.0) for i in range(min(args.quality, n_poses))]
        serve(q, ex, 1, args.mem_gb * 1e9)
        torch.cuda.synchronize()
        ref = api.Context(sync=True)
        ds = ex.scenes["s"]
        ps = []
        for r in q:
            f = ref.render_dominant(ds, r.cam_aff)["rgb"]
            mse = float(((r.out["rgb_aff"].clamp(0, 1).double() - f.clamp(0, 1).double()) ** 2).mean())
            ps.append(10 * math.log10(1 / max(mse, 1e-30)))
        s["psnr_aff_vs_full_db"] = round(float(np.mean(ps)), 3)
        s["psnr_poses"] = len(ps)
        if args.mode == "learned":
            s["quality_fallback_frac"] = round(float(np.mean([bool(r.fallback) for r in q])), 4)
    print(json.dumps(s), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
