"""CPU oracle of the learned gap/edge repair network (test infrastructure:
only the tests, the smoke check and the bench's CPU leg use it).

The network fills the holes the forward reprojection leaves in the
affiliated eye (Sec. 3.4-3.5: the warped image has disocclusions and
cracks that the method fills by interpolation and ROI re-rendering).  It
is a three-level convolutional U-Net:

    level 1 (H x W):      e1a 5->16, e1b 16->16
    level 2 (H/2 x W/2):  e2a 16->32, e2b 32->32   (input: 2x2 mean pool of e1b)
    level 3 (H/4 x W/4):  e3a 32->64, e3b 64->64   (input: 2x2 mean pool of e2b)
    level 2:              d2 (64+32)->32            (input: [nearest 2x upsample of e3b, e2b])
    level 1:              d1 (32+16)->16            (input: [upsample of d2, e1b])
    level 1:              out 16->4, no activation
    every other 3x3 convolution (zero padding, stride 1) is followed by ReLU.

Inputs per pixel: the warped RGB (0 at holes), the hole mask, and inverse
depth 1/z (0 at holes and for background).  Output channels 0-2 are a
residual on the holes only: pred = rgb + hole * r.  Channel 3, e, predicts
the pixel's squared error s = mean over channels of (pred - target)^2.  The
loss over hole pixels is
    sum_c (pred_c - target_c)^2 / (3 N) + sum (e - s)^2 / N,  N = max(1, holes),
with s held constant in the gradient (it is the error channel's target, not
a path back into the residual).  Training uses Adam (Kingma and Ba, 2015)
with bias correction.

Everything is computed in fp64.  The GPU stores activations, gradients
that feed matrix products, and weights in bfloat16; passing q=bf16 rounds
at exactly those points (round to nearest even from the fp32 value), so
the GPU result can be compared with fp32-accumulation tolerances.  With
q=None the oracle is the plain fp64 network, which the finite-difference
pins check.

Parameter layout (flat fp32): for each layer in the order above, the
weights W[cout][cin][3][3] then the bias b[cout].
"""
from __future__ import annotations

import numpy as np

# (name, cin, cout, relu)
LAYERS = [
    ("e1a", 5, 16, True), ("e1b", 16, 16, True),
    ("e2a", 16, 32, True), ("e2b", 32, 32, True),
    ("e3a", 32, 64, True), ("e3b", 64, 64, True),
    ("d2", 96, 32, True), ("d1", 48, 16, True),
    ("out", 16, 4, False),
]


def num_params() -> int:
    return sum(co * ci * 9 + co for _, ci, co, _ in LAYERS)


def unpack(params: np.ndarray) -> dict:
    """Flat parameter vector -> {name: (W[cout][cin][3][3], b[cout])}."""
    out, o = {}, 0
    for name, ci, co, _ in LAYERS:
        w = params[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = params[o:o + co]
        o += co
        out[name] = (w, b)
    assert o == params.size
    return out


def pack(grads: dict) -> np.ndarray:
    return np.concatenate([np.concatenate([grads[n][0].ravel(), grads[n][1].ravel()]) for n, *_ in LAYERS])


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) from the fp32 value; the
    result is returned as float64.  Values are finite here."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(x):
    return np.asarray(x, np.float64)


# --- layers (definitions written out) ---------------------------------------

def conv3x3(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """y[b, o, i, j] = sum_{c, u, v} w[o, c, u, v] x[b, c, i + u - 1, j + v - 1],
    zero outside the image.  x [B, C, H, W], w [O, C, 3, 3]."""
    B, C, H, W = x.shape
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((B, w.shape[0], H, W))
    for u in range(3):
        for v in range(3):
            y += np.einsum("oc,bchw->bohw", w[:, :, u, v], xp[:, :, u:u + H, v:v + W])
    return y


def conv3x3_grad_input(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of conv3x3 in x: dx[b, c, i, j] = sum_{o, u, v} w[o, c, u, v] g[b, o, i - u + 1, j - v + 1]."""
    B, O, H, W = g.shape
    dxp = np.zeros((B, w.shape[1], H + 2, W + 2))
    for u in range(3):
        for v in range(3):
            dxp[:, :, u:u + H, v:v + W] += np.einsum("oc,bohw->bchw", w[:, :, u, v], g)
    return dxp[:, :, 1:-1, 1:-1]


def conv3x3_grad_weight(g: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dw[o, c, u, v] = sum_{b, i, j} g[b, o, i, j] x[b, c, i + u - 1, j + v - 1]."""
    B, C, H, W = x.shape
    xp = np.zeros((B, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dw = np.zeros((g.shape[1], C, 3, 3))
    for u in range(3):
        for v in range(3):
            dw[:, :, u, v] = np.einsum("bohw,bchw->oc", g, xp[:, :, u:u + H, v:v + W])
    return dw


def pool2(x: np.ndarray) -> np.ndarray:
    """2x2 mean."""
    return 0.25 * (x[:, :, 0::2, 0::2] + x[:, :, 0::2, 1::2] + x[:, :, 1::2, 0::2] + x[:, :, 1::2, 1::2])


def pool2_grad(g: np.ndarray) -> np.ndarray:
    return 0.25 * up2(g)


def up2(x: np.ndarray) -> np.ndarray:
    """Nearest 2x upsample."""
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def up2_grad(g: np.ndarray) -> np.ndarray:
    return g[:, :, 0::2, 0::2] + g[:, :, 0::2, 1::2] + g[:, :, 1::2, 0::2] + g[:, :, 1::2, 1::2]


def net_input(rgb: np.ndarray, z: np.ndarray, hole: np.ndarray, q=_ident) -> np.ndarray:
    """[B, 5, H, W]: rgb with holes zeroed, hole mask, 1/z (0 at holes and
    for infinite depth)."""
    h = hole.astype(np.float64)
    z = np.asarray(z, np.float64)
    inv = np.where((h > 0) | ~np.isfinite(z), 0.0, 1.0 / np.where(np.isfinite(z) & (z != 0), z, 1.0))
    inv = np.asarray(inv.astype(np.float32), np.float64)  # the GPU forms 1/z in fp32
    x = np.concatenate([np.asarray(rgb, np.float64) * (1.0 - h)[:, None], h[:, None], inv[:, None]], axis=1)
    return q(x)


# --- network ----------------------------------------------------------------

def forward(params: np.ndarray, rgb, z, hole, q=None) -> dict:
    """Forward pass; returns every stored activation, r and pred."""
    q = q or _ident
    P = unpack(np.asarray(params, np.float64))
    Wq = {n: (q(P[n][0]), P[n][1]) for n in P}

    def layer(name, x):
        w, b = Wq[name]
        y = conv3x3(x, w) + b[None, :, None, None]
        return q(np.maximum(y, 0.0))

    a = {"x0": net_input(rgb, z, hole, q)}
    a["e1a"] = layer("e1a", a["x0"])
    a["e1b"] = layer("e1b", a["e1a"])
    a["p1"] = q(pool2(a["e1b"]))
    a["e2a"] = layer("e2a", a["p1"])
    a["e2b"] = layer("e2b", a["e2a"])
    a["p2"] = q(pool2(a["e2b"]))
    a["e3a"] = layer("e3a", a["p2"])
    a["e3b"] = layer("e3b", a["e3a"])
    a["cat2"] = np.concatenate([up2(a["e3b"]), a["e2b"]], axis=1)
    a["d2"] = layer("d2", a["cat2"])
    a["cat1"] = np.concatenate([up2(a["d2"]), a["e1b"]], axis=1)
    a["d1"] = layer("d1", a["cat1"])
    w, b = Wq["out"]
    a["r"] = np.asarray((conv3x3(a["d1"], w) + b[None, :, None, None]).astype(np.float32), np.float64) \
        if q is not _ident else conv3x3(a["d1"], w) + b[None, :, None, None]
    h = np.asarray(hole, np.float64)[:, None]
    a["pred"] = np.asarray(rgb, np.float64) + h * a["r"][:, :3]
    a["e"] = a["r"][:, 3]
    return a


def loss_and_grad(params: np.ndarray, rgb, z, hole, target, q=None, err_target=None):
    """Loss and gradient (flat, in the parameter layout).  err_target, if
    given, replaces the error channel's target s (finite differences hold
    it fixed, as the gradient does)."""
    qq = q or _ident
    a = forward(params, rgb, z, hole, q)
    P = unpack(np.asarray(params, np.float64))
    Wq = {n: qq(P[n][0]) for n in P}
    hp = np.asarray(hole, np.float64)
    h = hp[:, None]
    nh = max(1.0, float(np.sum(hole)))
    diff = (a["pred"] - np.asarray(target, np.float64)) * h
    s = np.mean(diff * diff, axis=1) if err_target is None else np.asarray(err_target, np.float64)
    de = (a["e"] - s) * hp
    loss = float(np.sum(diff * diff) / (3.0 * nh) + np.sum(de * de) / nh)
    g = {}

    def back(name, g_pre, x_in):
        g[name] = (conv3x3_grad_weight(g_pre, x_in), g_pre.sum(axis=(0, 2, 3)))

    def relu_mask(v, act):
        return v * (act > 0)

    g_r = qq(np.concatenate([2.0 * diff / (3.0 * nh), (2.0 * de / nh)[:, None]], axis=1))
    back("out", g_r, a["d1"])
    g_d1 = relu_mask(qq(conv3x3_grad_input(g_r, Wq["out"])), a["d1"])
    back("d1", g_d1, a["cat1"])
    g_cat1 = qq(conv3x3_grad_input(g_d1, Wq["d1"]))
    g_d2 = relu_mask(qq(up2_grad(g_cat1[:, :32])), a["d2"])
    back("d2", g_d2, a["cat2"])
    g_cat2 = qq(conv3x3_grad_input(g_d2, Wq["d2"]))
    g_e3b = relu_mask(qq(up2_grad(g_cat2[:, :64])), a["e3b"])
    back("e3b", g_e3b, a["e3a"])
    g_e3a = relu_mask(qq(conv3x3_grad_input(g_e3b, Wq["e3b"])), a["e3a"])
    back("e3a", g_e3a, a["p2"])
    g_p2 = qq(conv3x3_grad_input(g_e3a, Wq["e3a"]))
    g_e2b = relu_mask(qq(g_cat2[:, 64:] + pool2_grad(g_p2)), a["e2b"])
    back("e2b", g_e2b, a["e2a"])
    g_e2a = relu_mask(qq(conv3x3_grad_input(g_e2b, Wq["e2b"])), a["e2a"])
    back("e2a", g_e2a, a["p1"])
    g_p1 = qq(conv3x3_grad_input(g_e2a, Wq["e2a"]))
    g_e1b = relu_mask(qq(g_cat1[:, 32:] + pool2_grad(g_p1)), a["e1b"])
    back("e1b", g_e1b, a["e1a"])
    g_e1a = relu_mask(qq(conv3x3_grad_input(g_e1b, Wq["e1b"])), a["e1a"])
    back("e1a", g_e1a, a["x0"])
    return loss, pack(g)


def adam(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015, Algorithm 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
