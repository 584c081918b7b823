"""The repair network's oracle against what fixes it independently: a
library correlation, finite differences of its own fp64 loss, adjoint
identities, Adam's first step in closed form, and torch's bfloat16
rounding."""
import numpy as np
import pytest
import torch
from scipy.signal import correlate

from oracle import repair_oracle as R


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 7, 9))
    w = rng.normal(size=(4, 3, 3, 3))
    y = R.conv3x3(x, w)
    for b in range(2):
        for o in range(4):
            want = sum(correlate(x[b, c], w[o, c], mode="same", method="direct") for c in range(3))
            np.testing.assert_allclose(y[b, o], want, rtol=1e-12, atol=1e-12)


def test_conv_adjoints():
    # <conv(x, w), g> = <x, conv^T(g, w)> = <w, dW(g, x)>
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 5, 6, 8))
    w = rng.normal(size=(3, 5, 3, 3))
    g = rng.normal(size=(2, 3, 6, 8))
    lhs = np.sum(R.conv3x3(x, w) * g)
    assert np.sum(x * R.conv3x3_grad_input(g, w)) == pytest.approx(lhs, rel=1e-12)
    assert np.sum(w * R.conv3x3_grad_weight(g, x)) == pytest.approx(lhs, rel=1e-12)


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 3, 8, 12))
    y = rng.normal(size=(2, 3, 4, 6))
    assert np.sum(R.pool2(x) * y) == pytest.approx(np.sum(x * R.pool2_grad(y)), rel=1e-12)
    assert np.sum(R.up2(y) * x) == pytest.approx(np.sum(y * R.up2_grad(x)), rel=1e-12)
    # A constant image pools and upsamples to itself.
    c = np.full((1, 1, 4, 4), 0.7)
    np.testing.assert_allclose(R.pool2(c), 0.7)
    np.testing.assert_allclose(R.up2(R.pool2(c)), c)


def _problem(seed, B=2, H=8, W=12):
    rng = np.random.default_rng(seed)
    hole = (rng.uniform(size=(B, H, W)) < 0.3).astype(np.uint8)
    rgb = rng.uniform(size=(B, 3, H, W)) * (1 - hole[:, None])
    z = np.where(hole > 0, np.inf, rng.uniform(1.5, 4.0, size=(B, H, W)))
    target = rng.uniform(size=(B, 3, H, W))
    params = rng.normal(size=R.num_params()) * 0.15
    return params, rgb, z, hole, target


def test_gradient_matches_finite_differences():
    params, rgb, z, hole, target = _problem(3)
    # The error channel's target is held fixed, as in the gradient.
    s = np.mean(((R.forward(params, rgb, z, hole)["pred"] - target) * hole[:, None]) ** 2, axis=1)
    loss, g = R.loss_and_grad(params, rgb, z, hole, target, err_target=s)
    assert loss == R.loss_and_grad(params, rgb, z, hole, target)[0]
    assert loss > 0
    rng = np.random.default_rng(4)
    # A few coordinates of every layer (weights and bias).
    idx, o = [], 0
    for _, ci, co, _ in R.LAYERS:
        nw = co * ci * 9
        idx += list(o + rng.choice(nw, 3, replace=False)) + [o + nw + int(rng.integers(co))]
        o += nw + co
    h = 1e-6
    for i in idx:
        p1 = params.copy()
        p1[i] += h
        p0 = params.copy()
        p0[i] -= h
        fd = (R.loss_and_grad(p1, rgb, z, hole, target, err_target=s)[0]
              - R.loss_and_grad(p0, rgb, z, hole, target, err_target=s)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_zero_output_layer_gives_the_warped_image():
    # With the last layer zeroed, r = 0 and e = 0: pred = the warped image,
    # and the loss is the hole pixels' squared error over 3 x holes plus the
    # squared per-pixel mean squared error over holes.
    params, rgb, z, hole, target = _problem(5)
    P = R.unpack(params)
    P["out"][0][...] = 0
    P["out"][1][...] = 0
    a = R.forward(params, rgb, z, hole)
    np.testing.assert_array_equal(a["pred"], rgb)
    loss, _ = R.loss_and_grad(params, rgb, z, hole, target)
    h = hole[:, None] > 0
    d2 = ((rgb - target) * h) ** 2
    want = np.sum(d2) / (3 * hole.sum()) + np.sum(np.mean(d2, axis=1) ** 2) / hole.sum()
    assert loss == pytest.approx(want, rel=1e-12)
    np.testing.assert_array_equal(a["e"], 0.0)


def test_input_channels():
    params, rgb, z, hole, target = _problem(6)
    x = R.net_input(rgb, z, hole)
    np.testing.assert_array_equal(x[:, 3], hole)
    assert np.all(x[:, 4][hole > 0] == 0) and np.all(x[:, :3][np.repeat(hole[:, None] > 0, 3, 1)] == 0)
    np.testing.assert_allclose(x[:, 4][hole == 0], 1.0 / z[hole == 0], rtol=1e-7)


def test_adam_first_step_closed_form():
    # After one step from m = v = 0 the bias-corrected ratio is g / (|g| + eps).
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p, m, v = R.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-8)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-6, 6, size=4000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 1.0 + 2 ** -9]]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(R.bf16(x), want)
    assert R.bf16(1.0 + 2 ** -8) == 1.0  # a tie goes to the even neighbour


def test_param_layout():
    n = R.num_params()
    assert n == sum(co * ci * 9 + co for _, ci, co, _ in R.LAYERS)
    v = np.arange(n, dtype=np.float64)
    np.testing.assert_array_equal(R.pack({k: v_ for k, v_ in R.unpack(v).items()}), v)
    assert R.unpack(v)["e1a"][0].shape == (16, 5, 3, 3) and R.unpack(v)["out"][1].shape == (4,)
