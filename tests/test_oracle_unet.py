"""Pins of the FP64 U-Net oracle: convolution by two formulations, the
backward pass against central finite differences of the loss (FP64 mode),
pooling routing, the transposed convolution's adjoint, bfloat16 rounding,
and the identity map at initialization."""
import numpy as np
import pytest

from oracle import unet as U


def _theta(seed=0, head_scale=0.3):
    th = U.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    p = U.unpack(th)
    p["head"][0][:] = rng.normal(0, head_scale, p["head"][0].shape)
    for name, (w, b) in p.items():
        b[:] = rng.normal(0, 0.05, b.shape)
    return U.pack({k: v for k, v in p.items()})


def test_param_count():
    # hand count: 320 + 9248 + 18496 + 36928 + 73856 + 147584 + 32832 + 73792
    #             + 36928 + 8224 + 18464 + 9248 + 33
    assert U.param_count() == 465_953


def test_conv_two_formulations_agree():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 6, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    np.testing.assert_allclose(U.conv3x3(x, w, b), U.conv3x3_direct(x, w, b), rtol=1e-12, atol=1e-12)


def test_conv_and_upconv_adjoints():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 6, 4, 3))
    w = rng.normal(size=(5, 3, 3, 3))
    gy = rng.normal(size=(2, 6, 4, 5))
    dx, _, _ = U.conv3x3_backward(x, w, gy)
    lhs = np.sum(U.conv3x3(x, w, np.zeros(5)) * gy)
    assert abs(lhs - np.sum(x * dx)) < 1e-10 * abs(lhs)
    wu = rng.normal(size=(2, 2, 5, 3))
    gu = rng.normal(size=(2, 12, 8, 5))
    dxu, _, _ = U.upconv2_backward(x, wu, gu)
    lhs = np.sum(U.upconv2(x, wu, np.zeros(5)) * gu)
    assert abs(lhs - np.sum(x * dxu)) < 1e-10 * abs(lhs)


def test_maxpool_backward_routes_to_first_max():
    x = np.zeros((1, 2, 2, 1))
    x[0, 0, 1, 0] = 2.0
    x[0, 1, 0, 0] = 2.0        # tie: the first in scan order wins
    dx = U.maxpool2_backward(x, np.ones((1, 1, 1, 1)))
    assert dx[0, 0, 1, 0] == 1.0 and dx.sum() == 1.0


def test_identity_at_initialization():
    th = U.init_params(3)
    x = np.random.default_rng(2).uniform(0, 0.02, (1, 16, 16))
    out, _ = U.forward(th, x)
    np.testing.assert_array_equal(out, x)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 1e-3])
    r = U.bf16_round(v)
    assert r[0] == 1.0 and r[1] == 1.0                       # ties to even
    assert r[2] == 1.0 + 2 ** -7
    assert abs(r[3] + 3.140625) < 1e-12
    assert abs(r[4] - 1e-3) / 1e-3 < 2 ** -8


def test_gradient_matches_finite_differences():
    th = _theta(5)
    rng = np.random.default_rng(7)
    x = rng.uniform(0.0, 1.0, (2, 8, 8))
    t = x + rng.normal(0, 0.1, x.shape)
    mask = np.ones((8, 8), dtype=bool)
    mask[0, :] = False
    loss, g, _ = U.loss_and_grad(th, x, t, mask, 3.0, in_scale=1.7)
    idx = rng.choice(len(th), 40, replace=False)
    # also every layer's first weight and bias
    o = 0
    for name, ws, bs in U.param_shapes():
        nw = int(np.prod(ws))
        idx = np.concatenate([idx, [o, o + nw]])
        o += nw + int(np.prod(bs))
    h = 1e-6
    for k in idx:
        tp = th.copy(); tp[k] += h
        tm = th.copy(); tm[k] -= h
        fd = (U.loss_and_grad(tp, x, t, mask, 3.0, in_scale=1.7)[0]
              - U.loss_and_grad(tm, x, t, mask, 3.0, in_scale=1.7)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-5 * max(1.0, abs(g[k])) + 1e-7, (k, fd, g[k])


def test_adam_step_reduces_loss():
    th = _theta(9)
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 1.0, (1, 8, 8))
    t = x + 0.05
    mask = np.ones((8, 8), dtype=bool)
    m = np.zeros_like(th); v = np.zeros_like(th)
    l0 = U.loss_and_grad(th, x, t, mask, 10.0)[0]
    for k in range(1, 31):
        _, g, _ = U.loss_and_grad(th, x, t, mask, 10.0)
        th, m, v = U.adam_step(th, g, m, v, k, 1e-3)
    assert U.loss_and_grad(th, x, t, mask, 10.0)[0] < 0.5 * l0


def test_warmstart_layer_table_matches_the_oracle():
    """The pipeline's parameter layout (init, FLOP count) agrees with the
    oracle network's: same layers, shapes and order; the initial network is
    the identity (zero head)."""
    from paper_1402_4381_amd import warmstart as W
    a = [(n, tuple(w), tuple(b)) for n, w, b in W.layer_shapes()]
    b = [(n, tuple(w), tuple(bb)) for n, w, bb in U.param_shapes()]
    assert a == b
    th = W.init_params(3)
    assert th.size == U.param_count()
    x = np.random.default_rng(0).uniform(0, 0.03, (1, 8, 8))
    out, _ = U.forward(th.astype(np.float64), x, in_scale=50.0)
    assert np.array_equal(out, x)
    # FLOPs: 2 x (weights of each layer) x (pixels at its resolution)
    H = W_ = 16
    res = dict(e1a=1, e1b=1, e2a=4, e2b=4, e3a=16, e3b=16, up2=4, d2a=4, d2b=4, up1=1, d1a=1, d1b=1,
               head=1)
    f = sum(2 * np.prod(ws) * H * W_ / res[n] / (4 if n.startswith("up") else 1)
            for n, ws, _ in U.param_shapes())
    assert W.forward_flops(H, W_) == pytest.approx(f)


def test_adam_closed_forms():
    """Adam (Kingma & Ba) with bias correction, from zero moments:
    * a constant gradient g gives the step lr g / (|g| + eps) at every t
      (the corrected moments are exactly g and g^2);
    * alternating +a, -a gives the second step lr (1 - b1)/(1 + b1) sign(a)
      (corrected first moment -(1 - b1) a / (1 + b1), second moment a^2)."""
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    g = np.array([0.3, -2.0, 1e-3, 5.0])
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 8):
        th_new, m, v = U.adam_step(th, g, m, v, t, lr, b1, b2, eps)
        np.testing.assert_allclose(th_new - th, -lr * g / (np.abs(g) + eps), rtol=1e-9, atol=0)
        th = th_new
    a = np.array([0.7, -0.2])
    th1, m, v = U.adam_step(np.zeros(2), a, np.zeros(2), np.zeros(2), 1, lr, b1, b2, eps)
    np.testing.assert_allclose(th1, -lr * a / (np.abs(a) + eps), rtol=1e-12)
    th2, m, v = U.adam_step(th1, -a, m, v, 2, lr, b1, b2, eps)
    np.testing.assert_allclose(th2 - th1, lr * (1 - b1) / (1 + b1) * a / (np.abs(a) + eps),
                               rtol=1e-6)
    # a step without the bias correction fails the first closed form
    m0 = (1 - b1) * g
    v0 = (1 - b2) * g * g
    uncorrected = -lr * m0 / (np.sqrt(v0) + eps)
    assert np.abs(uncorrected + lr * g / (np.abs(g) + eps)).max() > 0.5 * lr


def test_upconv_against_direct_scatter():
    """2x2 stride-2 transposed convolution by its scatter definition: input
    pixel (i, j) adds W[a, c] x[i, j] to output pixel (2i + a, 2j + c), plus
    the bias; the output windows do not overlap at stride 2."""
    rng = np.random.default_rng(4)
    x = rng.normal(size=(2, 3, 4, 3))
    w = rng.normal(size=(2, 2, 5, 3))
    b = rng.normal(size=5)
    ref = np.zeros((2, 6, 8, 5))
    for n in range(2):
        for i in range(3):
            for j in range(4):
                for a in range(2):
                    for c in range(2):
                        for o in range(5):
                            ref[n, 2 * i + a, 2 * j + c, o] += sum(w[a, c, o, ci] * x[n, i, j, ci]
                                                                  for ci in range(3))
    ref += b
    np.testing.assert_allclose(U.upconv2(x, w, b), ref, rtol=1e-12, atol=1e-12)
