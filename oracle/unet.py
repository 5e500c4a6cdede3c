"""FP64 oracle of the learned warm-start network -- TEST INFRASTRUCTURE ONLY.

The warm start is not in the paper: it is a small 2D U-Net that maps an image
after a few OS-LALM iterations to the image after many iterations; plain
OS-LALM stays the fallback and the arbiter (by its cost value and by the RMS
difference to x*).  Architecture (3 levels, 3x3 convolutions, ReLU):

    e1a 1->32, e1b 32->32  | pool 2x2 | e2a 32->64, e2b 64->64 | pool 2x2 |
    e3a 64->128, e3b 128->128 | up2 (2x2 stride-2 transposed conv) 128->64,
    concat [up2, e2b] -> d2a 128->64, d2b 64->64 | up1 64->32, concat
    [up1, e1b] -> d1a 64->32, d1b 32->32 | head 1x1 32->1;
    output = x + head(...)   (residual)

Tensors are NHWC ``[B, H, W, C]``; 3x3 weights ``[Cout, 3, 3, Cin]`` with
zero padding 1; transposed-conv weights ``[2, 2, Cout, Cin]`` (output pixel
(2y+a, 2x+b) takes ``W[a, b] @ in[y, x]``); head ``[Cin]``.  Loss: mean over
the batch's ROI pixels of (HU scale x (output - target))^2.

``bf16=True`` rounds, like the GPU kernels' storage, the weights, the input
and every stored activation and gradient tensor to bfloat16 (round to nearest
even) while accumulating in FP64; ``bf16=False`` is plain FP64 (used for the
finite-difference checks).
"""
import numpy as np

LAYERS = [
    # name, kind, cin, cout
    ("e1a", "conv", 1, 32), ("e1b", "conv", 32, 32),
    ("e2a", "conv", 32, 64), ("e2b", "conv", 64, 64),
    ("e3a", "conv", 64, 128), ("e3b", "conv", 128, 128),
    ("up2", "up", 128, 64),
    ("d2a", "conv", 128, 64), ("d2b", "conv", 64, 64),
    ("up1", "up", 64, 32),
    ("d1a", "conv", 64, 32), ("d1b", "conv", 32, 32),
    ("head", "head", 32, 1),
]


def param_shapes():
    """Ordered (name, weight shape, bias shape) of the flat parameter vector:
    for every layer its weights then its biases."""
    out = []
    for name, kind, cin, cout in LAYERS:
        if kind == "conv":
            out.append((name, (cout, 3, 3, cin), (cout,)))
        elif kind == "up":
            out.append((name, (2, 2, cout, cin), (cout,)))
        else:
            out.append((name, (cin,), (1,)))
    return out


def param_count():
    return sum(int(np.prod(w)) + int(np.prod(b)) for _, w, b in param_shapes())


def unpack(theta):
    p, o = {}, 0
    for name, ws, bs in param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        p[name] = (theta[o:o + nw].reshape(ws), theta[o + nw:o + nw + nb].reshape(bs))
        o += nw + nb
    return p


def pack(grads):
    return np.concatenate([np.concatenate([grads[n][0].ravel(), grads[n][1].ravel()])
                           for n, _, _ in param_shapes()])


def init_params(seed):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; the head starts
    at zero so the initial network is the identity map."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, ws, bs in param_shapes():
        if name == "head":
            w = np.zeros(ws)
        else:
            fan_in = ws[-1] * (9 if len(ws) == 4 and ws[1] == 3 else 1)
            w = rng.normal(0.0, np.sqrt(2.0 / fan_in), ws)
        parts += [w.ravel(), np.zeros(int(np.prod(bs)))]
    return np.concatenate(parts)


def bf16_round(a):
    """Round to bfloat16 (nearest, ties to even) and back to float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ------------------------------------------------------------------ layers

def conv3x3(x, w, b):
    """Zero-padded 3x3 convolution (cross-correlation): y[p] = sum over taps
    (dy, dx) in {-1,0,1}^2 of W[:, dy+1, dx+1, :] @ x[p + (dy, dx)] + b."""
    B, H, W, C = x.shape
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((B, H, W, w.shape[0]))
    for ty in range(3):
        for tx in range(3):
            y += xp[:, ty:ty + H, tx:tx + W] @ w[:, ty, tx, :].T
    return y + b


def conv3x3_direct(x, w, b):
    """The same convolution by explicit loops (small inputs only)."""
    B, H, W, C = x.shape
    y = np.zeros((B, H, W, w.shape[0]))
    for n in range(B):
        for i in range(H):
            for j in range(W):
                acc = b.copy()
                for ty in range(3):
                    for tx in range(3):
                        ii, jj = i + ty - 1, j + tx - 1
                        if 0 <= ii < H and 0 <= jj < W:
                            acc = acc + w[:, ty, tx, :] @ x[n, ii, jj]
                y[n, i, j] = acc
    return y


def conv3x3_backward(x, w, dy):
    """Gradients of conv3x3 w.r.t. its input, weights and bias."""
    B, H, W, C = x.shape
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ty in range(3):
        for tx in range(3):
            dxp[:, ty:ty + H, tx:tx + W] += dy @ w[:, ty, tx, :]
            dw[:, ty, tx, :] = np.einsum("bhwo,bhwc->oc", dy, xp[:, ty:ty + H, tx:tx + W])
    return dxp[:, 1:-1, 1:-1], dw, dy.sum(axis=(0, 1, 2))


def maxpool2(x):
    B, H, W, C = x.shape
    v = x.reshape(B, H // 2, 2, W // 2, 2, C)
    return v.max(axis=(2, 4))


def maxpool2_backward(x, dy):
    """Route each output gradient to the first maximum of its 2x2 window in
    the order (0,0), (0,1), (1,0), (1,1)."""
    B, H, W, C = x.shape
    dx = np.zeros_like(x)
    v = x.reshape(B, H // 2, 2, W // 2, 2, C)
    m = v.max(axis=(2, 4))
    taken = np.zeros(m.shape, dtype=bool)
    for a in range(2):
        for c in range(2):
            hit = (v[:, :, a, :, c, :] == m) & ~taken
            dx[:, a::2, c::2, :] = np.where(hit, dy, 0.0)
            taken |= hit
    return dx


def upconv2(x, w, b):
    """2x2 stride-2 transposed convolution."""
    B, H, W, C = x.shape
    y = np.zeros((B, 2 * H, 2 * W, w.shape[2]))
    for a in range(2):
        for c in range(2):
            y[:, a::2, c::2, :] = x @ w[a, c].T + b
    return y


def upconv2_backward(x, w, dy):
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for a in range(2):
        for c in range(2):
            g = dy[:, a::2, c::2, :]
            dx += g @ w[a, c]
            dw[a, c] = np.einsum("bhwo,bhwc->oc", g, x)
    return dx, dw, dy.sum(axis=(0, 1, 2))


# ----------------------------------------------------------------- network

def forward(theta, x, bf16=False, in_scale=1.0):
    """x: [B, H, W] images; the network sees in_scale * x and the output is
    x + head / in_scale.  Returns (output [B, H, W], cache)."""
    r = bf16_round if bf16 else (lambda a: a)
    P = {k: (r(w), b) for k, (w, b) in unpack(theta).items()}
    a = {"x": r(in_scale * x[..., None])}
    relu = lambda z: np.maximum(z, 0.0)
    a["e1a"] = r(relu(conv3x3(a["x"], *P["e1a"])))
    a["e1b"] = r(relu(conv3x3(a["e1a"], *P["e1b"])))
    a["p1"] = maxpool2(a["e1b"])
    a["e2a"] = r(relu(conv3x3(a["p1"], *P["e2a"])))
    a["e2b"] = r(relu(conv3x3(a["e2a"], *P["e2b"])))
    a["p2"] = maxpool2(a["e2b"])
    a["e3a"] = r(relu(conv3x3(a["p2"], *P["e3a"])))
    a["e3b"] = r(relu(conv3x3(a["e3a"], *P["e3b"])))
    a["up2"] = r(upconv2(a["e3b"], *P["up2"]))
    a["c2"] = np.concatenate([a["up2"], a["e2b"]], axis=-1)
    a["d2a"] = r(relu(conv3x3(a["c2"], *P["d2a"])))
    a["d2b"] = r(relu(conv3x3(a["d2a"], *P["d2b"])))
    a["up1"] = r(upconv2(a["d2b"], *P["up1"]))
    a["c1"] = np.concatenate([a["up1"], a["e1b"]], axis=-1)
    a["d1a"] = r(relu(conv3x3(a["c1"], *P["d1a"])))
    a["d1b"] = r(relu(conv3x3(a["d1a"], *P["d1b"])))
    hw, hb = P["head"]
    out = x + (a["d1b"] @ hw + hb[0]) / in_scale
    return out, (P, a)


def loss_and_grad(theta, x, target, mask, hu_scale, bf16=False, in_scale=1.0):
    """Loss = mean over mask pixels of (hu_scale (out - target))^2, and its
    gradient w.r.t. theta (flat)."""
    r = bf16_round if bf16 else (lambda a: a)
    out, (P, a) = forward(theta, x, bf16, in_scale)
    m = np.broadcast_to(mask, out.shape).astype(np.float64)
    n = m.sum()
    e = (out - target) * m
    loss = float(np.sum((hu_scale * e) ** 2) / n)
    dout = 2.0 * hu_scale ** 2 * e / n / in_scale            # d loss / d head output
    G = {}
    hw, hb = P["head"]
    G["head"] = (np.einsum("bhwc,bhw->c", a["d1b"], dout), np.array([dout.sum()]))
    dA = r(dout[..., None] * hw)                              # d/d d1b
    relu_mask = lambda act, g: r(g * (act > 0))

    def conv_back(name, xin, act, dact):
        dz = relu_mask(act, dact)
        dx, dw, db = conv3x3_backward(xin, P[name][0], dz)
        G[name] = (dw, db)
        return dx

    d = conv_back("d1b", a["d1a"], a["d1b"], dA)
    d = conv_back("d1a", a["c1"], a["d1a"], r(d))
    # the transposed conv's output gradient is stored in bfloat16; the skip
    # part stays at full precision until the pooling path's gradient is added
    d_up1, d_e1b_skip = r(d[..., :32]), d[..., 32:]
    dx_, dw_, db_ = upconv2_backward(a["d2b"], P["up1"][0], d_up1)
    G["up1"] = (dw_, db_)
    d = conv_back("d2b", a["d2a"], a["d2b"], r(dx_))
    d = conv_back("d2a", a["c2"], a["d2a"], r(d))
    d_up2, d_e2b_skip = r(d[..., :64]), d[..., 64:]
    dx_, dw_, db_ = upconv2_backward(a["e3b"], P["up2"][0], d_up2)
    G["up2"] = (dw_, db_)
    d = conv_back("e3b", a["e3a"], a["e3b"], r(dx_))
    d = conv_back("e3a", a["p2"], a["e3a"], r(d))
    d_e2b = r(maxpool2_backward(a["e2b"], d) + d_e2b_skip)
    d = conv_back("e2b", a["e2a"], a["e2b"], d_e2b)
    d = conv_back("e2a", a["p1"], a["e2a"], r(d))
    d_e1b = r(maxpool2_backward(a["e1b"], d) + d_e1b_skip)
    d = conv_back("e1b", a["e1a"], a["e1b"], d_e1b)
    dz = relu_mask(a["e1a"], r(d))
    _, dw, db = conv3x3_backward(a["x"], P["e1a"][0], dz)
    G["e1a"] = (dw, db)
    return loss, pack(G), out


def adam_step(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba) with bias correction; returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
