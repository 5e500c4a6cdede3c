"""GPU parity of the warm-start U-Net (BF16 MFMA kernels through the C ABI)
against the FP64 oracle evaluated with the same bfloat16 storage points.

Tolerances: the kernels accumulate in FP32, the oracle in FP64; both round
every stored tensor to bfloat16, so an element whose FP32 and FP64 values
straddle a bfloat16 rounding boundary differs by one bfloat16 step (2^-8
relative).  Such flips are rare (~FP32 error / bf16 step ~ 1e-3 of the
elements) and propagate through at most 26 layers of the forward and
backward passes, hence: network correction (output - input) relative L2
<= 1e-2; loss relative 1e-3; per-layer gradients relative L2 <= 2e-2
(the first layers see the most propagated flips); Adam step 1e-6.
"""
import numpy as np
import pytest

from _helpers import ensure_built, rel_l2, say

from oracle import unet as U

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def L():
    ensure_built()
    from paper_1402_4381_amd import lalm
    return lalm


def _theta(seed):
    th = U.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    p = U.unpack(th)
    p["head"][0][:] = rng.normal(0, 0.3, p["head"][0].shape)
    for _, (w, b) in p.items():
        b[:] = rng.normal(0, 0.05, b.shape)
    return U.pack(p)


def g32(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV).to(dtype).contiguous()


@pytest.mark.parametrize("B,H,W", [(2, 16, 16), (1, 32, 24), (3, 8, 12)])
def test_forward_parity(L, B, H, W):
    say("unet forward", B, H, W)
    th = _theta(1)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.0, 1.0, (B, H, W))
    x = 0.02 * x
    ref, _ = U.forward(th, x, bf16=True, in_scale=50.0)
    net = L.lalm_unet_create(4, H, W)
    out = torch.empty(B * H * W, device=DEV)
    L.lalm_unet_forward(net, g32(th), g32(x).reshape(-1), out, B, in_scale=50.0)
    got = out.cpu().numpy().reshape(B, H, W).astype(np.float64)
    e = rel_l2(got - x, ref - x)
    say("  correction rel L2 %.2e" % e)
    assert e <= 1e-2


@pytest.mark.parametrize("B,H,W", [(2, 16, 16), (1, 32, 24)])
def test_loss_gradient_parity(L, B, H, W):
    say("unet grad", B, H, W)
    th = _theta(3)
    rng = np.random.default_rng(4)
    x = rng.uniform(0.0, 1.0, (B, H, W))
    t = x + rng.normal(0, 0.1, x.shape)
    mask = np.ones((H, W), dtype=bool)
    mask[:2, :] = False
    loss, g, _ = U.loss_and_grad(th, x, t, mask, 5.0, bf16=True, in_scale=2.0)
    net = L.lalm_unet_create(B, H, W)
    P = L.lalm_unet_param_count()
    grad = torch.zeros(P, device=DEV)
    lg = torch.zeros(1, dtype=torch.float64, device=DEV)
    L.lalm_unet_loss_grad(net, g32(th), g32(x).reshape(-1), g32(t).reshape(-1),
                          g32(mask.astype(np.uint8), torch.uint8).reshape(-1), 5.0, B, grad, lg, in_scale=2.0)
    gl = float(lg.item())
    gg = grad.cpu().numpy().astype(np.float64)
    say("  loss gpu %.8e oracle %.8e" % (gl, loss))
    assert abs(gl - loss) <= 1e-3 * abs(loss)
    o = 0
    for name, ws, bs in U.param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        ew = rel_l2(gg[o:o + nw], g[o:o + nw])
        eb = rel_l2(gg[o + nw:o + nw + nb], g[o + nw:o + nw + nb])
        say("  %-4s dW rel %.2e  db rel %.2e" % (name, ew, eb))
        assert ew <= 2e-2 and eb <= 2e-2
        o += nw + nb
    # deterministic
    grad2 = torch.zeros(P, device=DEV)
    L.lalm_unet_loss_grad(net, g32(th), g32(x).reshape(-1), g32(t).reshape(-1),
                          g32(mask.astype(np.uint8), torch.uint8).reshape(-1), 5.0, B, grad2, lg, in_scale=2.0)
    assert torch.equal(grad, grad2)


def test_adam_and_training_decreases_loss(L):
    th = U.init_params(11)
    P = L.lalm_unet_param_count()
    rng = np.random.default_rng(5)
    g = rng.normal(0, 1e-3, P)
    m = rng.normal(0, 1e-4, P)
    v = rng.uniform(0, 1e-6, P)
    ref, rm, rv = U.adam_step(th, g, m, v, 3, 1e-3)
    net = L.lalm_unet_create(2, 16, 16)
    pt, mt, vt = g32(th), g32(m), g32(v)
    L.lalm_unet_adam(net, pt, g32(g), mt, vt, 3, 1e-3)
    assert np.abs(pt.cpu().numpy() - ref).max() <= 1e-6 * max(1.0, np.abs(ref).max())
    # a few steps on a fixed batch lower the loss
    x = rng.uniform(0, 1, (2, 16, 16))
    t = x + 0.05 * np.sin(np.arange(16))[None, None, :]
    mask = g32(np.ones((16, 16), np.uint8), torch.uint8).reshape(-1)
    params = g32(U.init_params(12))
    m = torch.zeros(P, device=DEV)
    v = torch.zeros(P, device=DEV)
    grad = torch.zeros(P, device=DEV)
    lg = torch.zeros(1, dtype=torch.float64, device=DEV)
    xs, ts = g32(x).reshape(-1), g32(t).reshape(-1)
    losses = []
    for k in range(1, 41):
        L.lalm_unet_loss_grad(net, params, xs, ts, mask, 10.0, 2, grad, lg)
        losses.append(float(lg.item()))
        L.lalm_unet_adam(net, params, grad, m, v, k, 1e-3)
    say("  training losses", losses[0], losses[-1])
    assert losses[-1] < 0.5 * losses[0]
