"""GPU checks of the learned warm start on a held-out scan (the committed
network weights, the library's OS-LALM, the FP64 cost guard).

The gain is an empirical property of the trained network, not an identity:
the thresholds sit well inside what the evaluation over 20 held-out seeds
measured (network image about 3-6x closer to x* than the 2-iteration image
on seeds where the guard keeps it; after 2 + 10 iterations about 2x closer
than 12 plain iterations)."""
import numpy as np
import pytest

from _helpers import ensure_built, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def pipe():
    ensure_built()
    import synth
    from paper_1402_4381_amd import warmstart as WS
    return WS.Pipeline(synth.get_config("fan2d_512"))


def _scan(pipe, seed):
    d = pipe.synth.make_problem_data(pipe.cfg, seed)
    return pipe.problem(d["y"].astype(np.float32), d["w"].astype(np.float32))


def test_warm_start_gain_on_held_out_seed(pipe):
    from paper_1402_4381_amd import warmstart as WS
    ws = pipe.synth.configs.UNET_WARMSTART
    seed = ws["eval_seeds"][0] + 2
    say("warm start gain, seed", seed)
    prob = _scan(pipe, seed)
    params = torch.as_tensor(np.load(WS.WEIGHTS), device=DEV).contiguous()
    net = pipe.lalm.lalm_unet_create(1, pipe.H, pipe.W)
    st = pipe.zero_state()
    pipe.iterate(prob, st, ws["iters_in"])
    x_in = st.x.clone()
    pipe.iterate(prob, st, ws["iters_after"])
    x_plain = st.x.clone()
    xs, change = pipe.x_star(prob, x_plain, 1000)
    wst, kept, psi_in, psi_net, xt = pipe.warm_start(prob, params, net, ws["iters_in"])
    assert kept == (psi_net < psi_in)
    assert kept
    assert wst.step == 0                      # state reset: gradients recomputed at the new image
    assert float(xt.min().item()) >= 0.0      # non-negativity of the network image
    pipe.iterate(prob, wst, ws["iters_after"])
    r_in, r_net = pipe.rmsd_hu(x_in, xs), pipe.rmsd_hu(xt, xs)
    r_plain, r_warm = pipe.rmsd_hu(x_plain, xs), pipe.rmsd_hu(wst.x, xs)
    say("  x* change %.3f HU; RMSD x_in %.2f  net %.2f  plain %.2f  warm %.2f HU" %
        (change, r_in, r_net, r_plain, r_warm))
    assert r_net < 0.5 * r_in
    assert r_warm < 0.8 * r_plain


def test_cost_guard_rejects_a_bad_estimate(pipe):
    """A network whose output is off by a constant is rejected by the FP64
    cost, and the plain iteration state is kept (no reset)."""
    from paper_1402_4381_amd import warmstart as WS
    ws = pipe.synth.configs.UNET_WARMSTART
    prob = _scan(pipe, ws["eval_seeds"][0])
    th = WS.init_params(0)
    th[-1] = 5.0                              # head bias: +0.1 /mm everywhere
    params = torch.as_tensor(th, device=DEV)
    net = pipe.lalm.lalm_unet_create(1, pipe.H, pipe.W)
    wst, kept, psi_in, psi_net, xt = pipe.warm_start(prob, params, net, ws["iters_in"])
    say("  guard: psi_in %.6e psi_net %.6e kept %s" % (psi_in, psi_net, kept))
    assert not kept and psi_net > psi_in
    assert wst.step == ws["iters_in"] * pipe.M
    d = (xt - wst.x).abs()
    assert float(d.max().item()) > 0.05
