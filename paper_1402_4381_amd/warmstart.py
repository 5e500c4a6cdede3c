"""Learned warm start for 2D fan-beam OS-LALM (not part of the paper's method).

A small U-Net (the BF16-MFMA kernels of the library) maps the image after
two OS-LALM iterations to an estimate of the image after fifty.  Everything
runs through the library's C ABI on one GPU:

* pairs: for each training seed a synthetic scan (seeded phantom, Poisson
  counts) is reconstructed by the library's own OS-LALM (continuation rho,
  bit-reversal subset order, x0 = 0); the image after 2 iterations is the
  input and the one after 50 the target.  Sinograms are synthesised by CPU
  worker processes while the GPU iterates.
* training: mean squared error in HU over the reconstruction ROI, Adam with
  FP32 master weights, cosine learning-rate decay.
* evaluation on held-out seeds: 2 iterations -> U-Net -> cost guard (the
  estimate is kept only if its FP64 cost Psi is below that of the 2-iteration
  image) -> state reset (the aggregate gradients are recomputed at the new
  image, the continuation counter starts again) -> 10 iterations, against
  30 plain iterations; RMS difference to x* (one-subset OS-LALM with
  continuation run to convergence) over the ROI and wall time to 1 HU.

Plain OS-LALM stays the fallback and the arbiter: the network only proposes a
starting image and the method's own cost decides whether it is used.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(_HERE, "weights", "unet_fan2d_512.npy")

# Layer table of the network (order, shapes as the C ABI documents them).
LAYERS = (("e1a", "c3", 1, 32), ("e1b", "c3", 32, 32), ("e2a", "c3", 32, 64), ("e2b", "c3", 64, 64),
          ("e3a", "c3", 64, 128), ("e3b", "c3", 128, 128), ("up2", "up", 128, 64),
          ("d2a", "c3", 128, 64), ("d2b", "c3", 64, 64), ("up1", "up", 64, 32),
          ("d1a", "c3", 64, 32), ("d1b", "c3", 32, 32), ("head", "h", 32, 1))
# spatial scale of each layer's output (1 = full resolution)
_LEVEL = dict(e1a=1, e1b=1, e2a=4, e2b=4, e3a=16, e3b=16, up2=4, d2a=4, d2b=4, up1=1, d1a=1, d1b=1, head=1)


def layer_shapes():
    out = []
    for name, kind, cin, cout in LAYERS:
        if kind == "c3":
            out.append((name, (cout, 3, 3, cin), (cout,)))
        elif kind == "up":
            out.append((name, (2, 2, cout, cin), (cout,)))
        else:
            out.append((name, (cin,), (1,)))
    return out


def init_params(seed=0):
    """He-normal weights, zero biases, zero head (the network starts as the
    identity map)."""
    rng = np.random.default_rng(seed)
    parts = []
    for (name, kind, cin, cout), (_, ws, bs) in zip(LAYERS, layer_shapes()):
        fan_in = 9 * cin if kind == "c3" else cin
        w = np.zeros(ws) if kind == "h" else rng.normal(0.0, math.sqrt(2.0 / fan_in), ws)
        parts += [w.ravel(), np.zeros(int(np.prod(bs)))]
    return np.concatenate(parts).astype(np.float32)


def forward_flops(H, W):
    """Multiply-adds x 2 of one forward pass over an H x W image."""
    macs = 0.0
    for name, kind, cin, cout in LAYERS:
        px = H * W / _LEVEL[name]
        macs += px * cout * cin * (9 if kind == "c3" else 1)
    return 2.0 * macs


# ------------------------------------------------------------------ inputs

_WORKER = {}


def _worker_init(cfg):
    _WORKER["cfg"] = cfg


def _worker_sino(seed):
    """Natural-order float32 (y, w) of one synthetic scan (CPU worker)."""
    import synth
    d = synth.make_problem_data(_WORKER["cfg"], seed, workers=1)
    return seed, d["y"].astype(np.float32), d["w"].astype(np.float32)


class Problem:
    """One scan resident on the GPU: subset-major y, w and the SQS denominator."""

    def __init__(self, lalm, torch, plan, y_nat, w_nat, dev):
        vos = torch.as_tensor(plan.view_of_slot, dtype=torch.long, device=dev)
        yd = torch.as_tensor(y_nat, device=dev)
        wd = torch.as_tensor(w_nat, device=dev)
        self.y = yd.index_select(0, vos).reshape(-1).contiguous()
        self.w = wd.index_select(0, vos).reshape(-1).contiguous()
        self.denom = torch.empty(plan.image_elems, device=dev)
        lalm.lalm_sqs_denom(plan, self.w, self.denom)


class Pipeline:
    def __init__(self, cfg, dev="cuda:0", n_inner=1):
        import torch
        import synth
        from paper_1402_4381_amd import lalm
        self.torch, self.synth, self.lalm = torch, synth, lalm
        self.cfg, self.dev = cfg, dev
        self.M = cfg["M"]
        # inner FISTA iterations per subset step of every OS-LALM run of the
        # pipeline (pairs, plain and warm-started evaluation runs); x* always
        # uses the one-subset method with n = 1
        self.n_inner = int(n_inner)
        self.plan = lalm.lalm_plan_geometry(synth.geometry_of(cfg), self.M)
        self.beta = cfg["beta"]
        self.delta = synth.configs.delta_mu(cfg)
        self.H, self.W = cfg["ny"], cfg["nx"]
        self.in_scale = 1.0 / synth.MU_WATER
        self.hu = synth.HU_PER_MU
        self.radius = synth.roi_radius(cfg)
        self.mask = torch.as_tensor(synth.roi_mask(cfg)[0].astype(np.uint8).reshape(-1), device=dev)
        self._r = torch.zeros(1, dtype=torch.float64, device=dev)
        self._c = torch.zeros(3, dtype=torch.float64, device=dev)

    # -------------------------------------------------------------- helpers
    def zero_state(self):
        return self.lalm.LalmState.zeros_like(self.torch.zeros(self.plan.image_elems, device=self.dev))

    def iterate(self, prob, state, n_iters):
        self.lalm.lalm_iterate(self.plan, prob.y, prob.w, prob.denom, self.beta, self.delta, state,
                               n_iters * self.M, n_inner=self.n_inner)

    def rmsd_hu(self, a, b):
        self.lalm.lalm_roi_rmsd_f64(self.plan, a, b, self.radius, self._r)
        return float(self._r.item()) * self.hu

    def cost(self, prob, x):
        self.lalm.lalm_cost_f64(self.plan, prob.y, prob.w, self.beta, self.delta, x, self._c)
        return float(self._c[0].item())

    def problem(self, y_nat, w_nat):
        return Problem(self.lalm, self.torch, self.plan, y_nat, w_nat, self.dev)

    # ---------------------------------------------------------------- pairs
    def generate_pairs(self, seeds, iters_in, iters_target, pool, batch=16):
        """Training pairs (x after iters_in iterations, x after iters_target)
        for the seeds, ``batch`` scans reconstructed together by one batched
        plan (every kernel launch covers the batch's images)."""
        torch, lalm = self.torch, self.lalm
        n = len(seeds)
        npix = self.H * self.W
        X = torch.empty(n, npix, device=self.dev)
        T = torch.empty(n, npix, device=self.dev)
        plan = lalm.lalm_plan_geometry(self.synth.geometry_of(self.cfg), self.M, batch=batch)
        vos = torch.as_tensor(plan.view_of_slot, dtype=torch.long, device=self.dev)
        sino = plan.sino_elems
        Y = torch.zeros(batch, sino, device=self.dev)
        Wt = torch.zeros(batch, sino, device=self.dev)
        D = torch.empty(batch * npix, device=self.dev)
        t0 = time.perf_counter()
        gpu_s = 0.0
        it = pool.imap(_worker_sino, seeds, chunksize=1)
        for k0 in range(0, n, batch):
            nb = min(batch, n - k0)
            for b in range(nb):
                _, y, w = next(it)
                Y[b].copy_(torch.as_tensor(y, device=self.dev).index_select(0, vos).reshape(-1))
                Wt[b].copy_(torch.as_tensor(w, device=self.dev).index_select(0, vos).reshape(-1))
            # a short last batch repeats its first scan in the unused images
            for b in range(nb, batch):
                Y[b].copy_(Y[0])
                Wt[b].copy_(Wt[0])
            g0 = time.perf_counter()
            lalm.lalm_sqs_denom(plan, Wt, D)
            st = lalm.LalmState.zeros_like(torch.zeros(batch * npix, device=self.dev), batch=batch)
            lalm.lalm_iterate(plan, Y, Wt, D, self.beta, self.delta, st, iters_in * self.M, n_inner=self.n_inner)
            X[k0:k0 + nb].copy_(st.x.view(batch, npix)[:nb])
            lalm.lalm_iterate(plan, Y, Wt, D, self.beta, self.delta, st, (iters_target - iters_in) * self.M,
                              n_inner=self.n_inner)
            T[k0:k0 + nb].copy_(st.x.view(batch, npix)[:nb])
            torch.cuda.synchronize()
            gpu_s += time.perf_counter() - g0
            if (k0 // batch + 1) % max(1, n // batch // 20) == 0 or k0 + nb == n:
                print("pairs %d/%d  %.1f s (GPU %.1f s)" % (k0 + nb, n, time.perf_counter() - t0, gpu_s),
                      flush=True)
        return X, T, dict(n=n, batch=batch, wall_s=round(time.perf_counter() - t0, 2), gpu_s=round(gpu_s, 2))

    # ------------------------------------------------------------- training
    def train(self, X, T, epochs, batch, lr, seed=0, params=None, log_every=50):
        torch, lalm = self.torch, self.lalm
        n = X.shape[0]
        P = lalm.lalm_unet_param_count()
        net = lalm.lalm_unet_create(batch, self.H, self.W)
        p = torch.as_tensor(init_params(seed) if params is None else params, device=self.dev).contiguous()
        m = torch.zeros(P, device=self.dev)
        v = torch.zeros(P, device=self.dev)
        grad = torch.zeros(P, device=self.dev)
        loss = torch.zeros(1, dtype=torch.float64, device=self.dev)
        xb = torch.empty(batch, self.H * self.W, device=self.dev)
        tb = torch.empty(batch, self.H * self.W, device=self.dev)
        steps_per_epoch = n // batch
        total = max(1, epochs * steps_per_epoch)
        rng = np.random.default_rng(seed)
        hist, k = [], 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(n), dtype=torch.long, device=self.dev)
            acc, cnt = torch.zeros(1, dtype=torch.float64, device=self.dev), 0
            for s in range(steps_per_epoch):
                idx = perm[s * batch:(s + 1) * batch]
                torch.index_select(X, 0, idx, out=xb)
                torch.index_select(T, 0, idx, out=tb)
                lalm.lalm_unet_loss_grad(net, p, xb, tb, self.mask, self.hu, batch, grad, loss,
                                         in_scale=self.in_scale)
                k += 1
                lr_k = lr * 0.5 * (1.0 + math.cos(math.pi * (k - 1) / total))
                lalm.lalm_unet_adam(net, p, grad, m, v, k, lr_k)
                acc += loss
                cnt += 1
                if k % log_every == 0:
                    print("train step %d/%d  epoch %d  loss(HU^2) %.3f  %.1f s" %
                          (k, total, ep, float(loss.item()), time.perf_counter() - t0), flush=True)
            ep_loss = float(acc.item()) / max(cnt, 1)
            hist.append(round(ep_loss, 4))
            print("epoch %d  mean loss(HU^2) %.4f  (RMS %.3f HU)  %.1f s" %
                  (ep, ep_loss, math.sqrt(ep_loss), time.perf_counter() - t0), flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        info = dict(epochs=epochs, batch=batch, lr=lr, steps=k, wall_s=round(wall, 2),
                    ms_per_step=round(1e3 * wall / max(k, 1), 3), epoch_loss_hu2=hist,
                    train_tflops=round(3.0 * forward_flops(self.H, self.W) * batch * k / wall / 1e12, 1))
        return p, info

    # ----------------------------------------------------------- inference
    def unet_time(self, params, batch=1, reps=20):
        torch, lalm = self.torch, self.lalm
        net = lalm.lalm_unet_create(batch, self.H, self.W)
        x = torch.rand(batch * self.H * self.W, device=self.dev) * 0.02
        out = torch.empty_like(x)
        for _ in range(3):
            lalm.lalm_unet_forward(net, params, x, out, batch, self.in_scale, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            lalm.lalm_unet_forward(net, params, x, out, batch, self.in_scale, True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        fl = forward_flops(self.H, self.W) * batch
        return dict(batch=batch, ms=round(dt * 1e3, 4), gflop=round(fl / 1e9, 2),
                    tflops=round(fl / dt / 1e12, 1), frac_bf16_peak=round(fl / dt / 2.5e15, 4))

    def train_step_time(self, params, batch=8, reps=20):
        """Wall time of one training step (loss, gradient, Adam) on a
        synthetic batch, and its rate at 3x the forward FLOPs."""
        torch, lalm = self.torch, self.lalm
        net = lalm.lalm_unet_create(batch, self.H, self.W)
        P = lalm.lalm_unet_param_count()
        p = params.clone()
        m, v, grad = (torch.zeros(P, device=self.dev) for _ in range(3))
        loss = torch.zeros(1, dtype=torch.float64, device=self.dev)
        x = torch.rand(batch * self.H * self.W, device=self.dev) * 0.02
        t = x + 1e-4 * torch.rand_like(x)
        for k in range(3):
            lalm.lalm_unet_loss_grad(net, p, x, t, self.mask, self.hu, batch, grad, loss, in_scale=self.in_scale)
            lalm.lalm_unet_adam(net, p, grad, m, v, k + 1, 1e-4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(reps):
            lalm.lalm_unet_loss_grad(net, p, x, t, self.mask, self.hu, batch, grad, loss, in_scale=self.in_scale)
            lalm.lalm_unet_adam(net, p, grad, m, v, k + 4, 1e-4)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        fl = 3.0 * forward_flops(self.H, self.W) * batch
        return dict(batch=batch, ms=round(dt * 1e3, 4), tflops=round(fl / dt / 1e12, 1),
                    frac_bf16_peak=round(fl / dt / 2.5e15, 4))

    def warm_start(self, prob, params, net, iters_in, out=None):
        """iters_in plain iterations, U-Net, cost guard, state reset.
        Returns (state, kept, psi_in, psi_net, network image)."""
        torch, lalm = self.torch, self.lalm
        st = self.zero_state()
        self.iterate(prob, st, iters_in)
        xt = torch.empty_like(st.x) if out is None else out
        lalm.lalm_unet_forward(net, params, st.x, xt, 1, self.in_scale, True)
        psi_in = self.cost(prob, st.x)
        psi_net = self.cost(prob, xt)
        if psi_net < psi_in:
            # step 0: the next call recomputes the gradients at xt (state reset)
            st = self.lalm.LalmState(xt.clone(), torch.zeros_like(xt), torch.zeros_like(xt))
            return st, True, psi_in, psi_net, xt
        return st, False, psi_in, psi_net, xt

    def x_star(self, prob, x_init, iters):
        """One-subset OS-LALM with continuation from x_init, run to
        convergence; returns x* and its change over the last 100 iterations."""
        torch, lalm, synth = self.torch, self.lalm, self.synth
        if not hasattr(self, "_p1"):
            self._p1 = lalm.lalm_plan_geometry(synth.geometry_of(self.cfg), 1)
        p1 = self._p1
        # the one-subset plan keeps the natural view order
        vo = torch.as_tensor(np.argsort(self.plan.view_of_slot), dtype=torch.long, device=self.dev)
        nr_nb = self.cfg["n_rows"] * self.cfg["n_bins"]
        sel = torch.as_tensor(p1.view_of_slot, dtype=torch.long, device=self.dev)
        y1 = prob.y.reshape(-1, nr_nb).index_select(0, vo).index_select(0, sel).reshape(-1).contiguous()
        w1 = prob.w.reshape(-1, nr_nb).index_select(0, vo).index_select(0, sel).reshape(-1).contiguous()
        d1 = torch.empty(p1.image_elems, device=self.dev)
        lalm.lalm_sqs_denom(p1, w1, d1)
        st = lalm.LalmState(x_init.clone(), torch.zeros_like(x_init), torch.zeros_like(x_init))
        lalm.lalm_iterate(p1, y1, w1, d1, self.beta, self.delta, st, max(iters - 100, 1))
        prev = st.x.clone()
        lalm.lalm_iterate(p1, y1, w1, d1, self.beta, self.delta, st, 100)
        return st.x, self.rmsd_hu(st.x, prev)

    def evaluate_seed(self, seed, params, net, ws, xstar_iters, max_iters, timing=True):
        """Held-out comparison on one seed: plain OS-LALM and the warm start,
        each run up to max_iters iterations in all; RMS difference to x*
        (ROI, HU) after every iteration, costs, iterations and wall time to
        1 HU."""
        synth = self.synth
        d = synth.make_problem_data(self.cfg, seed)
        prob = self.problem(d["y"].astype(np.float32), d["w"].astype(np.float32))
        it_in, it_after, it_plain = ws["iters_in"], ws["iters_after"], ws["iters_plain"]
        # plain OS-LALM from x0 = 0, one image per iteration
        st = self.zero_state()
        plain, psi_plain = [], None
        for k in range(max_iters):
            self.iterate(prob, st, 1)
            plain.append(st.x.clone())
            if k + 1 == it_plain:
                psi_plain = self.cost(prob, st.x)
        xs, xs_change = self.x_star(prob, st.x, xstar_iters)
        psi_star = self.cost(prob, xs)
        plain_hu = [self.rmsd_hu(x, xs) for x in plain]
        del plain
        # warm start, then plain iterations from the network's image
        wst, kept, psi_in, psi_net, xt = self.warm_start(prob, params, net, it_in)
        x_net_hu = self.rmsd_hu(xt, xs)
        warm_hu, psi_warm = [], None
        for k in range(max_iters - it_in):
            self.iterate(prob, wst, 1)
            warm_hu.append(self.rmsd_hu(wst.x, xs))
            if k + 1 == it_after:
                psi_warm = self.cost(prob, wst.x)
        rel = lambda v: (v - psi_star) / abs(psi_star)
        res = dict(seed=seed, kept=kept, xstar_last100_change_hu=round(xs_change, 5),
                   rmsd_hu_after_in=round(plain_hu[it_in - 1], 3), rmsd_hu_unet=round(x_net_hu, 3),
                   rmsd_hu_warm=[round(v, 3) for v in warm_hu],       # after it_in + 1, it_in + 2, ...
                   rmsd_hu_plain=[round(v, 3) for v in plain_hu],     # after 1, 2, ...
                   psi_rel={"in": rel(psi_in), "unet": rel(psi_net), "warm_%d" % (it_in + it_after): rel(psi_warm),
                            "plain_%d" % it_plain: rel(psi_plain)})
        k_plain = next((i + 1 for i, v in enumerate(plain_hu) if v < 1.0), None)
        k_warm = next((i + 1 for i, v in enumerate(warm_hu) if v < 1.0), None)
        res["iters_to_1hu_plain"] = k_plain
        res["iters_to_1hu_warm"] = None if k_warm is None else it_in + k_warm
        if timing:
            res["wall_s_to_1hu_plain"] = self._time_plain(prob, k_plain) if k_plain else None
            res["wall_s_to_1hu_warm"] = (self._time_warm(prob, params, net, it_in, k_warm, kept)
                                         if k_warm else None)
        return res

    def _time_plain(self, prob, k):
        torch = self.torch
        st = self.zero_state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.iterate(prob, st, k)
        torch.cuda.synchronize()
        return round(time.perf_counter() - t0, 5)

    def _time_warm(self, prob, params, net, it_in, k, kept_expected):
        torch = self.torch
        out = torch.empty(self.plan.image_elems, device=self.dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, kept, _, _, _ = self.warm_start(prob, params, net, it_in, out=out)
        self.iterate(prob, st, k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return round(dt, 5) if kept == kept_expected else None


def _summary(rows, ws):
    """Medians over the evaluated seeds."""
    it_in, it_after, it_plain = ws["iters_in"], ws["iters_after"], ws["iters_plain"]
    med = lambda v: None if not v else float(np.median(v))
    def at(r, key, k):                 # RMSD after k iterations in all
        if key == "rmsd_hu_plain":
            return r[key][k - 1]
        return r["rmsd_hu_unet"] if k == it_in else r[key][k - it_in - 1]
    k_a = it_in + it_after
    out = dict(n_seeds=len(rows), kept=sum(r["kept"] for r in rows),
               median_rmsd_hu_after_in=med([r["rmsd_hu_after_in"] for r in rows]),
               median_rmsd_hu_unet=med([r["rmsd_hu_unet"] for r in rows]))
    for k in sorted({k_a, it_plain, 2 * it_plain}):
        if k <= len(rows[0]["rmsd_hu_plain"]):
            out["median_rmsd_hu_at_%d" % k] = dict(plain=med([at(r, "rmsd_hu_plain", k) for r in rows]),
                                                   warm=med([at(r, "rmsd_hu_warm", k) for r in rows]))
    out["warm_%d_beats_plain_%d" % (k_a, it_plain)] = sum(
        at(r, "rmsd_hu_warm", k_a) < at(r, "rmsd_hu_plain", it_plain) for r in rows)
    for key in ("iters_to_1hu_plain", "iters_to_1hu_warm", "wall_s_to_1hu_plain", "wall_s_to_1hu_warm"):
        v = [r.get(key) for r in rows]
        out["median_" + key] = med([x for x in v if x is not None])
        out["reached_" + key] = sum(x is not None for x in v)
    sp = [r["wall_s_to_1hu_plain"] / r["wall_s_to_1hu_warm"] for r in rows
          if r.get("wall_s_to_1hu_plain") and r.get("wall_s_to_1hu_warm")]
    out["median_speedup_to_1hu"] = med(sp)
    return out


def run_volume(name, weights, iters_in=2, iters_ref=150, inner_ref=10, max_iters=150, inners=(5, 10, 16),
               batch=8, dev="cuda:0"):
    """Run to 1 HU on a 3D workload, with the per-slice warm start.

    The reference is OS-LALM with continuation and inner_ref inner FISTA
    iterations (Sec. IV-A) run for iters_ref iterations, an M-subset limit
    point (on the helical volume about 0.8 HU from the one-subset reference
    that eval_volume and the benchmark build); the inner iterations cost
    little here beside the projections while they speed up the regularizer
    part of each step, which dominates the denominator of a 26-neighbour 3D
    regularizer.  From x0 = 0 every method below runs until
    its ROI RMS difference to the reference is at most 1 HU (or max_iters):
    plain OS-LALM (n = 1), the same with n in `inners`, and the warm start
    (iters_in plain iterations, the network trained on 2D slices applied to
    every axial slice, the FP64 cost guard of the whole volume, the state
    reset).  A rejected network image leaves the state of the plain run
    after iters_in iterations, so the warm path then is the plain run plus
    the network and guard time."""
    import torch
    import synth
    from paper_1402_4381_amd import lalm
    cfg = synth.get_config(name)
    M = cfg["M"]
    nz, ny, nx = cfg["nz"], cfg["ny"], cfg["nx"]
    t0 = time.perf_counter()
    data = synth.make_problem_data(cfg)
    t_data = time.perf_counter() - t0
    print("volume %s: inputs in %.1f s" % (name, t_data), flush=True)
    plan = lalm.lalm_plan_geometry(synth.geometry_of(cfg), M)
    vos = torch.as_tensor(plan.view_of_slot, dtype=torch.long, device=dev)
    y = torch.as_tensor(data["y"].astype(np.float32), device=dev).index_select(0, vos).reshape(-1).contiguous()
    w = torch.as_tensor(data["w"].astype(np.float32), device=dev).index_select(0, vos).reshape(-1).contiguous()
    del data
    denom = torch.empty(plan.image_elems, device=dev)
    lalm.lalm_sqs_denom(plan, w, denom)
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    radius, hu, in_scale = synth.roi_radius(cfg), synth.HU_PER_MU, 1.0 / synth.MU_WATER
    r64 = torch.zeros(1, dtype=torch.float64, device=dev)
    c64 = torch.zeros(3, dtype=torch.float64, device=dev)

    def step(state, n, n_inner=1):
        torch.cuda.synchronize()
        t = time.perf_counter()
        lalm.lalm_iterate(plan, y, w, denom, beta, delta, state, n * M, n_inner=n_inner)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    def rmsd(a, b):
        lalm.lalm_roi_rmsd_f64(plan, a, b, radius, r64)
        return float(r64.item()) * hu

    def cost(x):
        lalm.lalm_cost_f64(plan, y, w, beta, delta, x, c64)
        return float(c64[0].item())

    zero = lambda: lalm.LalmState.zeros_like(torch.zeros(plan.image_elems, device=dev))
    # reference
    st = zero()
    t_ref = []
    for k in range(iters_ref):
        t_ref.append(step(st, 1, inner_ref))
        if k + 1 == iters_ref - 10:
            x_prev10 = st.x.clone()
        if (k + 1) % 10 == 0:
            print("  reference (n = %d) iteration %d  (%.3f s per iteration)" % (inner_ref, k + 1, t_ref[-1]),
                  flush=True)
    x_ref = st.x
    ref_change = rmsd(x_ref, x_prev10)
    del x_prev10
    print("  reference change over its last 10 iterations: %.4f HU" % ref_change, flush=True)

    def to_1hu(label, n_inner, state=None, k0=0):
        st = zero() if state is None else state
        hist, times = [], []
        for k in range(k0, max_iters):
            times.append(step(st, 1, n_inner))
            hist.append(rmsd(st.x, x_ref))
            if (k + 1) % 10 == 0 or hist[-1] <= 1.0:
                print("  %s iteration %d: %.3f HU  (%.3f s per iteration)" % (label, k + 1, hist[-1], times[-1]),
                      flush=True)
            if hist[-1] <= 1.0:
                break
        return hist, times, st

    curves = {}
    plain_hist, plain_t, _ = to_1hu("plain n=1", 1)
    curves["n=1"] = (plain_hist, plain_t)
    for ni in inners:
        h, t, _ = to_1hu("n=%d" % ni, ni)
        curves["n=%d" % ni] = (h, t)
    # warm start
    params = torch.as_tensor(np.load(weights), device=dev).contiguous()
    net = lalm.lalm_unet_create(batch, ny, nx)
    st2 = zero()
    t_in = step(st2, iters_in)
    x_in = st2.x.clone()
    xt = torch.empty_like(x_in)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hw = ny * nx
    for z0 in range(0, nz, batch):
        b = min(batch, nz - z0)
        lalm.lalm_unet_forward(net, params, x_in[z0 * hw:(z0 + b) * hw], xt[z0 * hw:(z0 + b) * hw], b,
                               in_scale, True)
    torch.cuda.synchronize()
    t_net = time.perf_counter() - t1
    t1 = time.perf_counter()
    psi_in, psi_net = cost(x_in), cost(xt)
    t_guard = time.perf_counter() - t1
    kept = psi_net < psi_in
    print("  network on %d slices: %.3f s; guard %.3f s; Psi %.6e -> %.6e, kept %s"
          % (nz, t_net, t_guard, psi_in, psi_net, kept), flush=True)
    rmsd_in, rmsd_net = rmsd(x_in, x_ref), rmsd(xt, x_ref)
    if kept:
        st2 = lalm.LalmState(xt.clone(), torch.zeros_like(xt), torch.zeros_like(xt))
        wh, wt, _ = to_1hu("warm", 1, st2, iters_in)
        warm_hist = plain_hist[:iters_in] + wh
        warm_s = [t_in + t_net + t_guard + sum(wt[:k + 1]) for k in range(len(wt))]
    else:
        warm_hist = plain_hist
        warm_s = [t_in + t_net + t_guard + sum(plain_t[iters_in:k + 1]) for k in range(iters_in, len(plain_t))]
    del st2, xt, x_in

    def reached(h, times):
        k = next((i for i, e in enumerate(h) if e <= 1.0), None)
        return (None, None) if k is None else (k + 1, round(sum(times[:k + 1]), 3))

    res = dict(workload=name, M=M, iters_in=iters_in, iters_ref=iters_ref, inner_ref=inner_ref,
               max_iters=max_iters, kept=kept, inputs_s=round(t_data, 1),
               s_per_iteration_ref=round(float(np.median(t_ref)), 4),
               unet_s=round(t_net, 4), unet_slices=nz, guard_s=round(t_guard, 4), psi_in=psi_in, psi_net=psi_net,
               ref_last10_change_hu=round(ref_change, 4),
               rmsd_hu_in=round(rmsd_in, 3), rmsd_hu_unet=round(rmsd_net, 3), methods={})
    for key, (h, t) in curves.items():
        it, sec = reached(h, t)
        res["methods"][key] = dict(iters_to_1hu=it, wall_s_to_1hu=sec, s_per_iteration=round(float(np.median(t)), 4),
                                   rmsd_hu_at_30=round(h[29], 3) if len(h) >= 30 else None,
                                   rmsd_hu=[round(v, 3) for v in h])
    kw = next((i for i, e in enumerate(warm_hist) if e <= 1.0 and i >= iters_in), None)
    res["methods"]["warm"] = dict(iters_to_1hu=None if kw is None else kw + 1,
                                  wall_s_to_1hu=None if kw is None else round(warm_s[kw - iters_in], 3),
                                  rmsd_hu=[round(v, 3) for v in warm_hist])
    return res


def _volume_inputs(lalm, torch, synth, cfg, plan, seed, dev):
    """Subset-major device sinogram y, weights w and D_L of one synthetic
    scan of a 3D workload (seed None: the workload's own scan), and the
    host data (for plans with another subset count)."""
    data = synth.make_problem_data(cfg, seed)
    vos = torch.as_tensor(plan.view_of_slot, dtype=torch.long, device=dev)
    y = torch.as_tensor(data["y"].astype(np.float32), device=dev).index_select(0, vos).reshape(-1).contiguous()
    w = torch.as_tensor(data["w"].astype(np.float32), device=dev).index_select(0, vos).reshape(-1).contiguous()
    denom = torch.empty(plan.image_elems, device=dev)
    lalm.lalm_sqs_denom(plan, w, denom)
    return data, y, w, denom


def train_volume(name, seeds, weights_out, iters_in=2, iters_target=30, n_inner=16, epochs=10, batch=8, lr=1e-3,
                 dev="cuda:0"):
    """Train the warm-start network on the axial slices of 3D scans.

    For every seed a synthetic scan of the workload (its geometry, noise and
    beta, another phantom) is reconstructed by OS-LALM with continuation and
    n_inner inner FISTA iterations; the pairs are the slices after iters_in
    iterations and after iters_target iterations (with n_inner = 16 the
    latter lie within about 1 HU of x*).  The network, loss and optimizer
    are the 2D pipeline's (512^2 slices, ROI mask, HU loss, Adam)."""
    import torch
    import synth
    from paper_1402_4381_amd import lalm
    cfg = synth.get_config(name)
    if cfg["kind"] == 0:
        raise SystemExit("train_volume is for the 3D workloads")
    M = cfg["M"]
    nz, ny, nx = cfg["nz"], cfg["ny"], cfg["nx"]
    plan = lalm.lalm_plan_geometry(synth.geometry_of(cfg), M)
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    X = torch.empty(len(seeds) * nz, ny * nx, device=dev)
    T = torch.empty(len(seeds) * nz, ny * nx, device=dev)
    t0 = time.perf_counter()
    gpu_s = 0.0
    for i, seed in enumerate(seeds):
        _, y, w, denom = _volume_inputs(lalm, torch, synth, cfg, plan, seed, dev)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        st = lalm.LalmState.zeros_like(torch.zeros(plan.image_elems, device=dev))
        lalm.lalm_iterate(plan, y, w, denom, beta, delta, st, iters_in * M, n_inner=n_inner)
        X[i * nz:(i + 1) * nz].copy_(st.x.view(nz, ny * nx))
        lalm.lalm_iterate(plan, y, w, denom, beta, delta, st, (iters_target - iters_in) * M, n_inner=n_inner)
        T[i * nz:(i + 1) * nz].copy_(st.x.view(nz, ny * nx))
        torch.cuda.synchronize()
        gpu_s += time.perf_counter() - g0
        print("volume pairs %d/%d (seed %d): %.1f s (GPU %.1f s)" % (i + 1, len(seeds), seed,
                                                                    time.perf_counter() - t0, gpu_s), flush=True)
        del y, w, denom, st
    torch.cuda.empty_cache()
    # 512^2 slices on the same in-plane grid and field of view as the 2D workload
    pipe = Pipeline(synth.get_config("fan2d_512"), dev=dev)
    params, tinfo = pipe.train(X, T, epochs, batch, lr)
    os.makedirs(os.path.dirname(os.path.abspath(weights_out)), exist_ok=True)
    np.save(weights_out, params.cpu().numpy())
    print("weights written to", weights_out, flush=True)
    return dict(workload=name, seeds=[int(v) for v in seeds], slices=int(X.shape[0]), iters_in=iters_in,
                iters_target=iters_target, n_inner=n_inner, pairs_wall_s=round(time.perf_counter() - t0, 1),
                pairs_gpu_s=round(gpu_s, 1), train=tinfo)


def eval_volume(name, weights, n_inner=16, iters_in=2, max_iters=60, warm_iters=20, polish_tol_hu=0.005,
                polish_budget_s=240.0, batch=8, dev="cuda:0"):
    """Run to 1 HU on the workload's own 3D scan (held out from training),
    plain against warm-started, both with n_inner inner FISTA iterations.

    x* is built as the benchmark builds it (Sec. V measures against a
    converged one-subset reference): OS-LALM-M-c-n for warm_iters
    iterations, then the one-subset method from that image until its change
    over 10 iterations is below polish_tol_hu (or the time budget).  The warm
    start: iters_in iterations, the network on every axial slice, the FP64
    cost guard of the whole volume, the state reset, then iterations."""
    import torch
    import synth
    from paper_1402_4381_amd import lalm
    cfg = synth.get_config(name)
    M = cfg["M"]
    nz, ny, nx = cfg["nz"], cfg["ny"], cfg["nx"]
    plan = lalm.lalm_plan_geometry(synth.geometry_of(cfg), M)
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    radius, hu, in_scale = synth.roi_radius(cfg), synth.HU_PER_MU, 1.0 / synth.MU_WATER
    t0 = time.perf_counter()
    data, y, w, denom = _volume_inputs(lalm, torch, synth, cfg, plan, None, dev)
    print("eval volume %s: inputs in %.1f s" % (name, time.perf_counter() - t0), flush=True)
    r64 = torch.zeros(1, dtype=torch.float64, device=dev)
    c64 = torch.zeros(3, dtype=torch.float64, device=dev)

    def rmsd(a, b):
        lalm.lalm_roi_rmsd_f64(plan, a, b, radius, r64)
        return float(r64.item()) * hu

    def cost(x):
        lalm.lalm_cost_f64(plan, y, w, beta, delta, x, c64)
        return float(c64[0].item())

    def timed(f):
        torch.cuda.synchronize()
        t = time.perf_counter()
        f()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    zero = lambda: lalm.LalmState.zeros_like(torch.zeros(plan.image_elems, device=dev))
    # x*
    st = zero()
    timed(lambda: lalm.lalm_iterate(plan, y, w, denom, beta, delta, st, warm_iters * M, n_inner=n_inner))
    p1 = lalm.lalm_plan_geometry(synth.geometry_of(cfg), 1)
    vos = torch.as_tensor(p1.view_of_slot, dtype=torch.long, device=dev)
    y1 = torch.as_tensor(data["y"].astype(np.float32), device=dev).index_select(0, vos).reshape(-1).contiguous()
    w1 = torch.as_tensor(data["w"].astype(np.float32), device=dev).index_select(0, vos).reshape(-1).contiguous()
    del data
    xs = zero()
    xs.x.copy_(st.x)
    del st
    prev = xs.x.clone()
    k, t_pol, change = 0, 0.0, None
    while t_pol < polish_budget_s:
        t_pol += timed(lambda: lalm.lalm_iterate(p1, y1, w1, denom, beta, delta, xs, 10, n_inner=n_inner))
        k += 10
        change = rmsd(xs.x, prev)
        prev.copy_(xs.x)
        print("  x* one-subset iteration %d: change over 10 iterations %.4f HU (%.1f s)" % (k, change, t_pol),
              flush=True)
        if change < polish_tol_hu:
            break
    x_star = xs.x
    del y1, w1, p1, prev
    torch.cuda.empty_cache()

    def to_1hu(label, st, k0):
        hist, times = [], []
        for k in range(k0, max_iters):
            times.append(timed(lambda: lalm.lalm_iterate(plan, y, w, denom, beta, delta, st, M, n_inner=n_inner)))
            hist.append(round(rmsd(st.x, x_star), 3))
            if (k + 1) % 5 == 0 or hist[-1] <= 1.0:
                print("  %s iteration %d: %.3f HU" % (label, k + 1, hist[-1]), flush=True)
            if hist[-1] <= 1.0:
                break
        return hist, times

    plain_hist, plain_t = to_1hu("plain", zero(), 0)
    # warm start
    params = torch.as_tensor(np.load(weights), device=dev).contiguous()
    net = lalm.lalm_unet_create(batch, ny, nx)
    st2 = zero()
    t_in = timed(lambda: lalm.lalm_iterate(plan, y, w, denom, beta, delta, st2, iters_in * M, n_inner=n_inner))
    x_in = st2.x.clone()
    xt = torch.empty_like(x_in)
    hw = ny * nx

    def network():
        for z0 in range(0, nz, batch):
            b = min(batch, nz - z0)
            lalm.lalm_unet_forward(net, params, x_in[z0 * hw:(z0 + b) * hw], xt[z0 * hw:(z0 + b) * hw], b,
                                   in_scale, True)

    t_net = timed(network)
    t1 = time.perf_counter()
    psi_in, psi_net = cost(x_in), cost(xt)
    t_guard = time.perf_counter() - t1
    kept = psi_net < psi_in
    rmsd_in, rmsd_net = rmsd(x_in, x_star), rmsd(xt, x_star)
    print("  warm: %d iterations %.2f HU; network on %d slices %.3f s -> %.2f HU; guard %.3f s, Psi %.6e -> %.6e, "
          "kept %s" % (iters_in, rmsd_in, nz, t_net, rmsd_net, t_guard, psi_in, psi_net, kept), flush=True)
    if kept:
        st2 = lalm.LalmState(xt.clone(), torch.zeros_like(xt), torch.zeros_like(xt))
    del xt, x_in
    wh, wt = to_1hu("warm", st2, iters_in)
    warm_hist = wh
    lalm.lalm_unet_destroy(net)

    def reached(hist, times, k0, extra):
        i = next((j for j, e in enumerate(hist) if e <= 1.0), None)
        return (None, None) if i is None else (k0 + i + 1, round(extra + sum(times[:i + 1]), 3))

    ip, sp = reached(plain_hist, plain_t, 0, 0.0)
    iw, sw = reached(warm_hist, wt, iters_in, t_in + t_net + t_guard)
    return dict(workload=name, M=M, n_inner=n_inner, iters_in=iters_in, max_iters=max_iters,
                xstar=("OS-LALM-%d-c-%d for %d iterations, then one-subset OS-LALM-1-c-%d for %d iterations "
                       "(last change over 10 iterations %.4f HU)" % (M, n_inner, warm_iters, n_inner, k, change)),
                kept=bool(kept), psi_in=psi_in, psi_net=psi_net, rmsd_hu_in=round(rmsd_in, 3),
                rmsd_hu_unet=round(rmsd_net, 3), unet_s=round(t_net, 4), guard_s=round(t_guard, 4),
                plain=dict(iters_to_1hu=ip, wall_s_to_1hu=sp, rmsd_hu=plain_hist,
                           s_per_iteration=round(float(np.median(plain_t)), 4)),
                warm=dict(iters_to_1hu=iw, wall_s_to_1hu=sw, rmsd_hu_after_in=warm_hist))


def main(argv=None):
    ap = argparse.ArgumentParser(description="U-Net warm start for OS-LALM: pairs, training, evaluation")
    ap.add_argument("--workload", default="fan2d_512")
    ap.add_argument("--pairs", type=int, default=4000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--eval-seeds", type=int, default=20)
    ap.add_argument("--xstar-iters", type=int, default=6000)
    ap.add_argument("--max-iters", type=int, default=150, help="iterations per method in the evaluation")
    ap.add_argument("--workers", type=int, default=14)
    ap.add_argument("--weights", default=WEIGHTS, help="weights file to write (train) or read (eval only)")
    ap.add_argument("--eval-only", action="store_true")
    ap.add_argument("--pair-batch", type=int, default=16, help="scans reconstructed together for the pairs")
    ap.add_argument("--n-inner", type=int, default=1,
                    help="inner FISTA iterations per subset step of the plain and warm-started runs")
    ap.add_argument("--volume", default=None,
                    help="3D workload: per-slice warm start with the committed weights (no training)")
    ap.add_argument("--volume-train", type=int, default=0, metavar="K",
                    help="with --volume: train on the slices of K synthetic scans of that workload, write --weights, "
                         "then run to 1 HU on the workload's own scan with those weights")
    ap.add_argument("--volume-eval", action="store_true",
                    help="with --volume: run to 1 HU on the workload's own scan with --weights, plain against "
                         "warm-started, both with --n-inner")
    ap.add_argument("--out", default=None, help="JSON summary path")
    ap.add_argument("--iters-target", type=int, default=None,
                    help="iterations behind a training target (default: the warm-start settings' value)")
    ap.add_argument("--pairs-only", action="store_true",
                    help="only generate the training pairs and report their timing")
    ap.add_argument("--unet-timing", action="store_true",
                    help="only time the network: forward at batch 1 and 8, a training step at batch 8")
    args = ap.parse_args(argv)

    import multiprocessing as mp
    import synth
    if args.volume and (args.volume_train or args.volume_eval):
        res = {}
        if args.volume_train:
            seeds = list(range(310000, 310000 + args.volume_train))
            res["train"] = train_volume(args.volume, seeds, args.weights, n_inner=args.n_inner,
                                        iters_target=args.iters_target or 30, epochs=args.epochs)
        res["eval"] = eval_volume(args.volume, args.weights, n_inner=args.n_inner, max_iters=args.max_iters)
        ev = res["eval"]
        print(json.dumps({k: v for k, v in ev.items() if k not in ("plain", "warm")}), flush=True)
        print(json.dumps({k: {a: b for a, b in ev[k].items() if a not in ("rmsd_hu", "rmsd_hu_after_in")}
                          for k in ("plain", "warm")}), flush=True)
        if args.out:
            os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
            with open(args.out, "w") as f:
                json.dump(res, f, indent=1)
        return res
    if args.volume:
        res = run_volume(args.volume, args.weights)
        print(json.dumps({k: v for k, v in res.items() if k != "methods"}), flush=True)
        print(json.dumps({k: {a: b for a, b in v.items() if a != "rmsd_hu"} for k, v in res["methods"].items()}),
              flush=True)
        if args.out:
            os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
            with open(args.out, "w") as f:
                json.dump(res, f, indent=1)
        return res
    cfg = synth.get_config(args.workload)
    if cfg["kind"] != 0:
        raise SystemExit("the warm start is 2D (one network per slice image)")
    ws = dict(synth.configs.UNET_WARMSTART)
    if args.iters_target is not None:
        ws["iters_target"] = args.iters_target
    pool = None
    if not args.eval_only and not args.unet_timing:
        # CPU workers are forked before the GPU is touched
        pool = mp.get_context("fork").Pool(args.workers, initializer=_worker_init, initargs=(cfg,))

    pipe = Pipeline(cfg, n_inner=args.n_inner)
    torch = pipe.torch
    if args.unet_timing:
        params = torch.as_tensor(np.load(args.weights), device=pipe.dev).contiguous()
        res = dict(forward=[pipe.unet_time(params, b) for b in (1, 8)], train=pipe.train_step_time(params, 8))
        print(json.dumps(res), flush=True)
        return res
    report = dict(workload=args.workload, warmstart=ws, n_inner=args.n_inner)
    if args.eval_only:
        params = torch.as_tensor(np.load(args.weights), device=pipe.dev).contiguous()
    else:
        lo, hi = ws["train_seeds"]
        seeds = list(range(lo, min(hi, lo + args.pairs)))
        X, T, info = pipe.generate_pairs(seeds, ws["iters_in"], ws["iters_target"], pool, batch=args.pair_batch)
        pool.close()
        pool.join()
        report["pairs"] = info
        if args.pairs_only:
            print(json.dumps(report), flush=True)
            return report
        params, tinfo = pipe.train(X, T, args.epochs, args.batch, args.lr)
        report["train"] = tinfo
        del X, T
        os.makedirs(os.path.dirname(os.path.abspath(args.weights)), exist_ok=True)
        np.save(args.weights, params.cpu().numpy())
        print("weights written to", args.weights, flush=True)
    report["unet_forward"] = [pipe.unet_time(params, b) for b in (1, 8)]
    print("unet forward", report["unet_forward"], flush=True)
    net = pipe.lalm.lalm_unet_create(1, pipe.H, pipe.W)
    lo, hi = ws["eval_seeds"]
    rows = []
    for seed in range(lo, min(hi, lo + args.eval_seeds)):
        r = pipe.evaluate_seed(seed, params, net, ws, args.xstar_iters, args.max_iters)
        rows.append(r)
        print("eval seed %d kept %s  x%d %.2f HU  unet %.2f HU  warm(%d+%d) %.2f HU  plain(%d) %.2f HU  "
              "to 1 HU: plain %s it %s s, warm %s it %s s  (x* last-100 change %.3f HU)" %
              (seed, r["kept"], ws["iters_in"], r["rmsd_hu_after_in"], r["rmsd_hu_unet"], ws["iters_in"],
               ws["iters_after"], r["rmsd_hu_warm"][ws["iters_after"] - 1], ws["iters_plain"],
               r["rmsd_hu_plain"][ws["iters_plain"] - 1], r["iters_to_1hu_plain"], r.get("wall_s_to_1hu_plain"),
               r["iters_to_1hu_warm"], r.get("wall_s_to_1hu_warm"), r["xstar_last100_change_hu"]), flush=True)
    report["eval"] = rows
    report["eval_settings"] = dict(xstar_iters=args.xstar_iters, max_iters=args.max_iters)
    report["summary"] = _summary(rows, ws)
    print(json.dumps(report["summary"]), flush=True)
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        with open(args.out, "w") as f:
            json.dump(report, f, indent=1)
    return report


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(_HERE))
    main()
