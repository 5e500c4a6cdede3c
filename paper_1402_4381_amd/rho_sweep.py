"""Fixed-rho sweep of OS-LALM against the continuation, on one GPU.

Sec. V compares OS-LALM with a fixed AL penalty rho in {1, 0.2, 0.1, 0.05}
(rho = 1 is the standard OS algorithm with the same majorizer) and with the
deterministic downward continuation, by the RMS difference over the ROI
between x^(k) and an almost converged x*, and reports acceleration of about
5, 10 and 20 times over rho = 1 for rho = 0.2, 0.1 and 0.05, and below 1 HU
within 30 iterations for the continuation.  This runs the same comparison on
the synthetic 2D fan-beam workload with the library's own kernels:

* x*: one-subset OS-LALM with continuation (convergent) run long; for a
  volume, OS-LALM with the workload's subsets, continuation and several
  inner FISTA iterations per step, run until its change over the last 10
  iterations is far below 1 HU (an M-subset limit point: on the helical
  volume it lies about 0.8 HU from the one-subset reference the benchmark
  builds, which matters only for differences near 1 HU);
* every method from x0 = 0 with the workload's subsets and bit-reversal
  order, RMSD to x* after every iteration;
* acceleration of rho over rho = 1 at a level R: iterations rho = 1 needs to
  reach R divided by the iterations rho needs (rho = 1 runs long enough to
  reach the levels that matter);
* the continuation with n = 2 and 5 inner FISTA iterations (Sec. IV-A: the
  paper finds the gain from n > 1 slight), and with the Barzilai-Borwein
  scaling of D_L (supplement: about 2x in early iterations), with the time
  per iteration.
"""
import argparse
import json
import os
import sys
import time

import numpy as np


def run(workload="fan2d_512", rhos=(1.0, 0.2, 0.1, 0.05), iters=60, iters_rho1=600, xstar_iters=6000,
        seed=None, inners=(2, 5), dev="cuda:0", xstar_inner=None, bb=True, beta_scale=1.0):
    import torch
    import synth
    from paper_1402_4381_amd import lalm
    cfg = synth.get_config(workload)
    M = cfg["M"]
    data = synth.make_problem_data(cfg, seed)
    geom = synth.geometry_of(cfg)
    beta, delta = cfg["beta"] * beta_scale, synth.configs.delta_mu(cfg)
    radius, hu = synth.roi_radius(cfg), synth.HU_PER_MU
    r64 = torch.zeros(1, dtype=torch.float64, device=dev)

    def problem(plan):
        vos = torch.as_tensor(plan.view_of_slot, dtype=torch.long, device=dev)
        y = torch.as_tensor(data["y"].astype(np.float32), device=dev).index_select(0, vos).reshape(-1).contiguous()
        w = torch.as_tensor(data["w"].astype(np.float32), device=dev).index_select(0, vos).reshape(-1).contiguous()
        d = torch.empty(plan.image_elems, device=dev)
        lalm.lalm_sqs_denom(plan, w, d)
        return y, w, d

    def rmsd(plan, a, b):
        lalm.lalm_roi_rmsd_f64(plan, a, b, radius, r64)
        return float(r64.item()) * hu

    plan = lalm.lalm_plan_geometry(geom, M)
    y, w, d = problem(plan)
    t0 = time.perf_counter()
    if xstar_inner is None:
        # x*: one subset, continuation
        p1 = lalm.lalm_plan_geometry(geom, 1)
        y1, w1, d1 = problem(p1)
        xs = lalm.LalmState.zeros_like(torch.zeros(p1.image_elems, device=dev))
        lalm.lalm_iterate(p1, y1, w1, d1, beta, delta, xs, xstar_iters - 100)
        prev = xs.x.clone()
        lalm.lalm_iterate(p1, y1, w1, d1, beta, delta, xs, 100)
        change = rmsd(p1, xs.x, prev)
        del p1, y1, w1, d1
        print("x*: %d one-subset iterations in %.1f s, last-100 change %.4f HU"
              % (xstar_iters, time.perf_counter() - t0, change), flush=True)
    else:
        # x*: M subsets, continuation, xstar_inner inner FISTA iterations
        xs = lalm.LalmState.zeros_like(torch.zeros(plan.image_elems, device=dev))
        for k in range(xstar_iters):
            if k == xstar_iters - 10:
                prev = xs.x.clone()
            lalm.lalm_iterate(plan, y, w, d, beta, delta, xs, M, n_inner=xstar_inner)
            if (k + 1) % 10 == 0:
                print("  x* iteration %d (%.1f s)" % (k + 1, time.perf_counter() - t0), flush=True)
        change = rmsd(plan, xs.x, prev)
        print("x*: %d iterations with n = %d in %.1f s, last-10 change %.4f HU"
              % (xstar_iters, xstar_inner, time.perf_counter() - t0, change), flush=True)
    curves = {}
    runs = [("continuation", True, 1.0, iters, 1, False)] + \
        ([("continuation bb", True, 1.0, iters, 1, True)] if bb else []) + \
        [("continuation n=%d" % ni, True, 1.0, iters, ni, False) for ni in inners] + \
        [("rho=%g" % r, False, r, iters_rho1 if r == 1.0 else iters, 1, False) for r in rhos]
    wall = {}
    for name, cont, rho, n, ni, bb in runs:
        st = lalm.LalmState.zeros_like(torch.zeros(plan.image_elems, device=dev), bb=bb)
        hist = []
        t_run = 0.0
        for _ in range(n):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            lalm.lalm_iterate(plan, y, w, d, beta, delta, st, M, continuation=cont, rho_fixed=rho, n_inner=ni,
                              bb=bb)
            t_run += time.perf_counter() - t1
            hist.append(round(rmsd(plan, st.x, xs.x), 4))
            if len(hist) % 25 == 0:
                print("  %s: %d iterations, %.2f HU" % (name, len(hist), hist[-1]), flush=True)
        curves[name] = hist
        wall[name] = round(t_run / n * 1e3, 3)
        print("%-13s RMSD after 10/30/%d iterations: %.2f / %.2f / %.2f HU"
              % (name, n, hist[9], hist[29], hist[-1]), flush=True)

    def first_below(h, level):
        return next((k + 1 for k, v in enumerate(h) if v <= level), None)

    levels = [50.0, 20.0, 10.0, 5.0, 2.0, 1.0]
    accel = {}
    for r in rhos:
        if r == 1.0:
            continue
        row = {}
        for L in levels:
            k1, kr = first_below(curves["rho=1"], L), first_below(curves["rho=%g" % r], L)
            row["%g" % L] = None if (k1 is None or kr is None) else round(k1 / kr, 2)
        accel["rho=%g" % r] = row
    iters_to = {name: {"%g" % L: first_below(h, L) for L in levels} for name, h in curves.items()}
    return dict(workload=workload, M=M, beta=beta, beta_scale=beta_scale, xstar_iters=xstar_iters,
                xstar_inner=xstar_inner,
                xstar_last100_change_hu=round(change, 5) if xstar_inner is None else None,
                xstar_last10_change_hu=round(change, 5) if xstar_inner is not None else None,
                iterations_to_level=iters_to, acceleration_over_rho1=accel,
                rmsd_hu_at_30={k: v[29] for k, v in curves.items()}, ms_per_iteration=wall, curves=curves)


def main(argv=None):
    ap = argparse.ArgumentParser(description="fixed-rho sweep of OS-LALM against the continuation")
    ap.add_argument("--workload", default="fan2d_512")
    ap.add_argument("--iters", type=int, default=60)
    ap.add_argument("--iters-rho1", type=int, default=600)
    ap.add_argument("--xstar-iters", type=int, default=6000)
    ap.add_argument("--xstar-inner", type=int, default=None,
                    help="x* from M-subset OS-LALM with this many inner FISTA iterations (volumes)")
    ap.add_argument("--inners", default="2,5", help="inner FISTA counts of the extra continuation runs")
    ap.add_argument("--no-bb", action="store_true")
    ap.add_argument("--beta-scale", type=float, default=1.0, help="factor on the workload's beta")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    inners = tuple(int(v) for v in args.inners.split(",") if v)
    res = run(args.workload, iters=args.iters, iters_rho1=args.iters_rho1, xstar_iters=args.xstar_iters,
              inners=inners, xstar_inner=args.xstar_inner, bb=not args.no_bb, beta_scale=args.beta_scale)
    print(json.dumps({k: v for k, v in res.items() if k != "curves"}), flush=True)
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
