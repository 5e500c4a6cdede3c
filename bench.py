#!/usr/bin/env python3
"""OS-LALM benchmark on one MI355X.

One step = one OS-LALM subset iteration of the whole hot path: x-update
(regularizer majorizer, continuation rho), forward projection of the next
subset with fused weighted residual, matched back-projection with the fused
g-update, regularizer gradient and FP64 restart indicator, and the
continuation decision.  In 2D the back-projection epilogue and the next
x-update are one kernel (it computes the next x for both values the pending
decision can give rho; the forward projection takes the decision and reads
the chosen one).  The workload is the 512^2 fan-beam problem
(984 views x 888 bins, M = 24 subsets, 40-ellipse seeded phantom, Poisson
counts at I0 = 5e4); all inputs are resident in GPU memory before timing.

Printed: one JSON line with the throughput (subset iterations / s), the
roofline figure of the dominant kernel (algorithmic bytes / measured kernel
time against the 8 TB/s HBM peak) and the FP64 CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources of each kernel class (2D: the update class is the fused step kernel)
_CSRC = "paper_1402_4381_amd/csrc/"
KERNEL_SOURCES = {"project": [_CSRC + "project.hip", _CSRC + "lalm_internal.h"],
                  "backproject": [_CSRC + "backproject.hip", _CSRC + "lalm_internal.h"],
                  "update": [_CSRC + "backproject.hip", _CSRC + "project.hip", _CSRC + "lalm_internal.h"]}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(rels):
    h = hashlib.sha256()
    for rel in rels:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, or None
    when none exists or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256_16") != source_hash(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(cfg, data, beta, delta, budget_s):
    """The FP64 oracle's OS-LALM timed on a bounded number of subset steps
    (its D_L is computed once beforehand, outside the timing, as the GPU's is)."""
    import oracle as ora
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    DL = ora.sqs_denom(cfg, data["w"])
    t0 = time.perf_counter()
    ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=cfg["M"], n_steps=3, denom=DL)
    per = (time.perf_counter() - t0) / 3.0
    n = max(3, int(budget_s / max(per, 1e-4)))
    t0 = time.perf_counter()
    ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=cfg["M"], n_steps=n, denom=DL)
    dt = time.perf_counter() - t0
    return dict(value=round(n / dt, 3), unit="subset_iters/s", cores=threads, kind="oracle",
                sample="%d OS-LALM subset steps of %s (M=%d, from x0 = 0, incl. the initial "
                       "subset gradient) with the FP64 oracle: %.1f s" % (n, cfg["name"], cfg["M"], dt))


def oracle_timing(cfg, data, beta, delta, reps=5):
    """The FP64 oracle's pieces on one workload, medians of ``reps`` warm runs
    with the threads the OpenMP runtime gives it (OMP_NUM_THREADS): one
    subset's forward projection and back-projection, and one OS-LALM subset
    step (a call of two steps minus a call of one, so the initial subset
    gradient cancels); a full iteration is M such steps."""
    import statistics
    import numpy as np
    import oracle as ora
    M = cfg["M"]
    views = ora.subset_views(cfg["n_views"], M)[ora.bit_reversal_order(M)[1]]
    x = np.random.default_rng(0).uniform(0.0, 0.02, ora.image_shape(cfg))
    DL = ora.sqs_denom(cfg, data["w"])

    def med(f):
        f()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            f()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts)

    t_fp = med(lambda: ora.forward(cfg, x, views))
    r = ora.forward(cfg, x, views)
    t_bp = med(lambda: ora.back(cfg, r, views))
    t1 = med(lambda: ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=M, n_steps=1, denom=DL))
    t2 = med(lambda: ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=M, n_steps=2, denom=DL))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return dict(workload=cfg["name"], threads=threads, reps=reps, subset_views=len(views),
                fp_subset_s=round(t_fp, 5), bp_subset_s=round(t_bp, 5), step_s=round(t2 - t1, 5),
                iteration_s=round(M * (t2 - t1), 4), kind="oracle")


def time_to_1hu(lalm, torch, synth, cfg, data, plan, y, w, denom, beta, delta, dev,
                xstar_iters, max_iters, inner=(5,)):
    """Wall time of plain OS-LALM (M subsets, continuation, x0 = 0) to reach
    1 HU ROI RMS difference from x*.  x* is the one-subset continuation run of
    the same library (convergent; it reaches the same minimizer as one-subset
    FISTA with restart).  The same figure for n > 1 inner FISTA iterations
    (the listed n) and from the FBP initial image (its time included) is
    reported beside it."""
    geom = synth.geometry_of(cfg)
    p1 = lalm.lalm_plan_geometry(geom, 1)
    y1 = torch.as_tensor(data["y"][p1.view_of_slot], dtype=torch.float32, device=dev).reshape(-1).contiguous()
    w1 = torch.as_tensor(data["w"][p1.view_of_slot], dtype=torch.float32, device=dev).reshape(-1).contiguous()
    d1 = torch.empty(p1.image_elems, device=dev)
    lalm.lalm_sqs_denom(p1, w1, d1)
    xs = lalm.LalmState.zeros_like(torch.zeros(p1.image_elems, device=dev))
    t0 = time.perf_counter()
    lalm.lalm_iterate(p1, y1, w1, d1, beta, delta, xs, xstar_iters)
    t_xs = time.perf_counter() - t0
    prev = xs.x.clone()
    lalm.lalm_iterate(p1, y1, w1, d1, beta, delta, xs, 100)
    radius = synth.roi_radius(cfg)
    out = torch.zeros(1, dtype=torch.float64, device=dev)
    lalm.lalm_roi_rmsd_f64(plan, xs.x, prev, radius, out)
    change = float(out.item()) * synth.HU_PER_MU
    M = plan.M

    def start(from_fbp):
        st = lalm.LalmState.zeros_like(torch.zeros(plan.image_elems, device=dev))
        if from_fbp:
            lalm.lalm_fbp(plan, y, st.x)
            torch.clamp_(st.x, min=0.0)           # x0 in the constraint set
        return st

    def run(n_inner, from_fbp=False):
        st = start(from_fbp)
        k, hist = 0, []
        while k < max_iters:
            lalm.lalm_iterate(plan, y, w, denom, beta, delta, st, M, n_inner=n_inner)
            k += 1
            lalm.lalm_roi_rmsd_f64(plan, st.x, xs.x, radius, out)
            hist.append(round(float(out.item()) * synth.HU_PER_MU, 3))
            if hist[-1] < 1.0:
                break
        r = dict(reached=hist[-1] < 1.0, iters=k, rmsd_hu_at_stop=hist[-1], rmsd_hu_per_iter=hist[:40])
        if r["reached"]:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = start(from_fbp)
            lalm.lalm_iterate(plan, y, w, denom, beta, delta, st, k * M, n_inner=n_inner)
            torch.cuda.synchronize()
            r["wall_s"] = round(time.perf_counter() - t0, 5)
        else:
            r["wall_s"] = None
        return r

    res = run(1)
    res.update(xstar_iters=xstar_iters + 100, xstar_last100_change_hu=round(change, 5), xstar_wall_s=round(t_xs, 3))
    for n in inner:
        r = run(n)
        res["inner_%d" % n] = {k: v for k, v in r.items() if k != "rmsd_hu_per_iter"}
    if cfg["kind"] == 0:
        r = run(1, from_fbp=True)
        res["from_fbp"] = {k: v for k, v in r.items() if k != "rmsd_hu_per_iter"}
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=960, help="timed subset steps (40 iterations x 24)")
    ap.add_argument("--warmup", type=int, default=48)
    ap.add_argument("--workload", default="fan2d_512")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-1hu", action="store_true")
    ap.add_argument("--xstar-iters", type=int, default=6000)
    ap.add_argument("--max-iters-1hu", type=int, default=300)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="only time the FP64 oracle's projector pair and subset step (CPU; "
                         "threads from OMP_NUM_THREADS)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the multi-GPU path (views of a subset sharded across GPUs, "
              "one image all-reduce per subset step) is not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import synth
    if args.oracle_timing:
        cfg = synth.get_config(args.workload)
        data = synth.make_problem_data(cfg)
        print(json.dumps(oracle_timing(cfg, data, cfg["beta"], synth.configs.delta_mu(cfg))))
        return
    import torch
    from paper_1402_4381_amd import lalm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = "cuda:0"
    if args.copy_probe:
        src = torch.ones(64 * 1024 * 1024, device=dev)     # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": src.numel() * 4, "copy_probe_bytes_written": src.numel() * 4}))
        return
    cfg = synth.get_config(args.workload)
    M = cfg["M"]
    log("bench: generating %s inputs" % args.workload)
    data = synth.make_problem_data(cfg)
    plan = lalm.lalm_plan_geometry(synth.geometry_of(cfg), M)
    y = torch.as_tensor(data["y"][plan.view_of_slot], dtype=torch.float32, device=dev).reshape(-1).contiguous()
    w = torch.as_tensor(data["w"][plan.view_of_slot], dtype=torch.float32, device=dev).reshape(-1).contiguous()
    denom = torch.empty(plan.image_elems, device=dev)
    lalm.lalm_sqs_denom(plan, w, denom)
    beta = cfg["beta"]
    if beta is None:
        # workload without a tabulated median: beta from this run's own D_L
        roi = torch.as_tensor(synth.roi_mask(cfg).reshape(-1), device=dev)
        beta = synth.configs.BETA_REL * float(denom[roi].median().item())
    delta = synth.configs.delta_mu(cfg)
    state = lalm.LalmState.zeros_like(torch.zeros(plan.image_elems, device=dev))

    log("bench: warmup %d steps" % args.warmup)
    lalm.lalm_iterate(plan, y, w, denom, beta, delta, state, args.warmup)
    torch.cuda.synchronize()

    # timed region: K subset steps, no instrumentation
    log("bench: timing %d steps" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lalm.lalm_iterate(plan, y, w, denom, beta, delta, state, args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps / dt

    # per-kernel HIP events over a second pass of the same K steps
    log("bench: kernel timing pass")
    lalm.lalm_profile_begin(plan)
    step0 = state.step
    t1 = time.perf_counter()
    lalm.lalm_iterate(plan, y, w, denom, beta, delta, state, args.steps)
    dt_prof = time.perf_counter() - t1
    ms, cnt = lalm.lalm_profile_read(plan)
    lalm.lalm_profile_end(plan)
    avg_ms = ms / np.maximum(cnt, 1)

    # algorithmic bytes per launch, averaged over the subsets the steps visit.
    # 2D: the back-projection class is the line kernel (taps, residual, the
    # two partial images written); the update class is the step kernel that
    # fuses the back-projection epilogue with the next x-update (reads the
    # partial images, G, g, x, D_L; writes G, g, x and both x candidates
    # with their two projector layouts).  3D: the voxel-driven kernel with
    # its epilogue (G, g, x read; G, g, grad R written), and the x-update.
    fused = cfg["kind"] == 0
    taps = 4 if cfg["kind"] != 0 else 2
    nvox = plan.image_elems
    fp_b = bp_b = 0.0
    for j in range(step0, step0 + args.steps):
        m = int(plan.order[(j + 1) % M])
        s = float(plan.subset_samples[m])
        rays = float(plan.subset_rays(m))
        fp_b += s * taps * 4 + rays * 12          # taps + y, w read + residual write
        bp_b += s * taps * 4 + rays * 4 + nvox * (8 if fused else 24)
    fp_b /= args.steps
    bp_b /= args.steps
    upd_b = nvox * (60.0 if fused else 32.0)
    kern = {"update": (avg_ms[0], upd_b), "project": (avg_ms[1], fp_b), "backproject": (avg_ms[2], bp_b)}
    dom = max(kern, key=lambda k: kern[k][0])
    t_ms, b = kern[dom]
    achieved = b / (t_ms * 1e-3) / 1e9
    traffic = traffic_from_profiles(dom, args.workload) if dom in KERNEL_SOURCES else None
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=dom,
                    kernel_avg_us=round(t_ms * 1e3, 3),
                    kernels_avg_us={k: round(v[0] * 1e3, 3) for k, v in kern.items()},
                    kernels_gbs={k: round(v[1] / (v[0] * 1e-3) / 1e9, 1) for k, v in kern.items()},
                    bytes_per_launch=int(b))

    t1hu = None
    if not args.no_time_to_1hu and cfg["kind"] == 0:
        log("bench: x* and wall time to 1 HU")
        t1hu = time_to_1hu(lalm, torch, synth, cfg, data, plan, y, w, denom, beta, delta, dev,
                           args.xstar_iters, args.max_iters_1hu)

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline (~%.0f s)" % args.cpu_seconds)
        cpu = cpu_baseline(cfg, data, beta, delta, args.cpu_seconds)

    out = {
        "metric": "OS-LALM subset iters/sec",
        "value": round(value, 2),
        "unit": "subset_iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "image": [cfg["nz"], cfg["ny"], cfg["nx"]],
                   "views": cfg["n_views"], "bins": cfg["n_bins"], "rows": cfg["n_rows"],
                   "subsets": M, "continuation": True, "inner_iters": 1},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "profiled_pass_ms_per_step": round(dt_prof / args.steps * 1e3, 5),
        "time_to_1hu": t1hu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
