#!/usr/bin/env python3
"""OS-LALM benchmark on one MI355X.

One step = one OS-LALM subset iteration of the whole hot path: x-update
(regularizer majorizer, continuation rho), forward projection of the next
subset with fused weighted residual, matched back-projection with the fused
g-update, regularizer gradient and FP64 restart indicator, and the
continuation decision.  The default workload is the helical cone-beam volume:
512 x 512 x 256 voxels (0.98 x 0.98 x 0.625 mm), 6888 views (7 turns of 984)
of 64 rows x 888 channels, pitch 1, M = 12 subsets, a 60-ellipsoid seeded
phantom and Poisson counts at I0 = 5e4.  All inputs are resident in GPU
memory before timing.

Printed: one JSON line with
* the throughput (subset iterations / s) and the roofline figure of the
  dominant kernel (algorithmic bytes / event-timed kernel time against the
  8 TB/s HBM peak), next to the HBM traffic, DRAM rate, L2 hit rate and
  VALU issue use that rocprofv3 counters measured for that kernel;
* the FP64 CPU oracle timed on a bounded sample of the same workload (a few
  views of one subset and a slab of the x-update, extrapolated to one
  subset step) and the GPU-vs-oracle error on that sample;
* the wall time to 1 HU ROI RMS difference from x* (x* and its convergence
  figure stated in the record);
* the same throughput and roofline figures for the 512^2 fan-beam workload
  (984 views x 888 bins, M = 24) under the key "fan2d_512".
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
DEFAULT_WORKLOAD = "cone_helical_512x256"
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


def profile_record(kind, kernel, workload):
    """A committed rocprofv3 counter summary (``profiles/<kind>_<kernel>_
    <workload>.json``), or None when none exists or the kernel's sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_%s.json" % (kind, kernel, workload))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256_16") != source_hash(KERNEL_SOURCES[kernel]):
        return None
    return rec


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE record."""
    rec = profile_record("traffic", kernel, workload)
    return None if rec is None else rec.get("hbm_bytes_per_launch")


def threads_used():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))


# ------------------------------------------------------------ device inputs

def load_inputs(lalm, torch, synth, cfg, data, M, dev):
    """Plan, subset-major y and w on the device, D_L and beta."""
    plan = lalm.lalm_plan_geometry(synth.geometry_of(cfg), M)
    vos = torch.as_tensor(plan.view_of_slot, dtype=torch.long, device=dev)
    y = torch.as_tensor(data["y"].astype("float32"), device=dev).index_select(0, vos).reshape(-1).contiguous()
    w = torch.as_tensor(data["w"].astype("float32"), device=dev).index_select(0, vos).reshape(-1).contiguous()
    denom = torch.empty(plan.image_elems, device=dev)
    lalm.lalm_sqs_denom(plan, w, denom)
    beta = cfg["beta"]
    if beta is None:
        # workload without a tabulated median: beta from this run's own D_L
        roi = torch.as_tensor(synth.roi_mask(cfg).reshape(-1), device=dev)
        beta = synth.configs.BETA_REL * float(denom[roi].median().item())
    return plan, y, w, denom, beta


# ------------------------------------------------------------- throughput

def throughput(lalm, torch, np, cfg, plan, y, w, denom, beta, delta, steps, warmup, dev):
    """Warm-up, the timed K steps, then a second pass of K steps with
    per-dispatch HIP events for the kernel classes; returns the record, the
    roofline of the dominant class and the state."""
    M = plan.M
    state = lalm.LalmState.zeros_like(torch.zeros(plan.image_elems, device=dev))
    log("bench: %s warmup %d steps" % (cfg["name"], warmup))
    lalm.lalm_iterate(plan, y, w, denom, beta, delta, state, warmup)
    torch.cuda.synchronize()

    # timed region: K subset steps, no instrumentation
    log("bench: %s timing %d steps" % (cfg["name"], steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lalm.lalm_iterate(plan, y, w, denom, beta, delta, state, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # per-kernel HIP events over a second pass of the same K steps
    lalm.lalm_profile_begin(plan)
    step0 = state.step
    t1 = time.perf_counter()
    lalm.lalm_iterate(plan, y, w, denom, beta, delta, state, steps)
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
    for j in range(step0, step0 + steps):
        m = int(plan.order[(j + 1) % M])
        s = float(plan.subset_samples[m])
        rays = float(plan.subset_rays(m))
        fp_b += s * taps * 4 + rays * 12          # taps + y, w read + residual write
        bp_b += s * taps * 4 + rays * 4 + nvox * (8 if fused else 24)
    fp_b /= steps
    bp_b /= steps
    upd_b = nvox * (60.0 if fused else 32.0)
    kern = {"update": (avg_ms[0], upd_b), "project": (avg_ms[1], fp_b), "backproject": (avg_ms[2], bp_b)}
    dom = max(kern, key=lambda k: kern[k][0])
    t_ms, b = kern[dom]
    achieved = b / (t_ms * 1e-3) / 1e9
    wl = cfg["name"]
    traffic = traffic_from_profiles(dom, wl)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic, kernel=dom,
                    kernel_avg_us=round(t_ms * 1e3, 3),
                    kernels_avg_us={k: round(v[0] * 1e3, 3) for k, v in kern.items()},
                    kernels_gbs={k: round(v[1] / (v[0] * 1e-3) / 1e9, 1) for k, v in kern.items()},
                    bytes_per_launch=int(b))
    # what the counters say about the dominant kernel: the taps come from
    # L1 / L2, so DRAM moves a fraction of the algorithmic bytes; the limit
    # is instruction issue and gather latency, reported beside the HBM figure
    if traffic:
        roofline["dram_gbs"] = round(traffic / (t_ms * 1e-3) / 1e9, 1)
        roofline["dram_frac"] = round(roofline["dram_gbs"] / HBM_PEAK_GBS, 4)
    cnt_rec = profile_record("counters", dom, wl)
    if cnt_rec is not None:
        for key in ("l2_hit_rate", "valu_issue", "valu_insts_per_launch", "lds_bank_conflict_cycles"):
            if key in cnt_rec:
                roofline[key] = cnt_rec[key]
    rec = dict(value=round(steps / dt, 3), ms_per_step=round(dt / steps * 1e3, 5),
               profiled_pass_ms_per_step=round(dt_prof / steps * 1e3, 5), roofline=roofline)
    return rec, state


# ---------------------------------------------------------- CPU baseline

def cpu_baseline_2d(cfg, data, beta, delta, budget_s):
    """The FP64 oracle's OS-LALM timed on a bounded number of subset steps
    (its D_L is computed once beforehand, outside the timing, as the GPU's is)."""
    import oracle as ora
    DL = ora.sqs_denom(cfg, data["w"])
    t0 = time.perf_counter()
    ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=cfg["M"], n_steps=3, denom=DL)
    per = (time.perf_counter() - t0) / 3.0
    n = max(3, int(budget_s / max(per, 1e-4)))
    t0 = time.perf_counter()
    ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=cfg["M"], n_steps=n, denom=DL)
    dt = time.perf_counter() - t0
    return dict(value=round(n / dt, 3), unit="subset_iters/s", cores=threads_used(), kind="oracle",
                sample="%d OS-LALM subset steps of %s (M=%d, from x0 = 0, incl. the initial "
                       "subset gradient) with the FP64 oracle: %.1f s" % (n, cfg["name"], cfg["M"], dt))


def cpu_baseline_volume(lalm, torch, np, cfg, data, plan, beta, delta, dev, n_views=12, n_slices=16):
    """The FP64 oracle on a bounded sample of one subset step of a 3D
    workload, extrapolated to the whole step: the forward projection and the
    back-projection of ``n_views`` views from the middle of subset
    order[1] (scaled by the subset's view count), plus the x-update, g-update
    and restart dot on ``n_slices`` slices (scaled by the slice count).  The
    projector inputs are seeded: a uniform random image and, for the
    back-projection, standard normal residuals on the sampled views.  The
    same inputs, in FP32, go through the library's subset projection and
    back-projection, and their error against the oracle is reported."""
    import oracle as ora
    rng = np.random.default_rng(20140218)
    M = plan.M
    m = int(plan.order[1])
    views = plan.subset_views(m)
    a = len(views) // 2 - n_views // 2
    vs = np.asarray(views[a:a + n_views])
    shape = ora.image_shape(cfg)
    x32 = rng.uniform(0.0, 0.04, shape).astype(np.float32)
    x = x32.astype(np.float64)
    t0 = time.perf_counter()
    p = ora.forward(cfg, x, vs)
    t_fp = time.perf_counter() - t0
    r32 = rng.standard_normal(p.shape).astype(np.float32)
    t0 = time.perf_counter()
    b = ora.back(cfg, r32.astype(np.float64), vs)
    t_bp = time.perf_counter() - t0
    # the oracle's back-projection has a fixed part (image-sized partial
    # buffers and their reduction): time half the views as well and
    # extrapolate the difference, not the fixed part
    h = len(vs) // 2
    t0 = time.perf_counter()
    ora.back(cfg, r32[:h].astype(np.float64), vs[:h])
    t_bp_half = time.perf_counter() - t0
    bp_per_view = max(t_bp - t_bp_half, 0.0) / (len(vs) - h)
    # the size of the terms each voxel sums (outside the timing): with
    # residuals of both signs the sums cancel, so FP32 error is measured
    # against A'|r|
    b_abs = ora.back(cfg, np.abs(r32).astype(np.float64), vs)
    # x-update, g-update and xi on a slab (pointwise work; seeded values)
    nzs = min(n_slices, shape[0])
    xs = x[:nzs].copy()
    Gs = rng.standard_normal(xs.shape)
    gs = rng.standard_normal(xs.shape)
    DLs = rng.uniform(1.0, 2.0, xs.shape) * 1e10
    DRs = ora.reg_denom(xs.shape, beta, True)
    rho = 0.5
    t0 = time.perf_counter()
    s = rho * Gs + (1.0 - rho) * gs
    xn = ora.inner_fista(xs, s, DLs, DRs, rho, beta, delta, True, 1)
    Gn = Gs[::-1].copy()
    gn = (rho * Gn + gs) / (rho + 1.0)
    xi = float(np.sum((gs - Gn) * (Gn - Gs)))
    t_upd = time.perf_counter() - t0
    del xn, gn, xi
    t_bp_subset = t_bp + bp_per_view * (len(views) - len(vs))
    per_step = t_fp * len(views) / len(vs) + t_bp_subset + t_upd * shape[0] / nzs

    # the library on the same inputs
    rays_v = plan.rays_per_view
    slot0 = int(np.nonzero(views == vs[0])[0][0])
    xg = torch.as_tensor(x32.reshape(-1), device=dev)
    out = torch.empty(plan.subset_rays(m), device=dev)
    lalm.lalm_project_subset(plan, m, xg, out)
    pg = out[slot0 * rays_v:(slot0 + len(vs)) * rays_v].double().cpu().numpy()
    pr = p.reshape(-1)
    rsub = torch.zeros(plan.subset_rays(m), device=dev)
    rsub[slot0 * rays_v:(slot0 + len(vs)) * rays_v] = torch.as_tensor(r32.reshape(-1), device=dev)
    bg = torch.empty(plan.image_elems, device=dev)
    lalm.lalm_backproject_subset(plan, m, rsub, bg)
    bgn = bg.double().cpu().numpy()
    br = b.reshape(-1)
    err = dict(fp_rel_l2=float(np.linalg.norm(pg - pr) / np.linalg.norm(pr)),
               fp_max_abs_over_max=float(np.max(np.abs(pg - pr)) / np.max(np.abs(pr))),
               bp_rel_l2=float(np.linalg.norm(bgn - br) / np.linalg.norm(br)),
               bp_max_abs_over_max=float(np.max(np.abs(bgn - br)) / np.max(np.abs(br))),
               bp_max_abs_over_abs_terms=float(np.max(np.abs(bgn - br) / np.maximum(b_abs.reshape(-1),
                                                                                   1e-6 * np.max(b_abs)))),
               sample="A_m x and A_m' r of subset %d on %d views (%d rays), FP32 library vs FP64 oracle"
                      % (m, len(vs), len(vs) * rays_v))
    return dict(value=round(1.0 / per_step, 6), unit="subset_iters/s", cores=threads_used(), kind="oracle",
                sample=("extrapolated: FP64 oracle forward projection %.2f s of %d of the %d views of subset %d "
                        "(scaled x%.1f); back-projection %.2f s of the %d views and %.2f s of %d (the difference "
                        "per view extrapolated to %d views: %.1f s); x-update + g-update + restart dot %.2f s "
                        "on %d of %d slices (scaled x%.0f); one subset step of %s = %.1f s"
                        % (t_fp, len(vs), len(views), m, len(views) / len(vs), t_bp, len(vs), t_bp_half, h,
                           len(views), t_bp_subset, t_upd, nzs, shape[0], shape[0] / nzs, cfg["name"], per_step)),
                seconds_measured=round(t_fp + t_bp + t_bp_half + t_upd, 2), gpu_vs_oracle=err)


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
    return dict(workload=cfg["name"], threads=threads_used(), reps=reps, subset_views=len(views),
                fp_subset_s=round(t_fp, 5), bp_subset_s=round(t_bp, 5), step_s=round(t2 - t1, 5),
                iteration_s=round(M * (t2 - t1), 4), kind="oracle")


# ------------------------------------------------------------- time to 1 HU

def time_to_1hu_2d(lalm, torch, synth, cfg, data, plan, y, w, denom, beta, delta, dev,
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
    res.update(xstar="one-subset OS-LALM with continuation, n = 1, %d iterations from x0 = 0"
                     % (xstar_iters + 100),
               xstar_iters=xstar_iters + 100, xstar_last100_change_hu=round(change, 5),
               xstar_wall_s=round(t_xs, 3), beta=beta, n_inner=1)
    for n in inner:
        r = run(n)
        res["inner_%d" % n] = {k: v for k, v in r.items() if k != "rmsd_hu_per_iter"}
    r = run(1, from_fbp=True)
    res["from_fbp"] = {k: v for k, v in r.items() if k != "rmsd_hu_per_iter"}
    return res


def time_to_1hu_volume(lalm, torch, synth, cfg, data, plan, y, w, denom, beta, delta, dev,
                       warm_iters=20, polish_max=800, polish_tol_hu=0.005, polish_budget_s=270.0,
                       n_inner=16, max_iters=60, plain_iters=20):
    """Wall time of OS-LALM (M subsets, continuation, x0 = 0) to 1 HU ROI RMS
    difference from x* on a 3D workload.

    x* is the minimizer approached by a convergent method (Sec. V measures
    against a converged one-subset reference): OS-LALM with M subsets and
    n_inner FISTA iterations per step for warm_iters iterations (fast, but
    an M > 1 run ends in a limit cycle near the minimizer, Sec. III-A), then
    the one-subset method (M = 1, continuation, n_inner) from that image,
    ten iterations at a time, until its ROI RMS change over ten iterations
    is below polish_tol_hu or polish_max iterations or polish_budget_s
    seconds have run.  The record states which stop was reached.

    Timed from x0 = 0 against that x*: OS-LALM-M-c with n_inner inner
    iterations (until 1 HU, at most max_iters iterations), and the plain
    n = 1 method for plain_iters iterations (its RMSD at the stop)."""
    import numpy as np
    M = plan.M
    radius, hu = synth.roi_radius(cfg), synth.HU_PER_MU
    r64 = torch.zeros(1, dtype=torch.float64, device=dev)

    def rmsd(a, b):
        lalm.lalm_roi_rmsd_f64(plan, a, b, radius, r64)
        return float(r64.item()) * hu

    def zero():
        return lalm.LalmState.zeros_like(torch.zeros(plan.image_elems, device=dev))

    def timed(f):
        torch.cuda.synchronize()
        t = time.perf_counter()
        f()
        torch.cuda.synchronize()
        return time.perf_counter() - t

    st = zero()
    t_warm = timed(lambda: lalm.lalm_iterate(plan, y, w, denom, beta, delta, st, warm_iters * M, n_inner=n_inner))
    log("bench: x* warm start %d iterations in %.1f s" % (warm_iters, t_warm))
    x_warm = st.x
    del st
    p1 = lalm.lalm_plan_geometry(synth.geometry_of(cfg), 1)
    vos = torch.as_tensor(p1.view_of_slot, dtype=torch.long, device=dev)
    y1 = torch.as_tensor(data["y"].astype(np.float32), device=dev).index_select(0, vos).reshape(-1).contiguous()
    w1 = torch.as_tensor(data["w"].astype(np.float32), device=dev).index_select(0, vos).reshape(-1).contiguous()
    xs = zero()
    xs.x.copy_(x_warm)
    prev = x_warm.clone()
    k, change, t_pol, changes = 0, None, 0.0, []
    while k < polish_max and t_pol < polish_budget_s:
        t_pol += timed(lambda: lalm.lalm_iterate(p1, y1, w1, denom, beta, delta, xs, 10, n_inner=n_inner))
        k += 10
        change = rmsd(xs.x, prev)
        changes.append(round(change, 5))
        prev.copy_(xs.x)
        log("bench: x* one-subset iteration %d: change over 10 iterations %.4f HU (%.1f s)" % (k, change, t_pol))
        if change < polish_tol_hu:
            break
    warm_to_star = rmsd(x_warm, xs.x)
    # the changes decay geometrically; their sum over the iterations not run
    # estimates how far x* still is from the minimizer
    q = changes[-1] / changes[-2] if len(changes) > 1 and changes[-2] > 0 else None
    remaining = changes[-1] * q / (1.0 - q) if q is not None and q < 1.0 else None
    del y1, w1, p1, prev, x_warm
    torch.cuda.empty_cache()
    x_star = xs.x
    stop = ("change over 10 iterations below %.3g HU" % polish_tol_hu if change is not None and change < polish_tol_hu
            else ("%d-iteration cap" % polish_max if k >= polish_max else "%.0f s budget" % polish_budget_s))
    res = dict(xstar=("OS-LALM-%d-c-%d for %d iterations from x0 = 0, then one-subset OS-LALM-1-c-%d for %d "
                      "iterations (stopped at: %s)" % (M, n_inner, warm_iters, n_inner, k, stop)),
               xstar_one_subset_iters=k, xstar_last10_change_hu=changes[-1] if changes else None,
               xstar_est_distance_to_minimizer_hu=None if remaining is None else round(remaining, 4),
               xstar_change_per_10_hu=changes, xstar_rmsd_hu_from_M_subset_start=round(warm_to_star, 4),
               xstar_wall_s=round(t_warm + t_pol, 2), beta=beta)

    def start(from_fbp):
        s = zero()
        if from_fbp:
            lalm.lalm_fbp(plan, y, s.x)
            torch.clamp_(s.x, min=0.0)            # x0 in the constraint set
        return s

    def run(n, cap, from_fbp=False):
        s = start(from_fbp)
        hist, times = [], []
        if from_fbp:
            hist0 = round(rmsd(s.x, x_star), 3)
        for _ in range(cap):
            times.append(timed(lambda: lalm.lalm_iterate(plan, y, w, denom, beta, delta, s, M, n_inner=n)))
            hist.append(round(rmsd(s.x, x_star), 3))
            if hist[-1] < 1.0:
                break
        r = dict(n_inner=n, reached=hist[-1] < 1.0, iters=len(hist), rmsd_hu_at_stop=hist[-1],
                 rmsd_hu_per_iter=hist, s_per_iter=round(sum(times) / len(times), 4))
        if from_fbp:
            r["rmsd_hu_of_fbp"] = hist0
        # wall time of the iterate calls alone (and the FBP), without the
        # monitor between them
        r["wall_s"] = None
        if r["reached"]:
            def go():
                s2 = start(from_fbp)
                lalm.lalm_iterate(plan, y, w, denom, beta, delta, s2, len(hist) * M, n_inner=n)
            r["wall_s"] = round(timed(go), 4)
        return r

    res["inner_%d" % n_inner] = run(n_inner, max_iters)
    res["inner_1"] = run(1, plain_iters)
    if cfg["kind"] == 1 and cfg["n_views"] == cfg["n_views_per_turn"]:
        # the axial cone beam has an FDK initial image (Sec. V starts from FBP)
        res["from_fbp_inner_%d" % n_inner] = run(n_inner, max_iters, from_fbp=True)
        res["from_fbp_inner_1"] = run(1, plain_iters, from_fbp=True)
    return res


def batched_throughput(lalm, torch, np, synth, cfg, data, beta, delta, B, steps, dev):
    """Subset iterations per second summed over B independent scans of the
    workload reconstructed by one batched plan (every launch covers the B
    images), and the per-image kernel times; the scans are the workload's
    data with a different noise realization each."""
    M = cfg["M"]
    plan = lalm.lalm_plan_geometry(synth.geometry_of(cfg), M, batch=B)
    vos = torch.as_tensor(plan.view_of_slot, dtype=torch.long, device=dev)
    ys, ws = [], []
    for b in range(B):
        y_, w_ = synth.noisy_data(cfg, data["ybar"], 9000 + b)
        ys.append(torch.as_tensor(y_.astype("float32"), device=dev).index_select(0, vos).reshape(-1))
        ws.append(torch.as_tensor(w_.astype("float32"), device=dev).index_select(0, vos).reshape(-1))
    y, w = torch.cat(ys), torch.cat(ws)
    denom = torch.empty(B * plan.image_elems, device=dev)
    lalm.lalm_sqs_denom(plan, w, denom)
    st = lalm.LalmState.zeros_like(torch.zeros(B * plan.image_elems, device=dev), batch=B)
    lalm.lalm_iterate(plan, y, w, denom, beta, delta, st, 2 * M)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lalm.lalm_iterate(plan, y, w, denom, beta, delta, st, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lalm.lalm_profile_begin(plan)
    lalm.lalm_iterate(plan, y, w, denom, beta, delta, st, steps)
    ms, cnt = lalm.lalm_profile_read(plan)
    lalm.lalm_profile_end(plan)
    avg_us = ms / np.maximum(cnt, 1) * 1e3
    return dict(images=B, steps=steps, value=round(B * steps / dt, 2), unit="image subset_iters/s",
                ms_per_step=round(dt / steps * 1e3, 5),
                kernels_avg_us_per_launch={k: round(float(v), 3) for k, v in zip(("update", "project", "backproject"),
                                                                                  avg_us)})


def fan2d_figures(lalm, torch, np, synth, steps, warmup, dev, with_1hu):
    """Throughput, roofline and time to 1 HU of the 512^2 fan-beam workload."""
    cfg = synth.get_config("fan2d_512")
    data = synth.make_problem_data(cfg)
    plan, y, w, denom, beta = load_inputs(lalm, torch, synth, cfg, data, cfg["M"], dev)
    delta = synth.configs.delta_mu(cfg)
    rec, _ = throughput(lalm, torch, np, cfg, plan, y, w, denom, beta, delta, steps, warmup, dev)
    rec.update(steps=steps, warmup=warmup, workload="fan2d_512", subsets=cfg["M"])
    rec["batch_16"] = batched_throughput(lalm, torch, np, synth, cfg, data, beta, delta, 16, steps // 4, dev)
    if with_1hu:
        log("bench: fan2d_512 x* and wall time to 1 HU")
        rec["time_to_1hu"] = time_to_1hu_2d(lalm, torch, synth, cfg, data, plan, y, w, denom, beta, delta, dev,
                                            6000, 300)
    return rec


# ---------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=96, help="timed subset steps")
    ap.add_argument("--warmup", type=int, default=12)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle budget of the 2D workloads")
    ap.add_argument("--cpu-views", type=int, default=64, help="views of the 3D oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-1hu", action="store_true")
    ap.add_argument("--no-fan2d", action="store_true", help="skip the 512^2 fan-beam extra figures")
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
    is3d = cfg["kind"] != 0
    log("bench: generating %s inputs" % args.workload)
    t0 = time.perf_counter()
    data = synth.make_problem_data(cfg)
    log("bench: inputs in %.1f s" % (time.perf_counter() - t0))
    plan, y, w, denom, beta = load_inputs(lalm, torch, synth, cfg, data, M, dev)
    delta = synth.configs.delta_mu(cfg)
    rec, state = throughput(lalm, torch, np, cfg, plan, y, w, denom, beta, delta, args.steps, args.warmup, dev)

    t1hu = None
    if not args.no_time_to_1hu:
        log("bench: x* and wall time to 1 HU")
        if is3d:
            t1hu = time_to_1hu_volume(lalm, torch, synth, cfg, data, plan, y, w, denom, beta, delta, dev)
        else:
            t1hu = time_to_1hu_2d(lalm, torch, synth, cfg, data, plan, y, w, denom, beta, delta, dev, 6000, 300)

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        if is3d:
            cpu = cpu_baseline_volume(lalm, torch, np, cfg, data, plan, beta, delta, dev, n_views=args.cpu_views)
        else:
            cpu = cpu_baseline_2d(cfg, data, beta, delta, args.cpu_seconds)
    del data

    fan2d = None
    if is3d and not args.no_fan2d:
        log("bench: fan2d_512 figures")
        del y, w, denom, state
        torch.cuda.empty_cache()
        fan2d = fan2d_figures(lalm, torch, np, synth, 480, 48, dev, not args.no_time_to_1hu)

    out = {
        "metric": "OS-LALM subset iters/sec",
        "value": rec["value"],
        "unit": "subset_iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "image": [cfg["nz"], cfg["ny"], cfg["nx"]],
                   "views": cfg["n_views"], "bins": cfg["n_bins"], "rows": cfg["n_rows"],
                   "subsets": M, "continuation": True, "inner_iters": 1, "beta": beta},
        "roofline": rec["roofline"],
        "cpu_baseline": cpu,
        "profiled_pass_ms_per_step": rec["profiled_pass_ms_per_step"],
        "time_to_1hu": t1hu,
    }
    if fan2d is not None:
        out["fan2d_512"] = fan2d
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
