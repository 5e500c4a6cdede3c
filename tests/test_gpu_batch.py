"""GPU: a batch of B images planned together (lalm_plan_geometry's batch)
gives, image for image, the bits of B single-image runs -- every kernel
launch covers all B images, and each image's arithmetic and reduction order
are those of a single run.  Covers the fused 2D steps (continuation, fixed
rho, forced restarts, statistics), inner FISTA iterations, Barzilai-Borwein
scaling, a 3D cone-beam case, the projector pair, the SQS denominator, FBP
and the FP64 monitors."""
import numpy as np
import pytest

from _helpers import ensure_built, say

import oracle as ora
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

MED3D = dict(nx=64, ny=64, nz=16, dx=7.84, dy=7.84, dz=2.5, n_views=24, n_views_per_turn=24,
             n_bins=111, ds=8.0, n_rows=16, dt=4.4, n_ellipses=12)


@pytest.fixture(scope="module")
def L():
    ensure_built()
    from paper_1402_4381_amd import lalm
    assert torch.cuda.is_available()
    return lalm


def gpu(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV).to(dtype).contiguous()


def _data(cfg, seeds):
    return [synth.make_problem_data(cfg, seed=s, workers=1) for s in seeds]


def _inputs(L, cfg, M, datas):
    """Plans (batched and single) and subset-major y, w stacked per image."""
    B = len(datas)
    pb = L.lalm_plan_geometry(synth.geometry_of(cfg), M, batch=B)
    p1 = L.lalm_plan_geometry(synth.geometry_of(cfg), M)
    ys = [gpu(d["y"][p1.view_of_slot]).reshape(-1) for d in datas]
    ws = [gpu(d["w"][p1.view_of_slot]).reshape(-1) for d in datas]
    return pb, p1, ys, ws


CASES = [("fan2d_128", {}, 4, 3, dict()),
         ("fan2d_128", {}, 4, 3, dict(continuation=False, rho_fixed=0.2)),
         ("fan2d_128", {}, 4, 2, dict(n_inner=3)),
         ("fan2d_128", {}, 4, 3, dict(bb=True)),
         ("cone_axial_512x64", MED3D, 3, 2, dict())]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,over,M,n_iter,kw", CASES)
def test_batch_iterate_equals_single_runs(L, name, over, M, n_iter, kw):
    cfg = synth.get_config(name, **over)
    seeds = [31, 32, 33, 34] if not over else [41, 42]
    B = len(seeds)
    datas = _data(cfg, seeds)
    pb, p1, ys, ws = _inputs(L, cfg, M, datas)
    n = pb.image_elems
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    # SQS denominators: batched equals single
    db = torch.empty(B * n, device=DEV)
    L.lalm_sqs_denom(pb, torch.cat(ws), db)
    d1 = []
    for k in range(B):
        d = torch.empty(n, device=DEV)
        L.lalm_sqs_denom(p1, ws[k], d)
        d1.append(d)
        assert torch.equal(db[k * n:(k + 1) * n], d), "D_L of image %d" % k
    n_steps = n_iter * M
    bb = kw.get("bb", False)
    stb = L.LalmState.zeros_like(torch.zeros(B * n, device=DEV), bb=bb, batch=B)
    stats_b = dict(rho=torch.zeros(B * n_steps, dtype=torch.float64, device=DEV),
                   xi=torch.zeros(B * n_steps, dtype=torch.float64, device=DEV),
                   restart=torch.zeros(B * n_steps, dtype=torch.uint8, device=DEV))
    # two calls, so that the batch also resumes from its per-image state
    h = n_steps // 2 + 1
    L.lalm_iterate(pb, torch.cat(ys), torch.cat(ws), db, beta, delta, stb, h, stats=stats_b, **kw)
    L.lalm_iterate(pb, torch.cat(ys), torch.cat(ws), db, beta, delta, stb, n_steps - h, stats=stats_b, **kw)
    for k in range(B):
        s1 = L.LalmState.zeros_like(torch.zeros(n, device=DEV), bb=bb)
        st1 = {key: torch.zeros(n_steps, dtype=v.dtype, device=DEV) for key, v in stats_b.items()}
        L.lalm_iterate(p1, ys[k], ws[k], d1[k], beta, delta, s1, n_steps, stats=st1, **kw)
        sl = slice(k * n, (k + 1) * n)
        same = (torch.equal(stb.x[sl], s1.x) and torch.equal(stb.g[sl], s1.g) and torch.equal(stb.grad[sl], s1.grad))
        say("%s %s image %d: bit-identical %s, l %d/%d, rho %.6f/%.6f, restarts %d"
            % (name, kw, k, same, stb.l_b[k], s1.l, stb.rho_b[k], s1.rho, int(st1["restart"].sum())))
        assert same
        assert stb.l_b[k] == s1.l and stb.rho_b[k] == s1.rho and stb.alpha_b[k] == s1.alpha
        for key in st1:
            assert torch.equal(stats_b[key][k * n_steps:(k + 1) * n_steps], st1[key]), key
    assert stb.step == n_steps and stb.l == stb.l_b[0] and stb.rho == stb.rho_b[0]
    # images differ (different data): the batch is not one image repeated
    assert not torch.equal(stb.x[:n], stb.x[n:2 * n])


def test_batch_forced_restarts_per_image(L):
    cfg = synth.get_config("fan2d_128")
    datas = _data(cfg, [51, 52])
    pb, p1, ys, ws = _inputs(L, cfg, 4, datas)
    n, n_steps = pb.image_elems, 16
    db = torch.empty(2 * n, device=DEV)
    L.lalm_sqs_denom(pb, torch.cat(ws), db)
    pats = np.zeros((2, n_steps), dtype=np.uint8)
    pats[0, [2, 3, 9]] = 1
    pats[1, [5, 12]] = 1
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    stb = L.LalmState.zeros_like(torch.zeros(2 * n, device=DEV), batch=2)
    rs = torch.zeros(2 * n_steps, dtype=torch.uint8, device=DEV)
    stats = dict(rho=torch.zeros(2 * n_steps, dtype=torch.float64, device=DEV),
                 xi=torch.zeros(2 * n_steps, dtype=torch.float64, device=DEV), restart=rs)
    L.lalm_iterate(pb, torch.cat(ys), torch.cat(ws), db, beta, delta, stb, n_steps,
                   forced_restart=gpu(pats.reshape(-1), torch.uint8), stats=stats)
    assert np.array_equal(rs.cpu().numpy().reshape(2, n_steps), pats)
    for k in range(2):
        d = torch.empty(n, device=DEV)
        L.lalm_sqs_denom(p1, ws[k], d)
        s1 = L.LalmState.zeros_like(torch.zeros(n, device=DEV))
        L.lalm_iterate(p1, ys[k], ws[k], d, beta, delta, s1, n_steps, forced_restart=gpu(pats[k], torch.uint8))
        assert torch.equal(stb.x[k * n:(k + 1) * n], s1.x)


@pytest.mark.parametrize("name,over,M", [("fan2d_128", {}, 4), ("cone_axial_512x64", MED3D, 3),
                                         ("cone_helical_512x256", dict(MED3D, n_views=48, pitch=1.0,
                                                                        kind=2), 4)])
def test_batch_projector_pair_fbp_and_monitors(L, name, over, M):
    cfg = synth.get_config(name, **over)
    B = 3
    pb = L.lalm_plan_geometry(synth.geometry_of(cfg), M, batch=B)
    p1 = L.lalm_plan_geometry(synth.geometry_of(cfg), M)
    n = pb.image_elems
    rng = np.random.default_rng(7)
    xs = [gpu(rng.uniform(0, 0.03, n).astype(np.float32)) for _ in range(B)]
    m = int(pb.order[1])
    nm = pb.subset_rays(m)
    out = torch.empty(B * nm, device=DEV)
    L.lalm_project_subset(pb, m, torch.cat(xs), out)
    rs = [gpu(rng.normal(size=nm).astype(np.float32)) for _ in range(B)]
    back = torch.empty(B * n, device=DEV)
    L.lalm_backproject_subset(pb, m, torch.cat(rs), back, scale=1.5)
    sinos = [gpu(rng.uniform(0, 2, pb.sino_elems).astype(np.float32)) for _ in range(B)]
    wts = [gpu(rng.uniform(0.5, 2, pb.sino_elems).astype(np.float32)) for _ in range(B)]
    cost_b = torch.zeros(3 * B, dtype=torch.float64, device=DEV)
    L.lalm_cost_f64(pb, torch.cat(sinos), torch.cat(wts), 1e3, 2e-4, torch.cat(xs), cost_b)
    rm_b = torch.zeros(B, dtype=torch.float64, device=DEV)
    L.lalm_roi_rmsd_f64(pb, torch.cat(xs), torch.cat(xs[1:] + xs[:1]), 30.0, rm_b)
    fbp_ok = cfg["kind"] != 2
    if fbp_ok:
        fb = torch.empty(B * n, device=DEV)
        L.lalm_fbp(pb, torch.cat(sinos), fb)
    for k in range(B):
        o1 = torch.empty(nm, device=DEV)
        L.lalm_project_subset(p1, m, xs[k], o1)
        assert torch.equal(out[k * nm:(k + 1) * nm], o1), "A_m x, image %d" % k
        b1 = torch.empty(n, device=DEV)
        L.lalm_backproject_subset(p1, m, rs[k], b1, scale=1.5)
        assert torch.equal(back[k * n:(k + 1) * n], b1), "A_m' r, image %d" % k
        c1 = torch.zeros(3, dtype=torch.float64, device=DEV)
        L.lalm_cost_f64(p1, sinos[k], wts[k], 1e3, 2e-4, xs[k], c1)
        assert torch.equal(cost_b[3 * k:3 * k + 3], c1), "cost, image %d" % k
        r1 = torch.zeros(1, dtype=torch.float64, device=DEV)
        L.lalm_roi_rmsd_f64(p1, xs[k], xs[(k + 1) % B], 30.0, r1)
        assert torch.equal(rm_b[k:k + 1], r1)
        if fbp_ok:
            f1 = torch.empty(n, device=DEV)
            L.lalm_fbp(p1, sinos[k], f1)
            assert torch.equal(fb[k * n:(k + 1) * n], f1), "FBP, image %d" % k
    say("%s: batch of %d bit-identical for A_m x, A_m' r, cost, ROI RMSD%s" % (name, B, ", FBP" if fbp_ok else ""))
