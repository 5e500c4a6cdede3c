"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Tolerances (FP32 kernels vs FP64 oracle):
* projections and back-projections: relative L2 error <= 1e-5 per subset,
  and max abs error <= 1e-5 x max |oracle|;
* adjoint test on the GPU (FP32 kernels, FP64 inner products):
  |<A x, r> - <x, A' r>| <= 1e-6 x sum_i |(A x)_i r_i| (the size of the
  terms the inner product sums; with r of random sign the inner product
  itself can cancel, so it is not the scale of the rounding), on the medium
  geometries for every subset and at full size for one subset;
* Joseph sample counts and subset bookkeeping: exact;
* images after a fixed number of OS-LALM iterations: ROI RMS difference
  <= 0.5 HU (free-running), also reported with the oracle's restart sequence
  replayed;
* cost: relative 1e-4 (the weighted residual A x - y cancels about four
  digits of FP32 against the data).
"""
import os

import numpy as np
import pytest

from _helpers import ensure_built, rel_l2, say

import oracle as ora
import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    ensure_built()
    from paper_1402_4381_amd import lalm
    assert torch.cuda.is_available()
    return lalm


DEV = "cuda:0"


def gpu(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV).to(dtype).contiguous()


MED3D = dict(nx=64, ny=64, nz=16, dx=7.84, dy=7.84, dz=2.5, n_views=24, n_views_per_turn=24,
             n_bins=111, ds=8.0, n_rows=16, dt=4.4, n_ellipses=12)
MEDHEL = dict(nx=48, ny=48, nz=24, dx=10.0, dy=10.0, dz=5.0, n_views=72, n_views_per_turn=24,
              n_bins=101, ds=9.0, n_rows=12, dt=8.0, pitch=1.0, n_ellipses=8)
RAGGED2D = dict(nx=37, ny=29, dx=2.9, dy=3.3, n_views=90, n_views_per_turn=90, n_bins=101, ds=2.9)

CASES = [
    ("tiny2d", {}, 3),
    ("tiny3d", {}, 2),
    ("tiny_helical", {}, 4),
    ("fan2d_128", {}, 4),
    ("fan2d_128", RAGGED2D, 7),             # ragged tiles, ragged subsets
    ("cone_axial_512x64", MED3D, 5),
    ("cone_helical_512x256", MEDHEL, 6),
    # detectors of one and two rows: the cone back-projector's gathered row
    # pair then starts at row 0 (one row: row 0 twice, the second weighed by a
    # padding row)
    ("tiny3d", {"n_rows": 1}, 2),
    ("tiny3d", {"n_rows": 2}, 2),
]


def _image(cfg, seed=0):
    ph = synth.make_phantom(cfg)
    x = synth.pixelize(cfg, ph, ss=2)
    rng = np.random.default_rng(seed)
    return x + rng.uniform(0.0, 0.002, x.shape)


@pytest.mark.parametrize("name,over,M", CASES)
def test_project_backproject_parity(L, name, over, M):
    cfg = synth.get_config(name, **over)
    say("case", name, over, "M", M)
    plan = L.lalm_plan_geometry(synth.geometry_of(cfg), M)
    # subset bookkeeping
    subs = ora.subset_views(cfg["n_views"], M)
    assert list(plan.order) == list(ora.bit_reversal_order(M))
    x = _image(cfg)
    xg = gpu(x)
    rng = np.random.default_rng(1)
    for m in range(M):
        views = plan.subset_views(m)
        assert list(views) == list(subs[m])
        assert int(plan.subset_samples[m]) == ora.count_samples(cfg, views)
        ref = ora.forward(cfg, x, views)
        out = torch.empty(plan.subset_rays(m), device=DEV)
        L.lalm_project_subset(plan, m, xg, out)
        got = out.cpu().numpy().reshape(ref.shape)
        e = rel_l2(got, ref)
        say("  fp m=%d rel=%.2e" % (m, e))
        assert e <= 1e-5
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
        r = rng.normal(size=ref.shape)
        refb = ora.back(cfg, r, views)
        xb = torch.empty(plan.image_elems, device=DEV)
        L.lalm_backproject_subset(plan, m, gpu(r).reshape(-1), xb, scale=1.0)
        gotb = xb.cpu().numpy().reshape(refb.shape)
        eb = rel_l2(gotb, refb)
        say("  bp m=%d rel=%.2e" % (m, eb))
        assert eb <= 1e-5
        assert np.abs(gotb - refb).max() <= 1e-5 * np.abs(refb).max()


@pytest.mark.parametrize("name,over,M", [CASES[0], CASES[3], CASES[5], CASES[6]])
def test_residual_mode_and_accumulate(L, name, over, M):
    cfg = synth.get_config(name, **over)
    plan = L.lalm_plan_geometry(synth.geometry_of(cfg), M)
    x = _image(cfg)
    rng = np.random.default_rng(2)
    m = M - 1
    views = plan.subset_views(m)
    ref = ora.forward(cfg, x, views)
    y = ref + rng.normal(0, 0.05, ref.shape)
    w = rng.uniform(0.5, 3.0, ref.shape)
    out = torch.empty(plan.subset_rays(m), device=DEV)
    L.lalm_project_subset(plan, m, gpu(x), out, y=gpu(y).reshape(-1), w=gpu(w).reshape(-1))
    got = out.cpu().numpy().reshape(ref.shape)
    want = w * (ref - y)
    assert np.abs(got - want).max() <= 1e-5 * np.abs(ref).max() * w.max()
    # accumulate = 1 adds to what is there
    r = rng.normal(size=ref.shape)
    base = rng.normal(size=ora.image_shape(cfg))
    xb = gpu(base).reshape(-1)
    L.lalm_backproject_subset(plan, m, gpu(r).reshape(-1), xb, scale=2.5, accumulate=True)
    want = base + 2.5 * ora.back(cfg, r, views)
    assert rel_l2(xb.cpu().numpy().reshape(want.shape), want) <= 1e-5


def _adjoint_check(L, plan, m, xg, rg):
    """<A_m x, r> and <x, A_m' r> (FP64 dots of the FP32 kernels' outputs)
    and the sum of |(A_m x)_i r_i|."""
    n = plan.subset_rays(m)
    ax = torch.empty(n, device=DEV)
    L.lalm_project_subset(plan, m, xg, ax)
    atr = torch.empty(plan.image_elems, device=DEV)
    L.lalm_backproject_subset(plan, m, rg, atr)
    d = torch.zeros(3, dtype=torch.float64, device=DEV)
    L.lalm_dot_f64(plan, ax, rg, d[0:1])
    L.lalm_dot_f64(plan, xg, atr, d[1:2])
    L.lalm_dot_f64(plan, ax.abs().contiguous(), rg.abs().contiguous(), d[2:3])
    return d.cpu().numpy()


@pytest.mark.parametrize("name,over,M", [CASES[3], CASES[4], CASES[5], CASES[6]])
def test_adjoint_identity_on_gpu(L, name, over, M):
    cfg = synth.get_config(name, **over)
    plan = L.lalm_plan_geometry(synth.geometry_of(cfg), M)
    rng = np.random.default_rng(3)
    xg = gpu(rng.uniform(0, 1, ora.image_shape(cfg))).reshape(-1)
    for m in range(M):
        rg = gpu(rng.normal(size=plan.subset_rays(m)))
        a, b, terms = _adjoint_check(L, plan, m, xg, rg)
        say("  adjoint m=%d <Ax,r>=%.9e <x,A'r>=%.9e |diff|/sum|Ax_i r_i|=%.2e" % (m, a, b, abs(a - b) / terms))
        assert abs(a - b) <= 1e-6 * terms


@pytest.mark.timeout(300)
@pytest.mark.parametrize("name,M", [("fan2d_512", 24), ("cone_axial_512x64", 12), ("cone_helical_512x256", 12)])
def test_adjoint_identity_full_size(L, name, M):
    """The matched pair at full size in the benchmark's launch configuration
    (the subset the first step projects): the 2D line kernel's staging and
    wide-window paths, the 3D forward projector's segment split and the
    helical view-range search all take part."""
    cfg = synth.get_config(name)
    say("full-size adjoint", name, "M", M)
    plan = L.lalm_plan_geometry(synth.geometry_of(cfg), M)
    rng = np.random.default_rng(4)
    xg = gpu(rng.uniform(0, 1, ora.image_shape(cfg)).astype(np.float32)).reshape(-1)
    m = int(plan.order[1])
    rg = gpu(rng.normal(size=plan.subset_rays(m)).astype(np.float32))
    a, b, terms = _adjoint_check(L, plan, m, xg, rg)
    say("  adjoint m=%d <Ax,r>=%.12e <x,A'r>=%.12e |diff|/sum|Ax_i r_i|=%.2e" % (m, a, b, abs(a - b) / terms))
    assert abs(a - b) <= 1e-6 * terms


@pytest.mark.parametrize("name,over", [("fan2d_128", {}), ("cone_axial_512x64", MED3D)])
def test_fp64_monitors_against_oracle(L, name, over):
    """lalm_dot_f64 against the FP64 sum of the same FP32 products (a length
    that is not a multiple of any block size) and lalm_roi_rmsd_f64 against
    the oracle's ROI RMS difference (Sec. V) of the same FP32 images."""
    cfg = synth.get_config(name, **over)
    plan = L.lalm_plan_geometry(synth.geometry_of(cfg), 2)
    rng = np.random.default_rng(21)
    n = 1_000_003
    a32 = rng.normal(size=n).astype(np.float32)
    b32 = rng.normal(size=n).astype(np.float32)
    out = torch.zeros(1, dtype=torch.float64, device=DEV)
    L.lalm_dot_f64(plan, gpu(a32), gpu(b32), out)
    a64, b64 = a32.astype(np.float64), b32.astype(np.float64)
    want = float(np.dot(a64, b64))
    terms = float(np.sum(np.abs(a64 * b64)))
    got = float(out.item())
    say("%s dot gpu %.15e oracle %.15e |diff|/sum|a_i b_i| %.2e" % (name, got, want, abs(got - want) / terms))
    assert abs(got - want) <= 1e-11 * terms
    shape = ora.image_shape(cfg)
    x1 = rng.uniform(0.0, 0.03, shape).astype(np.float32)
    x2 = (x1 + rng.normal(0.0, 1e-4, shape)).astype(np.float32)
    L.lalm_roi_rmsd_f64(plan, gpu(x1).reshape(-1), gpu(x2).reshape(-1), synth.roi_radius(cfg), out)
    got = float(out.item())
    want = ora.rmsd_hu(x1, x2, synth.roi_mask(cfg), 1.0)
    say("%s ROI RMSD gpu %.15e oracle %.15e" % (name, got, want))
    assert abs(got - want) <= 1e-11 * want


def _problem(cfg, seed=None):
    d = synth.make_problem_data(cfg, seed=seed, workers=1)
    return d


def _gpu_problem(L, cfg, M, data):
    plan = L.lalm_plan_geometry(synth.geometry_of(cfg), M)
    y = gpu(data["y"][plan.view_of_slot]).reshape(-1)
    w = gpu(data["w"][plan.view_of_slot]).reshape(-1)
    denom = torch.empty(plan.image_elems, device=DEV)
    L.lalm_sqs_denom(plan, w, denom)
    return plan, y, w, denom


@pytest.mark.parametrize("name,over,M", [CASES[0], CASES[1], CASES[3], CASES[5], CASES[6]])
def test_sqs_denominator_and_cost(L, name, over, M):
    """D_L = A^T (w .* A 1) and the FP64 cost.  In 3D the library's own
    projection pair passes residuals that already carry each ray's scale, so
    the cone cases check that path against the oracle's plain A^T W A 1."""
    cfg = synth.get_config(name, **over)
    data = _problem(cfg)
    plan, y, w, denom = _gpu_problem(L, cfg, M, data)
    ref = ora.sqs_denom(cfg, data["w"])
    got = denom.cpu().numpy().reshape(ref.shape)
    assert rel_l2(got, ref) <= 1e-5
    x = _image(cfg)
    beta = 1e-3 * float(np.median(ref[ref > 0]))
    delta = synth.configs.delta_mu(cfg)
    out = torch.zeros(3, dtype=torch.float64, device=DEV)
    L.lalm_cost_f64(plan, y, w, beta, delta, gpu(x).reshape(-1), out)
    c = out.cpu().numpy()
    # the oracle sees the same FP32-rounded image
    xr = gpu(x).cpu().numpy().astype(np.float64)
    cr = np.array(ora.cost(cfg, xr, data["y"], data["w"], beta, delta))
    say("cost gpu", c, "oracle", cr)
    assert abs(c[2] - cr[2]) <= 1e-9 * abs(cr[2])          # regularizer: FP64 from the same image
    assert abs(c[1] - cr[1]) <= 1e-4 * abs(cr[1])
    assert abs(c[0] - cr[0]) <= 1e-4 * abs(cr[0])


def _run_both(L, cfg, M, n_iter, continuation=True, rho_fixed=1.0, seed=None, n_inner=1):
    data = _problem(cfg, seed)
    beta = cfg["beta"]
    delta = synth.configs.delta_mu(cfg)
    n_steps = n_iter * M
    ref = ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=M, n_steps=n_steps,
                      continuation=continuation, rho_fixed=rho_fixed, n_inner=n_inner)
    plan, y, w, denom = _gpu_problem(L, cfg, M, data)
    st = L.LalmState.zeros_like(torch.zeros(plan.image_elems, device=DEV))
    stats = dict(rho=torch.zeros(n_steps, dtype=torch.float64, device=DEV),
                 xi=torch.zeros(n_steps, dtype=torch.float64, device=DEV),
                 restart=torch.zeros(n_steps, dtype=torch.uint8, device=DEV))
    L.lalm_iterate(plan, y, w, denom, beta, delta, st, n_steps, continuation=continuation,
                   rho_fixed=rho_fixed, stats=stats, n_inner=n_inner)
    return data, ref, plan, (y, w, denom, beta, delta), st, stats


def _report(cfg, ref, st, stats):
    mask = synth.roi_mask(cfg)
    xg = st.x.cpu().numpy().reshape(ora.image_shape(cfg))
    d = ora.rmsd_hu(xg, ref["x"], mask, synth.HU_PER_MU)
    rs = stats["restart"].cpu().numpy().astype(bool)
    xi = stats["xi"].cpu().numpy()
    mism = int(np.sum(rs != ref["restart"]))
    return d, mism, rs, xi


@pytest.mark.parametrize("name,M,n_iter", [("fan2d_128", 4, 20), ("tiny2d", 3, 10)])
def test_os_lalm_parity_free_running_and_replay(L, name, M, n_iter):
    cfg = synth.get_config(name)
    data, ref, plan, prob, st, stats = _run_both(L, cfg, M, n_iter)
    d, mism, rs, xi = _report(cfg, ref, st, stats)
    say("%s free-running: RMSD %.4f HU, restart mismatches %d / %d, restarts %d"
        % (name, d, mism, len(rs), int(rs.sum())))
    assert d <= 0.5
    # replay the oracle's restart sequence on the GPU
    y, w, denom, beta, delta = prob
    st2 = L.LalmState.zeros_like(torch.zeros(plan.image_elems, device=DEV))
    forced = gpu(ref["restart"].astype(np.uint8), torch.uint8)
    L.lalm_iterate(plan, y, w, denom, beta, delta, st2, len(ref["restart"]), forced_restart=forced)
    d2 = ora.rmsd_hu(st2.x.cpu().numpy().reshape(ora.image_shape(cfg)), ref["x"],
                     synth.roi_mask(cfg), synth.HU_PER_MU)
    say("%s replay: RMSD %.4f HU" % (name, d2))
    assert d2 <= 0.5
    rho_g = stats["rho"].cpu().numpy()
    if mism == 0:
        np.testing.assert_allclose(rho_g, ref["rho"], rtol=1e-12)


def _marginal(ref, hist, tol=1e-5):
    """Steps whose restart decision is marginal: |xi| < tol ||g - G+|| ||G+ - G||
    (g, G before the step, G+ after it), with that product per step."""
    g, G = hist["g"], hist["G"]
    n = len(ref["xi"])
    prod = np.array([np.linalg.norm(g[j] - G[j + 1]) * np.linalg.norm(G[j + 1] - G[j]) for j in range(n)])
    return np.nonzero(np.abs(ref["xi"]) < tol * prod)[0], prod


@pytest.mark.timeout(300)
def test_natural_restarts_free_running_and_replay(L):
    """One-subset OS-LALM with continuation on the 128^2 fan-beam problem
    restarts on its own (xi > 0, Sec. III-B) several times within 40 steps.
    Free-running, the GPU takes the same restart decisions as the FP64 oracle
    (a mismatch is allowed only at a marginal decision, |xi| below 1e-5
    ||g - G+|| ||G+ - G||, and the run after it is then a different valid
    trajectory), its FP64 xi agrees with the oracle's to 1e-3 of that scale,
    and the image is within 0.5 HU; replaying the oracle's restart bits
    gives the same."""
    cfg = synth.get_config("fan2d_128")
    M, n = 1, 40
    data = _problem(cfg)
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    hist = {"g": [], "G": []}
    ref = ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=M, n_steps=n, history=hist)
    n_rs = int(ref["restart"].sum())
    marg, prod = _marginal(ref, hist)
    say("oracle: %d restarts at steps %s; %d marginal decisions %s"
        % (n_rs, list(np.nonzero(ref["restart"])[0]), len(marg), list(marg)))
    assert n_rs >= 3
    plan, y, w, denom = _gpu_problem(L, cfg, M, data)
    st = L.LalmState.zeros_like(torch.zeros(plan.image_elems, device=DEV))
    stats = dict(rho=torch.zeros(n, dtype=torch.float64, device=DEV),
                 xi=torch.zeros(n, dtype=torch.float64, device=DEV),
                 restart=torch.zeros(n, dtype=torch.uint8, device=DEV))
    L.lalm_iterate(plan, y, w, denom, beta, delta, st, n, stats=stats)
    rs = stats["restart"].cpu().numpy().astype(bool)
    xi = stats["xi"].cpu().numpy()
    mism = np.nonzero(rs != ref["restart"])[0]
    first = int(mism[0]) if len(mism) else n
    exi = np.abs(xi[:first] - ref["xi"][:first]) / prod[:first]
    d = ora.rmsd_hu(st.x.cpu().numpy().reshape(ora.image_shape(cfg)), ref["x"], synth.roi_mask(cfg),
                    synth.HU_PER_MU)
    say("gpu free-running: %d restarts, mismatches at %s, max |xi err| / scale %.2e, RMSD %.2e HU"
        % (int(rs.sum()), list(mism), exi.max(), d))
    assert first == n or first in set(marg.tolist())
    assert exi.max() <= 1e-3
    assert d <= 0.5
    st2 = L.LalmState.zeros_like(torch.zeros(plan.image_elems, device=DEV))
    stats2 = {k: torch.zeros_like(v) for k, v in stats.items()}
    forced = gpu(ref["restart"].astype(np.uint8), torch.uint8)
    L.lalm_iterate(plan, y, w, denom, beta, delta, st2, n, forced_restart=forced, stats=stats2)
    d2 = ora.rmsd_hu(st2.x.cpu().numpy().reshape(ora.image_shape(cfg)), ref["x"], synth.roi_mask(cfg),
                     synth.HU_PER_MU)
    say("gpu replay: RMSD %.2e HU" % d2)
    assert np.array_equal(stats2["restart"].cpu().numpy().astype(bool), ref["restart"])
    np.testing.assert_allclose(stats2["rho"].cpu().numpy(), ref["rho"], rtol=1e-12)
    assert d2 <= 0.5


CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_cache")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,iters", [("cone_axial_512x64", "1 2 20"), ("cone_helical_512x256", "1 2")])
def test_full_size_iterations_against_oracle(L, name, iters):
    """The full 3D workloads (512x512x64 axial: 984 views, 888 x 64
    detector; 512x512x256 helical: 6888 views over 7 turns; M = 12,
    continuation, x0 = 0) against the FP64 oracle's own run of them, stored
    by tests/make_oracle_cache.py: D_L, and after every stored iteration
    count K the image on the sampled slices (ROI RMS difference <= 0.5 HU),
    the FP64 cost of the whole volume (relative 1e-4) and the restart
    decisions of every step so far."""
    path = os.path.join(CACHE, name + ".npz")
    if not os.path.exists(path):
        pytest.skip("no stored oracle run: python tests/make_oracle_cache.py %s --iters %s" % (name, iters))
    c = np.load(path)
    cfg = synth.get_config(name)
    M, beta, delta = int(c["M"]), float(c["beta"]), float(c["delta"])
    assert M == cfg["M"] and beta == cfg["beta"]
    ks = sorted(int(k[3:]) for k in c.files if k.startswith("x_k"))
    assert ks, "the stored run holds no image yet"
    sl = c["slices"]
    shape = ora.image_shape(cfg)
    say("full-size %s: synthetic data (host workers)" % name)
    # the default host worker pool: one worker takes many minutes on the helical scan
    data = synth.make_problem_data(cfg)
    say("full-size %s: data ready, planning and D_L" % name)
    plan, y, w, denom = _gpu_problem(L, cfg, M, data)
    e_dl = rel_l2(denom.reshape(shape)[sl].cpu().numpy(), c["DL"])
    say("full-size %s: D_L rel %.2e on slices %s; stored K %s" % (name, e_dl, list(sl), ks))
    assert e_dl <= 1e-5
    n = ks[-1] * M
    st = L.LalmState.zeros_like(torch.zeros(plan.image_elems, device=DEV))
    stats = dict(rho=torch.zeros(n, dtype=torch.float64, device=DEV),
                 xi=torch.zeros(n, dtype=torch.float64, device=DEV),
                 restart=torch.zeros(n, dtype=torch.uint8, device=DEV))
    mask = synth.roi_mask(cfg)[sl]
    out = torch.zeros(3, dtype=torch.float64, device=DEV)
    done = 0
    for K in ks:
        L.lalm_iterate(plan, y, w, denom, beta, delta, st, K * M - done, stats=stats)
        done = K * M
        xg = st.x.reshape(shape)[sl].cpu().numpy()
        d = ora.rmsd_hu(xg, c["x_k%d" % K], mask, synth.HU_PER_MU)
        L.lalm_cost_f64(plan, y, w, beta, delta, st.x, out)
        cg, co = out.cpu().numpy(), c["cost_k%d" % K]
        nr = min(done, len(c["restart"]))
        mism = int(np.sum(stats["restart"].cpu().numpy()[:nr].astype(bool) != c["restart"][:nr].astype(bool)))
        say("  K=%d: RMSD %.2e HU, Psi gpu %.9e oracle %.9e, restart mismatches %d / %d, restarts %d"
            % (K, d, cg[0], co[0], mism, nr, int(c["restart"][:nr].sum())))
        assert d <= 0.5
        assert abs(cg[0] - co[0]) <= 1e-4 * abs(co[0])


@pytest.mark.timeout(900)
def test_os_lalm_parity_fan2d_512(L):
    cfg = synth.get_config("fan2d_512")
    data, ref, plan, prob, st, stats = _run_both(L, cfg, cfg["M"], cfg["n_iter"])
    d, mism, rs, xi = _report(cfg, ref, st, stats)
    say("fan2d_512 free-running: RMSD %.4f HU, restart mismatches %d / %d" % (d, mism, len(rs)))
    assert d <= 0.5


@pytest.mark.parametrize("name,over,M,n_iter", [("cone_axial_512x64", MED3D, 5, 4),
                                                ("cone_helical_512x256", MEDHEL, 6, 3)])
def test_os_lalm_parity_3d(L, name, over, M, n_iter):
    """Free-running OS-LALM on medium 3D geometries (26-neighbour
    regularizer, cone-beam projector pair), beta from the problem's own D_L."""
    cfg = synth.get_config(name, **over)
    data = _problem(cfg)
    dl = ora.sqs_denom(cfg, data["w"])
    cfg["beta"] = synth.configs.BETA_REL * float(np.median(dl[synth.roi_mask(cfg)]))
    data, ref, plan, prob, st, stats = _run_both(L, cfg, M, n_iter)
    d, mism, rs, xi = _report(cfg, ref, st, stats)
    size = ora.rmsd_hu(ref["x"], np.zeros_like(ref["x"]), synth.roi_mask(cfg), synth.HU_PER_MU)
    say("%s (medium) free-running: RMSD %.2e HU (image RMS %.0f HU), restart mismatches %d / %d"
        % (name, d, size, mism, len(rs)))
    assert size > 20.0                      # a non-trivial image
    assert d <= 0.5


# full-size workloads with the subset counts the benchmark runs them with
FULL = [("fan2d_512", 24, 20), ("cone_axial_512x64", 12, 20), ("cone_helical_512x256", 12, 12)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,M,n_vox", FULL)
def test_full_size_sampled_parity(L, name, M, n_vox):
    """Full-size geometry in the benchmark's launch configuration: sampled
    rays of A_m x against the oracle's ray integrals, sampled voxels of
    A_m' r against the oracle's per-entry sums (same FP32-rounded inputs)."""
    cfg = synth.get_config(name)
    say("full-size sampled parity", name, "M", M)
    plan = L.lalm_plan_geometry(synth.geometry_of(cfg), M)
    shape = ora.image_shape(cfg)
    rng = np.random.default_rng(11)
    x32 = rng.uniform(0.0, 0.03, shape).astype(np.float32)
    xo = x32.astype(np.float64)
    m = int(plan.order[1])                       # the subset the first step projects
    n = plan.subset_rays(m)
    views = plan.subset_views(m)
    nr, nb = cfg["n_rows"], cfg["n_bins"]
    out = torch.empty(n, device=DEV)
    L.lalm_project_subset(plan, m, gpu(x32).reshape(-1), out)
    torch.cuda.synchronize()
    q = np.concatenate([rng.choice(n, 200, replace=False),
                        [0, nb - 1, nr * nb - 1, n - nb, n - 1, (n // 2) // nb * nb]])
    got = out.cpu().numpy()[q].astype(np.float64)
    ref = np.array([ora.ray_integral(cfg, xo, int(views[k // (nr * nb)]), int((k // nb) % nr), int(k % nb))
                    for k in q])
    efp = np.abs(got - ref).max() / np.abs(ref).max()
    say("  A_m x: %d rays, max err / max %.2e" % (len(q), efp))
    assert efp <= 1e-5
    r32 = rng.uniform(0.0, 1.0, n).astype(np.float32)
    xb = torch.empty(plan.image_elems, device=DEV)
    L.lalm_backproject_subset(plan, m, gpu(r32), xb)
    torch.cuda.synchronize()
    nz, ny, nx = shape
    vox = [(nz // 2, ny // 2, nx // 2), (0, ny // 2, 0), (nz - 1, ny // 3, nx - 1), (0, 0, 0)]
    vox += [tuple(int(rng.integers(0, d)) for d in shape) for _ in range(n_vox - len(vox))]
    gotb = xb.cpu().numpy().reshape(shape)[tuple(np.array(vox).T)].astype(np.float64)
    refb = ora.back_at_c(cfg, r32.astype(np.float64).reshape(len(views), nr, nb), views, vox)
    ebp = np.abs(gotb - refb).max() / np.abs(refb).max()
    say("  A_m' r: %d voxels, max err / max %.2e" % (len(vox), ebp))
    assert ebp <= 1e-5


@pytest.mark.parametrize("name,over,M,n_iter,n_inner", [("fan2d_128", {}, 4, 10, 2), ("fan2d_128", {}, 4, 10, 5),
                                                        ("cone_axial_512x64", MED3D, 5, 3, 3)])
def test_os_lalm_parity_inner_fista(L, name, over, M, n_iter, n_inner):
    """n_inner FISTA iterations on the inner problem (Sec. IV-A) against the
    oracle's, free-running; the inner iterates differ from n = 1, so the
    image must too."""
    cfg = synth.get_config(name, **over)
    if over:
        data = _problem(cfg)
        dl = ora.sqs_denom(cfg, data["w"])
        cfg["beta"] = synth.configs.BETA_REL * float(np.median(dl[synth.roi_mask(cfg)]))
    data, ref, plan, prob, st, stats = _run_both(L, cfg, M, n_iter, n_inner=n_inner)
    d, mism, rs, xi = _report(cfg, ref, st, stats)
    one = ora.os_lalm(cfg, data["y"], data["w"], cfg["beta"], synth.configs.delta_mu(cfg), M=M,
                      n_steps=n_iter * M)
    gap = ora.rmsd_hu(one["x"], ref["x"], synth.roi_mask(cfg), synth.HU_PER_MU)
    say("%s n_inner=%d: RMSD to oracle %.2e HU, restart mismatches %d / %d; n=1 vs n=%d differ by %.3f HU"
        % (name, n_inner, d, mism, len(rs), n_inner, gap))
    assert d <= 0.5
    assert gap > 10 * max(d, 1e-3)


@pytest.mark.parametrize("name,over,M,n_iter", [("fan2d_128", {}, 4, 12), ("cone_axial_512x64", MED3D, 5, 4)])
def test_os_lalm_parity_bb(L, name, over, M, n_iter):
    """Barzilai-Borwein scaling of D_L (supplement) against the oracle:
    images within 0.5 HU, the scale alpha of the last iteration to 1e-4, and
    splitting the run over two calls (the history lives in the caller's
    state) is bit-identical to one call."""
    cfg = synth.get_config(name, **over)
    data = _problem(cfg)
    if over:
        dl = ora.sqs_denom(cfg, data["w"])
        cfg["beta"] = synth.configs.BETA_REL * float(np.median(dl[synth.roi_mask(cfg)]))
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    n_steps = n_iter * M
    ref = ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=M, n_steps=n_steps, bb=True)
    plan, y, w, denom = _gpu_problem(L, cfg, M, data)
    st = L.LalmState.zeros_like(torch.zeros(plan.image_elems, device=DEV), bb=True)
    L.lalm_iterate(plan, y, w, denom, beta, delta, st, n_steps, bb=True)
    d = ora.rmsd_hu(st.x.cpu().numpy().reshape(ora.image_shape(cfg)), ref["x"], synth.roi_mask(cfg),
                    synth.HU_PER_MU)
    say("%s bb: RMSD %.2e HU, alpha gpu %.6f oracle %.6f (alphas %s)"
        % (name, d, st.alpha, ref["alpha"][-1], np.unique(np.round(ref["alpha"], 4))))
    assert d <= 0.5
    assert abs(st.alpha - ref["alpha"][-1]) <= 1e-4 * ref["alpha"][-1]
    assert ref["alpha"][-1] < 0.999
    st2 = L.LalmState.zeros_like(torch.zeros(plan.image_elems, device=DEV), bb=True)
    L.lalm_iterate(plan, y, w, denom, beta, delta, st2, n_steps // 2 + 1, bb=True)
    L.lalm_iterate(plan, y, w, denom, beta, delta, st2, n_steps - (n_steps // 2 + 1), bb=True)
    assert torch.equal(st.x, st2.x) and st.alpha == st2.alpha


@pytest.mark.timeout(300)
@pytest.mark.parametrize("name", ["fan2d_128", "fan2d_512"])
def test_fbp_parity(L, name):
    """GPU FBP of the noisy data against the oracle's (same textbook
    equiangular fan-beam formula in FP64): relative L2 <= 1e-4 and max error
    <= 1e-4 x max (FP32 filtering sums ~ n_bins terms of both signs)."""
    cfg = synth.get_config(name)
    data = _problem(cfg)
    ref = ora.fbp_fan(cfg, data["y"])
    plan = L.lalm_plan_geometry(synth.geometry_of(cfg), cfg["M"])
    y = gpu(data["y"][plan.view_of_slot]).reshape(-1)
    x = torch.empty(plan.image_elems, device=DEV)
    L.lalm_fbp(plan, y, x)
    got = x.cpu().numpy().reshape(ref.shape)
    e = rel_l2(got, ref)
    emax = np.abs(got - ref).max() / np.abs(ref).max()
    say("  fbp %s: rel L2 %.2e, max %.2e" % (name, e, emax))
    assert e <= 1e-4 and emax <= 1e-4


def test_fbp_rejects_helical(L):
    cfg = synth.get_config("tiny_helical")
    plan = L.lalm_plan_geometry(synth.geometry_of(cfg), 2)
    with pytest.raises(L.LalmError):
        L.lalm_fbp(plan, torch.zeros(plan.sino_elems, device=DEV), torch.zeros(plan.image_elems, device=DEV))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,over", [("cone_axial_512x64", MED3D), ("cone_axial_512x64", {})])
def test_fdk_parity(L, name, over):
    """GPU FDK of the noisy data of an axial cone-beam workload against the
    oracle's (same textbook formula in FP64): on the medium geometry the
    whole image, at full size (512x512x64, 984 views, 888 x 64 detector)
    sampled voxels, each within 1e-4 of the image's maximum."""
    cfg = synth.get_config(name, **over)
    data = _problem(cfg)
    plan = L.lalm_plan_geometry(synth.geometry_of(cfg), cfg["M"])
    y = gpu(data["y"][plan.view_of_slot]).reshape(-1)
    x = torch.empty(plan.image_elems, device=DEV)
    L.lalm_fbp(plan, y, x)
    got = x.cpu().numpy().reshape(ora.image_shape(cfg)).astype(np.float64)
    if not over:
        rng = np.random.default_rng(12)
        nz, ny, nx = ora.image_shape(cfg)
        vox = [(0, ny // 2, nx // 2), (nz - 1, ny // 2, nx // 2), (nz // 2, 0, 0), (nz // 2, ny - 1, nx - 1)]
        vox += [(int(rng.integers(0, nz)), int(rng.integers(ny // 4, 3 * ny // 4)),
                 int(rng.integers(nx // 4, 3 * nx // 4))) for _ in range(60)]
        ref = ora.fbp_cone_axial(cfg, data["y"], voxels=vox)
        g = np.array([got[v] for v in vox])
        scale = np.abs(got).max()
        emax = np.abs(g - ref).max() / scale
        say("  fdk %s: %d sampled voxels, max err / max %.2e" % (name, len(vox), emax))
        assert emax <= 1e-4
        return
    ref = ora.fbp_cone_axial(cfg, data["y"])
    e = rel_l2(got, ref)
    emax = np.abs(got - ref).max() / np.abs(ref).max()
    say("  fdk %s (medium): rel L2 %.2e, max %.2e" % (name, e, emax))
    assert e <= 1e-4 and emax <= 1e-4


def test_fixed_rho_parity(L):
    cfg = synth.get_config("fan2d_128")
    data, ref, plan, prob, st, stats = _run_both(L, cfg, 4, 10, continuation=False, rho_fixed=0.1)
    d, mism, rs, xi = _report(cfg, ref, st, stats)
    assert d <= 0.5
    assert np.all(stats["rho"].cpu().numpy() == 0.1)


def test_single_subset_rho_one_cost_monotone(L):
    cfg = synth.get_config("fan2d_128", nx=64, ny=64, dx=2.0, dy=2.0, n_views=90,
                           n_views_per_turn=90, n_bins=128, ds=2.4, beta=None)
    data = _problem(cfg)
    plan, y, w, denom = _gpu_problem(L, cfg, 1, data)
    dn = denom.cpu().numpy()
    beta = synth.configs.BETA_REL * float(np.median(dn[synth.roi_mask(cfg).ravel()]))
    delta = synth.configs.delta_mu(cfg)
    st = L.LalmState.zeros_like(torch.zeros(plan.image_elems, device=DEV))
    out = torch.zeros(3, dtype=torch.float64, device=DEV)
    costs = []
    for k in range(30):
        L.lalm_iterate(plan, y, w, denom, beta, delta, st, 1, continuation=False, rho_fixed=1.0)
        L.lalm_cost_f64(plan, y, w, beta, delta, st.x, out)
        costs.append(float(out[0].item()))
    c = np.array(costs)
    assert np.all(np.diff(c) <= 1e-6 * abs(c[0]))
    assert c[-1] < c[0]


def test_determinism_and_checkpoint_resume(L):
    cfg = synth.get_config("fan2d_128")
    data = _problem(cfg)
    plan, y, w, denom = _gpu_problem(L, cfg, 4, data)
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    z = torch.zeros(plan.image_elems, device=DEV)
    a = L.LalmState.zeros_like(z.clone())
    L.lalm_iterate(plan, y, w, denom, beta, delta, a, 40)
    b = L.LalmState.zeros_like(z.clone())
    L.lalm_iterate(plan, y, w, denom, beta, delta, b, 40)
    assert torch.equal(a.x, b.x) and torch.equal(a.g, b.g) and a.rho == b.rho and a.l == b.l
    c = L.LalmState.zeros_like(z.clone())
    L.lalm_iterate(plan, y, w, denom, beta, delta, c, 17)
    saved = c.clone()
    del c
    plan2 = L.lalm_plan_geometry(synth.geometry_of(cfg), 4)    # resume on a fresh plan
    L.lalm_iterate(plan2, y, w, denom, beta, delta, saved, 23)
    assert saved.step == 40
    assert torch.equal(a.x, saved.x) and torch.equal(a.g, saved.g) and torch.equal(a.grad, saved.grad)
    assert a.rho == saved.rho and a.l == saved.l


@pytest.mark.parametrize("mode", ["continuation", "fixed", "forced"])
def test_fused_steps_equal_single_steps(L, mode):
    """Within one call of several 2D steps the step kernel also computes the
    next x for both values the pending decision can give rho, and the next
    forward projection picks one; single-step calls take no such shortcut.
    Both are the same arithmetic: x, g, G, rho, l and the recorded restart
    indicators are bit-identical, with the continuation, a fixed rho and a
    forced restart pattern."""
    cfg = synth.get_config("fan2d_128")
    data = _problem(cfg)
    M, n = 4, 36
    plan, y, w, denom = _gpu_problem(L, cfg, M, data)
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    kw = dict(continuation=mode != "fixed", rho_fixed=0.1)
    if mode == "forced":
        pat = np.zeros(n, dtype=np.uint8)
        pat[[3, 4, 11, 20, 21, 22, 30]] = 1
        kw["forced_restart"] = gpu(pat, torch.uint8)

    def stats():
        return dict(rho=torch.zeros(n, dtype=torch.float64, device=DEV),
                    xi=torch.zeros(n, dtype=torch.float64, device=DEV),
                    restart=torch.zeros(n, dtype=torch.uint8, device=DEV))
    z = torch.zeros(plan.image_elems, device=DEV)
    a, sa = L.LalmState.zeros_like(z.clone()), stats()
    L.lalm_iterate(plan, y, w, denom, beta, delta, a, n, stats=sa, **kw)
    b, sb = L.LalmState.zeros_like(z.clone()), stats()
    for _ in range(n):
        L.lalm_iterate(plan, y, w, denom, beta, delta, b, 1, stats=sb, **kw)
    restarts = int(sa["restart"].sum().item())
    say("fused vs single steps (%s): %d restarts, rho %.6f, l %d" % (mode, restarts, a.rho, a.l))
    assert torch.equal(a.x, b.x) and torch.equal(a.g, b.g) and torch.equal(a.grad, b.grad)
    assert a.rho == b.rho and a.l == b.l and a.step == b.step == n
    for k in ("rho", "xi", "restart"):
        assert torch.equal(sa[k], sb[k]), k
    if mode == "forced":
        assert np.array_equal(sa["restart"].cpu().numpy(), pat)


def test_nonfinite_data_is_reported_and_image_stays_finite(L):
    cfg = synth.get_config("fan2d_128")
    data = _problem(cfg)
    plan, y, w, denom = _gpu_problem(L, cfg, 4, data)
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    st = L.LalmState.zeros_like(torch.zeros(plan.image_elems, device=DEV))
    L.lalm_iterate(plan, y, w, denom, beta, delta, st, 6)
    good = st.x.clone()
    ybad = y.clone()
    s = plan.subset_slice(int(plan.order[(st.step + 1) % 4]))
    ybad[s.start + 100] = float("nan")
    with pytest.raises(L.LalmError) as ei:
        L.lalm_iterate(plan, ybad, w, denom, beta, delta, st, 5)
    assert ei.value.status == L.LALM_E_NONFINITE
    assert torch.isfinite(st.x).all()
    assert st.step == 7
    # the failing step's image update used finite gradients
    assert not torch.equal(st.x, good)


def test_fused_steps_stop_like_single_steps(L):
    """A non-finite restart indicator met a few steps into a call (the
    forward projection that takes the decision finds it): the call reports
    it and leaves x, g, G and the step count exactly as single-step calls do
    (x is the last accepted iterate, not a speculative candidate)."""
    cfg = synth.get_config("fan2d_128")
    data = _problem(cfg)
    M = 4
    plan, y, w, denom = _gpu_problem(L, cfg, M, data)
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    z = torch.zeros(plan.image_elems, device=DEV)
    a = L.LalmState.zeros_like(z.clone())
    L.lalm_iterate(plan, y, w, denom, beta, delta, a, 5)
    b = a.clone()
    # poison the subset projected three steps into the next call
    ybad = y.clone()
    s = plan.subset_slice(int(plan.order[(a.step + 3) % M]))
    ybad[s.start + 50] = float("nan")
    with pytest.raises(L.LalmError) as ea:
        L.lalm_iterate(plan, ybad, w, denom, beta, delta, a, 8)
    assert ea.value.status == L.LALM_E_NONFINITE
    for _ in range(8):
        try:
            L.lalm_iterate(plan, ybad, w, denom, beta, delta, b, 1)
        except L.LalmError as eb:
            assert eb.status == L.LALM_E_NONFINITE
            break
    else:
        raise AssertionError("single steps did not meet the non-finite indicator")
    say("stopped at step %d (fused call) / %d (single steps)" % (a.step, b.step))
    assert a.step == b.step
    assert torch.isfinite(a.x).all()
    assert torch.equal(a.x, b.x)
    assert torch.equal(torch.nan_to_num(a.g, nan=7.0), torch.nan_to_num(b.g, nan=7.0))
    assert torch.equal(torch.nan_to_num(a.grad, nan=7.0), torch.nan_to_num(b.grad, nan=7.0))


def test_edge_cases(L):
    # every subset a single view; one subset; zero steps
    cfg = synth.get_config("tiny2d")
    data = _problem(cfg)
    for M in (1, cfg["n_views"]):
        plan, y, w, denom = _gpu_problem(L, cfg, M, data)
        st = L.LalmState.zeros_like(torch.zeros(plan.image_elems, device=DEV))
        L.lalm_iterate(plan, y, w, denom, 1e-3, 2e-4, st, 0)
        assert st.step == 0 and torch.count_nonzero(st.x) == 0
        assert torch.count_nonzero(st.grad) > 0
        L.lalm_iterate(plan, y, w, denom, 1e-3, 2e-4, st, 2 * M)
        assert st.step == 2 * M and torch.isfinite(st.x).all()
    for bad in (0, 17):
        with pytest.raises(L.LalmError):
            L.lalm_iterate(plan, y, w, denom, 1e-3, 2e-4, st, 1, n_inner=bad)
    with pytest.raises(L.LalmError):
        L.lalm_project_subset(plan, M, torch.zeros(plan.image_elems, device=DEV),
                              torch.zeros(16, device=DEV))
