"""Pins of the FP64 oracle's algorithm against the paper and the mathematics.

* D_L = A'WA1 majorizes A'WA (dense eigenvalue check), Sec. II-A / IV-A;
* grad R against central finite differences; D_R majorizes R;
* the textbook linearized AL with u, d (Sec. II-A) and the gradient form
  (Sec. III-A) give the same iterates, and u + rho d = y (eq. "u_d_identity");
* the projector-based OS-LALM with M = 1 equals the dense gradient form;
* rho = 1, M = 1 is ISTA/majorize-minimize: the cost never increases;
* the toy quadratic's iteration matrix has the roots of eq. "char_poly_qp";
  critical damping, the over-damped rate and the measured contraction;
* the rho_l schedule equals the critical value at the estimated mu/L
  (both printed forms of eq. "opt_rho_r_qp"), decreases and hits rho_min;
* restarts on a quadratic come about every (pi/2) sqrt(L/mu) iterations;
* bit-reversal order; maximum number of subsets (Sec. IV-B vs Sec. V-B);
* M = 1 with continuation and FISTA with restart reach the same minimizer.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as ora
import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def small2d(**kw):
    base = dict(nx=32, ny=32, dx=4.0, dy=4.0, n_views=60, n_views_per_turn=60,
                n_bins=64, ds=4.8, n_ellipses=6, seed=21)
    base.update(kw)
    return synth.get_config("fan2d_128", **base)


def _beta(cfg, w):
    DL = ora.sqs_denom(cfg, w)
    mask = synth.roi_mask(cfg)
    return 2.0 ** -6 * float(np.median(DL[mask])), DL


def test_sqs_denominator_majorizes():
    cfg = synth.get_config("tiny2d")
    A = ora.dense(cfg)
    rng = np.random.default_rng(1)
    w = rng.uniform(0.5, 2.0, A.shape[0])
    DL = ora.sqs_denom(cfg, w.reshape(cfg["n_views"], 1, cfg["n_bins"])).ravel()
    np.testing.assert_allclose(DL, A.T @ (w * (A @ np.ones(A.shape[1]))), rtol=1e-12)
    H = A.T @ (w[:, None] * A)
    lam = np.linalg.eigvalsh(np.diag(DL) - H)
    assert lam.min() >= -1e-12 * np.abs(H).max()
    v = rng.normal(size=A.shape[1])
    assert v @ (DL * v) >= v @ H @ v


@pytest.mark.parametrize("is3d", [False, True])
def test_regularizer_gradient_and_majorizer(is3d):
    rng = np.random.default_rng(2)
    shape = (4, 6, 5) if is3d else (1, 7, 6)
    delta = 2e-4
    beta = 3.0
    x = rng.uniform(0.0, 1e-3, shape)
    g = ora.reg_grad(x, beta, delta, is3d)
    h = 1e-8
    for _ in range(12):
        idx = tuple(rng.integers(0, n) for n in shape)
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (ora.reg_value(xp, beta, delta, is3d) - ora.reg_value(xm, beta, delta, is3d)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(abs(g[idx]), 1e-3)
    DR = ora.reg_denom(shape, beta, is3d)
    # interior voxel: 2 beta (4 + 4/sqrt2) in 2D; 2 beta (6 + 12/sqrt2 + 8/sqrt3) in 3D
    c = (2, 3, 2) if is3d else (0, 3, 2)
    expect = 2 * beta * ((6 + 12 / math.sqrt(2) + 8 / math.sqrt(3)) if is3d else (4 + 4 / math.sqrt(2)))
    assert abs(DR[c] - expect) < 1e-12 * expect
    R0 = ora.reg_value(x, beta, delta, is3d)
    for _ in range(20):
        d = rng.normal(0.0, 1e-3, shape)
        assert ora.reg_value(x + d, beta, delta, is3d) <= R0 + np.sum(g * d) + 0.5 * np.sum(DR * d * d) + 1e-15


def _tiny_problem():
    cfg = synth.get_config("tiny2d")
    data = synth.make_problem_data(cfg, workers=1)
    A = ora.dense(cfg)
    y = data["y"].ravel()
    w = data["w"].ravel()
    DL = A.T @ (w * (A @ np.ones(A.shape[1])))
    return cfg, data, A, y, w, DL


@pytest.mark.parametrize("rho", [1.0, 0.5, 0.1])
def test_textbook_and_gradient_lalm_agree(rho):
    cfg, data, A, y, w, DL = _tiny_problem()
    shape = ora.image_shape(cfg)
    beta, delta = 1e-3 * float(np.median(DL)), 2e-4
    reg = lambda x: ora.reg_grad(x.reshape(shape), beta, delta, False).ravel()
    DR = ora.reg_denom(shape, beta, False).ravel()
    xs_t, ident = ora.lalm_textbook_dense(A, y, w, rho, 25, DL, reg=reg, DR=DR)
    xs_g = ora.lalm_gradient_dense(A, y, w, rho, 25, DL, reg=reg, DR=DR)
    scale = max(np.abs(xs_g[-1]).max(), 1e-12)
    for a, b in zip(xs_t, xs_g):
        assert np.abs(a - b).max() <= 1e-12 * scale * 10
    ys = np.sqrt(w) * y
    for v in ident:                       # eq. "u_d_identity"
        assert np.abs(v - ys).max() <= 1e-10 * np.abs(ys).max()
    assert np.abs(xs_g[-1] - xs_g[0]).max() > 0


def test_projector_os_lalm_matches_dense_gradient_form():
    cfg, data, A, y, w, DL = _tiny_problem()
    shape = ora.image_shape(cfg)
    beta, delta = 1e-3 * float(np.median(DL)), 2e-4
    reg = lambda x: ora.reg_grad(x.reshape(shape), beta, delta, False).ravel()
    DR = ora.reg_denom(shape, beta, False).ravel()
    for rho in (1.0, 0.3):
        xs_g = ora.lalm_gradient_dense(A, y, w, rho, 8, DL, reg=reg, DR=DR)
        out = ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=1, n_steps=8,
                          continuation=False, rho_fixed=rho)
        np.testing.assert_allclose(out["x"].ravel(), xs_g[-1], rtol=0,
                                   atol=1e-11 * np.abs(xs_g[-1]).max())


def test_rho_one_single_subset_is_monotone():
    cfg = small2d()
    data = synth.make_problem_data(cfg, workers=1)
    beta, DL = _beta(cfg, data["w"])
    delta = synth.configs.delta_mu(cfg)
    costs = []
    ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=1, n_steps=30,
                continuation=False, rho_fixed=1.0, denom=DL,
                callback=lambda j, x: costs.append(ora.cost(cfg, x, data["y"], data["w"], beta, delta)[0]))
    c = np.array(costs)
    assert np.all(np.diff(c) <= 1e-12 * abs(c[0]))
    assert c[-1] < c[0]


def test_continuation_is_not_monotone_but_faster():
    cfg = small2d()
    data = synth.make_problem_data(cfg, workers=1)
    beta, DL = _beta(cfg, data["w"])
    delta = synth.configs.delta_mu(cfg)
    f = lambda x: ora.cost(cfg, x, data["y"], data["w"], beta, delta)[0]
    a = ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=1, n_steps=40,
                    continuation=False, rho_fixed=1.0, denom=DL)
    b = ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=1, n_steps=40,
                    continuation=True, denom=DL)
    assert f(b["x"]) < f(a["x"])
    assert b["rho"][0] == 1.0 and b["rho"].min() < 0.5


@pytest.mark.parametrize("q,rho", [(0.3, 0.9), (0.05, 0.2), (0.7, 0.3), (0.01, 0.05), (0.5, 1.0)])
def test_toy_iteration_roots_match_characteristic_polynomial(q, rho):
    T = ora.toy_iteration_matrix(q, rho)
    eig = np.sort_complex(np.linalg.eigvals(T).astype(complex))
    roots = np.sort_complex(np.roots(ora.toy_char_poly(q, rho)).astype(complex))
    np.testing.assert_allclose(eig, roots, atol=1e-12)
    assert abs(max(abs(eig)) - ora.toy_rate(q, rho)) < 1e-10
    # measured per-component contraction of the full recursion: envelope of
    # |x_k| over windows longer than the oscillation period
    xs, _, _ = ora.toy_run([q], 1.0, 700, rho=rho)
    env = lambda k: np.abs(xs[k:k + 60, 0]).max()
    if env(600) > 1e-280:
        meas = (env(600) / env(100)) ** (1 / 500.0)
        assert abs(meas - ora.toy_rate(q, rho)) < 5e-3


def test_toy_critical_damping_and_under_damped_modulus():
    for q in (0.01, 0.2, 0.5, 0.8):
        rc = ora.toy_rho_critical(q)
        a, b, c = ora.toy_char_poly(q, rc)
        assert abs(b * b - 4 * a * c) < 1e-12                      # repeated root
        r = -b / (2 * a)
        assert abs(r - math.sqrt((1 - q) / (1 + rc))) < 1e-12      # eq. critical_damp_rate_qp
        assert ora.toy_rate(q, rc * 1.5) >= r - 1e-12               # over-damped is no faster
    # under-damped: the paper's printed rate is the real part of the root pair
    q, rho = 0.7, 0.3
    roots = np.roots(ora.toy_char_poly(q, rho))
    assert np.iscomplexobj(roots)
    printed = (1 - q + rho / 2) / (1 + rho)
    assert abs(roots[0].real - printed) < 1e-12
    assert abs(abs(roots[0]) - 0.48038446141526137) < 1e-9
    assert abs(ora.toy_rate(q, rho) - abs(roots[0])) < 1e-12


def test_rho_schedule():
    rho_min = GOLDEN["rho_min"]["value"]
    assert ora.rho_l(0, rho_min) == GOLDEN["rho_0"]["value"]
    prev = 1.0
    for l in range(1, 4000):
        r = ora.rho_l(l, rho_min)
        # second printed form of eq. "opt_rho_r_qp": the critical value at the
        # estimate sqrt(mu/L) = pi/(2r) with r = l + 1
        q = (math.pi / (2 * (l + 1))) ** 2
        assert abs(r - max(2 * math.sqrt(q * (1 - q)), rho_min)) < 1e-14
        assert r <= prev
        prev = r
    first_min = next(l for l in range(1, 10000) if ora.rho_l(l, rho_min) == rho_min)
    assert first_min == 3141
    assert abs(ora.rho_l(1) - 0.972309) < 1e-6 and abs(ora.rho_l(10) - 0.282672) < 1e-6


def test_restart_period_on_quadratic():
    """Sec. III-B: with a small rho, xi first turns positive about
    (pi/2) sqrt(L/mu) iterations after a (re)start, and then oscillates with
    period pi / psi_1 ~ pi sqrt(L/mu)."""
    L = 1.0
    for mu in (1e-3, 4e-4):
        expect = GOLDEN["restart_period_factor"]["value"] * math.sqrt(L / mu)
        # the slowest eigen-component alone
        _, _, xis = ora.toy_run([mu], L, 2000, rho=1e-3)
        pos = np.flatnonzero(xis > 0)
        starts = pos[np.r_[True, np.diff(pos) > 1]]
        assert abs(starts[0] - expect) <= 0.3 * expect
        assert abs(np.median(np.diff(starts)) - 2 * expect) <= 0.3 * 2 * expect
        # with faster components added, only the slowest one persists
        _, _, xis = ora.toy_run([mu, 0.3, L], L, 3000, rho=1e-3, x0=np.ones(3))
        pos = np.flatnonzero(xis[600:] > 0)
        starts = pos[np.r_[True, np.diff(pos) > 1]]
        assert abs(np.median(np.diff(starts)) - 2 * expect) <= 0.3 * 2 * expect
    # with the downward continuation, restarts recur and rho stays in (0, 1]
    _, restarts, _ = ora.toy_run([1e-3, 0.5, L], L, 1500, continuation=True, x0=np.ones(3))
    assert len(restarts) >= 3


def test_bit_reversal_order():
    assert list(ora.bit_reversal_order(4)) == [0, 2, 1, 3]
    assert list(ora.bit_reversal_order(8)) == [0, 4, 2, 6, 1, 5, 3, 7]
    assert list(ora.bit_reversal_order(1)) == [0]
    for M in (3, 12, 24, 41):
        o = ora.bit_reversal_order(M)
        assert sorted(o) == list(range(M))
        B = math.ceil(math.log2(M))
        full = [int(format(j, "0%db" % B)[::-1], 2) for j in range(1 << B)]
        assert list(o) == [v for v in full if v < M]


def test_max_subsets():
    s_ax = GOLDEN["s_axial"]["value"]
    n = GOLDEN["gepp_axial_views"]["value"]
    assert int(ora.max_subsets_axial(n, s_ax)) == GOLDEN["gepp_max_subsets_about"]["value"]
    # helical: inversely proportional to the pitch
    a = ora.max_subsets_helical(984, 541.0, 949.0, 0.5, GOLDEN["s_helical"]["value"])
    b = ora.max_subsets_helical(984, 541.0, 949.0, 1.0, GOLDEN["s_helical"]["value"])
    assert abs(a / b - 2.0) < 1e-12


@pytest.mark.slow
def test_single_subset_continuation_reaches_fista_minimizer():
    cfg = small2d()
    data = synth.make_problem_data(cfg, workers=1)
    beta, DL = _beta(cfg, data["w"])
    delta = synth.configs.delta_mu(cfg)
    x0 = np.zeros(ora.image_shape(cfg))
    xs = ora.fista_restart(cfg, data["y"], data["w"], beta, delta, x0, 1500, denom=DL)
    out = ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=1, n_steps=1500,
                      continuation=True, denom=DL)
    mask = synth.roi_mask(cfg)
    assert ora.rmsd_hu(out["x"], xs, mask, synth.HU_PER_MU) < 0.05


# ---------------------------------------------------------------- inner FISTA (n > 1)

def _inner_case(beta_scale=1.0, seed=7):
    cfg = synth.get_config("tiny2d")
    rng = np.random.default_rng(seed)
    shape = ora.image_shape(cfg)
    x = rng.uniform(0.0, 0.03, shape)
    x[0, 0, :3] = 0.0                                  # some voxels on the constraint
    DL = rng.uniform(0.5, 2.0, shape) * 1e3
    s = rng.normal(0.0, 20.0, shape)
    beta = beta_scale * 5.0
    delta = synth.configs.delta_mu(cfg)
    DR = ora.reg_denom(shape, beta, False)
    return x, s, DL, DR, beta, delta


def test_inner_fista_one_step_is_the_projected_gradient_step():
    x, s, DL, DR, beta, delta = _inner_case()
    rho = 0.3
    v = ora.inner_fista(x, s, DL, DR, rho, beta, delta, False, 1)
    ref = np.maximum(x - (s + ora.reg_grad(x, beta, delta, False)) / (rho * DL + DR), 0.0)
    assert np.array_equal(v, ref)


def test_inner_fista_without_regularizer_is_the_separable_closed_form():
    """beta = 0: the inner problem separates, z* = max(0, x - s / (rho D_L)),
    reached by the first step and kept by every later one."""
    x, s, DL, DR, beta, delta = _inner_case(beta_scale=0.0)
    rho = 0.2
    closed = np.maximum(x - s / (rho * DL), 0.0)
    for n in (1, 2, 5):
        v = ora.inner_fista(x, s, DL, DR, rho, 0.0, delta, False, n)
        np.testing.assert_allclose(v, closed, rtol=1e-12, atol=1e-15)


def test_inner_fista_converges_to_the_bound_constrained_minimizer():
    """Many FISTA iterations reach the minimizer found by an independent
    bound-constrained quasi-Newton solver (scipy L-BFGS-B), and the inner
    objective falls from n = 1 to n = 5."""
    from scipy.optimize import minimize
    x, s, DL, DR, beta, delta = _inner_case()
    rho = 0.1
    shape = x.shape
    f = lambda z: ora.inner_objective(z.reshape(shape), x, s, DL, rho, beta, delta, False)
    jac = lambda z: (rho * DL * (z.reshape(shape) - x) + s
                     + ora.reg_grad(z.reshape(shape), beta, delta, False)).ravel()
    res = minimize(f, x.ravel(), jac=jac, method="L-BFGS-B", bounds=[(0.0, None)] * x.size,
                   options=dict(ftol=1e-15, gtol=1e-12, maxiter=10000))
    v = ora.inner_fista(x, s, DL, DR, rho, beta, delta, False, 3000)
    assert np.max(np.abs(v.ravel() - res.x)) <= 1e-6 * max(1e-3, np.max(np.abs(res.x)))
    f1 = f(ora.inner_fista(x, s, DL, DR, rho, beta, delta, False, 1).ravel())
    f5 = f(ora.inner_fista(x, s, DL, DR, rho, beta, delta, False, 5).ravel())
    assert f5 < f1
    assert f(v.ravel()) <= f5 + 1e-12 * abs(f5)


def test_os_lalm_n_inner_one_matches_the_default():
    cfg = synth.get_config("tiny2d")
    d = synth.make_problem_data(cfg, workers=1)
    a = ora.os_lalm(cfg, d["y"], d["w"], cfg["beta"], synth.configs.delta_mu(cfg), M=3, n_steps=6)
    b = ora.os_lalm(cfg, d["y"], d["w"], cfg["beta"], synth.configs.delta_mu(cfg), M=3, n_steps=6, n_inner=1)
    assert np.array_equal(a["x"], b["x"])


# ---------------------------------------------------------------- Barzilai-Borwein scale

def test_bb_alpha_is_the_constrained_weighted_least_squares_fit():
    """alpha = argmin_{alpha <= 1} 1/2 ||y - alpha L s||^2_{L^-1}, checked by a
    bounded scalar minimization of that objective (independent of the closed
    form), for a fit below 1 and one capped at 1."""
    from scipy.optimize import minimize_scalar
    rng = np.random.default_rng(3)
    L = rng.uniform(0.5, 3.0, 200)
    s = rng.normal(size=200)
    for scale in (0.3, 4.0):
        yv = scale * L * s + rng.normal(0.0, 0.05, 200)
        obj = lambda a: 0.5 * np.sum((yv - a * L * s) ** 2 / L)
        ref = minimize_scalar(obj, bounds=(-10.0, 1.0), method="bounded", options=dict(xatol=1e-12)).x
        got = ora.bb_alpha(s, yv, L, 1e-3)
        assert got == pytest.approx(ref, abs=1e-6)
    assert ora.bb_alpha(s, -L * s, L, 1e-3) == 1.0               # no curvature information
    assert ora.bb_alpha(s, 1e-6 * L * s, L, 0.01) == 0.01        # floor


def test_bb_on_a_quadratic_fits_the_curvature_along_the_step():
    """One subset, beta = 0: y = A'WA s exactly, so alpha is the Rayleigh
    quotient s'A'WA s / s'D_L s of the step (below 1 because D_L majorizes
    A'WA), and the run records it from the second iteration on."""
    cfg = synth.get_config("tiny2d")
    d = synth.make_problem_data(cfg, workers=1)
    DL = ora.sqs_denom(cfg, d["w"])
    r = ora.os_lalm(cfg, d["y"], d["w"], 0.0, synth.configs.delta_mu(cfg), M=1, n_steps=4,
                    continuation=False, rho_fixed=1.0, bb=True, denom=DL)
    assert r["alpha"][0] == 1.0
    a = r["alpha"][1:]
    assert np.all((a > 0.0) & (a <= 1.0)) and np.any(a < 0.999)
    # alpha_1 recomputed from the first two iterates by the Rayleigh quotient
    r1 = ora.os_lalm(cfg, d["y"], d["w"], 0.0, synth.configs.delta_mu(cfg), M=1, n_steps=1,
                     continuation=False, rho_fixed=1.0, denom=DL)
    s = r1["x"] - np.zeros_like(r1["x"])
    Ad = ora.forward(cfg, s)
    rq = float(np.sum(d["w"] * Ad * Ad)) / float(np.sum(DL * s * s))
    assert a[0] == pytest.approx(rq, rel=1e-9)


def test_os_lalm_without_bb_is_unchanged():
    cfg = synth.get_config("tiny2d")
    d = synth.make_problem_data(cfg, workers=1)
    a = ora.os_lalm(cfg, d["y"], d["w"], cfg["beta"], synth.configs.delta_mu(cfg), M=3, n_steps=6)
    assert np.all(a["alpha"] == 1.0)


@pytest.mark.parametrize("is3d", [False, True])
def test_identical_subsets_reduce_to_one_subset(is3d):
    """Pin of the M > 1 path.  With V view angles per turn, V coprime to M,
    M turns (n_views = M V, the angle of view v is 2 pi v / V) and the data
    of an angle repeated in every turn, subset m = {v : v mod M = m} holds
    every angle exactly once, so M grad l_m = grad l exactly: the subset
    approximation of Sec. III-A is then exact, and OS-LALM with M subsets
    must follow, subset step for subset step, the one-subset method on the
    same data (itself pinned above against the dense gradient form and the
    textbook u, d form) -- the same images, the same restart decisions and
    rho values.  This pins what depends on M in the step (the factor M of the
    subset gradient, a per-step gradient taken on a subset rather than on all
    views); with identical subsets it cannot see which subset a step visits,
    so the subsets' own structure is checked as well: they partition the
    views, subset m starts at view m and steps by M (views spread uniformly
    over the scan, Sec. IV-B), and their sizes differ by at most one."""
    V, M = 13, 4
    assert math.gcd(V, M) == 1
    if is3d:    # axial cone beam: the angles also repeat every turn
        cfg = synth.get_config("tiny3d", nx=16, ny=16, nz=6, dx=2.0, dy=2.0, dz=2.0, dso=60.0,
                               dsd=120.0, n_bins=40, ds=2.5, n_rows=8, dt=2.0,
                               n_views=M * V, n_views_per_turn=V)
    else:
        cfg = small2d(n_views=M * V, n_views_per_turn=V)
    data = synth.make_problem_data(cfg, workers=1)
    y = np.concatenate([data["y"][:V]] * M)
    w = np.concatenate([data["w"][:V]] * M)
    for m, views in enumerate(ora.subset_views(cfg["n_views"], M)):
        assert sorted(int(v) % V for v in views) == list(range(V)), m
    for n_views, Ms in ((52, 4), (53, 4), (90, 7), (24, 24), (10, 1)):
        subs = [np.asarray(sv) for sv in ora.subset_views(n_views, Ms)]
        allv = np.sort(np.concatenate(subs))
        assert np.array_equal(allv, np.arange(n_views))
        sizes = [len(sv) for sv in subs]
        assert max(sizes) - min(sizes) <= 1
        for m, sv in enumerate(subs):
            assert sv[0] == m and np.all(np.diff(sv) == Ms)
    beta, DL = _beta(cfg, w)
    delta = synth.configs.delta_mu(cfg)
    n_steps = 10 * M
    rM = ora.os_lalm(cfg, y, w, beta, delta, M=M, n_steps=n_steps, denom=DL)
    r1 = ora.os_lalm(cfg, y, w, beta, delta, M=1, n_steps=n_steps, denom=DL)
    scale = float(np.abs(r1["x"]).max())
    assert scale > 0
    np.testing.assert_allclose(rM["x"], r1["x"], rtol=1e-9, atol=1e-12 * scale)
    np.testing.assert_allclose(rM["G"], r1["G"], rtol=1e-9, atol=1e-12 * float(np.abs(r1["G"]).max()))
    assert np.array_equal(rM["restart"], r1["restart"])
    np.testing.assert_allclose(rM["rho"], r1["rho"], rtol=0, atol=0)
    # the 2D run does restart and continue, so both branches of the rule are covered
    if not is3d:
        assert rM["restart"].any() and not rM["restart"].all()
    # and with genuinely different subsets (data of every view kept) the two differ
    rD = ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=M, n_steps=n_steps)
    r1D = ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=1, n_steps=n_steps)
    assert np.abs(rD["x"] - r1D["x"]).max() > 1e-6 * scale


# ------------------------------------------------ pins of xi and of the cost

def _dense_grad(A, y, w):
    """grad l(x) = A'W(Ax - y) from the per-entry dense matrix."""
    return lambda x: A.T @ (w * (A @ x - y))


def test_restart_indicator_is_the_papers_xi_with_restarts():
    """Sec. III-B, eq. "period_indicator_qp": with one subset the indicator
    is (g_k - grad l(x_{k+1}))'(grad l(x_{k+1}) - grad l(x_k)), g_k the split
    gradient before step k.  Recomputed from the dense matrix at the
    oracle's own iterates, on a run with several natural restarts."""
    cfg, data, A, y, w, DL = _tiny_problem()
    shape = ora.image_shape(cfg)
    beta = 2.0 ** -8 * float(np.median(DL[synth.roi_mask(cfg).ravel()]))
    delta = synth.configs.delta_mu(cfg)
    xs, hist = [np.zeros(A.shape[1])], {"g": []}
    out = ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=1, n_steps=200,
                      callback=lambda j, x: xs.append(x.ravel().copy()), history=hist)
    assert int(out["restart"].sum()) >= 3
    grad = _dense_grad(A, y, w)
    gl = [grad(x) for x in xs]
    g = [v.ravel() for v in hist["g"]]
    xi = np.array([(g[k] - gl[k + 1]) @ (gl[k + 1] - gl[k]) for k in range(200)])
    scale = np.array([np.linalg.norm(g[k] - gl[k + 1]) * np.linalg.norm(gl[k + 1] - gl[k])
                      for k in range(200)])
    np.testing.assert_allclose(out["xi"], xi, rtol=0, atol=1e-9 * scale.max())
    assert np.all(np.abs(out["xi"] - xi) <= 1e-9 * scale + 1e-300)
    # the restart rule is the sign of that value (l = 0 iff xi > 0)
    np.testing.assert_array_equal(out["restart"], xi > 0)
    # the comparison tells apart the plausible slips: the opposite sign, the
    # new split gradient in place of the old one, the gradient difference
    # taken against the wrong iterate
    for alt in (-xi,
                np.array([(g[k + 1] - gl[k + 1]) @ (gl[k + 1] - gl[k]) for k in range(200)]),
                np.array([(g[k] - gl[k + 1]) @ (gl[k + 1] - gl[max(k - 1, 0)]) for k in range(200)])):
        assert np.abs(out["xi"] - alt).max() > 1e-3 * scale.max()


def _cost_gradient_error(cost_fn, cfg, data, A, beta, delta, rng):
    """Largest relative gap between central differences of cost_fn and
    A'W(Ax - y) + grad R at random voxels."""
    shape = ora.image_shape(cfg)
    y, w = data["y"].ravel(), data["w"].ravel()
    x = rng.uniform(0.005, 0.03, shape)
    gexp = (A.T @ (w * (A @ x.ravel() - y))).reshape(shape) + ora.reg_grad(x, beta, delta, False)
    h = 1e-7
    err = 0.0
    for _ in range(16):
        idx = tuple(int(rng.integers(0, n)) for n in shape)
        xp = x.copy(); xp[idx] += h
        xm = x.copy(); xm[idx] -= h
        fd = (cost_fn(xp)[0] - cost_fn(xm)[0]) / (2 * h)
        err = max(err, abs(fd - gexp[idx]) / max(abs(gexp[idx]), 1e-12 * np.abs(gexp).max()))
    return err


def test_cost_gradient_is_the_weighted_residual_back_projection():
    """Sec. IV, eq. "ct_recon": Psi(x) = 1/2 ||y - Ax||_W^2 + R(x), so its
    gradient is A'W(Ax - y) + grad R (dense matrix and the regularizer
    gradient, both pinned elsewhere).  This fixes the 1/2 and the weights."""
    cfg, data, A, y, w, DL = _tiny_problem()
    beta, delta = 1e-3 * float(np.median(DL)), synth.configs.delta_mu(cfg)
    cost = lambda x: ora.cost(cfg, x, data["y"], data["w"], beta, delta)
    assert _cost_gradient_error(cost, cfg, data, A, beta, delta, np.random.default_rng(7)) < 1e-6
    # the parts add up
    x = np.random.default_rng(8).uniform(0.005, 0.03, ora.image_shape(cfg))
    tot, dat, reg = cost(x)
    assert tot == dat + reg
    assert abs(reg - ora.reg_value(x, beta, delta, False)) <= 1e-12 * abs(reg)
    # planted slips fail the pin: the data term without its 1/2, or unweighted
    no_half = lambda x: (2.0 * cost(x)[1] + cost(x)[2],)
    unweighted = lambda x: (ora.cost(cfg, x, data["y"], np.ones_like(data["w"]), beta, delta)[0],)
    for bad in (no_half, unweighted):
        assert _cost_gradient_error(bad, cfg, data, A, beta, delta, np.random.default_rng(7)) > 0.1
