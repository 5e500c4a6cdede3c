"""Pins of the FP64 oracle's projector against facts outside the oracle.

* brute force: every entry of A evaluated on its own (hat-function form)
  equals the ray march / scatter (floor-and-fraction form) on tiny geometries;
* the adjoint identity <A x, y> = <x, A' y>;
* a constant image integrates to c x (slices) x (path length per slice) on
  rays whose samples all lie inside the image;
* 90-degree rotation symmetry of the scanner;
* analytic line integrals of ellipse phantoms (computed by the independent
  input generator) agree with the Joseph projection of the supersampled
  pixelisation to discretisation accuracy, improving under refinement.
"""
import math
import os

import numpy as np
import pytest

import oracle as ora
import synth


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "tiny_helical"])
def test_dense_entries_match_ray_march(name):
    cfg = synth.get_config(name)
    A = ora.dense(cfg)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 1.0, ora.image_shape(cfg))
    p = ora.forward(cfg, x).ravel()
    np.testing.assert_allclose(A @ x.ravel(), p, rtol=0, atol=1e-13 * np.abs(p).max())
    s = rng.normal(size=p.shape)
    bp = ora.back(cfg, s).ravel()
    np.testing.assert_allclose(A.T @ s, bp, rtol=0, atol=1e-13 * np.abs(bp).max())
    # every ray of the tiny geometries meets the volume
    assert np.count_nonzero(A.sum(axis=1)) > 0.5 * A.shape[0]


def test_both_dominant_axes_occur_in_one_view():
    cfg = synth.get_config("tiny2d")
    doms = []
    for b in range(cfg["n_bins"]):
        _, u = ora.ray(cfg, 1, 0, b)
        doms.append(abs(u[0]) >= abs(u[1]))
    assert any(doms) and not all(doms)


@pytest.mark.parametrize("name", ["fan2d_128", "tiny3d", "tiny_helical"])
def test_adjoint_identity_fp64(name):
    cfg = synth.get_config(name)
    rng = np.random.default_rng(7)
    x = rng.uniform(0.0, 1.0, ora.image_shape(cfg))
    views = np.arange(0, cfg["n_views"], 3)
    y = rng.normal(size=(len(views), cfg["n_rows"], cfg["n_bins"]))
    lhs = float(np.sum(ora.forward(cfg, x, views) * y))
    rhs = float(np.sum(x * ora.back(cfg, y, views)))
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0) * 10


def test_constant_image_path_length():
    cfg = synth.get_config("fan2d_128")
    c = 0.02
    x = np.full(ora.image_shape(cfg), c)
    nx = cfg["nx"]
    X0 = -(nx - 1) / 2.0 * cfg["dx"]
    checked = 0
    for v in (0, 17, 45, 90, 133):
        p = ora.forward(cfg, x, [v])[0, 0]
        for b in range(0, cfg["n_bins"], 5):
            S, u = ora.ray(cfg, v, 0, b)
            xdom = abs(u[0]) >= abs(u[1])
            a, o = (0, 1) if xdom else (1, 0)
            # positions along the other axis at the first and last slice
            ts = [(X0 + s * cfg["dx"] - S[a]) / u[a] for s in (0, nx - 1)]
            eta = [(S[o] + t * u[o] - X0) / cfg["dx"] for t in ts]
            if min(eta) >= 0.0 and max(eta) <= nx - 1:
                expect = c * nx * cfg["dx"] / abs(u[a])
                assert abs(p[b] - expect) <= 1e-12 * expect
                checked += 1
    assert checked > 20


def test_rotation_symmetry_quarter_turn():
    cfg = synth.get_config("fan2d_128")
    n = cfg["n_views"]
    assert n % 4 == 0
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 1.0, ora.image_shape(cfg))
    N = cfg["nx"]
    # the scanner turned by +90 degrees sees the image turned by -90 degrees:
    # x_rot(X, Y) = x(-Y, X), i.e. x_rot[j][i] = x[i][N-1-j]
    xr = np.empty_like(x)
    jj, ii = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    xr[0] = x[0][ii, N - 1 - jj]
    for v in (0, 7, 30):
        p_rot_view = ora.forward(cfg, x, [v + n // 4])[0, 0]
        p_rot_img = ora.forward(cfg, xr, [v])[0, 0]
        keep = []
        for b in range(cfg["n_bins"]):
            _, u = ora.ray(cfg, v, 0, b)
            if abs(abs(u[0]) - abs(u[1])) > 1e-9:       # exact 45-degree ties excepted
                keep.append(b)
        np.testing.assert_allclose(p_rot_view[keep], p_rot_img[keep], rtol=1e-10, atol=1e-10)


def _analytic_vs_joseph(cfg):
    ph = synth.make_phantom(cfg)
    views = np.arange(0, cfg["n_views"], 6)
    ybar = synth.analytic_sinogram(cfg, ph, views=views)
    xt = synth.pixelize(cfg, ph, ss=4)
    p = ora.forward(cfg, xt, views)
    return np.linalg.norm(p - ybar) / np.linalg.norm(ybar)


def test_analytic_line_integrals_and_refinement():
    cfg = synth.get_config("fan2d_128")
    e1 = _analytic_vs_joseph(cfg)
    fine = synth.get_config("fan2d_128", nx=256, ny=256, dx=0.5, dy=0.5)
    e2 = _analytic_vs_joseph(fine)
    assert e1 < 1e-2
    assert e2 < 0.75 * e1


def _analytic_vs_joseph_3d(f):
    cfg = synth.get_config("cone_axial_512x64", nx=64 * f, ny=64 * f, nz=16 * f,
                           dx=7.84 / f, dy=7.84 / f, dz=2.5 / f, n_views=24,
                           n_views_per_turn=24, n_bins=111 * f, ds=8.0 / f,
                           n_rows=16 * f, dt=4.4 / f, n_ellipses=12)
    ph = synth.make_phantom(cfg)
    views = np.arange(0, cfg["n_views"], 4)
    ybar = synth.analytic_sinogram(cfg, ph, views=views)
    xt = synth.pixelize(cfg, ph, ss=3)
    p = ora.forward(cfg, xt, views)
    return np.linalg.norm(p - ybar) / np.linalg.norm(ybar)


def test_analytic_line_integrals_3d_refinement():
    e1 = _analytic_vs_joseph_3d(1)
    e2 = _analytic_vs_joseph_3d(2)
    assert e1 < 6e-2
    assert e2 < 0.75 * e1


def test_sample_count_bounds():
    cfg = synth.get_config("tiny2d")
    A = ora.dense(cfg)
    n = ora.count_samples(cfg)
    # a sample touches one column (x-dominant) or row (y-dominant): every
    # nonzero matrix entry belongs to one counted sample, at most 2 per sample
    nnz = np.count_nonzero(A)
    assert nnz <= 2 * n
    assert n <= nnz + cfg["n_views"] * cfg["n_bins"] * 2


@pytest.mark.parametrize("name", ["tiny2d", "tiny_helical"])
def test_back_at_entries_match_dense_and_full_back(name):
    """The per-entry back-projection used for sampled full-size checks gives
    the dense A' entries and the full back-projection at the same voxels."""
    cfg = synth.get_config(name)
    views = np.arange(cfg["n_views"])[1::3]
    rng = np.random.default_rng(5)
    sino = rng.uniform(-1, 1, (len(views), cfg["n_rows"], cfg["n_bins"]))
    sino[0, 0, :3] = 0.0
    full = ora.back(cfg, sino, views).reshape(ora.image_shape(cfg))
    nz, ny, nx = ora.image_shape(cfg)
    vox = [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (nz // 2, ny // 2, nx // 3), (0, ny - 1, 0)]
    got = ora.back_at_c(cfg, sino, views, vox)
    ref_loop = ora.back_at(cfg, sino, views, vox)
    A = ora.dense(cfg, views)
    ref_dense = (A.T @ sino.reshape(-1)).reshape(nz, ny, nx)
    for n, (k, j, i) in enumerate(vox):
        assert got[n] == pytest.approx(ref_dense[k, j, i], rel=1e-12, abs=1e-12)
        assert got[n] == pytest.approx(full[k, j, i], rel=1e-12, abs=1e-12)
        assert got[n] == pytest.approx(ref_loop[n], rel=1e-12, abs=1e-12)


# ---------------------------------------------------------------- FBP (initial image)

def test_fbp_of_a_uniform_disk_recovers_its_value():
    """The analytic sinogram of a centred uniform disk (independent chord
    generator) reconstructs to the disk's value inside it (mean within 1 %,
    every pixel within 5 %) and to zero mean outside."""
    cfg = synth.get_config("fan2d_128")
    mu, r = 0.02, 40.0
    ph = dict(cx=np.array([0.0]), cy=np.array([0.0]), cz=np.array([0.0]), ax=np.array([r]), ay=np.array([r]),
              az=np.array([1.0]), phi=np.array([0.0]), amp=np.array([mu]), is2d=True)
    sino = synth.analytic_sinogram(cfg, ph)
    f = ora.fbp_fan(cfg, sino)[0]
    X = (np.arange(cfg["nx"]) - (cfg["nx"] - 1) / 2.0) * cfg["dx"]
    R = np.hypot(X[None, :], X[:, None])
    inner = R < r - 4.0
    outer = (R > r + 8.0) & (R < 60.0)
    assert abs(np.mean(f[inner]) / mu - 1.0) < 0.01
    assert np.max(np.abs(f[inner] / mu - 1.0)) < 0.05
    # outside: view-aliasing streaks of the sharp edge (180 views) average out
    assert abs(np.mean(f[outer])) < 0.005 * mu
    assert np.sqrt(np.mean(f[outer] ** 2)) < 0.04 * mu


def test_fbp_of_the_phantom_is_close_to_the_pixelized_phantom():
    cfg = synth.get_config("fan2d_128")
    ph = synth.make_phantom(cfg)
    sino = synth.analytic_sinogram(cfg, ph)
    f = ora.fbp_fan(cfg, sino)
    truth = synth.pixelize(cfg, ph, ss=4)
    m = synth.roi_mask(cfg)
    rel = np.linalg.norm((f - truth)[m]) / np.linalg.norm(truth[m])
    assert rel < 0.08


def _brute_force_samples(cfg):
    """Joseph samples with at least one tap in the volume, counted from the
    per-entry dense matrix: for every ray, the number of distinct slices of
    its dominant in-plane axis that hold a non-zero entry of its row."""
    A = ora.dense(cfg)
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    total, q = 0, 0
    for v in range(cfg["n_views"]):
        for r in range(cfg["n_rows"]):
            for b in range(cfg["n_bins"]):
                _, u = ora.ray(cfg, v, r, b)
                cols = np.nonzero(A[q])[0]
                i = cols % nx
                j = (cols // nx) % ny
                total += len(np.unique(i if abs(u[0]) >= abs(u[1]) else j))
                q += 1
    assert q == A.shape[0] and nz * ny * nx == A.shape[1]
    return total


def _mutated_count(cfg, tmp_path, old, new):
    """og_count_samples of a copy of the oracle's C source with one planted
    change, compiled on the side."""
    import ctypes
    import subprocess
    from oracle import oracle as _oracle_mod
    src = open(os.path.join(os.path.dirname(_oracle_mod.__file__), "oracle.c")).read()
    assert src.count(old) == 1
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-std=c99", str(path), "-o", str(lib), "-lm"])
    L = ctypes.CDLL(str(lib))
    views = np.arange(cfg["n_views"], dtype=np.int32)
    L.og_count_samples.restype = ctypes.c_longlong
    return int(L.og_count_samples(ctypes.byref(_oracle_mod._geom(cfg)),
                                  views.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(views)))


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "tiny_helical"])
def test_sample_count_equals_brute_force(name, tmp_path):
    """The sample count behind every byte figure equals a brute-force count
    from the per-entry weights (which equal the ray march, pinned above);
    a count whose slice range is shifted by one differs from it."""
    cfg = synth.get_config(name)
    n = ora.count_samples(cfg)
    assert n == _brute_force_samples(cfg)
    # per view too (the GPU plan reports per subset)
    v0 = ora.count_samples(cfg, [0]) + ora.count_samples(cfg, list(range(1, cfg["n_views"])))
    assert v0 == n
    # planted slips: the in-volume test of the lower tap shifted by one
    assert _mutated_count(cfg, tmp_path, "if (lo < -1 || lo > no - 1) continue;",
                          "if (lo < 0 || lo > no - 1) continue;") != n
    assert _mutated_count(cfg, tmp_path, "if (lo < -1 || lo > no - 1) continue;",
                          "if (lo < -1 || lo > no - 2) continue;") != n
