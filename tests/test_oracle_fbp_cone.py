"""Pins of the oracle's axial cone-beam FDK (the x0 of the 3D workloads)
against what geometry and the mathematics fix, independently of the oracle's
own projector: analytic line integrals of a uniform infinite cylinder
(z-invariant: FDK is exact for it in the continuum) and of a uniform ball,
with the ray geometry written out here from the header's definitions, and
the reduction to the 2D fan-beam FBP for a single detector row.  Each pin
is shown to fail with a plausible mistake planted in a copy of the oracle
function."""
import inspect

import numpy as np
import pytest

import oracle as ora
import synth

MU = 0.02


def _cfg(**over):
    base = dict(kind=1, nx=48, ny=48, nz=32, dx=1.0, dy=1.0, dz=1.0, n_views=180, n_views_per_turn=180,
                n_bins=128, ds=1.0, n_rows=64, dt=2.0, dso=60.0, dsd=120.0, start_angle=0.0, pitch=0.0,
                channel_offset=0.0, detector=0)
    base.update(over)
    return base


def _rays(cfg):
    """Source points and unit directions of every ray, [view][row][bin][3],
    from the header's geometry: beta_v = 2 pi v / n, S = dso (cos, sin, 0),
    channel angle gamma_b = (b - (nb-1)/2) ds / dsd, in-plane direction at
    beta + pi + gamma_b, row height v_r = (r - (nr-1)/2) dt at distance dsd."""
    nv, nr, nb = cfg["n_views"], cfg["n_rows"], cfg["n_bins"]
    beta = 2.0 * np.pi * np.arange(nv) / cfg["n_views_per_turn"]
    gam = (np.arange(nb) - (nb - 1) / 2.0) * cfg["ds"] / cfg["dsd"]
    vr = (np.arange(nr) - (nr - 1) / 2.0) * cfg["dt"]
    B, R, G = np.meshgrid(beta, vr, gam, indexing="ij")
    phi = B + np.pi + G
    u = np.stack([cfg["dsd"] * np.cos(phi), cfg["dsd"] * np.sin(phi), R], axis=-1)
    u /= np.linalg.norm(u, axis=-1, keepdims=True)
    S = np.stack([cfg["dso"] * np.cos(B), cfg["dso"] * np.sin(B), np.zeros_like(B)], axis=-1)
    return S, u


def _cylinder_sino(cfg, radius):
    """Line integrals of mu over the infinite cylinder x^2 + y^2 <= radius^2:
    the in-plane chord divided by the cosine of the ray's cone angle."""
    S, u = _rays(cfg)
    uxy = np.linalg.norm(u[..., :2], axis=-1)
    d = np.abs(S[..., 0] * u[..., 1] - S[..., 1] * u[..., 0]) / uxy      # in-plane distance to the axis
    chord = 2.0 * np.sqrt(np.maximum(radius * radius - d * d, 0.0))
    return MU * chord / uxy


def _ball_sino(cfg, radius):
    """Line integrals of mu over the ball |p| <= radius at the isocentre."""
    S, u = _rays(cfg)
    d = np.linalg.norm(np.cross(S, u), axis=-1)
    return MU * 2.0 * np.sqrt(np.maximum(radius * radius - d * d, 0.0))


def _planted(old, new):
    """A copy of the oracle's fbp_cone_axial with one expression replaced."""
    src = inspect.getsource(ora.fbp_cone_axial)
    assert old in src
    ns = dict(inspect.getmodule(ora.fbp_cone_axial).__dict__)
    exec(src.replace(old, new), ns)
    return ns["fbp_cone_axial"]


def _centres(cfg):
    nz, ny, nx = cfg["nz"], cfg["ny"], cfg["nx"]
    Z = (np.arange(nz) - (nz - 1) / 2.0) * cfg["dz"]
    Y = (np.arange(ny) - (ny - 1) / 2.0) * cfg["dy"]
    X = (np.arange(nx) - (nx - 1) / 2.0) * cfg["dx"]
    return np.meshgrid(Z, Y, X, indexing="ij")


def _cylinder_error(fbp):
    cfg = _cfg()
    f = fbp(cfg, _cylinder_sino(cfg, 15.0))
    Z, Y, X = _centres(cfg)
    inner = np.sqrt(X * X + Y * Y) < 12.0
    return float(np.abs(f[inner] - MU).max() / MU)


def test_fdk_recovers_a_z_invariant_cylinder_in_every_slice():
    """FDK is exact for objects that do not vary along z; at a cone
    half-angle of 28 degrees every slice's interior must come back within
    1 % (discretization of the ramp filter and the interpolation)."""
    e = _cylinder_error(ora.fbp_cone_axial)
    assert e < 0.01, e


def test_cylinder_pin_fails_without_the_cone_weight():
    bad = _planted("* (dsd / np.sqrt(dsd * dsd + vr * vr))[None, :, None]", "")
    assert _cylinder_error(bad) > 0.02


def _ball_errors(fbp):
    cfg = _cfg()
    R = 10.0
    f = fbp(cfg, _ball_sino(cfg, R))
    Z, Y, X = _centres(cfg)
    r = np.sqrt(X * X + Y * Y + Z * Z)
    inside = r < R - 3.0
    outside = (r > R + 3.0) & (np.sqrt(X * X + Y * Y) < 20.0)
    return float(np.abs(f[inside] - MU).max() / MU), float(np.abs(f[outside]).max() / MU)


def test_fdk_recovers_a_ball():
    """A uniform ball of radius 10 mm (z-varying): inside 3 mm from its
    surface within 5 %, outside beyond 3 mm below 10 % of mu (the ball's
    edge rings and FDK's cone-beam approximation spreads it along z)."""
    ein, eout = _ball_errors(ora.fbp_cone_axial)
    assert ein < 0.05 and eout < 0.1, (ein, eout)


def test_ball_pin_fails_with_the_wrong_row_magnification():
    # the row height of a point measured at the isocentre instead of at the detector
    bad = _planted("rc = PZ * dsd / np.sqrt(L2)", "rc = PZ * D / np.sqrt(L2)")
    ein, eout = _ball_errors(bad)
    assert max(ein, eout) > 0.2


def test_one_row_reduces_to_the_fan_beam_fbp():
    cfg2 = synth.get_config("fan2d_128", nx=32, ny=32, dx=4.0, dy=4.0, n_views=60, n_views_per_turn=60,
                            n_bins=64, ds=4.8)
    cfg3 = dict(cfg2, kind=1, nz=1, n_rows=1, dt=1.0)
    s = np.random.default_rng(0).uniform(0, 1, (60, 1, 64))
    a = ora.fbp_fan(cfg2, s)
    b = ora.fbp_cone_axial(cfg3, s)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_selected_voxels_equal_the_whole_image():
    cfg = _cfg(nx=16, ny=16, nz=8, n_views=36, n_views_per_turn=36, n_bins=48, n_rows=16)
    s = np.random.default_rng(1).uniform(0, 1, (36, 16, 48))
    f = ora.fbp_cone_axial(cfg, s)
    vox = [(0, 0, 0), (7, 15, 15), (3, 8, 2), (5, 1, 12)]
    got = ora.fbp_cone_axial(cfg, s, voxels=vox)
    np.testing.assert_allclose(got, [f[v] for v in vox], rtol=1e-13, atol=0)


def test_helical_and_partial_turns_are_rejected():
    with pytest.raises(ValueError):
        ora.fbp_cone_axial(_cfg(kind=2, pitch=1.0), np.zeros((180, 64, 128)))
    with pytest.raises(ValueError):
        ora.fbp_cone_axial(_cfg(n_views=90), np.zeros((90, 64, 128)))
