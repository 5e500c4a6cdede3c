"""Workload definitions (geometry, phantom, noise and solver settings).

Every workload is a plain dict.  Geometry fields mirror the C ABI's
``lalm_geometry`` struct; lengths are in mm, angles in radians.

Scanner conventions (one reading of a paper that names no projector or
scanner model; stated once here and implemented independently by the input
generator, the oracle and the GPU planner):

* image voxel centres ``X_i = (i - (nx-1)/2) dx`` (same for y, z); the image
  centre is the isocentre;
* view angle ``beta_v = start_angle + 2 pi v / n_views_per_turn``; source
  ``S_v = (dso cos beta_v, dso sin beta_v, z_s(v))``;
* arc (equiangular) detector: channel angle
  ``gamma_b = (b - (n_bins-1)/2 - channel_offset) ds / dsd``, in-plane ray
  direction at angle ``beta_v + pi + gamma_b``;
* cylindrical detector rows at height ``v_r = (r - (n_rows-1)/2) dt`` at
  distance ``dsd`` from the source: the ray aims at
  ``S + dsd (cos, sin, 0) + (0, 0, v_r)``;
* helical source height ``z_s(v) = (v - (n_views-1)/2) feed / n_views_per_turn``
  with table feed per turn ``pitch * n_rows * dt * dso / dsd`` (pitch times
  the collimation at the isocentre), so the helix is centred on the volume.
"""
import copy
import math

# HU scale: 1000 HU per water attenuation, water = 0.02 / mm (a reading:
# the paper shows 800..1200 HU windows for soft tissue, i.e. water ~ 1000).
MU_WATER = 0.02
HU_PER_MU = 1000.0 / MU_WATER          # 1 HU = 2e-5 / mm

FAN2D, CONE_AXIAL, CONE_HELICAL = 0, 1, 2

_COMMON = dict(start_angle=0.0, pitch=0.0, channel_offset=0.0, detector=0,
               dso=541.0, dsd=949.0, delta_hu=10.0)

CONFIGS = {
    # 2D fan beam, 128^2 x 1 mm, 180 views / 360 deg, 256 x 1.2 mm bins;
    # 10 ellipses, I0 = 1e5; M = 4, 20 iterations.
    "fan2d_128": dict(_COMMON, kind=FAN2D, nx=128, ny=128, nz=1,
                      dx=1.0, dy=1.0, dz=1.0, n_views=180, n_views_per_turn=180,
                      n_bins=256, n_rows=1, ds=1.2, dt=1.0,
                      n_ellipses=10, seed=1, I0=1e5, M=4, n_iter=20,
                      beta=None),
    # 2D fan beam, 512^2 x 0.98 mm, 984 views, 888 x 1.0 mm bins;
    # 40 ellipses, I0 = 5e4; M = 24, 30 iterations with continuation.
    "fan2d_512": dict(_COMMON, kind=FAN2D, nx=512, ny=512, nz=1,
                      dx=0.98, dy=0.98, dz=1.0, n_views=984, n_views_per_turn=984,
                      n_bins=888, n_rows=1, ds=1.0, dt=1.0,
                      n_ellipses=40, seed=2, I0=5e4, M=24, n_iter=30,
                      beta=None),
    # 3D axial cone beam, 512x512x64 (0.98, 0.98, 0.625), 984 views,
    # 888 x 64 cylindrical detector (1.0 x 1.1 mm); 60 ellipsoids, I0 = 1e5;
    # M = 12, 20 iterations.
    "cone_axial_512x64": dict(_COMMON, kind=CONE_AXIAL, nx=512, ny=512, nz=64,
                              dx=0.98, dy=0.98, dz=0.625, n_views=984,
                              n_views_per_turn=984, n_bins=888, n_rows=64,
                              ds=1.0, dt=1.1, n_ellipses=60, seed=3, I0=1e5,
                              M=12, n_iter=20, beta=None),
    # 3D helical cone beam, 512x512x256, pitch 1.0, 984 views/turn x 7 turns,
    # 888 x 64 detector; 60 ellipsoids, I0 = 5e4; M = 12.
    "cone_helical_512x256": dict(_COMMON, kind=CONE_HELICAL, nx=512, ny=512,
                                 nz=256, dx=0.98, dy=0.98, dz=0.625,
                                 n_views=6888, n_views_per_turn=984,
                                 n_bins=888, n_rows=64, ds=1.0, dt=1.1,
                                 pitch=1.0, n_ellipses=60, seed=5, I0=5e4,
                                 M=12, n_iter=30, beta=None),
    # Tiny geometries for brute-force checks (wide fan so that both dominant
    # axes occur inside one view).
    "tiny2d": dict(_COMMON, kind=FAN2D, nx=8, ny=8, nz=1, dx=1.0, dy=1.0,
                   dz=1.0, n_views=12, n_views_per_turn=12, n_bins=16,
                   n_rows=1, ds=1.6, dt=1.0, dso=20.0, dsd=40.0,
                   n_ellipses=3, seed=11, I0=1e4, M=3, n_iter=5, beta=None),
    "tiny3d": dict(_COMMON, kind=CONE_AXIAL, nx=6, ny=6, nz=4, dx=1.0,
                   dy=1.0, dz=1.0, n_views=8, n_views_per_turn=8, n_bins=10,
                   n_rows=4, ds=2.0, dt=2.0, dso=20.0, dsd=40.0,
                   n_ellipses=3, seed=12, I0=1e4, M=2, n_iter=5, beta=None),
    "tiny_helical": dict(_COMMON, kind=CONE_HELICAL, nx=6, ny=6, nz=6,
                         dx=1.0, dy=1.0, dz=1.0, n_views=16,
                         n_views_per_turn=8, n_bins=10, n_rows=4, ds=2.0,
                         dt=1.0, dso=20.0, dsd=40.0, pitch=1.0,
                         n_ellipses=3, seed=13, I0=1e4, M=4, n_iter=5,
                         beta=None),
}

# The U-Net warm-start workload uses the 512^2 fan-beam geometry and noise
# model; training seeds 100000..103999, evaluation seeds 200000..200019.
UNET_WARMSTART = dict(base="fan2d_512", train_seeds=(100000, 104000),
                      eval_seeds=(200000, 200020), iters_in=2, iters_target=50,
                      iters_after=10, iters_plain=30)

# Regularization strength: beta = BETA_REL * median over the ROI of the SQS
# denominator A'WA1 of the workload (a reading: the paper does not give beta).
# The medians below were produced once by oracle/derive_beta.py (FP64 oracle)
# and are rounded to 4 significant digits; see that script.
BETA_REL = 2.0 ** -4
DL_MEDIAN = {
    "fan2d_128": 1.152e9,
    "fan2d_512": 1.446e9,
    "cone_axial_512x64": 2.781e10,
    "cone_helical_512x256": 1.844e10,
    "tiny2d": 1.188e6,
    "tiny3d": 4.765e5,
    "tiny_helical": 7.325e5,
}

GEOMETRY_KEYS = ("kind", "nx", "ny", "nz", "dx", "dy", "dz", "n_views",
                 "n_views_per_turn", "n_bins", "n_rows", "ds", "dt", "dso",
                 "dsd", "start_angle", "pitch", "channel_offset", "detector")


def get_config(name, **overrides):
    """Return a deep copy of a named workload with optional overrides."""
    cfg = copy.deepcopy(CONFIGS[name])
    cfg["name"] = name
    cfg.update(overrides)
    if cfg.get("beta") is None:
        med = DL_MEDIAN.get(name)
        if med is not None:
            cfg["beta"] = BETA_REL * med
    return cfg


def geometry_of(cfg):
    """The geometry sub-dict (the fields of ``lalm_geometry``)."""
    return {k: cfg[k] for k in GEOMETRY_KEYS}


def delta_mu(cfg):
    """Hyperbola potential parameter delta in 1/mm (10 HU by default)."""
    return cfg["delta_hu"] / HU_PER_MU


def helical_feed(cfg):
    """Table feed per turn in mm (pitch x collimation at the isocentre)."""
    return cfg["pitch"] * cfg["n_rows"] * cfg["dt"] * cfg["dso"] / cfg["dsd"]


def half_fan(cfg):
    return cfg["n_bins"] * cfg["ds"] / (2.0 * cfg["dsd"])


def fov_radius_of(cfg):
    return cfg["dso"] * math.sin(half_fan(cfg))
