"""Seeded ellipse / ellipsoid phantoms, analytic sinograms and Poisson data.

Recipe (one reading of the paper's unspecified workloads):

* one body ellipse(oid) plus ``n_ellipses - 1`` non-overlapping inner ones,
  placed by rejection sampling so that each inner one lies inside the body;
  attenuation values ``mu ~ U[0.015, 0.025] / mm``; inner objects carry the
  additive amplitude ``mu_k - mu_body`` so values stay in range and line
  integrals stay analytic; the object lies inside the reconstructed volume
  and inside the scanner's field of view;
* noiseless line integrals ``ybar_i = sum_e amp_e * chord_e(ray i)``;
* counts ``N_i ~ Poisson(I0 exp(-ybar_i))``, data ``y_i = ln(I0 / N_i)``,
  weights ``w_i = N_i``; a zero-count ray gets ``y_i = 0`` and ``w_i = 0``;
* random numbers: ``numpy.random.Generator(PCG64)`` seeded through
  ``SeedSequence(seed)``, whose first child draws the phantom and whose
  second child draws the noise.

Sinograms are returned in natural order ``[view][row][bin]``.
"""
import math
import os

import numpy as np

from .configs import FAN2D, helical_feed, fov_radius_of

MU_LO, MU_HI = 0.015, 0.025


def fov_radius(cfg):
    """Radius (mm) of the circle every view's fan covers."""
    return fov_radius_of(cfg)


def _rngs(seed):
    ss = np.random.SeedSequence(seed)
    a, b = ss.spawn(2)
    return np.random.Generator(np.random.PCG64(a)), np.random.Generator(np.random.PCG64(b))


def make_phantom(cfg, seed=None):
    """Random phantom: dict of float64 arrays (cx, cy, cz, ax, ay, az, phi, amp).

    Index 0 is the body.  For 2D workloads the z fields are unused
    (``az = inf``).
    """
    seed = cfg["seed"] if seed is None else seed
    rng, _ = _rngs(seed)
    is2d = cfg["kind"] == FAN2D
    half_w = 0.5 * min(cfg["nx"] * cfg["dx"], cfg["ny"] * cfg["dy"])
    rb = 0.9 * min(half_w, fov_radius(cfg))
    half_d = 0.5 * cfg["nz"] * cfg["dz"]
    n = int(cfg["n_ellipses"])
    cx = np.zeros(n); cy = np.zeros(n); cz = np.zeros(n)
    ax = np.zeros(n); ay = np.zeros(n); az = np.full(n, np.inf)
    phi = np.zeros(n); amp = np.zeros(n)
    # body
    ax[0] = rng.uniform(0.80, 0.95) * rb
    ay[0] = rng.uniform(0.65, 0.85) * rb
    phi[0] = rng.uniform(0.0, math.pi)
    if not is2d:
        az[0] = rng.uniform(0.70, 0.85) * half_d
    mu_body = rng.uniform(MU_LO, MU_HI)
    amp[0] = mu_body
    cb, sb = math.cos(phi[0]), math.sin(phi[0])
    bmin = min(ax[0], ay[0])
    placed = 1
    tries = 0
    scale = 1.0
    while placed < n:
        tries += 1
        if tries % 2000 == 0:
            scale *= 0.85          # crowded: shrink the inner objects
        ea = rng.uniform(0.04, 0.18) * rb * scale
        eb = rng.uniform(0.04, 0.18) * rb * scale
        ep = rng.uniform(0.0, math.pi)
        ez = rng.uniform(0.25, 0.8) * az[0] if not is2d else np.inf
        r = max(ea, eb)
        # centre uniformly in the body's bounding box, accept if the bounding
        # circle of the inner ellipse lies inside the body (normalised radius)
        px = rng.uniform(-ax[0], ax[0])
        py = rng.uniform(-ax[0], ax[0])
        pz = rng.uniform(-az[0], az[0]) if not is2d else 0.0
        u = (cb * px + sb * py) / ax[0]
        v = (-sb * px + cb * py) / ay[0]
        rho = math.hypot(u, v)
        if rho + r / bmin > 0.95:
            continue
        if not is2d:
            # z extent must stay inside the body ellipsoid's half height at
            # the normalised radius reached by the inner object
            rr = min(1.0, rho + r / bmin)
            hz = az[0] * math.sqrt(max(0.0, 1.0 - rr * rr))
            if abs(pz) + ez > 0.95 * hz:
                continue
        ok = True
        for k in range(1, placed):
            rk = max(ax[k], ay[k])
            if math.hypot(px - cx[k], py - cy[k]) < r + rk + 1e-9:
                if is2d or abs(pz - cz[k]) < ez + az[k]:
                    ok = False
                    break
        if not ok:
            continue
        cx[placed], cy[placed], cz[placed] = px, py, pz
        ax[placed], ay[placed], az[placed] = ea, eb, ez
        phi[placed] = ep
        amp[placed] = rng.uniform(MU_LO, MU_HI) - mu_body
        placed += 1
    return dict(cx=cx, cy=cy, cz=cz, ax=ax, ay=ay, az=az, phi=phi, amp=amp,
                is2d=is2d)


def ray_sources_directions(cfg, views):
    """Source points and unit directions of every ray of the given views.

    Returns ``S, u`` with shape ``[len(views), n_rows, n_bins, 3]`` (float64).
    """
    views = np.asarray(views, dtype=np.int64)
    nb, nr = cfg["n_bins"], cfg["n_rows"]
    beta = cfg["start_angle"] + 2.0 * math.pi * views / cfg["n_views_per_turn"]
    if cfg["kind"] == 2:
        zs = (views - (cfg["n_views"] - 1) / 2.0) * helical_feed(cfg) / cfg["n_views_per_turn"]
    else:
        zs = np.zeros(views.shape)
    gam = (np.arange(nb) - (nb - 1) / 2.0 - cfg["channel_offset"]) * cfg["ds"] / cfg["dsd"]
    vr = (np.arange(nr) - (nr - 1) / 2.0) * cfg["dt"]
    if cfg["kind"] == FAN2D:
        vr = np.zeros(1)
    th = beta[:, None] + math.pi + gam[None, :]                       # [V, B]
    ex, ey = np.cos(th), np.sin(th)
    dsd = cfg["dsd"]
    norm = np.sqrt(dsd * dsd + vr * vr)                                # [R]
    u = np.empty((len(views), nr, nb, 3))
    u[..., 0] = dsd * ex[:, None, :] / norm[None, :, None]
    u[..., 1] = dsd * ey[:, None, :] / norm[None, :, None]
    u[..., 2] = np.broadcast_to((vr / norm)[None, :, None], (len(views), nr, nb))
    S = np.empty_like(u)
    S[..., 0] = (cfg["dso"] * np.cos(beta))[:, None, None]
    S[..., 1] = (cfg["dso"] * np.sin(beta))[:, None, None]
    S[..., 2] = zs[:, None, None]
    return S, u


def _chords(S, u, ph):
    """Sum over ellipses of amplitude x chord length, vectorised over rays."""
    out = np.zeros(S.shape[:-1])
    n = len(ph["amp"])
    for e in range(n):
        c, s = math.cos(ph["phi"][e]), math.sin(ph["phi"][e])
        px = S[..., 0] - ph["cx"][e]
        py = S[..., 1] - ph["cy"][e]
        P0 = (c * px + s * py) / ph["ax"][e]
        P1 = (-s * px + c * py) / ph["ay"][e]
        D0 = (c * u[..., 0] + s * u[..., 1]) / ph["ax"][e]
        D1 = (-s * u[..., 0] + c * u[..., 1]) / ph["ay"][e]
        A = D0 * D0 + D1 * D1
        B = P0 * D0 + P1 * D1
        C = P0 * P0 + P1 * P1 - 1.0
        if not ph["is2d"]:
            P2 = (S[..., 2] - ph["cz"][e]) / ph["az"][e]
            D2 = u[..., 2] / ph["az"][e]
            A = A + D2 * D2
            B = B + P2 * D2
            C = C + P2 * P2
        disc = B * B - A * C
        pos = disc > 0
        out += np.where(pos, ph["amp"][e] * 2.0 * np.sqrt(np.where(pos, disc, 0.0)) / A, 0.0)
    return out


def _sino_chunk(args):
    cfg, ph, views = args
    S, u = ray_sources_directions(cfg, views)
    return _chords(S, u, ph)


_CHORDS_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "chords.c")
_CHORDS_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libchords.so")
_chords_lib = None


def build_chords(force=False):
    """Compile the C version of the chord sums (gcc, OpenMP)."""
    import subprocess
    if force or not os.path.exists(_CHORDS_LIB) or \
            os.path.getmtime(_CHORDS_LIB) < os.path.getmtime(_CHORDS_SRC):
        tmp = _CHORDS_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               _CHORDS_SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _CHORDS_LIB)
    return _CHORDS_LIB


def _chords_c(cfg, ph, views, n_threads=0):
    global _chords_lib
    import ctypes
    if _chords_lib is None:
        _chords_lib = ctypes.CDLL(build_chords())
    keys = ("kind", "nx", "ny", "nz", "dx", "dy", "dz", "n_views", "n_views_per_turn",
            "n_bins", "n_rows", "ds", "dt", "dso", "dsd", "start_angle", "pitch",
            "channel_offset")
    geo = np.array([float(cfg[k]) for k in keys])
    views = np.ascontiguousarray(np.asarray(views, dtype=np.int32))
    out = np.zeros((len(views), cfg["n_rows"], cfg["n_bins"]))
    arrs = [np.ascontiguousarray(ph[k], dtype=np.float64) for k in
            ("cx", "cy", "cz", "ax", "ay", "az", "phi", "amp")]
    dp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _chords_lib.synth_chords(dp(geo), ctypes.c_int(len(ph["amp"])), *[dp(a) for a in arrs],
                             ctypes.c_int(1 if ph["is2d"] else 0), dp(views),
                             ctypes.c_int(len(views)), dp(out), ctypes.c_int(int(n_threads)))
    return out


def analytic_sinogram(cfg, ph, views=None, workers=None, use_c=True):
    """Noiseless line integrals ``[n_views][n_rows][n_bins]`` (float64).
    ``use_c`` selects the compiled chord sums (same formulas as ``_chords``);
    ``workers`` is then its thread count (None: the OpenMP default)."""
    if views is None:
        views = np.arange(cfg["n_views"])
    views = np.asarray(views)
    if use_c:
        return _chords_c(cfg, ph, views, workers or 0)
    nr, nb = cfg["n_rows"], cfg["n_bins"]
    per = max(1, int(2_000_000 // (nr * nb)))
    chunks = [views[i:i + per] for i in range(0, len(views), per)]
    workers = workers or 1
    if workers > 1 and len(chunks) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, len(chunks))) as pool:
            parts = pool.map(_sino_chunk, [(cfg, ph, ch) for ch in chunks])
    else:
        parts = [_sino_chunk((cfg, ph, ch)) for ch in chunks]
    return np.concatenate(parts, axis=0)


def noisy_data(cfg, ybar, seed=None):
    """Poisson counts -> (y, w) float64 arrays of the sinogram's shape."""
    seed = cfg["seed"] if seed is None else seed
    _, rng = _rngs(seed)
    lam = cfg["I0"] * np.exp(-ybar)
    N = rng.poisson(lam).astype(np.float64)
    pos = N > 0
    y = np.where(pos, np.log(cfg["I0"] / np.where(pos, N, 1.0)), 0.0)
    return y, N


def pixelize(cfg, ph, ss=4):
    """Phantom averaged over ss^d sub-samples per voxel, ``[nz][ny][nx]``."""
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    X = (np.arange(nx) - (nx - 1) / 2.0) * cfg["dx"]
    Y = (np.arange(ny) - (ny - 1) / 2.0) * cfg["dy"]
    Z = (np.arange(nz) - (nz - 1) / 2.0) * cfg["dz"]
    off = (np.arange(ss) + 0.5) / ss - 0.5
    img = np.zeros((nz, ny, nx))
    zoffs = off if not ph["is2d"] else np.zeros(1)
    for oz in zoffs:
        zz = Z + oz * cfg["dz"]
        for oy in off:
            yy = Y + oy * cfg["dy"]
            for ox in off:
                xx = X + ox * cfg["dx"]
                gz, gy, gx = np.meshgrid(zz, yy, xx, indexing="ij")
                for e in range(len(ph["amp"])):
                    c, s = math.cos(ph["phi"][e]), math.sin(ph["phi"][e])
                    px = gx - ph["cx"][e]
                    py = gy - ph["cy"][e]
                    a = (c * px + s * py) / ph["ax"][e]
                    b = (-s * px + c * py) / ph["ay"][e]
                    r2 = a * a + b * b
                    if not ph["is2d"]:
                        cz = (gz - ph["cz"][e]) / ph["az"][e]
                        r2 = r2 + cz * cz
                    img += np.where(r2 <= 1.0, ph["amp"][e], 0.0)
    return img / (len(zoffs) * ss * ss)


def roi_radius(cfg):
    """Radius (mm) of the evaluation region (see :func:`roi_mask`)."""
    half_w = 0.5 * min(cfg["nx"] * cfg["dx"], cfg["ny"] * cfg["dy"])
    return min(fov_radius(cfg), half_w) - 2.0 * cfg["dx"]


def roi_mask(cfg):
    """Evaluation region: voxel centres within radius
    ``min(R_fov, image half-width) - 2 dx`` of the axis, all slices."""
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    X = (np.arange(nx) - (nx - 1) / 2.0) * cfg["dx"]
    Y = (np.arange(ny) - (ny - 1) / 2.0) * cfg["dy"]
    half_w = 0.5 * min(nx * cfg["dx"], ny * cfg["dy"])
    rad = min(fov_radius(cfg), half_w) - 2.0 * cfg["dx"]
    m2 = (X[None, :] ** 2 + Y[:, None] ** 2) <= rad * rad
    return np.broadcast_to(m2[None], (nz, ny, nx)).copy()


def make_problem_data(cfg, seed=None, workers=None, with_truth=False):
    """Phantom, noiseless and noisy sinograms (natural order), float64."""
    seed = cfg["seed"] if seed is None else seed
    ph = make_phantom(cfg, seed)
    if workers is None:
        workers = min(16, len(os.sched_getaffinity(0)))
    ybar = analytic_sinogram(cfg, ph, workers=workers)
    y, w = noisy_data(cfg, ybar, seed)
    out = dict(phantom=ph, ybar=ybar, y=y, w=w, seed=seed)
    if with_truth:
        out["x_true"] = pixelize(cfg, ph)
    return out
