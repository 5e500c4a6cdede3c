"""FP64 CPU oracle of OS-LALM for PWLS X-ray CT -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline
leg use this module; the GPU library never imports, links or calls it, and
it shares no code with the GPU library (only the seeded input generator in
``synth/`` serves both).

It is written for checking by eye against the paper (arXiv 1402.4381,
Nien & Fessler, "Fast X-ray CT image reconstruction using a linearized
augmented Lagrangian method with ordered subsets"):

* the system matrix (the Joseph projector in ``oracle.c``),
* the SQS denominator D_L = A'WA1 (Sec. IV-A),
* the edge-preserving regularizer, its gradient and its separable majorizer,
* the PWLS cost (Sec. IV, eq. "ct_recon"),
* OS-LALM (Sec. III-A, eq. "os_lalm_iterates") with the substitution of
  eq. "ct_substitution", one projected gradient step for the inner
  constrained-denoising problem (n = 1, Sec. IV-A), and the deterministic
  downward continuation of rho with adaptive restart (Sec. III-B,
  eqs. "period_indicator_qp" and "rho_l_formula_qp"),
* the textbook linearized-AL iterates with u and d (Sec. II-A,
  eq. "general_lal_iterates", and Sec. III-A, eq. "lalm_pls_u"),
* the second-order analysis of the toy quadratic (Sec. III-B,
  eqs. "char_poly_qp" .. "opt_rho_qp"),
* the maximum number of subsets (Sec. IV-B, eqs. "max_M_axial",
  "max_M_helical"),
* a reference solution x* by one-subset FISTA with adaptive restart
  (Sec. V) and the RMS-difference figure of merit in HU.

Images are float64 ``[nz][ny][nx]``; sinograms are float64
``[view][row][bin]`` in natural view order.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=False):
    """Compile the C part of the oracle (plain gcc, FP64, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c99", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("dz", ctypes.c_double), ("n_views", ctypes.c_int),
                ("n_views_per_turn", ctypes.c_int), ("n_bins", ctypes.c_int),
                ("n_rows", ctypes.c_int), ("ds", ctypes.c_double), ("dt", ctypes.c_double),
                ("dso", ctypes.c_double), ("dsd", ctypes.c_double),
                ("start_angle", ctypes.c_double), ("pitch", ctypes.c_double),
                ("channel_offset", ctypes.c_double), ("detector", ctypes.c_int)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        gp = ctypes.POINTER(_Geom)
        _lib.og_ray.argtypes = [gp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
        _lib.og_ray_integral.argtypes = [gp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        _lib.og_ray_integral.restype = ctypes.c_double
        _lib.og_forward.argtypes = [gp, dp, ip, ctypes.c_int, dp]
        _lib.og_back.argtypes = [gp, dp, ip, ctypes.c_int, dp]
        _lib.og_weight.argtypes = [gp] + [ctypes.c_int] * 6
        _lib.og_weight.restype = ctypes.c_double
        _lib.og_dense.argtypes = [gp, ip, ctypes.c_int, dp]
        _lib.og_count_samples.argtypes = [gp, ip, ctypes.c_int]
        _lib.og_count_samples.restype = ctypes.c_longlong
        _lib.og_back_at.argtypes = [gp, dp, ip, ctypes.c_int, ip, ctypes.c_int, dp]
    return _lib


def _geom(cfg):
    g = _Geom()
    for name, _ in _Geom._fields_:
        setattr(g, name, cfg[name])
    return g


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def image_shape(cfg):
    return (cfg["nz"], cfg["ny"], cfg["nx"])


def _views(cfg, views):
    if views is None:
        views = np.arange(cfg["n_views"])
    return np.ascontiguousarray(np.asarray(views, dtype=np.int32))


# ---------------------------------------------------------------- projector

def ray(cfg, v, r, b):
    """Source point and unit direction of one ray (FP64)."""
    S = np.zeros(3)
    u = np.zeros(3)
    _L().og_ray(ctypes.byref(_geom(cfg)), v, r, b, _dp(S), _dp(u))
    return S, u


def forward(cfg, x, views=None):
    """A x for the listed views: ``[len(views)][n_rows][n_bins]``."""
    views = _views(cfg, views)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(image_shape(cfg))
    out = np.zeros((len(views), cfg["n_rows"], cfg["n_bins"]))
    _L().og_forward(ctypes.byref(_geom(cfg)), _dp(x), _ip(views), len(views), _dp(out))
    return out


def back(cfg, sino, views=None):
    """A' sino for the listed views (the transpose of :func:`forward`)."""
    views = _views(cfg, views)
    sino = np.ascontiguousarray(sino, dtype=np.float64).reshape(
        len(views), cfg["n_rows"], cfg["n_bins"])
    img = np.zeros(image_shape(cfg))
    _L().og_back(ctypes.byref(_geom(cfg)), _dp(sino), _ip(views), len(views), _dp(img))
    return img


def ray_integral(cfg, x, v, r, b):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(image_shape(cfg))
    return _L().og_ray_integral(ctypes.byref(_geom(cfg)), _dp(x), v, r, b)


def weight(cfg, v, r, b, i, j, k):
    return _L().og_weight(ctypes.byref(_geom(cfg)), v, r, b, i, j, k)


def back_at(cfg, sino, views, voxels):
    """Selected entries of A' sino, each summed over every ray on its own."""
    views = _views(cfg, views)
    sino = np.asarray(sino, dtype=np.float64).reshape(len(views), cfg["n_rows"], cfg["n_bins"])
    out = np.zeros(len(voxels))
    for n, (k, j, i) in enumerate(voxels):
        acc = 0.0
        for kv, v in enumerate(views):
            for r in range(cfg["n_rows"]):
                for b in range(cfg["n_bins"]):
                    if sino[kv, r, b] != 0.0:
                        wgt = weight(cfg, int(v), r, b, int(i), int(j), int(k))
                        if wgt != 0.0:
                            acc += wgt * sino[kv, r, b]
        out[n] = acc
    return out


def back_at_c(cfg, sino, views, voxels):
    """:func:`back_at` in C (the same sums, OpenMP over the entries): fast
    enough for sampled entries of full-size geometries."""
    views = _views(cfg, views)
    sino = np.ascontiguousarray(sino, dtype=np.float64).reshape(len(views), cfg["n_rows"], cfg["n_bins"])
    vox = np.ascontiguousarray(np.asarray(voxels, dtype=np.int32).reshape(-1, 3))
    out = np.zeros(len(vox))
    _L().og_back_at(ctypes.byref(_geom(cfg)), _dp(sino), _ip(views), len(views), _ip(vox), len(vox), _dp(out))
    return out


def dense(cfg, views=None):
    """Dense system matrix, rows (view, row, bin), columns (k, j, i)."""
    views = _views(cfg, views)
    nray = len(views) * cfg["n_rows"] * cfg["n_bins"]
    nvox = cfg["nx"] * cfg["ny"] * cfg["nz"]
    A = np.zeros((nray, nvox))
    _L().og_dense(ctypes.byref(_geom(cfg)), _ip(views), len(views), _dp(A))
    return A


def count_samples(cfg, views=None):
    """Joseph samples with at least one tap inside the volume."""
    views = _views(cfg, views)
    return int(_L().og_count_samples(ctypes.byref(_geom(cfg)), _ip(views), len(views)))


# ------------------------------------------------------------------ subsets

def subset_views(n_views, M):
    """Subset m holds the views v with v mod M == m (views spread uniformly
    over each subset, Sec. IV-B; interleaving is the reading used)."""
    return [np.arange(m, n_views, M) for m in range(M)]


def bit_reversal_order(M):
    """Subset visiting order (Sec. IV-A: bit-reversal order).  For M not a
    power of two: reverse j in ceil(log2 M) bits for j = 0 .. 2^B - 1 and
    keep the values below M (a reading)."""
    B = max(0, math.ceil(math.log2(M))) if M > 1 else 0
    out = []
    for j in range(1 << B):
        r = int(format(j, "0%db" % B)[::-1], 2) if B > 0 else 0
        if r < M:
            out.append(r)
    return np.array(out, dtype=np.int64)


def max_subsets_axial(n_views, s_axial=40.0):
    """Sec. IV-B, eq. "max_M_axial"."""
    return n_views / s_axial


def max_subsets_helical(views_per_turn, dso, dsd, pitch, s_helical=24.0):
    """Sec. IV-B, eq. "max_M_helical"."""
    return views_per_turn * dso / (pitch * s_helical * dsd)


# ------------------------------------------------------ continuation of rho

def rho_l(l, rho_min=1e-3):
    """Sec. III-B, eq. "rho_l_formula_qp": 1 at l = 0, else
    max(pi/(l+1) sqrt(1 - (pi/(2l+2))^2), rho_min)."""
    if l == 0:
        return 1.0
    v = math.pi / (l + 1) * math.sqrt(1.0 - (math.pi / (2 * l + 2)) ** 2)
    return max(v, rho_min)


# -------------------------------------------------------------- regularizer

def neighbour_offsets(is3d):
    """Half of the 8- (2D) or 26- (3D) neighbourhood, one offset per unordered
    pair, as (dz, dy, dx, kappa) with kappa = 1 / |offset| (index units)."""
    offs = []
    rng_z = (-1, 0, 1) if is3d else (0,)
    for dz in rng_z:
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dz, dy, dx) == (0, 0, 0):
                    continue
                if (dz, dy, dx) > (0, 0, 0):          # lexicographic half
                    offs.append((dz, dy, dx, 1.0 / math.sqrt(dz * dz + dy * dy + dx * dx)))
    return offs


def _pair_slices(shape, off):
    a, b = [], []
    for n, o in zip(shape, off):
        if o >= 0:
            a.append(slice(0, n - o)); b.append(slice(o, n))
        else:
            a.append(slice(-o, n)); b.append(slice(0, n + o))
    return tuple(a), tuple(b)


def potential(t, delta):
    """Hyperbola potential psi(t) = delta^2 (sqrt(1 + (t/delta)^2) - 1)."""
    return delta * delta * (np.sqrt(1.0 + (t / delta) ** 2) - 1.0)


def dpotential(t, delta):
    """psi'(t) = t / sqrt(1 + (t/delta)^2)."""
    return t / np.sqrt(1.0 + (t / delta) ** 2)


def reg_value(x, beta, delta, is3d):
    """R(x) = beta sum over neighbour pairs kappa psi(x_j - x_k)."""
    total = 0.0
    for dz, dy, dx, kap in neighbour_offsets(is3d):
        a, b = _pair_slices(x.shape, (dz, dy, dx))
        total += kap * np.sum(potential(x[a] - x[b], delta))
    return beta * total


def reg_grad(x, beta, delta, is3d):
    """Gradient of :func:`reg_value`."""
    g = np.zeros_like(x)
    for dz, dy, dx, kap in neighbour_offsets(is3d):
        a, b = _pair_slices(x.shape, (dz, dy, dx))
        d = kap * dpotential(x[a] - x[b], delta)
        g[a] += d
        g[b] -= d
    return beta * g


def reg_denom(shape, beta, is3d):
    """Separable quadratic majorizer curvature of R: since psi'' <= 1 and
    (t - t0)^2 <= 2 (x_j - x_j0)^2 + 2 (x_k - x_k0)^2, each voxel gets
    2 beta sum_{k in N(j)} kappa_jk (pairs leaving the grid dropped)."""
    c = np.zeros(shape)
    for dz, dy, dx, kap in neighbour_offsets(is3d):
        a, b = _pair_slices(shape, (dz, dy, dx))
        c[a] += kap
        c[b] += kap
    return 2.0 * beta * c


# ------------------------------------------------------------- PWLS pieces

def sqs_denom(cfg, w):
    """D_L = A' W A 1 (Sec. IV-A)."""
    ones = np.ones(image_shape(cfg))
    return back(cfg, w * forward(cfg, ones))


def cost(cfg, x, y, w, beta, delta):
    """Psi(x) = 1/2 ||y - A x||_W^2 + R(x) (Sec. IV, eq. "ct_recon");
    returns (total, data term, regularizer)."""
    is3d = cfg["kind"] != 0
    r = forward(cfg, x) - y
    data = 0.5 * float(np.sum(w * r * r))
    reg = float(reg_value(x.reshape(image_shape(cfg)), beta, delta, is3d))
    return data + reg, data, reg


def subset_gradient(cfg, x, y, w, views, M):
    """M grad l_m(x) = M A_m' W_m (A_m x - y_m) for the views of subset m."""
    r = w[views] * (forward(cfg, x, views) - y[views])
    return M * back(cfg, r, views)


def _xstep(x, num, den, nonneg):
    """One projected, diagonally majorized gradient step; voxels whose
    majorizer curvature is zero stay unchanged."""
    safe = np.where(den > 0, den, 1.0)
    xn = np.where(den > 0, x - num / safe, x)
    return np.maximum(xn, 0.0) if nonneg else xn


def inner_objective(z, x, s, DL, rho, beta, delta, is3d):
    """Objective of the inner constrained-denoising problem of eq.
    "os_lalm_iterates" with h = R + i_Omega (Sec. IV-A), up to a constant:
    R(z) + rho/2 ||z - x||^2_{D_L} + <s, z - x>  (equal to
    R(z) + rho/2 ||z - (x - (rho D_L)^-1 s)||^2_{D_L} where D_L > 0); the
    constraint z >= 0 is not included."""
    d = z - x
    return float(reg_value(z, beta, delta, is3d) + 0.5 * rho * np.sum(DL * d * d) + np.sum(s * d))


def inner_fista(x, s, DL, DR, rho, beta, delta, is3d, n, nonneg=True):
    """n iterations of FISTA (Beck & Teboulle) on the inner problem of
    :func:`inner_objective`, from the warm start z = x (Sec. IV-A).  The
    smooth part's gradient rho D_L (z - x) + s + grad R(z) is majorized by the
    diagonal rho D_L + D_R; the proximal step is the projection onto Omega
    (the nonnegativity clamp).  Momentum: t_1 = 1,
    t_{i+1} = (1 + sqrt(1 + 4 t_i^2)) / 2, z <- v_i + (t_i - 1)/t_{i+1} (v_i - v_{i-1}).
    n = 1 is one projected gradient step from x."""
    den = rho * DL + DR
    v_prev, z, t = x, x, 1.0
    for _ in range(n):
        grad = rho * DL * (z - x) + s + reg_grad(z, beta, delta, is3d)
        v = _xstep(z, grad, den, nonneg)
        t_next = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        z = v + ((t - 1.0) / t_next) * (v - v_prev)
        v_prev, t = v, t_next
    return v_prev


def bb_alpha(s, yv, DL, alpha_min):
    """Barzilai-Borwein scale of the SQS Hessian (supplement, eq.
    "scale_factor_alpha_k"): alpha = argmin_{alpha <= 1} 1/2 ||y - alpha L s||^2_P
    with P = L^-1 and L = D_L, i.e. <s, y> / <s, L s> capped at 1.  Readings:
    a non-positive <s, y> or <s, L s> (no curvature information) gives 1, and
    alpha is kept at or above alpha_min."""
    sy = float(np.sum(s * yv))
    sls = float(np.sum(DL * s * s))
    if not (sy > 0.0 and sls > 0.0):
        return 1.0
    return min(1.0, max(alpha_min, sy / sls))


def os_lalm(cfg, y, w, beta, delta, M, n_steps, continuation=True, rho_fixed=1.0,
            rho_min=1e-3, x0=None, denom=None, forced_restart=None, nonneg=True,
            callback=None, n_inner=1, bb=False, bb_alpha_min=0.01, history=None):
    """OS-LALM, Sec. III-A eq. "os_lalm_iterates".

    The substitution of eq. "ct_substitution" makes grad l_m the weighted
    subset gradient; the inner constrained-denoising problem
    min_z R(z) + i_Omega(z) + rho/2 ||z - (x - (rho D_L)^-1 s)||^2_{D_L}
    gets n_inner FISTA iterations from the warm start z = x
    (:func:`inner_fista`); n_inner = 1 is one projected gradient step with
    the diagonal majorizer rho D_L + D_R (the first FISTA step has no
    momentum).

    bb: the Barzilai-Borwein acceleration of the supplement, H_k = alpha_k
    D_L in place of D_L.  Readings: k counts iterations (M subset steps);
    alpha_k (:func:`bb_alpha`) is computed at the start of iteration k >= 1
    from s = x - x_prev and y = G - G_prev, the images and the scaled
    gradients M grad l_{order[0]} held at the starts of iterations k and
    k - 1 (the same subset, so y is a gradient difference), and is used for
    the M steps of iteration k; alpha_0 = 1.

    Step j (0-based) visits subset order[(j + 1) mod M] for the gradient at
    the new image; the initial gradient is G = M grad l_{order[0]}(x0) and
    the split gradient starts as g = G (u0 = A x0, Sec. III-A).

    Continuation (Sec. III-B): after each subset step,
    xi = <g_old - G_new, G_new - G_old> (gradients replaced by the subset
    approximations); l is reset to 0 when xi > 0, else incremented; the next
    step uses rho_l.  ``forced_restart`` (bool per step) overrides the sign
    test, for replaying a restart sequence.

    ``callback(j, x)`` runs after step j; ``history``, a dict, receives the
    live per-step lists rho, xi and restart at the start (so a callback can
    read them while the run goes on); if it holds a list under "g", the
    split gradient g before every step and after the last is appended to it,
    and likewise the scaled subset gradient G for a list under "G".

    Returns a dict with x, g, G and per-step arrays rho, xi, restart.
    """
    is3d = cfg["kind"] != 0
    shape = image_shape(cfg)
    subsets = subset_views(cfg["n_views"], M)
    order = bit_reversal_order(M)
    x = np.zeros(shape) if x0 is None else np.array(x0, dtype=np.float64).reshape(shape)
    DL = sqs_denom(cfg, w) if denom is None else np.asarray(denom, dtype=np.float64).reshape(shape)
    DR = reg_denom(shape, beta, is3d)
    G = subset_gradient(cfg, x, y, w, subsets[order[0]], M)
    g = G.copy()
    l = 0
    rho = 1.0 if continuation else rho_fixed
    hist_rho, hist_xi, hist_rs, hist_alpha = [], [], [], []
    keep_g = history is not None and isinstance(history.get("g"), list)
    keep_G = history is not None and isinstance(history.get("G"), list)
    if history is not None:
        history.update(rho=hist_rho, xi=hist_xi, restart=hist_rs)
    if keep_g:
        history["g"].append(g.copy())
    if keep_G:
        history["G"].append(G.copy())
    alpha, x_prev, G_prev = 1.0, None, None
    for j in range(n_steps):
        if bb and j % M == 0:
            if j > 0:
                alpha = bb_alpha(x - x_prev, G - G_prev, DL, bb_alpha_min)
            x_prev, G_prev = x.copy(), G.copy()
        H = alpha * DL
        s = rho * G + (1.0 - rho) * g
        if n_inner == 1:
            x_new = _xstep(x, s + reg_grad(x, beta, delta, is3d), rho * H + DR, nonneg)
        else:
            x_new = inner_fista(x, s, H, DR, rho, beta, delta, is3d, n_inner, nonneg)
        hist_alpha.append(alpha)
        G_new = subset_gradient(cfg, x_new, y, w, subsets[order[(j + 1) % M]], M)
        g_new = (rho * G_new + g) / (rho + 1.0)
        xi = float(np.sum((g - G_new) * (G_new - G)))
        hist_rho.append(rho)
        hist_xi.append(xi)
        restart = False
        if continuation:
            restart = xi > 0.0
            if forced_restart is not None and j < len(forced_restart):
                restart = bool(forced_restart[j])
            l = 0 if restart else l + 1
            rho = rho_l(l, rho_min)
        hist_rs.append(restart)
        x, g, G = x_new, g_new, G_new
        if keep_g:
            history["g"].append(g.copy())
        if keep_G:
            history["G"].append(G.copy())
        if callback is not None:
            callback(j, x)
    return dict(x=x, g=g, G=G, rho=np.array(hist_rho), xi=np.array(hist_xi),
                restart=np.array(hist_rs), l=l, next_rho=rho, alpha=np.array(hist_alpha))


def fista_restart(cfg, y, w, beta, delta, x0, n_iter, denom=None, nonneg=True):
    """Reference solution x*: one-subset FISTA (Beck & Teboulle) with the
    separable majorizer D_L + D_R, projection onto x >= 0, and gradient-based
    adaptive restart (O'Donoghue & Candes): momentum is reset whenever
    <D (z - x_new), x_new - x> > 0 (Sec. V)."""
    is3d = cfg["kind"] != 0
    shape = image_shape(cfg)
    DL = sqs_denom(cfg, w) if denom is None else np.asarray(denom).reshape(shape)
    D = DL + reg_denom(shape, beta, is3d)
    x = np.array(x0, dtype=np.float64).reshape(shape)
    z = x.copy()
    t = 1.0
    for _ in range(n_iter):
        grad = back(cfg, w * (forward(cfg, z) - y)) + reg_grad(z, beta, delta, is3d)
        x_new = _xstep(z, grad, D, nonneg)
        if float(np.sum(D * (z - x_new) * (x_new - x))) > 0.0:
            t = 1.0
            z = x_new.copy()
        else:
            t_new = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
            z = x_new + ((t - 1.0) / t_new) * (x_new - x)
            t = t_new
        x = x_new
    return x


# ------------------------------------- textbook linearized AL (dense, M = 1)

def lalm_textbook_dense(A, y, w, rho, n_iter, DL, reg=None, DR=None, x0=None, nonneg=True):
    """Linearized AL iterates with split variable u and scaled multiplier d
    (Sec. II-A, eq. "general_lal_iterates"), for g(u) = 1/2 ||y - u||^2 after
    the substitution A <- W^1/2 A, y <- W^1/2 y (Sec. IV-A): the x-update is
    the diagonally majorized proximal step, the u-update is the closed form
    of eq. "lalm_pls_u", the d-update is the multiplier ascent.  Initial
    u0 = A x0 and d0 = (y - u0) / rho (Sec. III-A).  ``reg`` is a callable
    returning grad R (one majorized step with curvature rho D_L + D_R).

    Returns the list of iterates x^k and the list of u^k + rho d^k."""
    sw = np.sqrt(w)
    As = sw[:, None] * A
    ys = sw * y
    n = A.shape[1]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    u = As @ x
    d = (ys - u) / rho
    DR = np.zeros(n) if DR is None else DR
    xs, ident = [x.copy()], []
    for _ in range(n_iter):
        s = rho * (As.T @ (As @ x - u - d))
        num = s + (reg(x) if reg is not None else 0.0)
        x = _xstep(x, num, rho * DL + DR, nonneg)
        Ax = As @ x
        u = rho / (rho + 1.0) * (Ax - d) + ys / (rho + 1.0)
        d = d - Ax + u
        xs.append(x.copy())
        ident.append(u + rho * d)
    return xs, ident


def lalm_gradient_dense(A, y, w, rho, n_iter, DL, reg=None, DR=None, x0=None, nonneg=True):
    """Gradient-based LALM (Sec. III-A, eq. "lalm_iterates") on a dense
    matrix, M = 1, fixed rho, g0 = grad l(x0)."""
    grad = lambda x: A.T @ (w * (A @ x - y))
    n = A.shape[1]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    DR = np.zeros(n) if DR is None else DR
    gl = grad(x)
    g = gl.copy()
    xs = [x.copy()]
    for _ in range(n_iter):
        s = rho * gl + (1.0 - rho) * g
        num = s + (reg(x) if reg is not None else 0.0)
        x = _xstep(x, num, rho * DL + DR, nonneg)
        gl = grad(x)
        g = rho / (rho + 1.0) * gl + g / (rho + 1.0)
        xs.append(x.copy())
    return xs


# ------------------------------------------------------ toy quadratic (III-B)

def toy_iteration_matrix(lam_over_L, rho):
    """2x2 linear map of one eigen-component (x_i, g_i) of the gradient LALM
    on min 1/2 ||A x||^2 (Sec. III-B, eq. "ith_lalm_iterates_qp"), with
    lambda_i/L = q and g scaled by 1/L."""
    q = lam_over_L
    # x+ = x - q x - (1/rho - 1) g ;  g+ = rho/(rho+1) q x+ + g/(rho+1)
    a11, a12 = 1.0 - q, -(1.0 / rho - 1.0)
    b = rho / (rho + 1.0) * q
    return np.array([[a11, a12], [b * a11, b * a12 + 1.0 / (rho + 1.0)]])


def toy_char_poly(lam_over_L, rho):
    """Coefficients of (1+rho) r^2 - 2 (1 - q + rho/2) r + (1 - q)
    (eq. "char_poly_qp")."""
    q = lam_over_L
    return np.array([1.0 + rho, -2.0 * (1.0 - q + rho / 2.0), 1.0 - q])


def toy_rho_critical(lam_over_L):
    """eq. "critical_value_qp"."""
    q = lam_over_L
    return 2.0 * math.sqrt(q * (1.0 - q))


def toy_rate(lam_over_L, rho):
    """Per-iteration contraction of one eigen-component: the larger root
    modulus.  Over-damped: eq. "over_damp_rate_qp"; critical: eq.
    "critical_damp_rate_qp"; under-damped: the modulus of the complex pair,
    sqrt((1 - q) / (1 + rho)) (the product of the two roots) -- the paper's
    eq. "under_damp_rate_qp" prints the real part instead (a reading)."""
    q = lam_over_L
    rc = toy_rho_critical(q)
    if rho >= rc:
        return (1.0 - q + rho / 2.0 + math.sqrt(max(0.0, rho * rho / 4.0 - q * (1.0 - q)))) / (1.0 + rho)
    return math.sqrt((1.0 - q) / (1.0 + rho))


def toy_run(lams, L, n_iter, rho=None, continuation=False, rho_min=1e-3, x0=None):
    """Gradient LALM on min 1/2 ||A x||^2 with A'A = diag(lams)
    (Sec. III-B, eq. "lalm_iterates_qp"), optionally with the downward
    continuation.  Returns the x history, the restart steps and the restart
    indicator xi of eq. "period_indicator_qp" at every step."""
    lams = np.asarray(lams, dtype=np.float64)
    x = np.ones_like(lams) if x0 is None else np.array(x0, dtype=np.float64)
    gl = lams * x
    g = gl.copy()
    l = 0
    r = 1.0 if continuation else rho
    xs, restarts, xis = [x.copy()], [], []
    for k in range(n_iter):
        x_new = x - (gl + (1.0 / r - 1.0) * g) / L
        gl_new = lams * x_new
        g_new = r / (r + 1.0) * gl_new + g / (r + 1.0)
        xi = float(np.dot(g - gl_new, gl_new - gl))
        xis.append(xi)
        if continuation:
            if xi > 0.0:
                l = 0
                restarts.append(k)
            else:
                l += 1
            r = rho_l(l, rho_min)
        x, g, gl = x_new, g_new, gl_new
        xs.append(x.copy())
    return np.array(xs), restarts, np.array(xis)


# ------------------------------------------------------------ figure of merit

def rmsd_hu(a, b, mask, hu_per_mu):
    """RMS difference over the ROI, in HU (Sec. V)."""
    d = (np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))[mask]
    return float(np.sqrt(np.mean(d * d)) * hu_per_mu)


# ------------------------------------------------------------- FBP (x0)

def fbp_fan(cfg, sino):
    """Filtered back-projection for the 2D equiangular (arc-detector) fan
    beam over a full turn, the initial image the paper's experiments start
    from (figure captions).  The paper gives no formula; this is the textbook
    equiangular fan-beam reconstruction (reading): cosine-weighted data
    q = p D cos(gamma); the fan-beam ramp kernel
    g(n dgamma) = 1/2 (n dgamma / sin(n dgamma))^2 h(n dgamma) with the
    band-limited (Ram-Lak) ramp h(0) = 1/(4 dgamma^2), h(odd n) =
    -1/(n pi dgamma)^2, h(even n != 0) = 0; Q = dgamma (q * g); and
    f(P) = dbeta sum_views Q(gamma'(P)) / L(P)^2, with L the distance from
    the source to P and gamma'(P) the fan angle of the ray through P, Q
    interpolated linearly in channel (zero off the detector).

    sino: natural-order [n_views][1][n_bins] (or [n_views][n_bins]) line
    integrals.  Returns [1][ny][nx]."""
    if cfg["kind"] != 0 or cfg["n_views"] != cfg["n_views_per_turn"]:
        raise ValueError("fbp_fan: 2D fan beam over one full turn only")
    nb, nv = cfg["n_bins"], cfg["n_views"]
    p = np.asarray(sino, dtype=np.float64).reshape(nv, nb)
    dg = cfg["ds"] / cfg["dsd"]
    D = cfg["dso"]
    gam = (np.arange(nb) - (nb - 1) / 2.0 - cfg["channel_offset"]) * dg
    q = p * (D * np.cos(gam))[None, :]
    n = np.arange(-(nb - 1), nb)
    h = np.zeros(n.shape)
    h[n == 0] = 1.0 / (4.0 * dg * dg)
    odd = (n % 2) != 0
    h[odd] = -1.0 / (n[odd] * np.pi * dg) ** 2
    ratio = np.ones(n.shape)
    nz = n != 0
    ratio[nz] = (n[nz] * dg) / np.sin(n[nz] * dg)
    g = 0.5 * ratio * ratio * h
    Q = np.empty_like(q)
    for v in range(nv):
        Q[v] = dg * np.convolve(q[v], g)[nb - 1:2 * nb - 1]
    nx, ny = cfg["nx"], cfg["ny"]
    X = (np.arange(nx) - (nx - 1) / 2.0) * cfg["dx"]
    Y = (np.arange(ny) - (ny - 1) / 2.0) * cfg["dy"]
    PX, PY = np.meshgrid(X, Y)
    dbeta = 2.0 * np.pi / cfg["n_views_per_turn"]
    f = np.zeros((ny, nx))
    for v in range(nv):
        beta = cfg["start_angle"] + 2.0 * np.pi * v / cfg["n_views_per_turn"]
        sx, sy = D * np.cos(beta), D * np.sin(beta)
        dx_, dy_ = PX - sx, PY - sy
        along = -(dx_ * np.cos(beta) + dy_ * np.sin(beta))       # towards the isocentre
        perp = dx_ * np.sin(beta) - dy_ * np.cos(beta)           # central ray rotated +90 deg
        gp = np.arctan2(perp, along)
        bc = gp / dg + (nb - 1) / 2.0 + cfg["channel_offset"]
        b0 = np.floor(bc).astype(np.int64)
        t = bc - b0
        val = np.zeros_like(bc)
        for bb, wgt in ((b0, 1.0 - t), (b0 + 1, t)):
            ok = (bb >= 0) & (bb < nb)
            val[ok] += wgt[ok] * Q[v, bb[ok]]
        f += dbeta * val / (dx_ * dx_ + dy_ * dy_)
    return f[None]


def _fan_ramp_kernel(nb, dg):
    """The equiangular fan-beam Ram-Lak kernel of :func:`fbp_fan` on the
    offsets n = -(nb-1) .. nb-1: g(n dg) = 1/2 (n dg / sin(n dg))^2 h(n dg)."""
    n = np.arange(-(nb - 1), nb)
    h = np.zeros(n.shape)
    h[n == 0] = 1.0 / (4.0 * dg * dg)
    odd = (n % 2) != 0
    h[odd] = -1.0 / (n[odd] * np.pi * dg) ** 2
    ratio = np.ones(n.shape)
    nz = n != 0
    ratio[nz] = (n[nz] * dg) / np.sin(n[nz] * dg)
    return 0.5 * ratio * ratio * h


def fbp_cone_axial(cfg, sino, voxels=None):
    """Initial image for the axial cone beam: the FDK reconstruction
    (Feldkamp, Davis & Kress) for the cylindrical (arc) detector over a full
    turn; the paper's experiments start from an FBP image (figure captions)
    and give no formula, so this is the textbook reading:

    1. cosine weights of the fan and the cone angle,
       q = p D cos(gamma) dsd / sqrt(dsd^2 + v_r^2)  (D = dso, v_r the row
       height at the detector, which is a cylinder of radius dsd about the
       source);
    2. every detector row filtered along the channels with the fan-beam
       kernel of :func:`fbp_fan`, Q = dgamma (q * g);
    3. f(P) = dbeta sum_views Q(gamma'(P), v'(P)) / L(P)^2, L the in-plane
       distance from the source to P, gamma'(P) the fan angle of P and
       v'(P) = (z_P - z_s) dsd / L the height at which the ray through P
       meets the detector; Q interpolated bilinearly in (channel, row), zero
       off the detector.

    With one detector row at v = 0 and one slice it is :func:`fbp_fan`.

    sino: natural-order [n_views][n_rows][n_bins] line integrals.  Returns
    the image [nz][ny][nx], or, with voxels (a list of (k, j, i)), the
    values at those voxels only."""
    if cfg["kind"] != 1 or cfg["n_views"] != cfg["n_views_per_turn"]:
        raise ValueError("fbp_cone_axial: axial cone beam over one full turn only")
    nb, nr, nv = cfg["n_bins"], cfg["n_rows"], cfg["n_views"]
    p = np.asarray(sino, dtype=np.float64).reshape(nv, nr, nb)
    dg = cfg["ds"] / cfg["dsd"]
    D, dsd = cfg["dso"], cfg["dsd"]
    gam = (np.arange(nb) - (nb - 1) / 2.0 - cfg["channel_offset"]) * dg
    vr = (np.arange(nr) - (nr - 1) / 2.0) * cfg["dt"]
    q = p * (D * np.cos(gam))[None, None, :] * (dsd / np.sqrt(dsd * dsd + vr * vr))[None, :, None]
    g = _fan_ramp_kernel(nb, dg)
    # Toeplitz matrix of the convolution restricted to the detector: T[k, b] = g(b - k)
    kk, bb = np.meshgrid(np.arange(nb), np.arange(nb), indexing="ij")
    T = g[(bb - kk) + (nb - 1)]
    Q = dg * (q.reshape(-1, nb) @ T).reshape(nv, nr, nb)
    nx, ny, nz = cfg["nx"], cfg["ny"], cfg["nz"]
    if voxels is None:
        K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    else:
        vox = np.asarray(voxels, dtype=np.int64).reshape(-1, 3)
        K, J, I = vox[:, 0], vox[:, 1], vox[:, 2]
    PX = (I - (nx - 1) / 2.0) * cfg["dx"]
    PY = (J - (ny - 1) / 2.0) * cfg["dy"]
    PZ = (K - (nz - 1) / 2.0) * cfg["dz"]
    dbeta = 2.0 * np.pi / cfg["n_views_per_turn"]
    f = np.zeros(PX.shape)
    for v in range(nv):
        beta = cfg["start_angle"] + 2.0 * np.pi * v / cfg["n_views_per_turn"]
        sx, sy = D * np.cos(beta), D * np.sin(beta)
        dx_, dy_ = PX - sx, PY - sy
        along = -(dx_ * np.cos(beta) + dy_ * np.sin(beta))
        perp = dx_ * np.sin(beta) - dy_ * np.cos(beta)
        L2 = dx_ * dx_ + dy_ * dy_
        bc = np.arctan2(perp, along) / dg + (nb - 1) / 2.0 + cfg["channel_offset"]
        rc = PZ * dsd / np.sqrt(L2) / cfg["dt"] + (nr - 1) / 2.0
        b0 = np.floor(bc).astype(np.int64)
        r0 = np.floor(rc).astype(np.int64)
        tb, tr = bc - b0, rc - r0
        val = np.zeros(PX.shape)
        for rr, wr in ((r0, 1.0 - tr), (r0 + 1, tr)):
            for b_, wb in ((b0, 1.0 - tb), (b0 + 1, tb)):
                ok = (b_ >= 0) & (b_ < nb) & (rr >= 0) & (rr < nr)
                val[ok] += (wr * wb)[ok] * Q[v, rr[ok], b_[ok]]
        f += dbeta * val / L2
    return f
