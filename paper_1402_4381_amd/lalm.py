"""Python binding of ``liblalm.so`` (argument marshalling only).

Every function here has the name of the C ABI call it wraps (``include/
lalm.h``) and does nothing but check and pass pointers, sizes and the HIP
stream; all arithmetic runs in the library's gfx950 kernels.  Device buffers
are torch tensors on the GPU (float32, contiguous); the stream defaults to
torch's current stream.  The library must be built first
(``python -m paper_1402_4381_amd.build``); importing this module without it
raises ImportError, and there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblalm.so")

LALM_OK, LALM_E_INVALID, LALM_E_HIP, LALM_E_NOMEM, LALM_E_NONFINITE, LALM_E_STATE = 0, -1, -2, -3, -4, -5
FAN2D, CONE_AXIAL, CONE_HELICAL = 0, 1, 2

EXPORTS = ("lalm_last_error", "lalm_version", "lalm_plan_geometry", "lalm_plan_info",
           "lalm_plan_destroy", "lalm_project_subset", "lalm_backproject_subset",
           "lalm_sqs_denom", "lalm_fbp", "lalm_iterate", "lalm_cost_f64", "lalm_dot_f64",
           "lalm_roi_rmsd_f64", "lalm_profile_begin", "lalm_profile_read",
           "lalm_profile_end", "lalm_unet_param_count", "lalm_unet_create",
           "lalm_unet_destroy", "lalm_unet_forward", "lalm_unet_loss_grad", "lalm_unet_adam",
           "lalm_unet_capture_elems", "lalm_unet_capture", "lalm_dot_f64_noalloc")


class LalmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("lalm status %d: %s" % (status, msg))
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("dz", ctypes.c_double), ("n_views", ctypes.c_int32),
                ("n_views_per_turn", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("n_rows", ctypes.c_int32), ("ds", ctypes.c_double), ("dt", ctypes.c_double),
                ("dso", ctypes.c_double), ("dsd", ctypes.c_double),
                ("start_angle", ctypes.c_double), ("pitch", ctypes.c_double),
                ("channel_offset", ctypes.c_double), ("detector", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [("y", ctypes.c_void_p), ("w", ctypes.c_void_p), ("denom", ctypes.c_void_p),
                ("beta", ctypes.c_double), ("delta", ctypes.c_double), ("nonneg", ctypes.c_int32)]


class State(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("g", ctypes.c_void_p), ("grad", ctypes.c_void_p),
                ("step", ctypes.c_int64), ("l", ctypes.c_int64), ("rho", ctypes.c_double),
                ("x_prev", ctypes.c_void_p), ("grad_prev", ctypes.c_void_p), ("alpha", ctypes.c_double),
                ("l_b", ctypes.c_void_p), ("rho_b", ctypes.c_void_p), ("alpha_b", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("continuation", ctypes.c_int32), ("rho_fixed", ctypes.c_double),
                ("rho_min", ctypes.c_double), ("n_inner", ctypes.c_int32),
                ("forced_restart", ctypes.c_void_p), ("forced_len", ctypes.c_int64),
                ("bb", ctypes.c_int32), ("bb_alpha_min", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_void_p), ("xi", ctypes.c_void_p), ("restart", ctypes.c_void_p),
                ("capacity", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblalm.so is not built (python -m paper_1402_4381_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32, I64, F32, F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    sig = {
        "lalm_last_error": ([], ctypes.c_char_p),
        "lalm_version": ([], ctypes.c_char_p),
        "lalm_plan_geometry": ([ctypes.POINTER(Geometry), I32, I32, ctypes.POINTER(P)], I32),
        "lalm_plan_info": ([P, P, P, P, P, P, P], I32),
        "lalm_plan_destroy": ([P], I32),
        "lalm_project_subset": ([P, I32, P, P, P, P, P], I32),
        "lalm_backproject_subset": ([P, I32, P, P, F32, I32, P], I32),
        "lalm_sqs_denom": ([P, P, P, P], I32),
        "lalm_fbp": ([P, P, P, P], I32),
        "lalm_iterate": ([P, ctypes.POINTER(Problem), ctypes.POINTER(State), I64,
                          ctypes.POINTER(Options), ctypes.POINTER(Stats), P], I32),
        "lalm_cost_f64": ([P, ctypes.POINTER(Problem), P, P, P], I32),
        "lalm_dot_f64": ([P, P, P, I64, P, P], I32),
        "lalm_dot_f64_noalloc": ([P, P, I64, P, P], I32),
        "lalm_roi_rmsd_f64": ([P, P, P, F64, P, P], I32),
        "lalm_profile_begin": ([P], I32),
        "lalm_profile_read": ([P, P, P], I32),
        "lalm_profile_end": ([P], I32),
        "lalm_unet_param_count": ([], I64),
        "lalm_unet_create": ([I32, I32, I32, ctypes.POINTER(P)], I32),
        "lalm_unet_destroy": ([P], I32),
        "lalm_unet_forward": ([P, P, P, P, I32, F64, I32, P], I32),
        "lalm_unet_loss_grad": ([P, P, P, P, P, F64, F64, I32, P, P, P], I32),
        "lalm_unet_adam": ([P, P, P, P, P, I64, F64, P], I32),
        "lalm_unet_capture_elems": ([I32, I32, I32], I64),
        "lalm_unet_capture": ([P, P, P, P, P, F64, F64, I32, P, P, P, I64, P], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()


def _check(status):
    if status != LALM_OK:
        raise LalmError(status, _lib.lalm_last_error().decode())


def _dev(t, name, dtype="float32", numel=None, allow_none=False):
    """Device address of a contiguous GPU tensor (validated)."""
    if t is None:
        if allow_none:
            return None
        raise ValueError("%s: a tensor is required" % name)
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s: expected a GPU tensor" % name)
    if str(t.dtype) != "torch." + dtype:
        raise ValueError("%s: expected %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s: expected a contiguous tensor" % name)
    if numel is not None and t.numel() < numel:
        raise ValueError("%s: needs %d elements, has %d" % (name, numel, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def lalm_version():
    return _lib.lalm_version().decode()


def lalm_last_error():
    return _lib.lalm_last_error().decode()


class Plan:
    """Owner of a ``lalm_plan`` handle and its host-side facts.  ``batch``
    images are planned together; image_elems and sino_elems are those of
    one image."""

    def __init__(self, handle, geom, n_subsets, batch=1):
        self.handle = handle
        self.geom = dict(geom)
        self.M = n_subsets
        self.B = int(batch)
        n_views = geom["n_views"]
        img = ctypes.c_int64()
        sino = ctypes.c_int64()
        off = np.zeros(n_subsets + 1, dtype=np.int64)
        order = np.zeros(n_subsets, dtype=np.int32)
        vos = np.zeros(n_views, dtype=np.int32)
        samp = np.zeros(n_subsets, dtype=np.int64)
        _check(_lib.lalm_plan_info(handle, ctypes.byref(img), ctypes.byref(sino),
                                   off.ctypes.data_as(ctypes.c_void_p),
                                   order.ctypes.data_as(ctypes.c_void_p),
                                   vos.ctypes.data_as(ctypes.c_void_p),
                                   samp.ctypes.data_as(ctypes.c_void_p)))
        self.image_elems = img.value
        self.sino_elems = sino.value
        self.subset_ray_offset = off
        self.order = order
        self.view_of_slot = vos
        self.subset_samples = samp
        self.image_shape = (geom["nz"], geom["ny"], geom["nx"])
        self.rays_per_view = geom["n_rows"] * geom["n_bins"]

    def subset_rays(self, m):
        if not 0 <= m < self.M:
            return 0          # out-of-range subsets are rejected by the library
        return int(self.subset_ray_offset[m + 1] - self.subset_ray_offset[m])

    def subset_slice(self, m):
        return slice(int(self.subset_ray_offset[m]), int(self.subset_ray_offset[m + 1]))

    def subset_views(self, m):
        a = self.subset_ray_offset[m] // self.rays_per_view
        b = self.subset_ray_offset[m + 1] // self.rays_per_view
        return self.view_of_slot[a:b]

    def to_subset_major(self, sino):
        """Natural-order sinogram ``[n_views, rows, bins]`` -> flat subset-major
        (a permutation of whole views)."""
        return sino[self.view_of_slot].reshape(-1)

    def from_subset_major(self, flat):
        nv = self.geom["n_views"]
        s = flat.reshape(nv, self.geom["n_rows"], self.geom["n_bins"])
        out = s.clone() if hasattr(s, "clone") else s.copy()
        out[self.view_of_slot] = s
        return out

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                _lib.lalm_plan_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def _geometry(geom):
    g = Geometry()
    for name, _ in Geometry._fields_:
        setattr(g, name, geom[name])
    return g


def lalm_plan_geometry(geom, n_subsets, batch=1):
    """Plan a geometry (a dict with the ``lalm_geometry`` fields) for
    ``batch`` images reconstructed together."""
    h = ctypes.c_void_p()
    _check(_lib.lalm_plan_geometry(ctypes.byref(_geometry(geom)), int(n_subsets), int(batch), ctypes.byref(h)))
    return Plan(h, geom, int(n_subsets), int(batch))


def lalm_plan_info(plan):
    return dict(image_elems=plan.image_elems, sino_elems=plan.sino_elems,
                subset_ray_offset=plan.subset_ray_offset.copy(), order=plan.order.copy(),
                view_of_slot=plan.view_of_slot.copy(), subset_samples=plan.subset_samples.copy())


def lalm_plan_destroy(plan):
    if plan.handle:
        _check(_lib.lalm_plan_destroy(plan.handle))
        plan.handle = None


def lalm_project_subset(plan, m, x, out, y=None, w=None, stream=None):
    n = plan.subset_rays(m) * plan.B
    _check(_lib.lalm_project_subset(plan.handle, int(m), _dev(x, "x", numel=plan.image_elems * plan.B),
                                    _dev(out, "out", numel=n), _dev(y, "y", numel=n, allow_none=True),
                                    _dev(w, "w", numel=n, allow_none=True), _stream(stream)))


def lalm_backproject_subset(plan, m, r, x_out, scale=1.0, accumulate=False, stream=None):
    _check(_lib.lalm_backproject_subset(plan.handle, int(m), _dev(r, "r", numel=plan.subset_rays(m) * plan.B),
                                        _dev(x_out, "x_out", numel=plan.image_elems * plan.B), float(scale),
                                        1 if accumulate else 0, _stream(stream)))


def lalm_sqs_denom(plan, w_full, denom, stream=None):
    _check(_lib.lalm_sqs_denom(plan.handle, _dev(w_full, "w_full", numel=plan.sino_elems * plan.B),
                               _dev(denom, "denom", numel=plan.image_elems * plan.B), _stream(stream)))


def lalm_fbp(plan, y_full, x_out, stream=None):
    _check(_lib.lalm_fbp(plan.handle, _dev(y_full, "y_full", numel=plan.sino_elems * plan.B),
                         _dev(x_out, "x_out", numel=plan.image_elems * plan.B), _stream(stream)))


def _problem(plan, y, w, denom, beta, delta, nonneg):
    B = plan.B
    return Problem(_dev(y, "y", numel=plan.sino_elems * B), _dev(w, "w", numel=plan.sino_elems * B),
                   _dev(denom, "denom", numel=plan.image_elems * B) if denom is not None else None,
                   float(beta), float(delta), 1 if nonneg else 0)


class LalmState:
    """Caller-owned iteration state: GPU images x, g, grad, the scalars and,
    for the Barzilai-Borwein option, the images at the start of the current
    iteration (x_prev, grad_prev) and the scale alpha.  For a batch of B
    images the tensors hold B images and ``l_b``, ``rho_b``, ``alpha_b``
    (numpy arrays of B entries) the continuation state of each image; the
    scalar fields then mirror image 0."""

    def __init__(self, x, g, grad, step=0, l=0, rho=1.0, x_prev=None, grad_prev=None, alpha=1.0, batch=1):
        self.x, self.g, self.grad = x, g, grad
        self.step, self.l, self.rho = int(step), int(l), float(rho)
        self.x_prev, self.grad_prev, self.alpha = x_prev, grad_prev, float(alpha)
        self.batch = int(batch)
        self.l_b = np.full(self.batch, self.l, dtype=np.int64)
        self.rho_b = np.full(self.batch, self.rho, dtype=np.float64)
        self.alpha_b = np.full(self.batch, self.alpha, dtype=np.float64)

    @classmethod
    def zeros_like(cls, x, bb=False, batch=1):
        import torch
        z = torch.zeros_like
        return cls(x, z(x), z(x), x_prev=z(x) if bb else None, grad_prev=z(x) if bb else None, batch=batch)

    def clone(self):
        c = lambda t: None if t is None else t.clone()
        s = LalmState(self.x.clone(), self.g.clone(), self.grad.clone(), self.step, self.l, self.rho,
                      c(self.x_prev), c(self.grad_prev), self.alpha, self.batch)
        s.l_b, s.rho_b, s.alpha_b = self.l_b.copy(), self.rho_b.copy(), self.alpha_b.copy()
        return s


def lalm_iterate(plan, y, w, denom, beta, delta, state, n_steps, continuation=True,
                 rho_fixed=1.0, rho_min=1e-3, n_inner=1, nonneg=True, forced_restart=None,
                 stats=None, stream=None, bb=False, bb_alpha_min=0.01):
    """Run ``n_steps`` subset steps; ``state`` (LalmState) is updated in place.
    ``stats``: optional dict of GPU tensors rho (float64), xi (float64),
    restart (uint8) indexed by global step ([batch][capacity] for a batch).
    ``forced_restart``: optional uint8 GPU tensor indexed by global step
    ([batch][length] for a batch)."""
    prob = _problem(plan, y, w, denom, beta, delta, nonneg)
    nimg = plan.image_elems * plan.B
    if state.batch != plan.B:
        raise ValueError("state holds %d images, the plan %d" % (state.batch, plan.B))
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
    st = State(_dev(state.x, "x", numel=nimg), _dev(state.g, "g", numel=nimg),
               _dev(state.grad, "grad", numel=nimg), state.step, state.l, state.rho,
               _dev(state.x_prev, "x_prev", numel=nimg, allow_none=True),
               _dev(state.grad_prev, "grad_prev", numel=nimg, allow_none=True), state.alpha,
               ptr(state.l_b), ptr(state.rho_b), ptr(state.alpha_b))
    fr = _dev(forced_restart, "forced_restart", dtype="uint8", allow_none=True)
    opt = Options(1 if continuation else 0, float(rho_fixed), float(rho_min), int(n_inner), fr,
                  int(forced_restart.numel()) // plan.B if forced_restart is not None else 0,
                  1 if bb else 0, float(bb_alpha_min))
    sp = None
    if stats is not None:
        cap = min(stats["rho"].numel(), stats["xi"].numel(), stats["restart"].numel()) // plan.B
        sp = ctypes.byref(Stats(_dev(stats["rho"], "stats.rho", dtype="float64"),
                                _dev(stats["xi"], "stats.xi", dtype="float64"),
                                _dev(stats["restart"], "stats.restart", dtype="uint8"), cap))
    status = _lib.lalm_iterate(plan.handle, ctypes.byref(prob), ctypes.byref(st), int(n_steps),
                               ctypes.byref(opt), sp, _stream(stream))
    state.step, state.l, state.rho, state.alpha = st.step, st.l, st.rho, st.alpha
    _check(status)
    return state


def lalm_cost_f64(plan, y, w, beta, delta, x, out, stream=None):
    """out (float64 GPU tensor, 3 elements per image) = (Psi, data term, R)."""
    prob = _problem(plan, y, w, None, beta, delta, True)
    _check(_lib.lalm_cost_f64(plan.handle, ctypes.byref(prob), _dev(x, "x", numel=plan.image_elems * plan.B),
                              _dev(out, "out", dtype="float64", numel=3 * plan.B), _stream(stream)))


def lalm_dot_f64(plan, a, b, out, stream=None):
    n = min(a.numel(), b.numel())
    _check(_lib.lalm_dot_f64(plan.handle, _dev(a, "a"), _dev(b, "b"), int(n),
                             _dev(out, "out", dtype="float64", numel=1), _stream(stream)))


def lalm_dot_f64_noalloc(a, b, out, stream=None):
    """lalm_dot_f64 without a plan and without allocation (the library's
    per-GPU static scratch; calls overlapping on one GPU race)."""
    n = min(a.numel(), b.numel())
    _check(_lib.lalm_dot_f64_noalloc(_dev(a, "a"), _dev(b, "b"), int(n),
                                     _dev(out, "out", dtype="float64", numel=1), _stream(stream)))


def lalm_roi_rmsd_f64(plan, a, b, radius_mm, out, stream=None):
    """out (float64 GPU tensor, one element per image of the batch)."""
    n = plan.image_elems * plan.B
    _check(_lib.lalm_roi_rmsd_f64(plan.handle, _dev(a, "a", numel=n), _dev(b, "b", numel=n), float(radius_mm),
                                  _dev(out, "out", dtype="float64", numel=plan.B), _stream(stream)))


def lalm_profile_begin(plan):
    _check(_lib.lalm_profile_begin(plan.handle))


def lalm_profile_read(plan):
    """Per kernel class (update, project, backproject): total ms and counts."""
    ms = np.zeros(3, dtype=np.float64)
    n = np.zeros(3, dtype=np.int64)
    _check(_lib.lalm_profile_read(plan.handle, ms.ctypes.data_as(ctypes.c_void_p),
                                  n.ctypes.data_as(ctypes.c_void_p)))
    return ms, n


def lalm_profile_end(plan):
    _check(_lib.lalm_profile_end(plan.handle))


# ---------------------------------------------------------------- warm start

def lalm_unet_param_count():
    return int(_lib.lalm_unet_param_count())


class UNet:
    """Owner of a ``lalm_unet`` workspace."""

    def __init__(self, handle, batch_max, height, width):
        self.handle, self.batch_max, self.height, self.width = handle, batch_max, height, width

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                _lib.lalm_unet_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def lalm_unet_create(batch_max, height, width):
    h = ctypes.c_void_p()
    _check(_lib.lalm_unet_create(int(batch_max), int(height), int(width), ctypes.byref(h)))
    return UNet(h, int(batch_max), int(height), int(width))


def lalm_unet_destroy(net):
    if net.handle:
        _check(_lib.lalm_unet_destroy(net.handle))
        net.handle = None


def lalm_unet_forward(net, params, x, out, batch, in_scale=1.0, nonneg=False, stream=None):
    n = int(batch) * net.height * net.width
    _check(_lib.lalm_unet_forward(net.handle, _dev(params, "params", numel=lalm_unet_param_count()),
                                  _dev(x, "x", numel=n), _dev(out, "out", numel=n), int(batch),
                                  float(in_scale), 1 if nonneg else 0, _stream(stream)))


def lalm_unet_loss_grad(net, params, x, target, mask, hu_scale, batch, grad, loss, in_scale=1.0,
                        stream=None):
    n = int(batch) * net.height * net.width
    P = lalm_unet_param_count()
    _check(_lib.lalm_unet_loss_grad(net.handle, _dev(params, "params", numel=P), _dev(x, "x", numel=n),
                                    _dev(target, "target", numel=n),
                                    _dev(mask, "mask", dtype="uint8", numel=net.height * net.width),
                                    float(in_scale), float(hu_scale), int(batch), _dev(grad, "grad", numel=P),
                                    _dev(loss, "loss", dtype="float64", numel=1), _stream(stream)))


def lalm_unet_adam(net, params, grad, m, v, t, lr, stream=None):
    P = lalm_unet_param_count()
    _check(_lib.lalm_unet_adam(net.handle, _dev(params, "params", numel=P), _dev(grad, "grad", numel=P),
                               _dev(m, "m", numel=P), _dev(v, "v", numel=P), int(t), float(lr),
                               _stream(stream)))


# tensors of lalm_unet_capture, in order: (name, level, channels)
UNET_CAPTURE = (("e1a", 1, 32), ("e1b", 1, 32), ("p1", 2, 32), ("e2a", 2, 64), ("e2b", 2, 64), ("p2", 3, 64),
                ("e3a", 3, 128), ("e3b", 3, 128), ("up2", 2, 64), ("d2a", 2, 64), ("d2b", 2, 64),
                ("up1", 1, 32), ("d1a", 1, 32), ("d1b", 1, 32),
                ("dz_d1b", 1, 32), ("dz_d1a", 1, 32), ("dz_up1", 1, 32), ("dz_d2b", 2, 64),
                ("dz_d2a", 2, 64), ("dz_up2", 2, 64), ("dz_e3b", 3, 128), ("dz_e3a", 3, 128),
                ("dz_e2b", 2, 64), ("dz_e2a", 2, 64), ("dz_e1b", 1, 32), ("dz_e1a", 1, 32))


def lalm_unet_capture_elems(batch, height, width):
    return int(_lib.lalm_unet_capture_elems(int(batch), int(height), int(width)))


def lalm_unet_capture(net, params, x, target, mask, hu_scale, batch, grad, loss, capture, in_scale=1.0,
                      stream=None):
    """lalm_unet_loss_grad plus a copy of every stored tensor into ``capture``
    (float32 GPU tensor); returns a dict name -> view [batch, h, w, C]."""
    n = int(batch) * net.height * net.width
    P = lalm_unet_param_count()
    need = lalm_unet_capture_elems(batch, net.height, net.width)
    _check(_lib.lalm_unet_capture(net.handle, _dev(params, "params", numel=P), _dev(x, "x", numel=n),
                                  _dev(target, "target", numel=n),
                                  _dev(mask, "mask", dtype="uint8", numel=net.height * net.width),
                                  float(in_scale), float(hu_scale), int(batch), _dev(grad, "grad", numel=P),
                                  _dev(loss, "loss", dtype="float64", numel=1),
                                  _dev(capture, "capture", numel=need), int(capture.numel()), _stream(stream)))
    out, o = {}, 0
    for name, lv, ch in UNET_CAPTURE:
        h, w = net.height >> (lv - 1), net.width >> (lv - 1)
        cnt = int(batch) * h * w * ch
        out[name] = capture[o:o + cnt].view(int(batch), h, w, ch)
        o += cnt
    return out
