"""ctypes wrapper of the C FP64 oracle (``ddgs_oracle.c``).

Test infrastructure only.  Inputs are float32 arrays (the values the GPU path
receives); they are widened to float64 exactly before the oracle sees them.
Scenes and views are plain objects with the attributes used below (see the
seeded input generators); nothing here computes any part of the method.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

PROJ_COLS = 13
PROJ_FIELDS = ("valid", "mx", "my", "A00", "A01", "A11", "alpha", "c", "zkey",
               "S00", "S01", "S11", "z")

DEFAULT_OPTS = dict(kappa=3.0, dilation=0.3, t_min=0.0, z_near=1.0, sigma_max=0.99)


class _Model(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_iso", C.c_int64), ("k", C.c_int32), ("L", C.c_int32),
                ("mean", C.c_void_p), ("quat", C.c_void_p), ("log_scale", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("feat", C.c_void_p), ("b_iso", C.c_void_p),
                ("B_dir", C.c_void_p), ("entangled", C.c_int32)]


class _View(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("pitch_mm", C.c_double),
                ("sdd_mm", C.c_double), ("pose", C.c_double * 12)]


class _Opts(C.Structure):
    _fields_ = [("kappa", C.c_double), ("dilation", C.c_double), ("t_min", C.c_double),
                ("z_near", C.c_double), ("sigma_max", C.c_double), ("c_override", C.c_void_p)]


class _Grads(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in
                ("dmean", "dquat", "dlog_scale", "dopacity_logit", "dfeat", "db_iso", "dB_dir",
                 "dpose", "dc", "g2d")]


def lib():
    global _LIB
    if _LIB is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.orc_kl.argtypes = [C.c_int]
        L.orc_kl.restype = C.c_int
        L.orc_param_count.argtypes = [C.c_int, C.c_int, i64, vp, vp, vp]
        L.orc_sh.argtypes = [C.c_int, vp, vp, vp]
        L.orc_sh.restype = C.c_int
        L.orc_quat_to_rot.argtypes = [vp, vp]
        L.orc_project.argtypes = [vp, vp, C.c_int, vp, vp]
        L.orc_project.restype = C.c_int
        L.orc_render.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, C.c_int]
        L.orc_render.restype = C.c_int
        L.orc_render_pixels.argtypes = [vp, vp, C.c_int, vp, i64, vp, vp, C.c_int]
        L.orc_render_pixels.restype = C.c_int
        L.orc_pixel_margins.argtypes = [vp, vp, C.c_int, vp, i64, vp, vp, C.c_int]
        L.orc_pixel_margins.restype = C.c_int
        L.orc_backward.argtypes = [vp, vp, C.c_int, vp, i64, vp, vp, vp, C.c_int]
        L.orc_backward.restype = C.c_int
        L.orc_loss_l1ssim.argtypes = [vp, vp, C.c_int, C.c_int, C.c_double, vp, vp, vp]
        L.orc_loss_l1ssim.restype = C.c_int
        L.orc_loss_ncc.argtypes = [vp, vp, i64, C.c_double, vp, vp]
        L.orc_loss_ncc.restype = C.c_int
        _LIB = L
    return _LIB


def default_threads():
    return max(1, min(64, len(os.sched_getaffinity(0))))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _Keep:
    """Holds the float64 copies alive while the C structs point at them."""

    def __init__(self):
        self.items = []

    def add(self, a):
        self.items.append(a)
        return a


def _model(scene, keep):
    m = _Model()
    m.n = int(scene.n)
    m.n_iso = int(scene.n_iso)
    m.k = int(scene.k)
    m.L = int(scene.L)
    for name in ("mean", "quat", "log_scale", "opacity_logit", "feat", "b_iso", "B_dir"):
        setattr(m, name, _ptr(keep.add(_f64(getattr(scene, name)))))
    m.entangled = 1 if getattr(scene, "entangled", False) else 0
    return m


def _views(views):
    arr = (_View * max(1, len(views)))()
    for i, v in enumerate(views):
        arr[i].W = int(v.W)
        arr[i].H = int(v.H)
        arr[i].pitch_mm = float(np.float32(v.pitch))
        arr[i].sdd_mm = float(np.float32(v.sdd))
        pose = np.asarray(v.pose, dtype=np.float64).reshape(12)
        for j in range(12):
            arr[i].pose[j] = pose[j]
    return arr


def _opts(opts, keep, c_override=None):
    d = dict(DEFAULT_OPTS)
    if opts:
        d.update(opts)
    o = _Opts()
    o.kappa, o.dilation, o.t_min = d["kappa"], d["dilation"], d["t_min"]
    o.z_near, o.sigma_max = d["z_near"], d["sigma_max"]
    o.c_override = None if c_override is None else _ptr(keep.add(_f64(c_override)))
    return o


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def kl(L):
    return lib().orc_kl(int(L))


def param_count(k, L, n):
    out = np.zeros(3, dtype=np.int64)
    lib().orc_param_count(int(k), int(L), int(n), _ptr(out[0:1]), _ptr(out[1:2]), _ptr(out[2:3]))
    return int(out[0]), int(out[1]), int(out[2])


def sh(L, d):
    """Basis values and gradients at unit directions d of shape (M, 3)."""
    d = np.atleast_2d(_f64(d))
    K = kl(L)
    Y = np.zeros((d.shape[0], K))
    dY = np.zeros((d.shape[0], K, 3))
    for i in range(d.shape[0]):
        row = np.ascontiguousarray(d[i])
        y = np.zeros(K)
        g = np.zeros(3 * K)
        _check(lib().orc_sh(int(L), _ptr(row), _ptr(y), _ptr(g)), "sh")
        Y[i] = y
        dY[i] = g.reshape(K, 3)
    return Y, dY


def quat_to_rot(q):
    q = _f64(q)
    R = np.zeros(9)
    lib().orc_quat_to_rot(_ptr(q), _ptr(R))
    return R.reshape(3, 3)


def project(scene, view, opts=None, view_index=0, c_override=None):
    """Per-Gaussian projection records, shape (n, 13); see PROJ_FIELDS."""
    keep = _Keep()
    m = _model(scene, keep)
    vs = _views([view])
    o = _opts(opts, keep, c_override)
    out = np.zeros((scene.n, PROJ_COLS))
    _check(lib().orc_project(C.byref(m), vs, int(view_index), C.byref(o), _ptr(out)), "project")
    return out


def render(scene, views, opts=None, threads=None, c_override=None, stats=False):
    """Full images: list of (H, W) float64 arrays, one per view."""
    keep = _Keep()
    m = _model(scene, keep)
    vs = _views(views)
    o = _opts(opts, keep, c_override)
    total = sum(int(v.W) * int(v.H) for v in views)
    img = np.zeros(total)
    hsh = np.zeros(max(1, len(views)), dtype=np.uint64)
    cnt = np.zeros(max(1, len(views)), dtype=np.int64)
    rc = lib().orc_render(C.byref(m), vs, len(views), C.byref(o), _ptr(img), _ptr(hsh), _ptr(cnt),
                          int(threads or default_threads()))
    _check(rc, "render")
    out, base = [], 0
    for v in views:
        P = int(v.W) * int(v.H)
        out.append(img[base:base + P].reshape(int(v.H), int(v.W)))
        base += P
    if stats:
        return out, hsh[:len(views)].copy(), cnt[:len(views)].copy()
    return out


def render_pixels(scene, views, pix, opts=None, threads=None, c_override=None):
    """Values at pix, an int array (M, 3) of (view, u, v)."""
    keep = _Keep()
    m = _model(scene, keep)
    vs = _views(views)
    o = _opts(opts, keep, c_override)
    pix = np.ascontiguousarray(np.asarray(pix, dtype=np.int32).reshape(-1, 3))
    out = np.zeros(pix.shape[0])
    rc = lib().orc_render_pixels(C.byref(m), vs, len(views), C.byref(o), pix.shape[0], _ptr(pix),
                                 _ptr(out), int(threads or default_threads()))
    _check(rc, "render_pixels")
    return out


def pixel_margins(scene, views, pix, opts=None, threads=None, c_override=None):
    """Smallest relative gap of each pixel in pix (M, 3) to the cutoff, clamp
    and early-stop decisions of Eq. 1 (orc_pixel_margins)."""
    keep = _Keep()
    m = _model(scene, keep)
    vs = _views(views)
    o = _opts(opts, keep, c_override)
    pix = np.ascontiguousarray(np.asarray(pix, dtype=np.int32).reshape(-1, 3))
    out = np.zeros(pix.shape[0])
    rc = lib().orc_pixel_margins(C.byref(m), vs, len(views), C.byref(o), pix.shape[0], _ptr(pix),
                                 _ptr(out), int(threads or default_threads()))
    _check(rc, "pixel_margins")
    return out


def all_pixels(views):
    """(view, u, v) of every pixel, view-major then row-major."""
    rows = []
    for vi, v in enumerate(views):
        vv, uu = np.meshgrid(np.arange(int(v.H)), np.arange(int(v.W)), indexing="ij")
        rows.append(np.stack([np.full(uu.size, vi), uu.ravel(), vv.ravel()], axis=1))
    return np.concatenate(rows).astype(np.int32)


def backward(scene, views, pix, g, opts=None, threads=None, c_override=None, want_g2d=False):
    """Analytic FP64 gradient of sum_p g_p I(p) over the pixels pix (M, 3)."""
    keep = _Keep()
    m = _model(scene, keep)
    vs = _views(views)
    o = _opts(opts, keep, c_override)
    pix = np.ascontiguousarray(np.asarray(pix, dtype=np.int32).reshape(-1, 3))
    g = _f64(g).reshape(-1)
    n, k, V = int(scene.n), int(scene.k), len(views)
    K = kl(scene.L)
    res = dict(dmean=np.zeros((3, n)), dquat=np.zeros((4, n)), dlog_scale=np.zeros((3, n)),
               dopacity_logit=np.zeros(n), dfeat=np.zeros((k, n)), db_iso=np.zeros(k),
               dB_dir=np.zeros((K, k)), dpose=np.zeros((V, 6)), dc=np.zeros((V, n)))
    if want_g2d:
        res["g2d"] = np.zeros((V, n, 7))
    gr = _Grads()
    for name, arr in res.items():
        setattr(gr, name, _ptr(arr))
    rc = lib().orc_backward(C.byref(m), vs, V, C.byref(o), pix.shape[0], _ptr(pix), _ptr(g),
                            C.byref(gr), int(threads or default_threads()))
    _check(rc, "backward")
    return res


def loss_l1ssim(x, y, lam=0.2, want_grad=True):
    x, y = _f64(x), _f64(y)
    H, W = x.shape
    loss = np.zeros(1)
    sm = np.zeros(1)
    grad = np.zeros_like(x) if want_grad else None
    _check(lib().orc_loss_l1ssim(_ptr(x), _ptr(y), W, H, float(lam), _ptr(loss), _ptr(sm),
                                 _ptr(grad)), "loss_l1ssim")
    return float(loss[0]), float(sm[0]), grad


def loss_ncc(x, y, eps=1e-12, want_grad=True):
    x, y = _f64(x), _f64(y)
    loss = np.zeros(1)
    grad = np.zeros_like(x) if want_grad else None
    _check(lib().orc_loss_ncc(_ptr(x), _ptr(y), x.size, float(eps), _ptr(loss), _ptr(grad)),
           "loss_ncc")
    return float(loss[0]), grad
