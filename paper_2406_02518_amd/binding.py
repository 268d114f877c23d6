"""ctypes binding of libddgs.so (include/ddgs.h).

The ``ddgs_*`` functions below carry the C names and only marshal arguments:
every step of the render / backward / loss path runs in the HIP kernels of the
library.  ``Renderer`` is a small convenience layer that takes torch tensors
(device memory and streams come from torch) and keeps them alive while the
library borrows their pointers.  There is no CPU fallback: if the library has
not been built, ``lib()`` raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libddgs.so")

OK, ERR_INVALID_ARG, ERR_OOM, ERR_HIP, ERR_CAPACITY, ERR_NONFINITE, ERR_STATE, ERR_UNSUPPORTED = range(8)
LOSS_L1_DSSIM, LOSS_NCC, LOSS_LINEAR = 0, 1, 2
(DBG_RECORDS, DBG_DEPTH_KEYS, DBG_COUNTS, DBG_RECTS, DBG_TILE_KEYS_UNSORTED, DBG_TILE_VALS_UNSORTED,
 DBG_TILE_KEYS, DBG_TILE_VALS, DBG_RANGES, DBG_NLAST, DBG_TILE_BASE, DBG_FIT_MOMENTS, DBG_TILE_MASKS) = range(13)
T_PROJECT, T_SORT, T_RASTER_FWD, T_LOSS, T_RASTER_BWD, T_PROJECT_BWD, T_COUNT = range(7)
STAGES = ("project", "sort", "raster_fwd", "loss", "raster_bwd", "project_bwd")

EXPORTED = (
    "ddgs_create", "ddgs_destroy", "ddgs_set_stream", "ddgs_status_str", "ddgs_last_error",
    "ddgs_default_options", "ddgs_set_options", "ddgs_get_options", "ddgs_set_model", "ddgs_set_views",
    "ddgs_set_radiosity_override", "ddgs_set_workspace", "ddgs_workspace_size", "ddgs_set_pose_optimizer",
    "ddgs_get_views",
    "ddgs_image_size", "ddgs_render", "ddgs_backward", "ddgs_loss", "ddgs_step_capture", "ddgs_step_launch", "ddgs_step_set_target",
    "ddgs_check", "ddgs_autotune", "ddgs_param_count", "ddgs_num_rendered", "ddgs_debug_copy",
    "ddgs_debug_keep_unsorted", "ddgs_debug_sort_pairs", "ddgs_debug_exclusive_scan", "ddgs_debug_count_pairs",
    "ddgs_debug_pair_counts", "ddgs_enable_timing", "ddgs_stage_times", "ddgs_default_fit_options",
    "ddgs_set_fit_optimizer", "ddgs_set_densify_stats", "ddgs_densify_plan", "ddgs_densify_apply",
    "ddgs_fit_reset_opacity", "ddgs_rads_prepare", "ddgs_rads_sample", "ddgs_step_report", "ddgs_set_allocator",
    "ddgs_compose_pose", "ddgs_sort_pairs_noalloc")

# allocator callbacks of ddgs_set_allocator: alloc(user, bytes) -> device pointer, free(user, ptr)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class ddgs_model(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_iso", C.c_int64), ("k", C.c_int32), ("L", C.c_int32),
                ("mean", C.c_void_p), ("quat", C.c_void_p), ("log_scale", C.c_void_p),
                ("opacity_logit", C.c_void_p), ("feat", C.c_void_p), ("b_iso", C.c_void_p),
                ("B_dir", C.c_void_p), ("radiosity", C.c_int32), ("reserved", C.c_int32)]


RADIOSITY_DISENTANGLED, RADIOSITY_ENTANGLED = 0, 1


class ddgs_view(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("pitch_mm", C.c_float), ("sdd_mm", C.c_float),
                ("pose", C.c_float * 12)]


class ddgs_adam(C.Structure):
    _fields_ = [("lr_trans", C.c_float), ("lr_rot", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("pivot_mode", C.c_int32), ("pivot", C.c_float * 3)]


PIVOT_SOURCE, PIVOT_POINT = 0, 1


class ddgs_options(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("kappa", C.c_float), ("dilation", C.c_float),
                ("t_min", C.c_float), ("z_near", C.c_float), ("sigma_max", C.c_float),
                ("persistent", C.c_int32), ("split", C.c_int32), ("capacity", C.c_int64)]


class ddgs_grads(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("dmean", "dquat", "dlog_scale", "dopacity_logit", "dfeat", "db_iso",
                                          "dB_dir", "dpose")]


class ddgs_fit_opts(C.Structure):
    _fields_ = [("lr_mean_init", C.c_float), ("lr_mean_final", C.c_float), ("lr_mean_steps", C.c_int32),
                ("lr_quat", C.c_float), ("lr_log_scale", C.c_float), ("lr_opacity", C.c_float),
                ("lr_feat", C.c_float), ("lr_b_iso", C.c_float), ("lr_B_dir", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class ddgs_densify_opts(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("grad_threshold", "dense_scale", "min_opacity", "max_world_scale",
                                         "max_screen_radius", "split_factor")]


class ddgs_params(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("mean", "quat", "log_scale", "opacity_logit", "feat", "b_iso", "B_dir")]


class ddgs_volume(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("spacing", C.c_float * 3),
                ("origin", C.c_float * 3), ("hu", C.c_void_p)]


class DDGSError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


_LIB = None


def lib():
    """Loads libddgs.so; raises if it has not been built (no fallback)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2406_02518_amd/build.py "
                               "(the DRR renderer has no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, st = C.c_void_p, C.c_int32, C.c_int64, C.c_int
        sig = {
            "ddgs_create": ([C.POINTER(vp), C.c_int, vp], st),
            "ddgs_destroy": ([vp], None),
            "ddgs_set_stream": ([vp, vp], st),
            "ddgs_status_str": ([st], C.c_char_p),
            "ddgs_last_error": ([vp], C.c_char_p),
            "ddgs_default_options": ([C.POINTER(ddgs_options)], None),
            "ddgs_set_options": ([vp, C.POINTER(ddgs_options)], st),
            "ddgs_get_options": ([vp, C.POINTER(ddgs_options)], st),
            "ddgs_set_model": ([vp, C.POINTER(ddgs_model)], st),
            "ddgs_set_views": ([vp, C.POINTER(ddgs_view), C.c_int], st),
            "ddgs_set_radiosity_override": ([vp, vp], st),
            "ddgs_set_pose_optimizer": ([vp, C.POINTER(ddgs_adam)], st),
            "ddgs_get_views": ([vp, C.POINTER(ddgs_view), C.c_int], st),
            "ddgs_set_workspace": ([vp, vp, C.c_size_t], st),
            "ddgs_workspace_size": ([vp, i64, C.POINTER(C.c_size_t)], st),
            "ddgs_image_size": ([vp, C.POINTER(i64)], st),
            "ddgs_render": ([vp, vp], st),
            "ddgs_backward": ([vp, vp, C.POINTER(ddgs_grads)], st),
            "ddgs_loss": ([vp, C.c_int, vp, vp, C.c_float, vp, vp], st),
            "ddgs_step_capture": ([vp, C.c_int, vp, C.c_float, vp, vp, vp, C.POINTER(ddgs_grads)], st),
            "ddgs_step_launch": ([vp], st),
            "ddgs_step_set_target": ([vp, vp], st),
            "ddgs_check": ([vp, C.POINTER(C.c_uint32)], st),
            "ddgs_autotune": ([vp, C.c_char_p, C.c_int, C.POINTER(C.c_float)], st),
            "ddgs_param_count": ([C.c_int, C.c_int, i64, C.POINTER(i64), C.POINTER(i64)], st),
            "ddgs_num_rendered": ([vp, C.POINTER(i64)], st),
            "ddgs_debug_copy": ([vp, C.c_int, vp, C.c_size_t], st),
            "ddgs_debug_keep_unsorted": ([vp, C.c_int], st),
            "ddgs_debug_sort_pairs": ([vp, vp, vp, i64, C.c_int], st),
            "ddgs_debug_exclusive_scan": ([vp, vp, vp, i64, C.POINTER(C.c_uint64)], st),
            "ddgs_debug_count_pairs": ([vp, C.c_int], st),
            "ddgs_debug_pair_counts": ([vp, C.POINTER(i64), C.POINTER(i64)], st),
            "ddgs_enable_timing": ([vp, C.c_int], st),
            "ddgs_stage_times": ([vp, C.POINTER(C.c_float)], st),
            "ddgs_default_fit_options": ([C.POINTER(ddgs_fit_opts), C.c_float], None),
            "ddgs_set_fit_optimizer": ([vp, C.POINTER(ddgs_fit_opts)], st),
            "ddgs_set_densify_stats": ([vp, vp, vp, vp], st),
            "ddgs_densify_plan": ([vp, C.POINTER(ddgs_densify_opts), vp, C.POINTER(i64), C.POINTER(i64)], st),
            "ddgs_densify_apply": ([vp, C.POINTER(ddgs_params)], st),
            "ddgs_fit_reset_opacity": ([vp, C.c_float], st),
            "ddgs_rads_prepare": ([vp, C.POINTER(ddgs_volume), C.POINTER(C.c_float), C.POINTER(i64),
                                   C.POINTER(C.c_uint64)], st),
            "ddgs_rads_sample": ([vp, i64, vp, i64, vp, vp, vp, C.POINTER(i64)], st),
            "ddgs_step_report": ([vp, C.POINTER(i64), C.POINTER(i64)], st),
            "ddgs_set_allocator": ([vp, ALLOC_FN, FREE_FN, vp], st),
            "ddgs_compose_pose": ([C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_float)], st),
            "ddgs_sort_pairs_noalloc": ([vp, vp, vp, i64, C.c_int], st),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def status_name(s):
    try:
        return lib().ddgs_status_str(int(s)).decode()
    except Exception:  # noqa: BLE001 - message formatting must not fail
        return f"status {s}"


def _check(status, ctx=None):
    if status != OK:
        msg = lib().ddgs_last_error(ctx).decode() if ctx else ""
        raise DDGSError(status, msg)


# ------------------------------------------------------------ C-name wrappers

def ddgs_create(device=0, stream=0):
    h = C.c_void_p()
    _check(lib().ddgs_create(C.byref(h), int(device), C.c_void_p(stream or 0)))
    return h


def ddgs_destroy(ctx):
    lib().ddgs_destroy(ctx)


def ddgs_set_stream(ctx, stream):
    _check(lib().ddgs_set_stream(ctx, C.c_void_p(stream or 0)), ctx)


def ddgs_default_options():
    o = ddgs_options()
    lib().ddgs_default_options(C.byref(o))
    return o


def ddgs_set_options(ctx, opts):
    _check(lib().ddgs_set_options(ctx, C.byref(opts)), ctx)


def ddgs_get_options(ctx):
    o = ddgs_options()
    _check(lib().ddgs_get_options(ctx, C.byref(o)), ctx)
    return o


def ddgs_set_model(ctx, model):
    _check(lib().ddgs_set_model(ctx, C.byref(model)), ctx)


def ddgs_set_views(ctx, views_arr, n):
    _check(lib().ddgs_set_views(ctx, views_arr, int(n)), ctx)


def ddgs_set_radiosity_override(ctx, ptr):
    _check(lib().ddgs_set_radiosity_override(ctx, ptr), ctx)


def ddgs_set_pose_optimizer(ctx, adam):
    _check(lib().ddgs_set_pose_optimizer(ctx, None if adam is None else C.byref(adam)), ctx)


def ddgs_default_fit_options(extent):
    o = ddgs_fit_opts()
    lib().ddgs_default_fit_options(C.byref(o), float(extent))
    return o


def ddgs_set_fit_optimizer(ctx, opts):
    _check(lib().ddgs_set_fit_optimizer(ctx, None if opts is None else C.byref(opts)), ctx)


def ddgs_set_densify_stats(ctx, grad_ptr, cnt_ptr, rad_ptr):
    _check(lib().ddgs_set_densify_stats(ctx, grad_ptr, cnt_ptr, rad_ptr), ctx)


def ddgs_densify_plan(ctx, opts, noise_ptr):
    n_new, n_iso = C.c_int64(), C.c_int64()
    _check(lib().ddgs_densify_plan(ctx, C.byref(opts), noise_ptr, C.byref(n_new), C.byref(n_iso)), ctx)
    return n_new.value, n_iso.value


def ddgs_densify_apply(ctx, params):
    _check(lib().ddgs_densify_apply(ctx, C.byref(params)), ctx)


def ddgs_fit_reset_opacity(ctx, max_alpha):
    _check(lib().ddgs_fit_reset_opacity(ctx, float(max_alpha)), ctx)


def ddgs_rads_prepare(ctx, vol):
    level, m, w = C.c_float(), C.c_int64(), C.c_uint64()
    _check(lib().ddgs_rads_prepare(ctx, C.byref(vol), C.byref(level), C.byref(m), C.byref(w)), ctx)
    return level.value, m.value, w.value


def ddgs_rads_sample(ctx, n1, keys_ptr, n2, draws_ptr, points_ptr, log_scale_ptr):
    n_iso = C.c_int64()
    _check(lib().ddgs_rads_sample(ctx, int(n1), keys_ptr, int(n2), draws_ptr, points_ptr, log_scale_ptr,
                                  C.byref(n_iso)), ctx)
    return n_iso.value


def ddgs_get_views(ctx, n):
    arr = (ddgs_view * max(1, n))()
    _check(lib().ddgs_get_views(ctx, arr, int(n)), ctx)
    return arr


def ddgs_set_workspace(ctx, ptr, nbytes):
    _check(lib().ddgs_set_workspace(ctx, ptr, int(nbytes)), ctx)


def ddgs_workspace_size(ctx, capacity=0):
    n = C.c_size_t()
    _check(lib().ddgs_workspace_size(ctx, int(capacity), C.byref(n)), ctx)
    return n.value


def ddgs_image_size(ctx):
    n = C.c_int64()
    _check(lib().ddgs_image_size(ctx, C.byref(n)), ctx)
    return n.value


def ddgs_render(ctx, images_ptr):
    _check(lib().ddgs_render(ctx, C.c_void_p(images_ptr)), ctx)


def ddgs_backward(ctx, dl_ptr, grads):
    _check(lib().ddgs_backward(ctx, C.c_void_p(dl_ptr), C.byref(grads)), ctx)


def ddgs_loss(ctx, kind, images_ptr, target_ptr, lam, loss_ptr, dl_ptr):
    _check(lib().ddgs_loss(ctx, int(kind), C.c_void_p(images_ptr), C.c_void_p(target_ptr), float(lam),
                           C.c_void_p(loss_ptr or 0), C.c_void_p(dl_ptr or 0)), ctx)


def ddgs_step_capture(ctx, kind, target_ptr, lam, images_ptr, dl_ptr, loss_ptr, grads):
    _check(lib().ddgs_step_capture(ctx, int(kind), C.c_void_p(target_ptr), float(lam), C.c_void_p(images_ptr),
                                   C.c_void_p(dl_ptr), C.c_void_p(loss_ptr or 0), C.byref(grads)), ctx)


def ddgs_step_launch(ctx):
    _check(lib().ddgs_step_launch(ctx), ctx)


def ddgs_step_set_target(ctx, target_ptr):
    _check(lib().ddgs_step_set_target(ctx, C.c_void_p(int(target_ptr))), ctx)


def ddgs_check(ctx, raise_on_error=True):
    fl = C.c_uint32()
    st = lib().ddgs_check(ctx, C.byref(fl))
    if raise_on_error:
        _check(st, ctx)
    return st, fl.value


def ddgs_step_report(ctx):
    """(skipped replays, largest entry need) found by the last ddgs_check."""
    sk, need = C.c_int64(), C.c_int64()
    _check(lib().ddgs_step_report(ctx, C.byref(sk), C.byref(need)), ctx)
    return sk.value, need.value


def ddgs_set_allocator(ctx, alloc_fn, free_fn):
    """alloc_fn / free_fn: ALLOC_FN / FREE_FN objects (kept alive by the
    caller), or None for hipMalloc."""
    _check(lib().ddgs_set_allocator(ctx, alloc_fn or ALLOC_FN(), free_fn or FREE_FN(), None), ctx)


def ddgs_compose_pose(pose, delta):
    """Exp(delta) pose for a (3, 4) float32 pose and a 6-vector (rho, omega)
    tangent: the library composes in float64 and rounds once."""
    p = np.ascontiguousarray(np.asarray(pose, dtype=np.float32).reshape(12))
    d = np.ascontiguousarray(np.asarray(delta, dtype=np.float64).reshape(6))
    out = np.zeros(12, dtype=np.float32)
    _check(lib().ddgs_compose_pose(p.ctypes.data_as(C.POINTER(C.c_float)), d.ctypes.data_as(C.POINTER(C.c_double)),
                                   out.ctypes.data_as(C.POINTER(C.c_float))))
    return out.reshape(3, 4)


def ddgs_autotune(ctx, cache_path=None, repeats=5):
    ms = C.c_float()
    p = cache_path.encode() if cache_path else None
    _check(lib().ddgs_autotune(ctx, p, int(repeats), C.byref(ms)), ctx)
    return ms.value


def ddgs_param_count(k, L, n):
    per, sh = C.c_int64(), C.c_int64()
    _check(lib().ddgs_param_count(int(k), int(L), int(n), C.byref(per), C.byref(sh)))
    return per.value, sh.value


def ddgs_num_rendered(ctx):
    n = C.c_int64()
    _check(lib().ddgs_num_rendered(ctx, C.byref(n)), ctx)
    return n.value


def ddgs_debug_keep_unsorted(ctx, keep):
    _check(lib().ddgs_debug_keep_unsorted(ctx, int(bool(keep))), ctx)


def ddgs_debug_copy(ctx, what, dtype, count):
    out = np.zeros(int(count), dtype=dtype)
    _check(lib().ddgs_debug_copy(ctx, int(what), out.ctypes.data_as(C.c_void_p), out.nbytes), ctx)
    return out


def ddgs_debug_sort_pairs(ctx, keys_ptr, vals_ptr, n, bits):
    _check(lib().ddgs_debug_sort_pairs(ctx, C.c_void_p(keys_ptr), C.c_void_p(vals_ptr), int(n), int(bits)), ctx)


def ddgs_sort_pairs_noalloc(ctx, keys_ptr, vals_ptr, n, bits):
    _check(lib().ddgs_sort_pairs_noalloc(ctx, C.c_void_p(keys_ptr), C.c_void_p(vals_ptr), int(n), int(bits)), ctx)


def ddgs_debug_exclusive_scan(ctx, in_ptr, out_ptr, n):
    t = C.c_uint64()
    _check(lib().ddgs_debug_exclusive_scan(ctx, C.c_void_p(in_ptr), C.c_void_p(out_ptr), int(n), C.byref(t)), ctx)
    return t.value


def ddgs_debug_count_pairs(ctx, enable):
    _check(lib().ddgs_debug_count_pairs(ctx, int(bool(enable))), ctx)


def ddgs_debug_pair_counts(ctx):
    e, c = C.c_int64(), C.c_int64()
    _check(lib().ddgs_debug_pair_counts(ctx, C.byref(e), C.byref(c)), ctx)
    return e.value, c.value


def ddgs_enable_timing(ctx, enable):
    _check(lib().ddgs_enable_timing(ctx, int(bool(enable))), ctx)


def ddgs_stage_times(ctx):
    ms = (C.c_float * T_COUNT)()
    _check(lib().ddgs_stage_times(ctx, ms), ctx)
    return dict(zip(STAGES, list(ms)))


# --------------------------------------------------------- torch-facing layer

def _views_struct(views):
    arr = (ddgs_view * max(1, len(views)))()
    for i, v in enumerate(views):
        arr[i].W, arr[i].H = int(v.W), int(v.H)
        arr[i].pitch_mm, arr[i].sdd_mm = float(v.pitch), float(v.sdd)
        pose = np.asarray(v.pose, dtype=np.float32).reshape(12)
        for j in range(12):
            arr[i].pose[j] = float(pose[j])
    return arr


PARAM_NAMES = ("mean", "quat", "log_scale", "opacity_logit", "feat", "b_iso", "B_dir")
GRAD_NAMES = ("dmean", "dquat", "dlog_scale", "dopacity_logit", "dfeat", "db_iso", "dB_dir", "dpose")


class TorchAllocator:
    """Workspace allocator of a context backed by torch's caching allocator:
    every buffer the library asks for is a uint8 tensor allocated on the
    context's stream and kept here until the library frees it."""

    def __init__(self, torch, device, stream):
        self.blocks = {}

        def alloc(_user, nbytes):
            try:
                with torch.cuda.stream(stream):
                    t = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
            except RuntimeError:  # out of memory: the library reports DDGS_ERR_OOM
                return None
            self.blocks[t.data_ptr()] = t
            return t.data_ptr()

        def free(_user, ptr):
            self.blocks.pop(ptr, None)

        self.alloc_fn = ALLOC_FN(alloc)
        self.free_fn = FREE_FN(free)

    def bytes_held(self):
        return sum(t.numel() for t in self.blocks.values())


class Renderer:
    """Owns a ddgs context bound to a torch CUDA(HIP) device and stream.  The
    library's workspace comes from torch's caching allocator (TorchAllocator),
    so torch owns every byte of device memory the renderer uses."""

    def __init__(self, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = ddgs_create(device, self.stream.cuda_stream)
        self._keep = {}
        self.views = []
        self.n = 0
        self.k = 0
        self.L = 1
        self.render_id = 0   # bumped by every render and state change (the autograd function checks it)
        self.allocator = TorchAllocator(torch, self.device, self.stream)
        ddgs_set_allocator(self.ctx, self.allocator.alloc_fn, self.allocator.free_fn)

    def close(self):
        if self.ctx is not None:
            ddgs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    # inputs
    def set_options(self, **kw):
        o = ddgs_get_options(self.ctx)
        for k, v in kw.items():
            setattr(o, k, v)
        ddgs_set_options(self.ctx, o)
        self.render_id += 1

    def options(self):
        o = ddgs_get_options(self.ctx)
        return {f: getattr(o, f) for f, _ in o._fields_}

    def set_model(self, params, n_iso, L, entangled=False):
        """params: dict of float32 contiguous device tensors named as PARAM_NAMES.
        ``entangled``: both radiosity terms on every Gaussian (needs n_iso = 0)."""
        t = {}
        for name in PARAM_NAMES:
            x = params[name]
            if x.dtype != self.torch.float32 or x.device != self.device:
                raise ValueError(f"{name} must be a float32 tensor on {self.device}")
            t[name] = x.contiguous()
        m = ddgs_model()
        m.n = int(t["mean"].shape[1])
        m.n_iso = int(n_iso)
        m.k = int(t["feat"].shape[0])
        m.L = int(L)
        m.radiosity = RADIOSITY_ENTANGLED if entangled else RADIOSITY_DISENTANGLED
        for name in PARAM_NAMES:
            setattr(m, name, t[name].data_ptr())
        ddgs_set_model(self.ctx, m)
        self.render_id += 1
        self._keep["model"] = t
        self.n, self.k, self.L = m.n, m.k, m.L

    def set_scene(self, scene):
        p = {name: self.torch.from_numpy(np.ascontiguousarray(getattr(scene, name))).to(self.device)
             for name in PARAM_NAMES}
        self.set_model(p, scene.n_iso, scene.L, getattr(scene, "entangled", False))
        return p

    def set_views(self, views):
        self.views = list(views)
        ddgs_set_views(self.ctx, _views_struct(self.views), len(self.views))
        self.render_id += 1

    def set_radiosity_override(self, c):
        """c: float32 device tensor [n_views][n] used as the radiosity instead of
        Eq. 3, or None to restore Eq. 3 (the tensor is kept alive here)."""
        if c is None:
            self._c_override = None
            ddgs_set_radiosity_override(self.ctx, None)
            return
        if c.dtype != self.torch.float32 or c.device != self.device:
            raise ValueError(f"override must be a float32 tensor on {self.device}")
        self._c_override = c.contiguous()
        ddgs_set_radiosity_override(self.ctx, self._c_override.data_ptr())

    def set_pose_optimizer(self, lr_trans=None, lr_rot=None, beta1=0.9, beta2=0.999, eps=1e-8, pivot=None):
        """Adam on every view's pose tangent inside captured steps (None: off).
        ``pivot``: world point (mm) the rotation turns about; None turns it
        about the source (the left tangent)."""
        if lr_trans is None and lr_rot is None:
            ddgs_set_pose_optimizer(self.ctx, None)
            return
        a = ddgs_adam()
        a.lr_trans, a.lr_rot = float(lr_trans or 0.0), float(lr_rot or 0.0)
        a.beta1, a.beta2, a.eps = float(beta1), float(beta2), float(eps)
        if pivot is None:
            a.pivot_mode = PIVOT_SOURCE
        else:
            a.pivot_mode = PIVOT_POINT
            a.pivot[:] = [float(x) for x in pivot]
        ddgs_set_pose_optimizer(self.ctx, a)

    # ------------------------------------------------------------ fitting
    def set_fit_optimizer(self, extent=None, **rates):
        """Adam on every parameter group inside captured steps, updating the
        model tensors in place; defaults from ddgs_default_fit_options(extent)
        with any field overridden by keyword.  extent None turns it off."""
        if extent is None:
            ddgs_set_fit_optimizer(self.ctx, None)
            return
        o = ddgs_default_fit_options(extent)
        for k, v in rates.items():
            setattr(o, k, v)
        ddgs_set_fit_optimizer(self.ctx, o)

    def set_densify_stats(self, stats):
        """stats: dict of float32 [n] device tensors grad, count, radius (None: off)."""
        if stats is None:
            ddgs_set_densify_stats(self.ctx, None, None, None)
            self._keep.pop("stats", None)
            return
        ddgs_set_densify_stats(self.ctx, stats["grad"].data_ptr(), stats["count"].data_ptr(),
                               stats["radius"].data_ptr())
        self._keep["stats"] = stats

    def new_densify_stats(self):
        z = self.torch.zeros(self.n, device=self.device, dtype=self.torch.float32)
        return {"grad": z, "count": z.clone(), "radius": z.clone()}

    def densify(self, noise, grad_threshold=2e-4, dense_scale=1.0, min_opacity=0.005, max_world_scale=0.0,
                max_screen_radius=0.0, split_factor=1.6):
        """Plans and applies one densification; returns (params dict of new
        tensors, n_iso).  The caller sets the new model (set_model)."""
        o = ddgs_densify_opts(float(grad_threshold), float(dense_scale), float(min_opacity), float(max_world_scale),
                              float(max_screen_radius), float(split_factor))
        noise = noise.contiguous()
        cur = self._begin()
        n_new, n_iso = ddgs_densify_plan(self.ctx, o, noise.data_ptr())
        m = self._keep["model"]
        t = self.torch
        out = {"mean": t.empty((3, n_new), device=self.device), "quat": t.empty((4, n_new), device=self.device),
               "log_scale": t.empty((3, n_new), device=self.device), "opacity_logit": t.empty(n_new, device=self.device),
               "feat": t.empty((self.k, n_new), device=self.device), "b_iso": t.empty_like(m["b_iso"]),
               "B_dir": t.empty_like(m["B_dir"])}
        p = ddgs_params(*[out[name].data_ptr() if out[name].numel() else None for name in PARAM_NAMES])
        ddgs_densify_apply(self.ctx, p)
        self._end(cur, noise, *out.values())
        return out, n_iso

    def reset_opacity(self, max_alpha=0.01):
        ddgs_fit_reset_opacity(self.ctx, max_alpha)

    def fit_moments(self):
        """Adam moments (m, v) as flat float32 host arrays."""
        P = self.n * (11 + self.k) + self.k + self.L * (self.L + 2) * self.k
        out = ddgs_debug_copy(self.ctx, DBG_FIT_MOMENTS, np.float32, 2 * P)
        return out[:P], out[P:]

    def get_poses(self):
        """Current (3, 4) float32 world -> source poses of the views."""
        arr = ddgs_get_views(self.ctx, len(self.views))
        return [np.array(arr[i].pose[:], dtype=np.float32).reshape(3, 4) for i in range(len(self.views))]

    def workspace_size(self, capacity=0):
        return ddgs_workspace_size(self.ctx, capacity)

    def set_workspace(self, ws):
        """ws: a uint8 device tensor the library carves its workspace from
        (kept alive here), or None to return to the torch allocator."""
        if ws is None:
            self._ws = None
            ddgs_set_workspace(self.ctx, None, 0)
            ddgs_set_allocator(self.ctx, self.allocator.alloc_fn, self.allocator.free_fn)
            return
        if ws.dtype != self.torch.uint8 or ws.device != self.device or not ws.is_contiguous():
            raise ValueError(f"workspace must be a contiguous uint8 tensor on {self.device}")
        self._ws = ws
        ddgs_set_workspace(self.ctx, ws.data_ptr(), ws.numel())

    def check_step(self):
        """ddgs_check for a captured step.  Returns 0 when every replay since
        the previous check fitted its tile-entry capacity.  After an overflow
        it raises options.capacity to twice the largest need and returns the
        number of replays whose updates were skipped (the last ones launched
        before this check): the caller captures the step again and replays
        those iterations, in order.  Other errors raise."""
        st, _ = ddgs_check(self.ctx, raise_on_error=False)
        if st == OK:
            return 0
        if st != ERR_CAPACITY:
            _check(st, self.ctx)
        skipped, need = ddgs_step_report(self.ctx)
        self.set_options(capacity=int(min(max(2 * need, 1024), 0xFFFFFFF0)))
        return skipped

    def image_size(self):
        return ddgs_image_size(self.ctx)

    def split(self, flat):
        out, base = [], 0
        for v in self.views:
            P = int(v.W) * int(v.H)
            out.append(flat[base:base + P].view(int(v.H), int(v.W)))
            base += P
        return out

    # compute
    # Work runs on self.stream.  It first waits for torch's current stream
    # (where the inputs were produced), and the current stream then waits for
    # it, so results are ordered for any later torch work.
    def _begin(self):
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
        return cur

    def _end(self, cur, *outs):
        if cur != self.stream:
            for t in outs:
                if t is not None:
                    t.record_stream(self.stream)
            cur.wait_stream(self.stream)

    def render(self, out=None):
        cur = self._begin()
        if out is None:
            out = self.torch.empty(self.image_size(), device=self.device, dtype=self.torch.float32)
        ddgs_render(self.ctx, out.data_ptr())
        self.render_id += 1
        self._end(cur, out)
        return out

    def alloc_grads(self, which=GRAD_NAMES):
        m = self._keep["model"]
        shapes = dict(dmean=m["mean"].shape, dquat=m["quat"].shape, dlog_scale=m["log_scale"].shape,
                      dopacity_logit=m["opacity_logit"].shape, dfeat=m["feat"].shape, db_iso=m["b_iso"].shape,
                      dB_dir=m["B_dir"].shape, dpose=(len(self.views), 6))
        return {k: self.torch.empty(shapes[k], device=self.device, dtype=self.torch.float32) for k in which}

    @staticmethod
    def grads_struct(grads):
        g = ddgs_grads()
        for name in GRAD_NAMES:
            x = grads.get(name)
            setattr(g, name, x.data_ptr() if x is not None else None)
        return g

    def backward(self, dl, grads=None, which=GRAD_NAMES):
        cur = self._begin()
        if grads is None:
            grads = self.alloc_grads(which)
        dl = dl.contiguous()
        ddgs_backward(self.ctx, dl.data_ptr(), self.grads_struct(grads))
        self._end(cur, dl, *grads.values())
        return grads

    def loss(self, kind, images, target, lam=0.2, want_grad=True):
        cur = self._begin()
        loss = self.torch.empty(len(self.views), device=self.device, dtype=self.torch.float32)
        dl = self.torch.empty_like(images) if want_grad else None
        ddgs_loss(self.ctx, kind, images.data_ptr(), target.data_ptr(), lam, loss.data_ptr(),
                  dl.data_ptr() if dl is not None else 0)
        self._end(cur, loss, dl, images, target)
        return loss, dl

    def num_rendered(self):
        return ddgs_num_rendered(self.ctx)

    def debug(self, what, dtype, count):
        return ddgs_debug_copy(self.ctx, what, dtype, count)
