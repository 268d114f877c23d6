"""FP64 reference of the fitting loop's optimiser and densification (test
infrastructure, like the rest of oracle/; only tests import it).

Training (Sec. 4.1, implementation paragraph): Adam on every parameter group,
1.25e-4 for the two bases, 2.5e-3 for the features, and the 3D Gaussian
splatting defaults for the rest (Kerbl et al. 2023, which the paper cites for
them): position 1.6e-4 -> 1.6e-6 times the scene extent with log-linear decay
over 30000 steps, log-scales 5e-3, rotations 1e-3, opacity logits 5e-2,
beta = (0.9, 0.999), eps = 1e-15.  Points move, split and drop during training
(App., "move/split/drop"); the densification follows the same defaults:

* statistics per Gaussian over the views where it is visible (non-empty
  projected box): the sum of the norms of the 2D-mean gradient in normalised
  device units (pixel gradient times W/2 and H/2), the number of such views,
  and the largest projected radius kappa sqrt(lambda_max) in pixels;
* a Gaussian whose mean gradient norm reaches the threshold is cloned (an
  exact copy appended) when its largest scale is at most the dense scale, and
  split otherwise: the parent is replaced by two children at mu + R diag(s) eps
  (eps ~ N(0, I), passed in) with log-scales lowered by log(1.6);
* every resulting Gaussian is dropped when its opacity is below the minimum,
  and, when enabled, when its largest scale exceeds a world bound or (for
  Gaussians that existed before this step) its tracked radius exceeds a
  screen bound;
* each set keeps its own Gaussians: output order is, per set (isotropic then
  directional), kept originals, then clones, then children, each in parent
  order;
* new Gaussians start with zero optimiser moments.

Decisions are taken in float32 on float32 inputs against float32 thresholds
derived once in double, as the kernels take them, so both sides decide alike.
"""
import numpy as np

from . import ref

GROUPS = ("mean", "quat", "log_scale", "opacity_logit", "feat", "b_iso", "B_dir")
PER_GAUSSIAN = ("mean", "quat", "log_scale", "opacity_logit", "feat")


def expon_lr(t, lr0, lr1, steps):
    """Log-linear interpolation from lr0 at t = 0 to lr1 at t = steps, held after."""
    a = min(max(t / float(steps), 0.0), 1.0) if steps > 0 else 1.0
    return float(np.exp((1.0 - a) * np.log(lr0) + a * np.log(lr1)))


def adam(params, grads, m, v, t, lrs, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (bias-corrected, step t = 1, 2, ...) on every group.
    params, grads, m, v: dicts of arrays; lrs: dict of learning rates.
    Returns new (params, m, v) dicts."""
    out_p, out_m, out_v = {}, {}, {}
    for name in GROUPS:
        g = np.asarray(grads[name], np.float64)
        mm = beta1 * np.asarray(m[name], np.float64) + (1.0 - beta1) * g
        vv = beta2 * np.asarray(v[name], np.float64) + (1.0 - beta2) * g * g
        mhat = mm / (1.0 - beta1 ** t)
        vhat = vv / (1.0 - beta2 ** t)
        out_p[name] = np.asarray(params[name], np.float64) - lrs[name] * mhat / (np.sqrt(vhat) + eps)
        out_m[name], out_v[name] = mm, vv
    return out_p, out_m, out_v


def visible_boxes(scene, view, kappa=3.0, opts=None, band=0.05):
    """Visibility of every Gaussian in a view: projected (not culled) and its
    kappa box [mu -+ kappa sqrt(S_aa)] overlaps a pixel centre of the image.
    Returns (visible bool [n], stable bool [n]: the decision is the same when
    the box centre and half-widths move by -+(band + 1e-3 half-width) pixels,
    for tests that skip cases within rounding of the decision, radius
    kappa sqrt(lambda_max) in pixels)."""
    P = ref.project(scene, view, opts=opts)
    f = {name: P[:, i] for i, name in enumerate(ref.PROJ_FIELDS)}
    ok = f["valid"] > 0
    rx = kappa * np.sqrt(np.maximum(f["S00"], 0.0))
    ry = kappa * np.sqrt(np.maximum(f["S11"], 0.0))

    def decide(mx, my, hx, hy):
        # pixel centres u + 0.5 inside [mx - hx, mx + hx], clipped to the image
        u0 = np.maximum(np.ceil(mx - hx - 0.5), 0)
        u1 = np.minimum(np.floor(mx + hx - 0.5), view.W - 1)
        v0 = np.maximum(np.ceil(my - hy - 0.5), 0)
        v1 = np.minimum(np.floor(my + hy - 0.5), view.H - 1)
        return ok & (u0 <= u1) & (v0 <= v1)

    vis = decide(f["mx"], f["my"], rx, ry)
    stable = np.ones_like(vis)
    dx, dy = band + 1e-3 * rx, band + 1e-3 * ry
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sw in (-1, 1):
                stable &= decide(f["mx"] + sx * dx, f["my"] + sy * dy, rx + sw * dx, ry + sw * dy) == vis
    mid = 0.5 * (f["S00"] + f["S11"])
    lam = mid + np.sqrt(np.maximum(mid * mid - (f["S00"] * f["S11"] - f["S01"] ** 2), 0.0))
    radius = kappa * np.sqrt(np.maximum(lam, 0.0))
    return vis, stable | ~ok, np.where(ok, radius, 0.0)


def densify_stats(scene, views, g2d, opts=None):
    """Statistics accumulated over one backward of ``views`` from the oracle's
    per-view image-plane gradients g2d [V][n][7] (d mu^x, d mu^y first).
    Returns (grad_accum, denom, max_radius, stable) with stable as in
    visible_boxes, over all views."""
    n = scene.n
    acc, den, rad = np.zeros(n), np.zeros(n), np.zeros(n)
    stable = np.ones(n, bool)
    for vi, v in enumerate(views):
        vis, st, r = visible_boxes(scene, v, opts=opts)
        gx = g2d[vi, :, 0] * (0.5 * v.W)
        gy = g2d[vi, :, 1] * (0.5 * v.H)
        acc += np.where(vis, np.sqrt(gx * gx + gy * gy), 0.0)
        den += vis
        rad = np.maximum(rad, np.where(vis, r, 0.0))
        stable &= st
    return acc, den, rad, stable


def thresholds(grad_threshold, dense_scale, min_opacity, max_world_scale, max_screen_radius, split_factor=1.6):
    """float32 thresholds of the decisions, derived once in double."""
    f32 = np.float32
    return dict(grad=f32(grad_threshold), log_dense=f32(np.log(dense_scale)),
                logit_min_op=f32(np.log(min_opacity) - np.log1p(-min_opacity)),
                log_world=f32(np.log(max_world_scale)) if max_world_scale > 0 else None,
                screen=f32(max_screen_radius) if max_screen_radius > 0 else None,
                log_split=f32(np.log(split_factor)))


def densify(params, n_iso, grad_accum, denom, max_radius, noise, th):
    """One densification of float32 parameters (dict of (rows, n) / (n,)
    arrays) with float32 statistics and noise [n][2][3].  Returns
    (new params dict (float64 children means, float32 copies elsewhere),
    new n_iso, source index per output Gaussian, kind per output Gaussian
    (0 kept, 1 clone, 2 first child, 3 second child))."""
    f32 = np.float32
    n = params["mean"].shape[1]
    acc = np.asarray(grad_accum, f32)
    den = np.asarray(denom, f32)
    avg = np.where(den > 0, acc / np.where(den > 0, den, f32(1)), f32(0)).astype(f32)
    ls = np.asarray(params["log_scale"], f32)
    lmax = ls.max(axis=0)
    big_grad = avg >= th["grad"]
    clone = big_grad & (lmax <= th["log_dense"])
    split = big_grad & (lmax > th["log_dense"])
    op = np.asarray(params["opacity_logit"], f32)
    low_op = op < th["logit_min_op"]

    def too_big(lm):
        return (lm > th["log_world"]) if th["log_world"] is not None else np.zeros(lm.shape, bool)

    screen = (np.asarray(max_radius, f32) > th["screen"]) if th["screen"] is not None else np.zeros(n, bool)
    keep = ~split & ~(low_op | too_big(lmax) | screen)
    keep_clone = clone & ~(low_op | too_big(lmax))
    child_lmax = (lmax - th["log_split"]).astype(f32)
    keep_child = split & ~(low_op | too_big(child_lmax))

    R = [ref.quat_to_rot(params["quat"][:, i]) if keep_child[i] else None for i in range(n)]
    src, kind = [], []
    for lo, hi in ((0, n_iso), (n_iso, n)):
        idx = np.arange(lo, hi)
        src += [(i, 0) for i in idx[keep[lo:hi]]]
        src += [(i, 1) for i in idx[keep_clone[lo:hi]]]
        for i in idx[keep_child[lo:hi]]:
            src += [(i, 2), (i, 3)]
    n_iso_new = int(keep[:n_iso].sum() + keep_clone[:n_iso].sum() + 2 * keep_child[:n_iso].sum())
    out = {}
    for name in PER_GAUSSIAN:
        a = np.asarray(params[name], np.float64)
        a2 = a.reshape(-1, n)
        out[name] = np.stack([a2[:, i] for i, _ in src], axis=1) if src else np.zeros((a2.shape[0], 0))
    for j, (i, kd) in enumerate(src):
        if kd >= 2:
            s = np.exp(ls[:, i].astype(np.float64))
            out["mean"][:, j] = np.asarray(params["mean"][:, i], np.float64) + R[i] @ (s * noise[i, kd - 2])
            out["log_scale"][:, j] = (ls[:, i] - th["log_split"]).astype(f32)
    out["opacity_logit"] = out["opacity_logit"].reshape(-1)
    for name in ("b_iso", "B_dir"):
        out[name] = np.asarray(params[name], np.float64)
    return out, n_iso_new, np.array([i for i, _ in src], np.int64), np.array([kd for _, kd in src], np.int64)
