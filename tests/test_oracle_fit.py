"""Pins of the fitting loop's FP64 reference (oracle/fit_ref.py): the learning
rate schedule, Adam, the visibility / radius statistics and densification,
each against closed forms or hand-built cases whose outcome is known.  CPU
only."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import fit_ref, ref
from paper_2406_02518_amd import synth


def test_learning_rate_schedule():
    assert fit_ref.expon_lr(0, 1e-2, 1e-4, 100) == pytest.approx(1e-2, rel=1e-12)
    assert fit_ref.expon_lr(100, 1e-2, 1e-4, 100) == pytest.approx(1e-4, rel=1e-12)
    assert fit_ref.expon_lr(50, 1e-2, 1e-4, 100) == pytest.approx(1e-3, rel=1e-12)  # geometric midpoint
    assert fit_ref.expon_lr(500, 1e-2, 1e-4, 100) == pytest.approx(1e-4, rel=1e-12)  # held after the end


def test_adam_constant_gradient_moves_by_lr():
    rng = np.random.default_rng(1)
    shapes = dict(mean=(3, 5), quat=(4, 5), log_scale=(3, 5), opacity_logit=(5,), feat=(2, 5), b_iso=(2,),
                  B_dir=(3, 2))
    p = {k: rng.normal(size=s) for k, s in shapes.items()}
    g = {k: rng.normal(size=s) for k, s in shapes.items()}
    m = {k: np.zeros(s) for k, s in shapes.items()}
    v = {k: np.zeros(s) for k, s in shapes.items()}
    lrs = {k: 10.0 ** -(i + 1) for i, k in enumerate(shapes)}
    for t in range(1, 5):
        p2, m, v = fit_ref.adam(p, g, m, v, t, lrs)
        for k in shapes:
            np.testing.assert_allclose(p2[k] - p[k], -lrs[k] * np.sign(g[k]), rtol=1e-9)
        p = p2
    # a zero gradient leaves the parameter where it is
    z = {k: np.zeros(s) for k, s in shapes.items()}
    p3, _, _ = fit_ref.adam(p, z, z, z, 1, lrs)
    for k in shapes:
        np.testing.assert_array_equal(p3[k], p[k])


def test_radius_and_visibility_of_an_isotropic_gaussian():
    """A sphere of std sigma on the principal ray at depth z projects to
    Sigma^ = ((f sigma / z)^2 + 0.3) I (EWA plus the dilation), so its radius
    is 3 sqrt((f sigma / z)^2 + 0.3); moved far off the detector it is not
    visible."""
    sc = synth.random_scene(1, 2, k=4, L=1, iso_fraction=1.0, extent=1.0)
    sc.mean[:] = 0.0
    sc.mean[1, 1] = 500.0  # sideways, far outside the field of view
    sc.quat[:] = np.array([1.0, 0.0, 0.0, 0.0], np.float32)[:, None]
    sigma = np.float32(2.0)
    sc.log_scale[:] = np.log(sigma)
    v = synth.view(64, 64, 1.0, 1000.0, 600.0, 0.0)
    vis, stable, radius = fit_ref.visible_boxes(sc, v)
    f = 1000.0 / 1.0
    assert vis[0] and not vis[1] and stable.all()
    assert radius[0] == pytest.approx(3.0 * np.sqrt((f * float(sigma) / 600.0) ** 2 + 0.3), rel=1e-6)


def _params(n, rng):
    return dict(mean=rng.normal(size=(3, n)).astype(np.float32) * 10,
                quat=np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)),
                log_scale=np.full((3, n), np.log(0.5), np.float32),
                opacity_logit=np.zeros(n, np.float32),
                feat=rng.normal(size=(4, n)).astype(np.float32),
                b_iso=rng.normal(size=4).astype(np.float32),
                B_dir=rng.normal(size=(3, 4)).astype(np.float32))


def test_densify_hand_built_case():
    """Six Gaussians, three isotropic then three directional:
    g0 large gradient, small -> cloned;  g1 large gradient, large -> split;
    g2 small gradient -> kept;  g3 opacity below the minimum -> dropped;
    g4 large gradient, large, children beyond the world bound -> gone;
    g5 beyond the screen bound but large gradient and small -> the original
    is dropped, its clone (new, so not screen-tested) stays."""
    rng = np.random.default_rng(2)
    p = _params(6, rng)
    p["log_scale"][:, 1] = np.log([3.0, 1.0, 1.0])
    p["log_scale"][:, 4] = np.log([40.0, 1.0, 1.0])
    p["opacity_logit"][3] = -8.0
    p["quat"][:, 1] = Rotation.from_euler("z", 90, degrees=True).as_quat()[[3, 0, 1, 2]]
    acc = np.array([5e-3, 5e-3, 1e-5, 0.0, 5e-3, 5e-3], np.float32)
    den = np.ones(6, np.float32)
    rad = np.array([1, 1, 1, 1, 1, 50], np.float32)
    noise = rng.normal(size=(6, 2, 3)).astype(np.float32)
    th = fit_ref.thresholds(2e-4, 2.0, 0.005, 20.0, 20.0)
    out, n_iso, src, kind = fit_ref.densify(p, 3, acc, den, rad, noise, th)
    assert n_iso == 5
    assert src.tolist() == [0, 2, 0, 1, 1, 5]
    assert kind.tolist() == [0, 0, 1, 2, 3, 1]
    # copies are exact
    for j, i in ((0, 0), (1, 2), (2, 0), (5, 5)):
        for name in fit_ref.PER_GAUSSIAN:
            np.testing.assert_array_equal(out[name].reshape(-1, 6)[:, j], p[name].reshape(-1, 6)[:, i])
    # children: rotated by 90 degrees about z, scales (3, 1, 1): offset (-s_y e_y, s_x e_x, s_z e_z)
    for j, c in ((3, 0), (4, 1)):
        e = noise[1, c].astype(np.float64)
        off = np.array([-1.0 * e[1], 3.0 * e[0], 1.0 * e[2]])
        np.testing.assert_allclose(out["mean"][:, j], p["mean"][:, 1] + off, rtol=0, atol=1e-5)
        np.testing.assert_allclose(out["log_scale"][:, j], p["log_scale"][:, 1] - np.float32(np.log(1.6)), atol=0)
    # no screen bound: g5 stays too
    th2 = fit_ref.thresholds(2e-4, 2.0, 0.005, 20.0, 0.0)
    _, n_iso2, src2, kind2 = fit_ref.densify(p, 3, acc, den, rad, noise, th2)
    assert n_iso2 == 5 and src2.tolist() == [0, 2, 0, 1, 1, 5, 5] and kind2.tolist() == [0, 0, 1, 2, 3, 0, 1]
    # a view count of zero gives a zero mean gradient
    _, _, src3, _ = fit_ref.densify(p, 3, acc, np.zeros(6, np.float32), rad, noise, th2)
    assert src3.tolist() == [0, 1, 2, 5]  # g3 low opacity, g4 beyond the world bound


def test_densify_children_are_samples_of_the_parent():
    """Children means over many parents: (child - mu) R^T / s is the noise."""
    rng = np.random.default_rng(3)
    n = 50
    p = _params(n, rng)
    p["log_scale"] = np.log(rng.uniform(2.5, 4.0, size=(3, n))).astype(np.float32)
    p["quat"] = synth.random_unit_quaternions(rng, n).astype(np.float32)
    noise = rng.normal(size=(n, 2, 3)).astype(np.float32)
    th = fit_ref.thresholds(2e-4, 2.0, 0.005, 0.0, 0.0)
    out, n_iso, src, kind = fit_ref.densify(p, 20, np.ones(n, np.float32), np.ones(n, np.float32),
                                            np.zeros(n, np.float32), noise, th)
    assert n_iso == 40 and out["mean"].shape[1] == 2 * n
    for j in range(2 * n):
        i, c = src[j], kind[j] - 2
        R = Rotation.from_quat(p["quat"][[1, 2, 3, 0], i].astype(np.float64)).as_matrix()
        e = R.T @ (out["mean"][:, j] - p["mean"][:, i]) / np.exp(p["log_scale"][:, i].astype(np.float64))
        np.testing.assert_allclose(e, noise[i, c], rtol=1e-5, atol=1e-5)


def test_densify_stats_from_the_oracle_gradient():
    """Statistics from the oracle's per-view 2D gradients: the mean-gradient
    norm of a Gaussian seen in one view is the pixel-gradient norm scaled by
    (W/2, H/2), summed over the views that see it."""
    sc = synth.random_scene(4, 30, k=4, L=1, extent=10.0)
    views = [synth.view(40, 36, 1.5, 1000.0, 600.0, a) for a in (0.0, 70.0)]
    P = sum(v.W * v.H for v in views)
    g = np.random.default_rng(4).normal(size=P)
    o = ref.backward(sc, views, ref.all_pixels(views), g, want_g2d=True)
    acc, den, rad, _ = fit_ref.densify_stats(sc, views, o["g2d"])
    exp_acc = np.zeros(sc.n)
    for vi, v in enumerate(views):
        vis = fit_ref.visible_boxes(sc, v)[0]
        exp_acc += vis * np.hypot(o["g2d"][vi, :, 0] * v.W / 2, o["g2d"][vi, :, 1] * v.H / 2)
    np.testing.assert_allclose(acc, exp_acc, rtol=1e-12)
    assert den.max() == 2 and acc.max() > 0 and rad.max() > 0


def _iso_scene(means, std_mm, alpha=0.5, c=0.7):
    """Isotropic Gaussians at world means (3, n) with std std_mm and one
    radiosity c (features encode logit(c) along b_iso)."""
    means = np.asarray(means, np.float64)
    n = means.shape[1]
    b = np.array([1.0, 0.5, -0.25, 0.125])
    f = np.log(c / (1.0 - c)) * b / (b @ b)
    return synth.Scene(mean=means, quat=np.tile([[1.0], [0.0], [0.0], [0.0]], (1, n)),
                       log_scale=np.full((3, n), np.log(std_mm)),
                       opacity_logit=np.full(n, np.log(alpha / (1.0 - alpha))), feat=np.tile(f[:, None], (1, n)),
                       b_iso=b, B_dir=np.zeros((3, 4)), n_iso=n, L=1)


def test_densify_statistic_against_finite_differences_of_the_mean():
    """Independent pin of the densification statistic.  One isotropic Gaussian
    on the principal ray (source-frame mean (0, 0, z)): shifting it by x along
    the source-frame x axis moves its projected mean by f x / z pixels, while
    the projected covariance s^2 J J^T + dI changes only at order x^2 (J J^T
    = (f/z)^2 (I + (x, y)(x, y)^T / z^2)), so a central difference of the
    loss under that shift gives dL/du exactly up to O(h^2); likewise for y.
    Normalised device units are u_ndc = (2 u + 1) / W - 1, so the statistic is
    the norm of (dL/du W/2, dL/dv H/2).  The upstream weights vanish near the
    cut-off, so no pixel changes its contributor set under the shifts."""
    W, H, pitch, sdd, sid, std = 48, 40, 0.8, 1000.0, 600.0, 2.0
    v = synth.view(W, H, pitch, sdd, sid, 0.0)
    f = np.float64(np.float32(sdd)) / np.float64(np.float32(pitch))
    sig2 = (std * f / sid) ** 2 + 0.3
    vv, uu = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    d2 = ((uu - W / 2) ** 2 + (vv - H / 2) ** 2) / sig2
    g = np.random.default_rng(17).normal(size=(H, W)) * (d2 < 8.0)
    R = np.asarray(v.pose, np.float64)[:, :3]

    def loss(shift):
        sc = _iso_scene(np.asarray(shift, np.float64)[:, None], std)
        return float((ref.render(sc, [v])[0] * g).sum())

    h = 1e-3
    du = (loss(h * R[0]) - loss(-h * R[0])) / (2 * h) * sid / f
    dv = (loss(h * R[1]) - loss(-h * R[1])) / (2 * h) * sid / f
    expected = np.hypot(du * W / 2, dv * H / 2)
    sc = _iso_scene(np.zeros((3, 1)), std)
    o = ref.backward(sc, [v], ref.all_pixels([v]), g.ravel(), want_g2d=True)
    acc, den, rad, stable = fit_ref.densify_stats(sc, [v], o["g2d"])
    assert den[0] == 1 and stable[0]
    assert expected > 1e-3
    np.testing.assert_allclose(acc[0], expected, rtol=1e-6)
    # the tracked radius: kappa sqrt(lambda_max), isotropic here
    np.testing.assert_allclose(rad[0], 3.0 * np.sqrt(sig2), rtol=1e-12)


def test_visibility_rule_at_the_image_edges():
    """visible_boxes against boxes placed in closed form.  An isotropic
    Gaussian at source-frame (x, 0, z) projects to u = f x / z + W/2 with
    variance s^2 (f/z)^2 (1 + x^2 / z^2) + 0.3 along u (the pinhole Jacobian
    at y = 0), and likewise along v at (0, y, z).  A Gaussian counts as
    visible when its kappa box reaches a pixel centre u' + 0.5, u' = 0..W-1,
    on both axes.  Boxes whose inner edge lies 0.02 px inside the outermost
    centre on each of the four sides are visible, 0.02 px outside invisible."""
    from scipy.optimize import brentq

    W, H, pitch, sdd, sid, std, kappa = 50, 36, 1.0, 1000.0, 600.0, 1.5, 3.0
    v = synth.view(W, H, pitch, sdd, sid, 0.0)
    f = np.float64(np.float32(sdd)) / np.float64(np.float32(pitch))
    P = np.asarray(v.pose, np.float64)
    Rm, t = P[:, :3], P[:, 3]

    def half(off):
        return kappa * np.sqrt(std ** 2 * (f / sid) ** 2 * (1.0 + (off / sid) ** 2) + 0.3)

    cams, want = [], []
    for axis, size in ((0, W), (1, H)):
        for side in (-1, 1):
            for inside in (True, False):
                e = -0.02 if inside else 0.02
                if side > 0:   # left end of the box past the last centre, size - 0.5
                    target = lambda off: f * off / sid + size / 2 - half(off) - (size - 0.5 + e)  # noqa: E731
                else:          # right end of the box before the first centre, 0.5
                    target = lambda off: f * off / sid + size / 2 + half(off) - (0.5 - e)  # noqa: E731
                off = brentq(target, -sid, sid, xtol=1e-12)
                cam = np.array([0.0, 0.0, sid])
                cam[axis] = off
                cams.append(cam)
                want.append(inside)
    means = np.stack([Rm.T @ (cm - t) for cm in cams], axis=1)
    sc = _iso_scene(means, std)
    vis, stable, _ = fit_ref.visible_boxes(sc, v, kappa=kappa)
    np.testing.assert_array_equal(vis, np.array(want))
    # the projected means confirm the placement (box edges 0.02 px from the centres)
    pr = ref.project(sc, v)
    assert np.all(pr[:, 0] > 0)
