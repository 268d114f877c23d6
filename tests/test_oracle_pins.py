"""Pins of the FP64 oracle against facts fixed outside it: the paper's printed
numbers, closed forms, library routines (scipy), invariants and brute force.
CPU only."""
import json
import os

import numpy as np
import pytest
from scipy import special
from scipy.spatial.transform import Rotation

from oracle import ref
from paper_2406_02518_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def make_scene(means, stds, quats, alphas, feats=None, n_iso=None, k=4, L=1, b=None, B=None, seed=0):
    rng = np.random.default_rng(seed)
    n = len(means)
    kl = L * (L + 2)
    if feats is None:
        feats = rng.normal(0, 0.5, size=(k, n))
    if b is None:
        b = rng.normal(size=k)
    if B is None:
        B = rng.normal(size=(kl, k))
    a = np.asarray(alphas, dtype=np.float64)
    return synth.Scene(
        mean=np.ascontiguousarray(np.asarray(means, dtype=np.float32).T),
        quat=np.ascontiguousarray(np.asarray(quats, dtype=np.float32).T),
        log_scale=np.ascontiguousarray(np.log(np.asarray(stds, dtype=np.float64)).astype(np.float32).T),
        opacity_logit=(np.log(a) - np.log1p(-a)).astype(np.float32),
        feat=np.ascontiguousarray(np.asarray(feats, dtype=np.float32)),
        b_iso=np.asarray(b, dtype=np.float32), B_dir=np.asarray(B, dtype=np.float32),
        n_iso=n if n_iso is None else n_iso, L=L)


def f32(x):
    return np.float64(np.float32(x))


# --------------------------------------------------------------- printed values

def test_param_count_matches_paper():
    g = _load("param_count.json")
    per, shared, total = ref.param_count(g["k"], g["L"], g["n"])
    assert (per, shared, total) == (g["per_gaussian"], g["shared"], g["total"])


def test_basis_size_matches_eq3():
    g = _load("basis_size.json")
    for L, v in g["k_L"].items():
        assert ref.kl(int(L)) == v


def _two_step_scene(alpha, W=33):
    # two Gaussians at the isocentre project onto the centre of pixel (16, 16)
    return make_scene([[0, 0, 0], [0, 0, 0]], [[1, 1, 1]] * 2, [[1, 0, 0, 0]] * 2, [alpha, alpha])


def test_transmittance_worked_example():
    g = _load("transmittance_example.json")
    a1, a2 = g["step_attenuation"]
    assert a1 == a2 == 0.5
    sc = _two_step_scene(0.5)
    v = synth.view(33, 33, 0.5, 1000.0, 600.0, 0.0)
    c_one = np.ones((1, 2))
    val = ref.render_pixels(sc, [v], [[0, 16, 16]], c_override=c_one)[0]
    # with unit radiosity the pixel value is the total attenuation 1 - T
    assert val == pytest.approx(g["total_attenuation"], abs=1e-12)
    assert 1.0 - val == pytest.approx(g["transmittance"], abs=1e-12)


def test_early_termination_reading():
    # three co-located s = 0.5 steps; with t_min = 0.2 the third would push T
    # to 0.125 < 0.2, so compositing stops before it
    sc = make_scene([[0, 0, 0]] * 3, [[1, 1, 1]] * 3, [[1, 0, 0, 0]] * 3, [0.5] * 3)
    v = synth.view(33, 33, 0.5, 1000.0, 600.0, 0.0)
    c = np.ones((1, 3))
    full = ref.render_pixels(sc, [v], [[0, 16, 16]], c_override=c)[0]
    cut = ref.render_pixels(sc, [v], [[0, 16, 16]], c_override=c, opts=dict(t_min=0.2))[0]
    assert full == pytest.approx(0.875, abs=1e-12)
    assert cut == pytest.approx(0.75, abs=1e-12)


def test_sigma_clamp():
    sc = make_scene([[0, 0, 0]], [[1, 1, 1]], [[1, 0, 0, 0]], [0.999])
    v = synth.view(33, 33, 0.5, 1000.0, 600.0, 0.0)
    val = ref.render_pixels(sc, [v], [[0, 16, 16]], c_override=np.ones((1, 1)))[0]
    assert val == pytest.approx(0.99, abs=1e-12)


# ---------------------------------------------------------------- basis (Eq. 3)

def _real_sh_scipy(L, d):
    """Real orthonormal SH without Condon-Shortley phase from scipy's complex
    harmonics (which carry the phase)."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    cols = []
    for l in range(1, L + 1):
        for m in range(-l, l + 1):
            Yc = special.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                cols.append(np.sqrt(2) * (-1) ** m * Yc.real)
            elif m < 0:
                cols.append(np.sqrt(2) * (-1) ** m * Yc.imag)
            else:
                cols.append(Yc.real)
    return np.stack(cols, axis=1)


def _unit_dirs(n, seed=3):
    d = np.random.default_rng(seed).normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


@pytest.mark.parametrize("L", [1, 2, 3])
def test_sh_matches_scipy(L):
    d = _unit_dirs(64)
    Y, _ = ref.sh(L, d)
    np.testing.assert_allclose(Y, _real_sh_scipy(L, d), rtol=0, atol=1e-13)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for these degrees
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 24
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    w = (np.outer(wg, np.full(nphi, 2 * np.pi / nphi))).reshape(-1)
    Y, _ = ref.sh(3, d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(15), atol=1e-13)


def test_sh_gradient_by_central_differences():
    d = _unit_dirs(8) * 0.9
    _, dY = ref.sh(3, d)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        Yp, _ = ref.sh(3, d + e)
        Ym, _ = ref.sh(3, d - e)
        np.testing.assert_allclose((Yp - Ym) / (2 * h), dY[:, :, a], atol=1e-8)


def test_quaternion_rotation_matches_scipy():
    q = np.random.default_rng(5).normal(size=(10, 4)) * 3.0
    for qi in q:
        R = ref.quat_to_rot(qi)
        Rs = Rotation.from_quat([qi[1], qi[2], qi[3], qi[0]]).as_matrix()  # scalar-last
        np.testing.assert_allclose(R, Rs, atol=1e-14)


def test_isotropic_radiosity_reproduces_encoded_target():
    # the generator writes logit(c) along b; Eq. 3 must give back c
    sc = synth.random_scene(11, 300, k=16, L=3)
    rng = np.random.default_rng(np.random.SeedSequence(11).spawn(3)[1])
    c_target = np.clip(rng.uniform(0.0, 1.0, size=sc.n_iso), 1e-3, 1 - 1e-3)
    v = synth.view(64, 64, 1.0, 1000.0, 600.0, 0.0)
    proj = ref.project(sc, v)
    np.testing.assert_allclose(proj[:sc.n_iso, 7], c_target, rtol=2e-5, atol=0)


def test_directional_radiosity_closed_form():
    # directional blob at the isocentre: its ray direction is -src/|src|, so
    # c(theta) = sigmoid(Y(d(theta)) . B f) with Y from scipy
    rng = np.random.default_rng(2)
    k, L = 16, 3
    f = rng.normal(0, 0.5, size=(k, 1))
    B = rng.normal(size=(15, k))
    sc = make_scene([[0, 0, 0]], [[2, 2, 2]], [[1, 0, 0, 0]], [0.3], feats=f, n_iso=0, k=k, L=L, B=B)
    for th in (0.0, 33.0, 90.0, 211.0):
        v = synth.view(33, 33, 0.5, 1000.0, 600.0, th)
        R = v.pose[:, :3].astype(np.float64)
        t = v.pose[:, 3].astype(np.float64)
        so = -R.T @ t
        d = -so / np.linalg.norm(so)
        Y = _real_sh_scipy(L, d[None, :])[0]
        c = 1.0 / (1.0 + np.exp(-(Y @ (B.astype(np.float32).astype(np.float64) @
                                       f.astype(np.float32).astype(np.float64)[:, 0]))))
        val = ref.render_pixels(sc, [v], [[0, 16, 16]])[0]
        assert val == pytest.approx(c * 0.3, rel=1e-6)


# -------------------------------------------------------- projection closed form

def _pinhole(view, X):
    """pixel coordinates of a world point, written from the view geometry"""
    R = view.pose[:, :3].astype(np.float64)
    t = view.pose[:, 3].astype(np.float64)
    Xc = R @ X + t
    f = f32(view.sdd) / f32(view.pitch)
    return np.array([f * Xc[0] / Xc[2] + view.W / 2, f * Xc[1] / Xc[2] + view.H / 2])


def _expected_single(sc, view, kappa=3.0, dil=0.3):
    mu = sc.mean[:, 0].astype(np.float64)
    q = sc.quat[:, 0].astype(np.float64)
    s = np.exp(sc.log_scale[:, 0].astype(np.float64))
    Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    Sig = Rq @ np.diag(s ** 2) @ Rq.T
    # Jacobian of the pinhole map by central differences in world space
    h = 1e-4
    Jw = np.zeros((2, 3))
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        Jw[:, a] = (_pinhole(view, mu + e) - _pinhole(view, mu - e)) / (2 * h)
    S2 = Jw @ Sig @ Jw.T + dil * np.eye(2)
    A = np.linalg.inv(S2)
    m2 = _pinhole(view, mu)
    alpha = 1.0 / (1.0 + np.exp(-np.float64(sc.opacity_logit[0])))
    c = 1.0 / (1.0 + np.exp(-(sc.b_iso.astype(np.float64) @ sc.feat[:, 0].astype(np.float64))))
    vv, uu = np.meshgrid(np.arange(view.H) + 0.5, np.arange(view.W) + 0.5, indexing="ij")
    dx, dy = uu - m2[0], vv - m2[1]
    d2 = A[0, 0] * dx * dx + 2 * A[0, 1] * dx * dy + A[1, 1] * dy * dy
    val = c * np.minimum(0.99, alpha * np.exp(-0.5 * d2))
    val[d2 > kappa ** 2] = 0.0
    return val, m2, A, d2


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_single_gaussian_footprint_closed_form(seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-15, 15, size=3)
    std = rng.uniform(0.8, 4.0, size=3)
    q = rng.normal(size=4)
    sc = make_scene([mu], [std], [q], [0.4], seed=seed)
    v = synth.view(48, 40, 0.9, 1000.0, 600.0, float(rng.uniform(0, 360)))
    img = ref.render(sc, [v])[0]
    exp_img, m2, A, d2 = _expected_single(sc, v)
    # finite-difference Jacobian limits agreement to ~1e-9
    np.testing.assert_allclose(img, exp_img, atol=1e-8)
    assert (img > 0).sum() > 20
    proj = ref.project(sc, v)[0]
    np.testing.assert_allclose(proj[1:3], m2, atol=1e-9)
    np.testing.assert_allclose(proj[3:6], [A[0, 0], A[0, 1], A[1, 1]], rtol=1e-7)


@pytest.mark.parametrize("seed", [0, 1])
def test_pixel_margins_closed_form(seed):
    # one Gaussian: the margin is the relative gap of the closed-form d2 to
    # kappa^2, or of alpha exp(-d2/2) to sigma_max where it is considered
    rng = np.random.default_rng(seed)
    sc = make_scene([rng.uniform(-10, 10, size=3)], [rng.uniform(0.8, 4.0, size=3)], [rng.normal(size=4)],
                    [0.985], seed=seed)
    v = synth.view(40, 36, 0.9, 1000.0, 600.0, float(rng.uniform(0, 360)))
    _, _, _, d2 = _expected_single(sc, v)
    alpha = 1.0 / (1.0 + np.exp(-np.float64(sc.opacity_logit[0])))
    exp = np.abs(d2 - 9.0) / 9.0
    hit = d2 <= 9.0
    exp[hit] = np.minimum(exp[hit], np.abs(alpha * np.exp(-0.5 * d2[hit]) - 0.99) / 0.99)
    got = ref.pixel_margins(sc, [v], ref.all_pixels([v])).reshape(v.H, v.W)
    np.testing.assert_allclose(got, exp, atol=1e-7)
    assert got.min() < 1e-2


def test_pixel_margins_early_stop_steps():
    # three co-located s = 0.5 steps: T (1 - s) runs 0.5, 0.25, 0.125; with
    # t_min = 0.2 the closest is 0.25 (gap 0.25); without it, the clamp gap
    sc = make_scene([[0, 0, 0]] * 3, [[1, 1, 1]] * 3, [[1, 0, 0, 0]] * 3, [0.5] * 3)
    v = synth.view(33, 33, 0.5, 1000.0, 600.0, 0.0)
    got = ref.pixel_margins(sc, [v], [[0, 16, 16]], opts=dict(t_min=0.2))[0]
    assert got == pytest.approx(0.25, abs=1e-12)
    got = ref.pixel_margins(sc, [v], [[0, 16, 16]])[0]
    assert got == pytest.approx(0.49 / 0.99, abs=1e-12)


def test_parallel_beam_limit_equals_ray_maximum():
    """SID, SDD -> infinity at fixed ratio: the local-affine projection becomes
    exact and the footprint equals the maximum of the 3D Gaussian along each
    pixel ray (no dilation)."""
    rng = np.random.default_rng(7)
    mu = np.array([3.0, -2.0, 1.5])
    std = np.array([1.5, 0.7, 2.5])
    q = rng.normal(size=4)
    sc = make_scene([mu], [std], [q], [0.5], seed=1)
    sid, sdd, pitch = 1e7, 2e7, 0.25
    v = synth.view(40, 40, pitch, sdd, sid, 25.0)
    img = ref.render(sc, [v], opts=dict(dilation=0.0))[0]
    # ray geometry
    R = v.pose[:, :3].astype(np.float64)
    t = v.pose[:, 3].astype(np.float64)
    so = -R.T @ t
    mu32 = sc.mean[:, 0].astype(np.float64)
    qq = sc.quat[:, 0].astype(np.float64)
    s = np.exp(sc.log_scale[:, 0].astype(np.float64))
    Rq = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()
    Si = np.linalg.inv(Rq @ np.diag(s ** 2) @ Rq.T)
    alpha = 0.5
    c = 1.0 / (1.0 + np.exp(-(sc.b_iso.astype(np.float64) @ sc.feat[:, 0].astype(np.float64))))
    exp_img = np.zeros_like(img)
    for vv in range(v.H):
        for uu in range(v.W):
            pd = np.array([(uu + 0.5 - v.W / 2) * f32(pitch), (vv + 0.5 - v.H / 2) * f32(pitch), f32(sdd)])
            pw = R.T @ (pd - t)
            d = pw - so
            d /= np.linalg.norm(d)
            o = so + ((mu32 - so) @ d) * d          # ray point nearest to mu
            x = o - mu32
            m2 = x @ Si @ x - (d @ Si @ x) ** 2 / (d @ Si @ d)
            exp_img[vv, uu] = c * alpha * np.exp(-0.5 * m2) if m2 <= 9.0 else 0.0
    assert (exp_img > 0).sum() > 30
    np.testing.assert_allclose(img, exp_img, atol=2e-6)


def test_ray_quadrature_sanity_at_finite_distance():
    """Brute force: densely sampled maximum of the 3D Gaussians along each
    pixel ray, composited in depth order, matches the local-affine image to
    O(sigma / z) (a sanity bound, not parity)."""
    sc = make_scene([[0, 0, 0], [4, 3, -6]], [[2, 1, 1.5], [1.2, 1.2, 1.2]],
                    [[1, 0.2, 0.1, 0], [0.9, 0, 0.3, 0.1]], [0.3, 0.5], seed=4)
    v = synth.view(32, 32, 0.6, 1000.0, 600.0, 15.0)
    img = ref.render(sc, [v], opts=dict(dilation=0.0))[0]
    R = v.pose[:, :3].astype(np.float64)
    t = v.pose[:, 3].astype(np.float64)
    so = -R.T @ t
    proj = ref.project(sc, v, opts=dict(dilation=0.0))
    order = np.argsort(proj[:, 8], kind="stable")
    params = []
    for i in range(sc.n):
        qq = sc.quat[:, i].astype(np.float64)
        s = np.exp(sc.log_scale[:, i].astype(np.float64))
        Rq = Rotation.from_quat([qq[1], qq[2], qq[3], qq[0]]).as_matrix()
        params.append((sc.mean[:, i].astype(np.float64), np.linalg.inv(Rq @ np.diag(s ** 2) @ Rq.T),
                       proj[i, 6], proj[i, 7]))
    ts = np.linspace(550.0, 650.0, 20001)
    exp_img = np.zeros_like(img)
    for vv in range(v.H):
        for uu in range(v.W):
            pd = np.array([(uu + 0.5 - v.W / 2) * f32(v.pitch), (vv + 0.5 - v.H / 2) * f32(v.pitch),
                           f32(v.sdd)])
            d = R.T @ (pd - t) - so
            d /= np.linalg.norm(d)
            T, Cv = 1.0, 0.0
            for i in order:
                mu, Si, alpha, c = params[i]
                X = so[None, :] + ts[:, None] * d[None, :] - mu[None, :]
                m2 = np.einsum("ij,jk,ik->i", X, Si, X).min()
                if m2 > 9.0:
                    continue
                s_ = alpha * np.exp(-0.5 * m2)
                Cv += c * s_ * T
                T *= 1 - s_
            exp_img[vv, uu] = Cv
    assert np.abs(img - exp_img).max() < 1e-2 * max(1e-12, exp_img.max())


# ----------------------------------------------------------------- invariants

def test_linear_in_radiosity():
    sc = synth.random_scene(21, 200, k=8, L=1, extent=12.0)
    v = synth.view(40, 40, 0.8, 1000.0, 600.0, 30.0)
    rng = np.random.default_rng(1)
    c1 = rng.uniform(0, 1, size=(1, sc.n))
    c2 = rng.uniform(0, 1, size=(1, sc.n))
    i1 = ref.render(sc, [v], c_override=c1)[0]
    i2 = ref.render(sc, [v], c_override=c2)[0]
    i12 = ref.render(sc, [v], c_override=c1 + 2.5 * c2)[0]
    np.testing.assert_allclose(i12, i1 + 2.5 * i2, rtol=1e-12, atol=1e-14)


def test_permutation_invariance_within_sets():
    sc = synth.random_scene(22, 300, k=16, L=3, extent=12.0)
    v = synth.view(40, 40, 0.8, 1000.0, 600.0, 70.0)
    base = ref.render(sc, [v])[0]
    rng = np.random.default_rng(3)
    pi = rng.permutation(sc.n_iso)
    pd = sc.n_iso + rng.permutation(sc.n - sc.n_iso)
    perm = sc.subset(pi, pd)
    img = ref.render(perm, [v])[0]
    np.testing.assert_allclose(img, base, rtol=1e-13, atol=1e-15)


def test_isotropic_blob_is_pose_symmetric():
    s, alpha = 3.0, 0.6
    sc = make_scene([[0, 0, 0]], [[s, s, s]], [[1, 0, 0, 0]], [alpha], seed=9)
    c = 1.0 / (1.0 + np.exp(-(sc.b_iso.astype(np.float64) @ sc.feat[:, 0].astype(np.float64))))
    imgs = []
    for th in (0.0, 37.0, 90.0, 200.0, 333.0):
        v = synth.view(41, 41, 0.7, 1000.0, 600.0, th)
        imgs.append(ref.render(sc, [v])[0])
    for im in imgs[1:]:
        np.testing.assert_allclose(im, imgs[0], atol=1e-12)
    f = f32(1000.0) / f32(0.7)
    var = (np.float64(np.float32(s)) * f / 600.0) ** 2 + 0.3
    vv, uu = np.meshgrid(np.arange(41) + 0.5 - 20.5, np.arange(41) + 0.5 - 20.5, indexing="ij")
    r2 = (uu ** 2 + vv ** 2) / var
    exp_img = np.where(r2 <= 9.0, c * alpha * np.exp(-0.5 * r2), 0.0)
    np.testing.assert_allclose(imgs[0], exp_img, atol=1e-6)


def test_joint_rasterization_occlusion():
    """App. A.2: an opaque isotropic Gaussian in front hides a directional one
    behind it; rendering the two sets separately and adding is wrong."""
    # azimuth 0 puts the source at (600, 0, 0) looking along -x: the Gaussian
    # at x = +40 is in front of the one at x = -40, both on the principal ray
    sc = make_scene([[40, 0, 0], [-40, 0, 0]], [[3, 3, 3], [3, 3, 3]], [[1, 0, 0, 0]] * 2,
                    [0.999, 0.5], n_iso=1, k=4, L=1, seed=12)
    v = synth.view(33, 33, 0.5, 1000.0, 600.0, 0.0)
    proj = ref.project(sc, v)
    assert proj[0, 8] < proj[1, 8]
    pix = [[0, 16, 16]]
    joint = ref.render_pixels(sc, [v], pix)[0]
    a = ref.render_pixels(sc.subset([0], []), [v], pix)[0]
    b = ref.render_pixels(sc.subset([], [1]), [v], pix)[0]
    # the front Gaussian is clamped to s = 0.99, leaving T = 0.01 behind it
    assert a == pytest.approx(0.99 * proj[0, 7], rel=1e-12)
    assert joint == pytest.approx(a + 0.01 * b, rel=1e-12)
    assert abs(joint - (a + b)) > 0.9 * b


def test_iso_only_is_x_gaussian_special_case():
    """With n_iso = n every radiosity is sigmoid(b . f) (the X-Gaussian form
    the paper starts from, Sec. 3.1), independent of the view."""
    sc = synth.random_scene(23, 100, k=8, L=1, iso_fraction=1.0)
    p0 = ref.project(sc, synth.view(32, 32, 1.0, 1000.0, 600.0, 0.0))
    p1 = ref.project(sc, synth.view(32, 32, 1.0, 1000.0, 600.0, 123.0))
    np.testing.assert_array_equal(p0[:, 7], p1[:, 7])


# ----------------------------------------------------------------------- losses

def _ssim_scipy(x, y):
    from scipy.signal import correlate2d
    g = np.exp(-((np.arange(11) - 5) ** 2) / (2 * 1.5 ** 2))
    g /= g.sum()
    w = np.outer(g, g)

    def filt(a):
        return correlate2d(a, w, mode="same", boundary="fill", fillvalue=0.0)

    mx, my = filt(x), filt(y)
    vx, vy, cxy = filt(x * x) - mx ** 2, filt(y * y) - my ** 2, filt(x * y) - mx * my
    C1, C2 = 0.01 ** 2, 0.03 ** 2
    return (((2 * mx * my + C1) * (2 * cxy + C2)) / ((mx ** 2 + my ** 2 + C1) * (vx + vy + C2))).mean()


def test_ssim_matches_scipy_window():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, size=(23, 31))
    y = np.clip(x + rng.normal(0, 0.1, size=x.shape), 0, 1)
    loss, sm, _ = ref.loss_l1ssim(x, y, 0.2)
    assert sm == pytest.approx(_ssim_scipy(x, y), abs=1e-13)
    assert loss == pytest.approx(0.8 * np.abs(x - y).mean() + 0.2 * (1 - sm), abs=1e-14)


def test_ssim_identity_and_zero_gradient():
    x = np.random.default_rng(1).uniform(0, 1, size=(20, 20))
    loss, sm, g = ref.loss_l1ssim(x, x, 0.2)
    assert sm == pytest.approx(1.0, abs=1e-14)
    assert loss == pytest.approx(0.0, abs=1e-14)
    assert np.abs(g).max() < 1e-14


@pytest.mark.parametrize("which", ["l1ssim", "ncc"])
def test_loss_gradients_by_central_differences(which):
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, size=(14, 17))
    y = np.clip(0.7 * x + 0.2 + rng.normal(0, 0.1, size=x.shape), 0, 1)

    def L(z):
        return ref.loss_l1ssim(z, y, 0.2, want_grad=False)[0] if which == "l1ssim" else \
            ref.loss_ncc(z, y, want_grad=False)[0]

    g = ref.loss_l1ssim(x, y, 0.2)[2] if which == "l1ssim" else ref.loss_ncc(x, y)[1]
    h = 1e-6
    for idx in [(0, 0), (3, 4), (7, 8), (13, 16), (10, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        assert (L(xp) - L(xm)) / (2 * h) == pytest.approx(g[idx], rel=1e-6, abs=1e-10)


def test_ncc_matches_corrcoef_and_affine_invariance():
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, size=500)
    y = rng.uniform(0, 1, size=500) + 0.5 * x
    loss, _ = ref.loss_ncc(x, y, eps=0.0)
    assert 1 - loss == pytest.approx(np.corrcoef(x, y)[0, 1], abs=1e-13)
    loss2, g2 = ref.loss_ncc(2.5 * y + 0.3, y, eps=0.0)
    assert loss2 == pytest.approx(0.0, abs=1e-14)
    assert np.abs(g2).max() < 1e-14


# ------------------------------------------------------ pose optimiser step

def test_pose_step_reference_pins():
    from oracle import pose_opt
    rng = np.random.default_rng(4)
    # Exp equals scipy's rotation of the same rotation vector, small and large
    for w in (rng.normal(size=3) * 1e-7, rng.normal(size=3) * 0.3, np.array([0.0, 2.5, -1.0])):
        np.testing.assert_allclose(pose_opt.exp_so3(w), Rotation.from_rotvec(w).as_matrix(), atol=1e-12)
    # Adam's first bias-corrected step moves every component by lr against the
    # gradient's sign (|mhat| / sqrt(vhat) = 1 at t = 1 up to eps)
    g = rng.normal(size=6)
    lr = np.array([1.0, 1.0, 1.0, 0.01, 0.01, 0.01])
    d, m, s = pose_opt.adam_step(g, np.zeros(6), np.zeros(6), 1, lr, 0.9, 0.999, 1e-12)
    np.testing.assert_allclose(d, -lr * np.sign(g), rtol=1e-9)
    # a constant gradient keeps the step at lr (bias correction exact)
    for t in range(2, 6):
        d, m, s = pose_opt.adam_step(g, m, s, t, lr, 0.9, 0.999, 1e-12)
        np.testing.assert_allclose(d, -lr * np.sign(g), rtol=1e-9)
    # re-basing is the left action: source position moves by -R'^T rho rotated, and
    # a pure translation tangent shifts t only
    P = synth.azimuth_pose(30.0, 600.0)
    Q = pose_opt.rebase(P, np.array([1.0, -2.0, 3.0, 0.0, 0.0, 0.0]))
    np.testing.assert_allclose(Q[:, :3], P[:, :3], atol=1e-15)
    np.testing.assert_allclose(Q[:, 3], P[:, 3] + [1.0, -2.0, 3.0], atol=1e-12)
    # errors: a rotation by 5 degrees about the isocentre gives 5 degrees and a
    # source displacement of 2 SID sin(2.5 deg)
    w = np.array([0.0, 0.0, np.radians(5.0)])
    P2 = synth.perturbed_pose(P, w, np.zeros(3))
    ang, dso = pose_opt.pose_errors(P2, P)
    assert ang == pytest.approx(5.0, abs=1e-9)
    assert dso == pytest.approx(2 * 600.0 * np.sin(np.radians(2.5)), rel=1e-9)
    # projection distance: points at one camera depth z shifted sideways by d
    # move by f d / z pixels; a rotation about the optical axis by a moves a
    # point at image radius r by 2 r sin(a / 2)
    I = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    pts = np.concatenate([rng.uniform(-50, 50, size=(20, 2)), np.full((20, 1), 700.0)], axis=1)
    T = I.copy()
    T[:, 3] = [3.0, -4.0, 0.0]
    assert pose_opt.projection_distance(T, I, 2000.0, pts) == pytest.approx(2000.0 * 5.0 / 700.0, rel=1e-12)
    assert pose_opt.projection_distance(I, I, 2000.0, pts) == 0.0
    Rz = np.concatenate([Rotation.from_rotvec([0, 0, 0.1]).as_matrix(), np.zeros((3, 1))], axis=1)
    r = 2000.0 * np.linalg.norm(pts[:, :2], axis=1) / 700.0
    assert pose_opt.projection_distance(Rz, I, 2000.0, pts) == pytest.approx(np.mean(2 * r * np.sin(0.05)), rel=1e-12)
    # rotation about a pivot: the pivot's image stays put under a pure rotation,
    # and pivot_gradient matches central differences of a smooth function of
    # the projected points through rebase_about, given the left-tangent
    # gradient from central differences through rebase
    piv = np.array([5.0, -8.0, 12.0])
    Q = pose_opt.rebase_about(P, np.array([0.0, 0.0, 0.0, 0.1, -0.2, 0.05]), piv)
    np.testing.assert_allclose(Q[:, :3] @ piv + Q[:, 3], P[:, :3] @ piv + P[:, 3], atol=1e-9)
    wpts = rng.normal(size=(30, 3)) * 40.0

    def lossf(pose):
        x = wpts @ pose[:, :3].T + pose[:, 3]
        u = 1000.0 * x[:, :2] / x[:, 2:3]
        return float(np.sum(np.sin(u / 37.0)) + np.sum(u[:, 0] * u[:, 1]) * 1e-4)

    def fd(step_fn):
        out = np.zeros(6)
        for q in range(6):
            e = np.zeros(6)
            e[q] = 1e-6
            out[q] = (lossf(step_fn(e)) - lossf(step_fn(-e))) / 2e-6
        return out

    g_left = fd(lambda e: pose_opt.rebase(P, e))
    g_piv = fd(lambda e: pose_opt.rebase_about(P, e, piv))
    np.testing.assert_allclose(pose_opt.pivot_gradient(g_left, P, piv), g_piv, rtol=1e-5, atol=1e-6 * np.abs(g_piv).max())
    # the world origin is the source-frame point t
    np.testing.assert_allclose(pose_opt.rebase_about(P, np.array([1.0, 2.0, 3.0, 0.1, 0.0, 0.0]), np.zeros(3))[:, 3],
                               P[:, 3] + [1.0, 2.0, 3.0], atol=1e-9)


def test_entangled_radiosity_reductions_and_logit_sum():
    """Co-located ablation: with B_dir = 0 it is the all-isotropic model, with
    b_iso = 0 the all-directional one (same images), and in general each
    Gaussian's radiosity logit is the isotropic logit plus the directional one
    (read from the per-Gaussian projection records of the three models)."""
    from dataclasses import replace
    base = synth.random_scene(5, 40, k=8, L=2, iso_fraction=0.0, extent=8.0, std_range=(1.0, 2.5),
                              alpha_range=(0.1, 0.6))
    ent = replace(base, n_iso=0, entangled=True)
    v = synth.view(32, 28, 0.6, 1000.0, 600.0, 25.0)
    iso_only = replace(base, n_iso=base.n)
    dir_only = replace(base, n_iso=0)
    zero_B = replace(ent, B_dir=np.zeros_like(base.B_dir))
    zero_b = replace(ent, b_iso=np.zeros_like(base.b_iso))
    np.testing.assert_allclose(ref.render(zero_B, [v])[0], ref.render(replace(iso_only, B_dir=zero_B.B_dir), [v])[0],
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(ref.render(zero_b, [v])[0], ref.render(replace(dir_only, b_iso=zero_b.b_iso), [v])[0],
                               rtol=0, atol=1e-15)
    ci = ref.project(iso_only, v)[:, ref.PROJ_FIELDS.index("c")]
    cd = ref.project(dir_only, v)[:, ref.PROJ_FIELDS.index("c")]
    ce = ref.project(ent, v)[:, ref.PROJ_FIELDS.index("c")]
    ok = ref.project(ent, v)[:, 0] > 0
    assert ok.sum() > 20

    def logit(c):
        return np.log(c) - np.log1p(-c)

    np.testing.assert_allclose(logit(ce[ok]), logit(ci[ok]) + logit(cd[ok]), rtol=1e-9, atol=1e-9)
    # the entangled image differs from both single-term models
    img_e = ref.render(ent, [v])[0]
    assert np.abs(img_e - ref.render(iso_only, [v])[0]).max() > 1e-3
    assert np.abs(img_e - ref.render(dir_only, [v])[0]).max() > 1e-3
    # an entangled model must have no separate isotropic set
    with pytest.raises(Exception):
        ref.render(replace(ent, n_iso=3), [v])
