"""The oracle's analytic FP64 backward checked against central differences of
its own forward (which the pins in test_oracle_pins tie to closed forms),
plus exact identities of the pose gradient.  CPU only."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import ref
from paper_2406_02518_amd import synth


def _scene64(seed, n=24, k=8, L=3, extent=6.0):
    sc = synth.random_scene(seed, n, k=k, L=L, iso_fraction=0.5, extent=extent,
                            std_range=(0.8, 2.5), alpha_range=(0.05, 0.6))
    s = sc.copy()
    for name, a in s.arrays().items():
        setattr(s, name, np.array(a, dtype=np.float64))
    return s


def _view(theta=40.0, W=26, H=22):
    v = synth.view(W, H, 0.5, 1000.0, 600.0, theta)
    v.pose = v.pose.astype(np.float64)
    return v


def _loss(scene, v, g, c_override=None):
    img, h, _ = ref.render(scene, [v], stats=True, c_override=c_override)
    return float((img[0].ravel() * g).sum()), int(h[0])


def _fd_group(scene, v, g, name, h, base_hash, max_coords=None, seed=0):
    arr = getattr(scene, name)
    flat = arr.reshape(-1)
    idx = np.arange(flat.size)
    if max_coords is not None and flat.size > max_coords:
        idx = np.random.default_rng(seed).choice(flat.size, max_coords, replace=False)
    fd = np.full(flat.size, np.nan)
    skipped = 0
    for i in idx:
        old = flat[i]
        # a pixel crossing the cut-off radius makes the image jump; shrink the
        # step until the set of contributing pairs is unchanged on both sides
        for hh in (h, h / 10, h / 100):
            flat[i] = old + hh
            lp, hp = _loss(scene, v, g)
            flat[i] = old - hh
            lm, hm = _loss(scene, v, g)
            flat[i] = old
            if hp == base_hash and hm == base_hash:
                fd[i] = (lp - lm) / (2 * hh)
                break
        else:
            skipped += 1
    return fd, skipped


GROUPS = [("mean", "dmean", 1e-5), ("quat", "dquat", 1e-6), ("log_scale", "dlog_scale", 1e-6),
          ("opacity_logit", "dopacity_logit", 1e-6), ("feat", "dfeat", 1e-6),
          ("b_iso", "db_iso", 1e-6), ("B_dir", "dB_dir", 1e-6)]


@pytest.mark.parametrize("seed", [31, 32])
def test_parameter_gradients_by_central_differences(seed):
    sc = _scene64(seed)
    v = _view(theta=17.0 * seed)
    g = np.random.default_rng(seed).normal(size=v.W * v.H)
    _, base_hash = _loss(sc, v, g)
    grads = ref.backward(sc, [v], ref.all_pixels([v]), g)
    for name, gname, h in GROUPS:
        fd, skipped = _fd_group(sc, v, g, name, h, base_hash)
        an = grads[gname].reshape(-1)
        ok = ~np.isnan(fd)
        assert ok.sum() >= 0.9 * fd.size, (name, skipped)
        err = np.linalg.norm(fd[ok] - an[ok]) / max(1e-300, np.linalg.norm(an[ok]))
        assert err < 1e-6, (name, err)
        assert np.linalg.norm(an) > 0, name


@pytest.mark.parametrize("seed,L,k", [(33, 3, 8), (34, 1, 4)])
def test_entangled_gradients_by_central_differences(seed, L, k):
    """The co-located ablation (both radiosity terms under one sigmoid on every
    Gaussian): every parameter group, both bases included, by central
    differences."""
    from dataclasses import replace
    sc = replace(_scene64(seed, k=k, L=L), n_iso=0, entangled=True)
    v = _view(theta=11.0 * seed)
    g = np.random.default_rng(seed).normal(size=v.W * v.H)
    _, base_hash = _loss(sc, v, g)
    grads = ref.backward(sc, [v], ref.all_pixels([v]), g)
    for name, gname, h in GROUPS:
        fd, skipped = _fd_group(sc, v, g, name, h, base_hash)
        an = grads[gname].reshape(-1)
        ok = ~np.isnan(fd)
        assert ok.sum() >= 0.9 * fd.size, (name, skipped)
        err = np.linalg.norm(fd[ok] - an[ok]) / max(1e-300, np.linalg.norm(an[ok]))
        assert err < 1e-6, (name, err)
        assert np.linalg.norm(an) > 0, name


def _exp_pose(v, delta):
    """pose' = Exp(delta) pose with delta = (rho, omega): R' = Exp(w) R,
    t' = Exp(w) t + rho."""
    P = np.asarray(v.pose, dtype=np.float64)
    E = Rotation.from_rotvec(delta[3:]).as_matrix()
    w = synth.View(W=v.W, H=v.H, pitch=v.pitch, sdd=v.sdd, pose=None)
    w.pose = np.concatenate([E @ P[:, :3], (E @ P[:, 3] + delta[:3])[:, None]], axis=1)
    return w


@pytest.mark.parametrize("seed", [41, 42])
def test_pose_gradient_by_central_differences(seed):
    sc = _scene64(seed)
    v = _view(theta=23.0 * seed)
    g = np.random.default_rng(seed).normal(size=v.W * v.H)
    _, base_hash = _loss(sc, v, g)
    an = ref.backward(sc, [v], ref.all_pixels([v]), g)["dpose"][0]
    fd = np.zeros(6)
    for a in range(6):
        for h in ((1e-5, 1e-6, 1e-7) if a < 3 else (1e-7, 1e-8, 1e-9)):
            d = np.zeros(6)
            d[a] = h
            lp, hp = _loss(sc, _exp_pose(v, d), g)
            lm, hm = _loss(sc, _exp_pose(v, -d), g)
            if hp == base_hash and hm == base_hash:
                fd[a] = (lp - lm) / (2 * h)
                break
        else:
            raise AssertionError(f"cut-off flips at every step for pose coordinate {a}")
    np.testing.assert_allclose(an, fd, rtol=2e-6, atol=1e-9 * np.abs(an).max())


def test_radiosity_gradient_by_central_differences():
    sc = _scene64(51)
    v = _view(theta=5.0)
    g = np.random.default_rng(5).normal(size=v.W * v.H)
    c = np.random.default_rng(6).uniform(0.1, 0.9, size=(1, sc.n))
    an = ref.backward(sc, [v], ref.all_pixels([v]), g, c_override=c)["dc"][0]
    # the image is linear in c, so differences are exact up to rounding
    for i in range(sc.n):
        e = np.zeros_like(c)
        e[0, i] = 1e-3
        lp, _ = _loss(sc, v, g, c + e)
        lm, _ = _loss(sc, v, g, c - e)
        assert (lp - lm) / 2e-3 == pytest.approx(an[i], rel=1e-9, abs=1e-12)


def test_translation_identity():
    """Moving every Gaussian by a equals moving the source frame by rho = R a,
    so sum_i dL/dmu_i = R^T g_rho exactly."""
    sc = _scene64(61, n=40)
    v = _view(theta=77.0)
    g = np.random.default_rng(7).normal(size=v.W * v.H)
    res = ref.backward(sc, [v], ref.all_pixels([v]), g)
    R = np.asarray(v.pose, dtype=np.float64)[:, :3]
    np.testing.assert_allclose(res["dmean"].sum(axis=1), R.T @ res["dpose"][0, :3], rtol=1e-10,
                               atol=1e-12 * np.abs(res["dmean"]).sum())


def test_multi_view_backward_is_sum_of_single_views():
    sc = _scene64(71)
    va, vb = _view(theta=10.0), _view(theta=130.0, W=20, H=30)
    pa, pb = ref.all_pixels([va]), ref.all_pixels([vb])
    ga = np.random.default_rng(1).normal(size=len(pa))
    gb = np.random.default_rng(2).normal(size=len(pb))
    both = ref.backward(sc, [va, vb], np.concatenate([pa, pb + np.array([1, 0, 0])]), np.concatenate([ga, gb]))
    ra = ref.backward(sc, [va], pa, ga)
    rb = ref.backward(sc, [vb], pb, gb)
    for key in ("dmean", "dquat", "dlog_scale", "dopacity_logit", "dfeat", "db_iso", "dB_dir"):
        np.testing.assert_allclose(both[key], ra[key] + rb[key], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(both["dpose"], np.stack([ra["dpose"][0], rb["dpose"][0]]), rtol=1e-12)


def test_sampled_pixel_backward_equals_sparse_full_backward():
    sc = _scene64(81)
    v = _view(theta=200.0)
    allp = ref.all_pixels([v])
    rng = np.random.default_rng(8)
    sel = rng.choice(len(allp), 40, replace=False)
    g = np.zeros(len(allp))
    g[sel] = rng.normal(size=40)
    full = ref.backward(sc, [v], allp, g)
    part = ref.backward(sc, [v], allp[sel], g[sel])
    for key in ("dmean", "dfeat", "dpose"):
        np.testing.assert_allclose(part[key], full[key], rtol=1e-12, atol=1e-15)
    vals = ref.render_pixels(sc, [v], allp[sel])
    np.testing.assert_allclose(vals, ref.render(sc, [v])[0].ravel()[sel], rtol=0, atol=0)
