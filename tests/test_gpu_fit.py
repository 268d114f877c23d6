"""Fitting loop on the GPU against the FP64 reference (oracle/fit_ref.py):
the Adam step inside the captured graph, the densification statistics of
the backward, densification itself (bit-exact decisions and copies, children
within rounding), the carried optimiser moments, the opacity reset, and a
short fitting run that lowers the loss."""
from dataclasses import replace

import numpy as np
import pytest

from gpu_common import make_renderer, rel_l2
from oracle import fit_ref, ref
from paper_2406_02518_amd import binding, fit, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture()
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = binding.Renderer(0, stream=torch.cuda.Stream())
    yield r
    r.close()


def _dev(scene):
    return {name: torch.from_numpy(np.ascontiguousarray(getattr(scene, name))).cuda() for name in binding.PARAM_NAMES}


def _host(p):
    return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in p.items()}


def _lrs(o, t):
    return dict(mean=fit_ref.expon_lr(t, o.lr_mean_init, o.lr_mean_final, o.lr_mean_steps), quat=o.lr_quat,
                log_scale=o.lr_log_scale, opacity_logit=o.lr_opacity, feat=o.lr_feat, b_iso=o.lr_b_iso,
                B_dir=o.lr_B_dir)


def _flat(d):
    return np.concatenate([np.asarray(d[k], np.float64).ravel() for k in fit_ref.GROUPS])


def test_adam_step_matches_reference(R):
    true = synth.random_scene(21, 300, k=8, L=2, iso_fraction=0.5, extent=15.0, std_range=(0.8, 2.5),
                              alpha_range=(0.05, 0.5))
    sc = synth.perturb_scene(22, true)
    v = synth.view(48, 40, 1.6, 1000.0, 600.0, 35.0)
    target = torch.from_numpy(ref.render(true, [v])[0].astype(np.float32).ravel()).cuda()
    p = _dev(sc)
    R.set_model(p, sc.n_iso, sc.L)
    R.set_views([v])
    R.set_fit_optimizer(15.0, lr_mean_steps=7)   # a short decay so the schedule moves
    o = binding.ddgs_default_fit_options(15.0)
    o.lr_mean_steps = 7
    img = torch.empty(v.W * v.H, device="cuda")
    dl = torch.empty_like(img)
    loss = torch.empty(1, device="cuda")
    g = R.alloc_grads()
    with torch.cuda.stream(R.stream):
        binding.ddgs_step_capture(R.ctx, binding.LOSS_L1_DSSIM, target.data_ptr(), 0.2, img.data_ptr(),
                                  dl.data_ptr(), loss.data_ptr(), R.grads_struct(g))
    z = {k: np.zeros_like(a) for k, a in _host(p).items()}
    m, s = dict(z), dict(z)
    for t in (1, 2, 3):
        before = _host(p)
        binding.ddgs_step_launch(R.ctx)
        binding.ddgs_check(R.ctx)
        grads = {k[1:]: a for k, a in _host(g).items() if k != "dpose"}
        exp, m, s = fit_ref.adam(before, grads, m, s, t, _lrs(o, t), o.beta1, o.beta2, o.eps)
        after = _host(p)
        lrs = _lrs(o, t)
        for k in fit_ref.GROUPS:
            tol = 1e-4 * lrs[k] + 2e-7 * np.abs(before[k])
            assert np.all(np.abs(after[k] - exp[k]) <= tol), (t, k, np.abs(after[k] - exp[k]).max())
            assert np.abs(after[k] - before[k]).max() > 0, (t, k)
        gm, gv = R.fit_moments()
        assert rel_l2(gm, _flat(m)) < 1e-5 and rel_l2(gv, _flat(s)) < 1e-5, t
    R.set_fit_optimizer(None)


def test_densify_stats_match_oracle(R):
    sc = synth.random_scene(31, 250, k=8, L=1, iso_fraction=0.6, extent=18.0, std_range=(0.6, 2.5),
                            alpha_range=(0.05, 0.5))
    views = [synth.view(48, 40, 1.6, 1000.0, 600.0, 10.0), synth.view(48, 40, 1.6, 1000.0, 600.0, 100.0)]
    R.set_scene(sc)
    R.set_views(views)
    stats = R.new_densify_stats()
    R.set_densify_stats(stats)
    dlh = np.random.default_rng(31).normal(size=2 * 48 * 40)
    dl = torch.from_numpy(dlh.astype(np.float32)).cuda()
    R.render()
    R.backward(dl)
    torch.cuda.synchronize()
    o = ref.backward(sc, views, ref.all_pixels(views), dlh, want_g2d=True)
    acc, den, rad, ok = fit_ref.densify_stats(sc, views, o["g2d"])
    assert ok.sum() > 0.8 * sc.n
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in stats.items()}
    np.testing.assert_array_equal(got["count"][ok], den[ok])
    assert rel_l2(got["grad"][ok], acc[ok]) < 1e-4
    np.testing.assert_allclose(got["radius"][ok], rad[ok], rtol=1e-5, atol=1e-5)
    # a second backward adds the same again
    R.render()
    R.backward(dl)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(stats["count"].cpu().numpy()[ok], 2 * den[ok])
    R.set_densify_stats(None)


def _dense_case(seed, n, n_iso):
    rng = np.random.default_rng(seed)
    sc = synth.random_scene(seed, n, k=8, L=2, iso_fraction=n_iso / n, extent=20.0, std_range=(0.5, 4.0),
                            alpha_range=(0.002, 0.5))
    acc = rng.uniform(0.0, 1.2e-3, n).astype(np.float32)
    cnt = rng.integers(0, 4, n).astype(np.float32)
    rad = rng.uniform(0.0, 40.0, n).astype(np.float32)
    noise = rng.normal(size=(n, 2, 3)).astype(np.float32)
    return sc, acc, cnt, rad, noise


@pytest.mark.parametrize("n,n_iso,world,screen", [(600, 300, 3.0, 20.0), (600, 300, 0.0, 0.0), (400, 0, 3.0, 20.0),
                                                  (400, 400, 3.0, 0.0), (1, 1, 0.0, 0.0)])
def test_densify_matches_reference(R, n, n_iso, world, screen):
    sc, acc, cnt, rad, noise = _dense_case(40 + n + n_iso, n, n_iso)
    p = _dev(sc)
    R.set_model(p, sc.n_iso, sc.L)
    stats = {"grad": torch.from_numpy(acc).cuda(), "count": torch.from_numpy(cnt).cuda(),
             "radius": torch.from_numpy(rad).cuda()}
    R.set_densify_stats(stats)
    out, ni = R.densify(torch.from_numpy(noise).cuda(), grad_threshold=2e-4, dense_scale=1.5, min_opacity=0.005,
                        max_world_scale=world, max_screen_radius=screen)
    torch.cuda.synchronize()
    th = fit_ref.thresholds(2e-4, 1.5, 0.005, world, screen)
    host = {k: getattr(sc, k) for k in binding.PARAM_NAMES}
    exp, exp_iso, src, kind = fit_ref.densify(host, sc.n_iso, acc, cnt, rad, noise, th)
    assert ni == exp_iso and out["mean"].shape[1] == len(src), (ni, exp_iso, out["mean"].shape, len(src))
    if n > 1:
        assert (kind == 1).any() and (kind >= 2).any() and len(src) != n
    got = {k: v.cpu().numpy() for k, v in out.items()}
    copy = kind < 2
    for name in ("quat", "opacity_logit", "feat"):
        np.testing.assert_array_equal(got[name].reshape(-1, len(src)), exp[name].reshape(-1, len(src)).astype(np.float32))
    np.testing.assert_array_equal(got["mean"][:, copy], exp["mean"][:, copy].astype(np.float32))
    np.testing.assert_allclose(got["mean"][:, ~copy], exp["mean"][:, ~copy], rtol=0, atol=2e-5)
    np.testing.assert_array_equal(got["log_scale"], exp["log_scale"].astype(np.float32))
    np.testing.assert_array_equal(got["b_iso"], sc.b_iso)
    np.testing.assert_array_equal(got["B_dir"], sc.B_dir)
    R.set_densify_stats(None)


def test_moments_follow_densification_and_opacity_reset(R):
    """One captured step creates moments; densification keeps a kept
    Gaussian's moments and zeroes new ones; the opacity reset clamps the
    logits and zeroes only the opacity moments."""
    true = synth.random_scene(51, 300, k=8, L=2, iso_fraction=0.5, extent=15.0, std_range=(0.8, 3.0),
                              alpha_range=(0.05, 0.5))
    sc = synth.perturb_scene(52, true)
    v = synth.view(48, 40, 1.6, 1000.0, 600.0, 35.0)
    target = torch.from_numpy(ref.render(true, [v])[0].astype(np.float32).ravel()).cuda()
    p = _dev(sc)
    R.set_model(p, sc.n_iso, sc.L)
    R.set_views([v])
    R.set_fit_optimizer(15.0)
    stats = R.new_densify_stats()
    R.set_densify_stats(stats)
    img = torch.empty(v.W * v.H, device="cuda")
    dl, loss = torch.empty_like(img), torch.empty(1, device="cuda")
    g = R.alloc_grads()
    with torch.cuda.stream(R.stream):
        binding.ddgs_step_capture(R.ctx, binding.LOSS_L1_DSSIM, target.data_ptr(), 0.2, img.data_ptr(),
                                  dl.data_ptr(), loss.data_ptr(), R.grads_struct(g))
    binding.ddgs_step_launch(R.ctx)
    binding.ddgs_check(R.ctx)
    m0, v0 = R.fit_moments()
    n, k, kl = sc.n, sc.k, sc.L * (sc.L + 2)
    st = {kk: t.cpu().numpy() for kk, t in stats.items()}
    thr = float(np.quantile(st["grad"][st["count"] > 0] / st["count"][st["count"] > 0], 0.7))
    noise = torch.randn((n, 2, 3), device="cuda")
    out, ni = R.densify(noise, grad_threshold=thr, dense_scale=1.5)
    th = fit_ref.thresholds(thr, 1.5, 0.005, 0.0, 0.0)
    host = {kk: getattr(sc, kk) for kk in binding.PARAM_NAMES}
    host.update({kk: p[kk].cpu().numpy() for kk in binding.PARAM_NAMES})  # after the step
    _, exp_iso, src, kind = fit_ref.densify(host, sc.n_iso, st["grad"], st["count"], st["radius"],
                                            noise.cpu().numpy(), th)
    assert ni == exp_iso and (kind == 1).any() and (kind >= 2).any()
    R.set_model(out, ni, sc.L)
    m1, v1 = R.fit_moments()
    nn = len(src)
    off_old = np.cumsum([0, 3 * n, 4 * n, 3 * n, n, k * n])
    off_new = np.cumsum([0, 3 * nn, 4 * nn, 3 * nn, nn, k * nn])
    for gi, rows in enumerate((3, 4, 3, 1, k)):
        for mo, mn in ((m0, m1), (v0, v1)):
            old = mo[off_old[gi]:off_old[gi + 1]].reshape(rows, n)
            new = mn[off_new[gi]:off_new[gi + 1]].reshape(rows, nn)
            exp = np.where(kind[None, :] == 0, old[:, src], 0.0)
            np.testing.assert_array_equal(new, exp.astype(np.float32))
    np.testing.assert_array_equal(m1[off_new[-1]:], m0[off_old[-1]:])
    # opacity reset
    before = out["opacity_logit"].cpu().numpy().copy()
    R.reset_opacity(0.01)
    torch.cuda.synchronize()
    cap = np.float32(np.log(0.01) - np.log1p(-0.01))
    np.testing.assert_array_equal(out["opacity_logit"].cpu().numpy(), np.minimum(before, cap))
    m2, v2 = R.fit_moments()
    np.testing.assert_array_equal(m2[off_new[3]:off_new[4]], 0.0)
    np.testing.assert_array_equal(v2[off_new[3]:off_new[4]], 0.0)
    np.testing.assert_array_equal(m2[:off_new[3]], m1[:off_new[3]])
    R.set_fit_optimizer(None)
    R.set_densify_stats(None)


def test_fitting_loop_lowers_the_loss(R):
    c = synth.config("C3", scale=0.02)
    true = c.extra["true_scene"]
    views = c.views[::3]
    targets = [torch.from_numpy(t.astype(np.float32).ravel()).cuda() for t in ref.render(true, views)]
    sched = fit.FitSchedule(densify_from=40, densify_until=200, densify_every=40, opacity_reset_every=0)
    extent = float(np.abs(c.scene.mean).max())
    params, n_iso, hist = fit.fit(R, _dev(c.scene), c.scene.n_iso, c.scene.L, views, targets, iters=240,
                                  extent=extent, schedule=sched, log_every=40)
    print("history", hist)
    assert hist[-1][2] < 0.8 * hist[0][2]
    assert params["mean"].shape[1] == hist[-1][1]
    assert any(h[1] != c.scene.n for h in hist)
    assert all(torch.isfinite(t).all() for t in params.values())


def test_training_from_dual_sampling(R):
    """The paper's path end to end on a small phantom: dual-sampling
    initialisation from the volume, then fitting to targets rendered by the
    oracle from a model of the same phantom, with densification.  The loss
    falls and densification adds Gaussians to both sets."""
    from paper_2406_02518_amd import rads
    seed = 61
    ss = np.random.SeedSequence(seed)
    ph = synth.phantom(40, np.random.default_rng(ss.spawn(1)[0]))
    true = synth.scene_from_phantom(seed, 40, 3000, 0.15, k=8, L=1)
    views = [synth.view(48, 48, 1.2, 1000.0, 600.0, 30.0 * j) for j in range(12)]
    targets = [torch.from_numpy(t.astype(np.float32).ravel()).cuda() for t in ref.render(true, views)]
    hu = torch.from_numpy(np.ascontiguousarray(ph.transpose(2, 1, 0))).cuda()
    pts, ls, n_iso, _ = rads.sample(R, hu, (1.0, 1.0, 1.0), (-19.5, -19.5, -19.5), n1=1500, n2=1000, seed=2)
    g = torch.Generator().manual_seed(3)
    p = rads.initial_model(pts, ls, 8, 1, b_iso=torch.randn(8, generator=g).cuda(),
                           B_dir=0.1 * torch.randn((3, 8), generator=g).cuda())
    n0 = p["mean"].shape[1]
    sched = fit.FitSchedule(densify_from=50, densify_until=250, densify_every=50, opacity_reset_every=0,
                            grad_threshold=1e-5)
    params, n_iso_end, hist = fit.fit(R, p, n_iso, 1, views, targets, iters=300, extent=20.0, schedule=sched,
                                      log_every=50)
    print("history", hist, "n_iso", n_iso, "->", n_iso_end)
    assert hist[-1][2] < 0.7 * hist[0][2]
    assert params["mean"].shape[1] > n0 and n_iso_end > n_iso and params["mean"].shape[1] - n_iso_end > n0 - n_iso
    assert all(torch.isfinite(t).all() for t in params.values())
