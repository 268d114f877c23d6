"""Edge cases of Eq. 1 on the GPU against the FP64 oracle -- the sigma_max
clamp (forward value and the zero gradient of a clamped step) and the early
stop (t_min > 0) in the backward -- plus the boundary's ownership rules: the
torch-owned workspace, the autograd function at a non-zero pose tangent and
with interleaved forwards, and the captured step's overflow retry."""
import numpy as np
import pytest

from gpu_common import make_renderer, rel_l2, unique_pixels
from oracle import ref
from paper_2406_02518_amd import binding, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GROUPS = ("dmean", "dquat", "dlog_scale", "dopacity_logit", "dfeat", "db_iso", "dB_dir")
TOL = 1e-4


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = make_renderer()
    yield r
    r.close()


def _opaque_scene(seed=11, n=300):
    """Large footprints (std 1..3 mm -> ~3..10 px) with opacities in
    (0.3, 0.999) and every third one in (0.991, 0.999), so that alpha G
    exceeds sigma_max around many centres and the transmittance falls below
    0.3 (and below 1e-4) on many pixels."""
    sc = synth.random_scene(seed, n, k=8, L=2, extent=14.0, iso_fraction=0.6, std_range=(1.0, 3.0),
                            alpha_range=(0.3, 0.999))
    a = np.random.default_rng(seed + 100).uniform(0.991, 0.999, size=sc.opacity_logit[::3].shape)
    sc.opacity_logit[::3] = np.log(a / (1.0 - a)).astype(np.float32)
    return sc


def _view():
    return synth.view(64, 64, 0.5, 1000.0, 600.0, 20.0)


def _parity(R, sc, v, opts, seed):
    """Image and every gradient group against the oracle on the pixels whose
    Eq. 1 decisions are unique at the FP32/FP64 band (the upstream gradient
    is zero elsewhere)."""
    R.set_scene(sc)
    R.set_views([v])
    pix = unique_pixels(sc, [v], ref.all_pixels([v]), opts=opts)
    assert len(pix) > 0.5 * v.W * v.H
    img = R.render().cpu().numpy().astype(np.float64)
    exp = ref.render(sc, [v], opts=opts)[0].ravel()
    lin = pix[:, 2] * v.W + pix[:, 1]
    assert rel_l2(img[lin], exp[lin]) < TOL
    w = np.random.default_rng(seed).normal(size=len(pix))
    dl = np.zeros(v.W * v.H)
    dl[lin] = w
    g = R.backward(torch.from_numpy(dl.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    o = ref.backward(sc, [v], pix, w, opts=opts)
    for k in GROUPS:
        assert rel_l2(g[k].cpu().numpy(), o[k]) < TOL, k
    assert rel_l2(g["dpose"].cpu().numpy()[0], o["dpose"][0]) < TOL
    return img


@pytest.mark.parametrize("sigma_max", [0.99, 0.6])
def test_sigma_max_clamp_matches_oracle(R, sigma_max):
    sc = _opaque_scene()
    v = _view()
    opts = dict(sigma_max=sigma_max)
    # the clamp is reached: alpha G > sigma_max at the centre of many Gaussians
    pr = ref.project(sc, v, opts=opts)
    assert np.sum(pr[:, 0] * (pr[:, 6] > sigma_max)) >= 20
    try:
        R.set_options(sigma_max=sigma_max)
        _parity(R, sc, v, opts, seed=1)
    finally:
        R.set_options(sigma_max=0.99)


@pytest.mark.parametrize("t_min", [0.3, 1e-4])
def test_backward_with_early_stop_matches_oracle(R, t_min):
    sc = _opaque_scene(seed=12, n=500)
    v = _view()
    opts = dict(t_min=t_min)
    # the stop is taken: the image differs from the one without it
    assert np.abs(ref.render(sc, [v], opts=opts)[0] - ref.render(sc, [v])[0]).max() > 0.0
    try:
        R.set_options(t_min=t_min)
        _parity(R, sc, v, opts, seed=2)
    finally:
        R.set_options(t_min=0.0)


def test_default_workspace_is_torch_owned(R):
    """The renderer's workspace comes from torch's caching allocator; the same
    render through hipMalloc and through a caller region is bit-identical."""
    c = synth.config("C2", scale=0.05)
    R.set_scene(c.scene)
    R.set_views(c.views)
    a = R.render().cpu().numpy()
    assert R.allocator.bytes_held() > 0
    held = R.allocator.bytes_held()
    before = torch.cuda.memory_allocated()
    assert before >= held
    try:
        binding.ddgs_set_allocator(R.ctx, None, None)   # library hipMalloc
        assert R.allocator.bytes_held() == 0
        b = R.render().cpu().numpy()
        need = R.workspace_size(max(R.num_rendered(), 1))
        ws = torch.empty(int(need * 1.5), dtype=torch.uint8, device="cuda")
        R.set_workspace(ws)
        c2 = R.render().cpu().numpy()
    finally:
        R.set_workspace(None)   # back to the torch allocator
    d = R.render().cpu().numpy()
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c2)
    np.testing.assert_array_equal(a, d)
    assert R.allocator.bytes_held() > 0


def test_autograd_with_pose_tangent_against_oracle(R):
    """Non-zero tangent: the library composes Exp(delta) pose; the oracle
    renders at the pose composed independently (scipy, float64 rounded once)."""
    from scipy.spatial.transform import Rotation

    from paper_2406_02518_amd import autograd
    c = synth.config("C2", scale=0.05)
    views = [c.views[0], synth.view(40, 40, 5.0, 1000.0, 600.0, 90.0)]
    d = np.array([[1.5, -0.8, 2.0, 0.02, -0.015, 0.03], [-2.0, 1.0, 0.5, -0.01, 0.025, 0.005]])
    params = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda().requires_grad_(True)
              for k, v in c.scene.arrays().items()}
    delta = torch.tensor(d, dtype=torch.float32, device="cuda", requires_grad=True)
    img = autograd.render(R, views, params, c.scene.n_iso, c.scene.L, pose_tangent=delta)
    w = torch.from_numpy(np.random.default_rng(3).normal(size=img.numel()).astype(np.float32)).cuda()
    (img * w).sum().backward()
    composed = []
    for v, dv in zip(views, delta.detach().cpu().numpy().astype(np.float64)):
        P = np.asarray(v.pose, np.float64)
        E = Rotation.from_rotvec(dv[3:]).as_matrix()
        pose = np.concatenate([E @ P[:, :3], (E @ P[:, 3] + dv[:3])[:, None]], axis=1).astype(np.float32)
        composed.append(synth.view(v.W, v.H, v.pitch, v.sdd, v.sid, v.azimuth_deg, pose=pose))
    exp = np.concatenate([x.ravel() for x in ref.render(c.scene, composed)])
    assert rel_l2(img.detach().cpu().numpy(), exp) < TOL
    o = ref.backward(c.scene, composed, ref.all_pixels(composed), w.cpu().numpy())
    for k in ("mean", "quat", "log_scale", "opacity_logit", "feat", "b_iso", "B_dir"):
        assert rel_l2(params[k].grad.cpu().numpy(), o["d" + k]) < TOL, k
    for vi in range(len(views)):
        assert rel_l2(delta.grad[vi].cpu().numpy(), o["dpose"][vi]) < TOL


def test_autograd_interleaved_forwards(R):
    """Two forwards on one renderer summed into one loss: each backward
    differentiates its own render."""
    from paper_2406_02518_amd import autograd
    c = synth.config("C2", scale=0.05)
    va = [c.views[0]]
    vb = [synth.view(48, 40, 4.0, 1000.0, 600.0, 70.0)]
    params = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda().requires_grad_(True)
              for k, v in c.scene.arrays().items()}
    ia = autograd.render(R, va, params, c.scene.n_iso, c.scene.L)
    ib = autograd.render(R, vb, params, c.scene.n_iso, c.scene.L)
    rng = np.random.default_rng(4)
    wa = torch.from_numpy(rng.normal(size=ia.numel()).astype(np.float32)).cuda()
    wb = torch.from_numpy(rng.normal(size=ib.numel()).astype(np.float32)).cuda()
    ((ia * wa).sum() + (ib * wb).sum()).backward()
    oa = ref.backward(c.scene, va, ref.all_pixels(va), wa.cpu().numpy())
    ob = ref.backward(c.scene, vb, ref.all_pixels(vb), wb.cpu().numpy())
    for k in ("mean", "quat", "log_scale", "opacity_logit", "feat", "b_iso", "B_dir"):
        assert rel_l2(params[k].grad.cpu().numpy(), oa["d" + k] + ob["d" + k]) < TOL, k


# --------------------------------------------------------- overflow retry

@pytest.fixture(scope="module")
def RS():
    """A renderer on a stream of its own (a captured step needs one)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = binding.Renderer(0, stream=torch.cuda.Stream())
    yield r
    r.close()


def test_overflowed_replay_changes_nothing(RS):
    """A captured step whose tile entries exceed its capacity leaves the
    poses, the optimiser state and the model untouched, reports the overflow
    and the need, and the replays it skipped."""
    R = RS
    c = synth.config("C4", scale=0.03)
    views = c.views[:3]
    R.set_scene(c.scene)
    R.set_views(views)
    R.render()
    need = R.num_rendered()
    n = R.image_size()
    tgt = torch.rand(n, device="cuda")
    img, dl = torch.empty(n, device="cuda"), torch.empty(n, device="cuda")
    lo = torch.empty(len(views), device="cuda")
    grads = R.alloc_grads(("dpose",))
    try:
        R.set_options(capacity=max(need // 4, 1))
        R.set_pose_optimizer(1.0, 0.01, pivot=(0.0, 0.0, 0.0))
        with torch.cuda.stream(R.stream):
            binding.ddgs_step_capture(R.ctx, binding.LOSS_NCC, tgt.data_ptr(), 0.0, img.data_ptr(), dl.data_ptr(),
                                      lo.data_ptr(), R.grads_struct(grads))
        before = R.get_poses()
        for _ in range(3):
            binding.ddgs_step_launch(R.ctx)
        st, flags = binding.ddgs_check(R.ctx, raise_on_error=False)
        assert st == binding.ERR_CAPACITY and flags & 1
        skipped, got_need = binding.ddgs_step_report(R.ctx)
        assert skipped == 3 and got_need == need
        after = R.get_poses()
        for a, b in zip(before, after):
            np.testing.assert_array_equal(a, b)
    finally:
        R.set_pose_optimizer(None)
        R.set_options(capacity=0)


def test_registration_retries_overflow_exactly(RS):
    """register() from a too-small capacity ends bit-identical to a run with
    ample capacity: the overflowed iterations are replayed after growing."""
    R = RS
    from paper_2406_02518_amd import register
    c = synth.config("C4", scale=0.03)
    views = c.views[:4]
    R.set_scene(c.scene)
    R.set_views([c.extra["gt_view"]] * len(views))
    tgt = R.render().clone()
    runs = []
    for cap in (0, 64):
        R.set_views(views)
        R.set_options(capacity=cap)
        try:
            poses, hist = register.register(R, tgt, iters=12, check_every=4, rel_tol=0.0, abs_tol=0.0)
        finally:
            R.set_options(capacity=0)
        runs.append((poses, hist))
    for a, b in zip(runs[0][0], runs[1][0]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(runs[0][1][-1][1], runs[1][1][-1][1])


def test_fitting_retries_overflow_exactly(RS):
    """fit() from a too-small capacity ends bit-identical to a run with ample
    capacity (the fused Adam of an overflowed replay is skipped, the replay
    is run again after the capacity grows)."""
    R = RS
    from paper_2406_02518_amd import fit
    c = synth.config("C3", scale=0.02)
    views = c.views[:6]
    R.set_scene(c.scene)
    R.set_views(views)
    targets = [t.reshape(-1).clone() for t in R.split(R.render())]
    results = []
    for cap in (0, 64):
        p = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in c.scene.arrays().items()}
        p["mean"] += 0.3
        R.set_options(capacity=cap)
        try:
            out, n_iso, hist = fit.fit(R, p, c.scene.n_iso, c.scene.L, views, targets, iters=10, extent=100.0,
                                       schedule=fit.FitSchedule(densify_from=10 ** 9), log_every=5)
        finally:
            R.set_options(capacity=0)
        results.append(({k: v.cpu().numpy() for k, v in out.items()}, hist))
    for k in results[0][0]:
        np.testing.assert_array_equal(results[0][0][k], results[1][0][k])
    assert [h[2] for h in results[0][1]] == [h[2] for h in results[1][1]]
