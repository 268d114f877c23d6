"""Radiodensity-aware dual sampling on the GPU against the FP64 reference
(oracle/rads_ref.py): level, crossing count and total weight exactly, the
interface points and the drawn voxel centres within float32 rounding, the
set split, and the nearest-neighbour scales; small ragged volumes, edge
cases and the 256^3 phantom of the fitting workload with the paper's set
sizes."""
import ctypes

import numpy as np
import pytest

from oracle import rads_ref
from paper_2406_02518_amd import binding, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture()
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = binding.Renderer(0, stream=torch.cuda.Stream())
    yield r
    r.close()


def _volume(hu, spacing, origin):
    t = torch.from_numpy(np.ascontiguousarray(hu)).cuda()
    f3 = ctypes.c_float * 3
    v = binding.ddgs_volume(hu.shape[2], hu.shape[1], hu.shape[0], f3(*spacing), f3(*origin), t.data_ptr())
    return v, t


def _run(R, hu, spacing, origin, n1, n2, seed, full_knn=True):
    vol, keep = _volume(hu, spacing, origin)
    level, M, W = binding.ddgs_rads_prepare(R.ctx, vol)
    iso = rads_ref.iso_level(hu)
    assert level == iso
    pmc, _ = rads_ref.crossings(hu, iso, spacing, origin)
    assert M == len(pmc)
    assert W == int(rads_ref.weights(hu).astype(np.uint64).sum())
    rng = np.random.default_rng(seed)
    keys = rng.integers(0, 1 << 32, max(M, 1), dtype=np.uint64).astype(np.uint32)
    keys[: min(8, M)] = keys[0]  # a few equal keys: ties go by edge order
    draws = rng.integers(0, max(W, 1), max(n2, 1), dtype=np.uint64)
    N = min(n1, M) + n2
    pts = torch.empty((3, max(N, 1)), device="cuda")
    ls = torch.empty((3, max(N, 1)), device="cuda")
    kd = torch.from_numpy(keys).cuda()
    dd = torch.from_numpy(draws.view(np.int64)).cuda()
    n_iso = binding.ddgs_rads_sample(R.ctx, n1, kd.data_ptr(), n2, dd.data_ptr(), pts.data_ptr(), ls.data_ptr())
    torch.cuda.synchronize()
    exp_pts, exp_iso, _ = (rads_ref.rads(hu, spacing, origin, n1, keys[:M], draws[:n2]) if full_knn else
                           (None, None, None))
    if not full_knn:
        order = np.lexsort((np.arange(M), keys[:M]))[:n1]
        exp_pts = np.concatenate([pmc[order], rads_ref.weighted_draws(hu, draws[:n2], spacing, origin)[0]])
        exp_iso = len(order) + n2 // 2
    got = pts.cpu().numpy()[:, :N].T.astype(np.float64)
    assert n_iso == exp_iso
    np.testing.assert_allclose(got, exp_pts, rtol=0, atol=2e-4)
    rows = np.arange(N) if full_knn else np.random.default_rng(seed).choice(N, 400, replace=False)
    exp_ls = rads_ref.knn_log_scale(exp_pts, rows=rows)
    got_ls = ls.cpu().numpy()[:, :N]
    np.testing.assert_array_equal(got_ls[0], got_ls[1])
    np.testing.assert_array_equal(got_ls[0], got_ls[2])
    np.testing.assert_allclose(got_ls[0][rows], exp_ls, rtol=0, atol=1e-4)
    return M, W, N


@pytest.mark.parametrize("shape,n1,n2", [((12, 17, 23), 300, 200), ((40, 33, 37), 1500, 1000),
                                         ((5, 6, 7), 10_000, 50), ((9, 8, 7), 0, 30), ((9, 8, 7), 40, 0)])
def test_rads_matches_reference(R, shape, n1, n2):
    nz, ny, nx = shape
    ph = synth.phantom(max(shape), np.random.default_rng(sum(shape)))  # [x][y][z]
    hu = np.ascontiguousarray(ph[:nx, :ny, :nz].transpose(2, 1, 0))
    M, W, N = _run(R, hu, (0.9, 1.1, 1.3), (-20.0, -25.0, -30.0), n1, n2, seed=nx + n1)
    assert M > 0 and W > 0 and N == min(n1, M) + n2


def test_rads_constant_volume(R):
    hu = np.full((4, 5, 6), 7.0, np.float32)
    vol, keep = _volume(hu, (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
    level, M, W = binding.ddgs_rads_prepare(R.ctx, vol)
    assert level == 7.0 and M == 0 and W == 0
    assert binding.ddgs_rads_sample(R.ctx, 10, None, 0, None, None, None) == 0
    with pytest.raises(binding.DDGSError):
        d = torch.zeros(4, dtype=torch.int64, device="cuda")
        p = torch.empty((3, 4), device="cuda")
        binding.ddgs_rads_sample(R.ctx, 0, None, 4, d.data_ptr(), p.data_ptr(), None)


def test_rads_full_phantom(R):
    """The 256^3 phantom of the fitting workload, n1 = 15000, n2 = 10000."""
    ph = synth.phantom(256, np.random.default_rng(1003))
    hu = np.ascontiguousarray(ph.transpose(2, 1, 0))
    M, W, N = _run(R, hu, (1.0, 1.0, 1.0), (-127.5, -127.5, -127.5), 15000, 10000, seed=7, full_knn=False)
    assert N == 25000 and M > 15000


def test_initial_model_renders(R):
    """The dual-sampling helper's starting model (sampled means, nearest-
    neighbour scales, identity rotations, opacity 0.1) renders a finite,
    non-empty image and matches the oracle on it."""
    from oracle import ref
    from paper_2406_02518_amd import rads
    ph = synth.phantom(48, np.random.default_rng(5))
    hu = torch.from_numpy(np.ascontiguousarray(ph.transpose(2, 1, 0))).cuda()
    pts, ls, n_iso, info = rads.sample(R, hu, (1.0, 1.0, 1.0), (-23.5, -23.5, -23.5), n1=800, n2=400, seed=3)
    assert pts.shape == (3, 1200) and n_iso == 1000 and info["crossings"] > 800
    k, L = 8, 1
    g = torch.Generator().manual_seed(1)
    b = torch.randn(k, generator=g).cuda()
    B = torch.randn((3, k), generator=g).cuda()
    p = rads.initial_model(pts, ls, k, L, b_iso=b, B_dir=B)
    R.set_model(p, n_iso, L)
    v = synth.view(48, 48, 1.2, 1000.0, 600.0, 30.0)
    R.set_views([v])
    img = R.render().cpu().numpy()
    assert np.isfinite(img).all() and img.max() > 0
    host = synth.Scene(**{name: p[name].cpu().numpy() for name in binding.PARAM_NAMES}, n_iso=n_iso, L=L)
    o = ref.render(host, [v])[0].ravel()
    assert np.linalg.norm(img - o) / np.linalg.norm(o) < 1e-4
