"""Full-size parity in the launch configuration the benchmark times: the
uneven 1M-Gaussian batch of 16 mixed-size views and the 64-pose batch.  The
oracle evaluates sampled pixels one by one; the backward is checked with an
upstream gradient that is non-zero only on those pixels (so the oracle's
gradient over those pixels is the exact reference).  Sampled pixels exclude
those within rounding of a hit decision, where FP32 and FP64 may both be
right and differ by a whole contribution."""
import numpy as np
import pytest

from gpu_common import make_renderer, rel_l2, unique_pixels
from oracle import ref
from paper_2406_02518_amd import binding, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = make_renderer()
    yield r
    r.close()


def _sample(scene, views, per_view, seed):
    # draw twice the count per view, keep the pixels whose hit decisions are
    # unique (about half at full size), then at most per_view of them
    rng = np.random.default_rng(seed)
    cand = []
    for vi, v in enumerate(views):
        cand.append(np.stack([np.full(2 * per_view, vi), rng.integers(0, v.W, 2 * per_view),
                              rng.integers(0, v.H, 2 * per_view)], 1))
    keep = unique_pixels(scene, views, np.concatenate(cand).astype(np.int32))
    pix = np.concatenate([keep[keep[:, 0] == vi][:per_view] for vi in range(len(views))])
    assert len(pix) >= len(views) * per_view // 3
    base = np.cumsum([0] + [v.W * v.H for v in views])
    flat = base[pix[:, 0]] + pix[:, 2] * np.array([views[i].W for i in pix[:, 0]]) + pix[:, 1]
    return pix, flat


def _check_sampled(R, scene, views, per_view, seed, options=None):
    if options:
        R.set_options(**options)
    R.set_scene(scene)
    R.set_views(views)
    img = R.render()
    pix, flat = _sample(scene, views, per_view, seed)
    # forward at the sampled pixels
    got = img.cpu().numpy()[flat]
    exp = ref.render_pixels(scene, views, pix)
    assert rel_l2(got, exp) < 1e-4
    # backward of a loss that weights only the sampled pixels
    w = np.random.default_rng(seed + 1).normal(size=len(flat))
    dl = np.zeros(img.numel())
    np.add.at(dl, flat, w)
    g = R.backward(torch.from_numpy(dl.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    o = ref.backward(scene, views, pix, w)
    errs = {k: rel_l2(g[k].cpu().numpy(), o[k])
            for k in ("dmean", "dquat", "dlog_scale", "dopacity_logit", "dfeat", "db_iso", "dB_dir")}
    gp = g["dpose"].cpu().numpy()
    errs["dpose"] = max(rel_l2(gp[v], o["dpose"][v]) for v in range(len(views))
                        if np.linalg.norm(o["dpose"][v]) > 0)
    assert max(errs.values()) < 1e-4, errs


def test_uneven_batch_full_size(R):
    c = synth.config("C5")
    try:
        for opts in (dict(tile_w=16, tile_h=16, split=256), dict(tile_w=8, tile_h=8, split=1024, persistent=1)):
            _check_sampled(R, c.scene, c.views, 24, 5, opts)
    finally:
        R.set_options(tile_w=16, tile_h=16, split=256, persistent=0)


def test_pose_batch_full_size(R):
    c = synth.config("C4")
    _check_sampled(R, c.scene, c.views[:16], 20, 6)
