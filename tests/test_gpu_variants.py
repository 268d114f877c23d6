"""Model variants of the ablations (Sec. 4, ablation and feature-size
studies) against the FP64 oracle: the disentangled model with both sets, an
isotropic set alone (n_iso = n), a directional set alone (n_iso = 0) and the
co-located "direct-entangled" form (both terms under one sigmoid on every
Gaussian), each at every degree L = 1..3 and feature size
k in {1, 4, 8, 16, 32}.  Forward images and every gradient group, the pose
included, to the same tolerance as the main parity tests."""
from dataclasses import replace

import numpy as np
import pytest

from gpu_common import make_renderer, rel_l2
from oracle import ref
from paper_2406_02518_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-4
GROUPS = ("dmean", "dquat", "dlog_scale", "dopacity_logit", "dfeat", "db_iso", "dB_dir")
VARIANTS = ("disentangled", "iso_only", "dir_only", "entangled")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = make_renderer()
    yield r
    r.close()


def _scene(variant, L, k, seed):
    sc = synth.random_scene(seed, 400, k=k, L=L, iso_fraction=0.5, extent=20.0, std_range=(0.8, 2.5),
                            alpha_range=(0.03, 0.4))
    if variant == "iso_only":
        return replace(sc, n_iso=sc.n)
    if variant == "dir_only":
        return replace(sc, n_iso=0)
    if variant == "entangled":
        return replace(sc, n_iso=0, entangled=True)
    return sc


@pytest.mark.parametrize("k", [1, 4, 8, 16, 32])
@pytest.mark.parametrize("L", [1, 2, 3])
@pytest.mark.parametrize("variant", VARIANTS)
def test_variant_matches_oracle(R, variant, L, k):
    seed = 700 + 10 * L + k + 100 * VARIANTS.index(variant)
    sc = _scene(variant, L, k, seed)
    views = [synth.view(48, 40, 1.8, 1000.0, 600.0, 30.0 * (seed % 12)),
             synth.view(37, 45, 1.7, 1000.0, 560.0, 30.0 * (seed % 12) + 95.0)]
    R.set_scene(sc)
    R.set_views(views)
    img = R.render().cpu().numpy().astype(np.float64)
    o_img = np.concatenate([x.ravel() for x in ref.render(sc, views)])
    assert rel_l2(img, o_img) < TOL, (variant, L, k, "image", rel_l2(img, o_img))
    dl = np.random.default_rng(seed).normal(size=img.size)
    g = R.backward(torch.from_numpy(dl.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    o = ref.backward(sc, views, ref.all_pixels(views), dl)
    for name in GROUPS:
        got = g[name].cpu().numpy().astype(np.float64)
        if variant == "iso_only" and name == "dB_dir" or variant == "dir_only" and name == "db_iso":
            # the basis of the absent set gets exactly zero
            assert np.all(got == 0.0) and np.all(o[name] == 0.0), (variant, name)
            continue
        err = rel_l2(got, o[name])
        assert err < TOL, (variant, L, k, name, err)
        assert np.linalg.norm(o[name]) > 0, (variant, L, k, name)
    gp = g["dpose"].cpu().numpy().astype(np.float64).reshape(-1, 6)
    for v in range(len(views)):
        err = rel_l2(gp[v], o["dpose"][v])
        assert err < TOL, (variant, L, k, "dpose", v, err)


def test_entangled_model_rejects_isotropic_set(R):
    from paper_2406_02518_amd import binding
    sc = replace(_scene("entangled", 2, 8, 1), n_iso=5)
    with pytest.raises(binding.DDGSError):
        R.set_scene(sc)
