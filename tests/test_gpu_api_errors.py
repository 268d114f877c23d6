"""Error handling of the registration, fitting and dual-sampling entry points:
invalid arguments and calls out of order return their status (as
binding.DDGSError) and leave the context usable."""
import ctypes

import numpy as np
import pytest

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


def _status(fn, *args):
    with pytest.raises(binding.DDGSError) as e:
        fn(*args)
    return e.value.status


def test_optimiser_arguments(R):
    sc = synth.random_scene(1, 50, k=4, L=1)
    R.set_scene(sc)
    R.set_views([synth.view(24, 24, 2.0, 1000.0, 600.0, 0.0)])
    bad = binding.ddgs_default_fit_options(10.0)
    bad.beta1 = 1.0
    assert _status(binding.ddgs_set_fit_optimizer, R.ctx, bad) == binding.ERR_INVALID_ARG
    bad = binding.ddgs_default_fit_options(10.0)
    bad.lr_mean_steps = 0
    assert _status(binding.ddgs_set_fit_optimizer, R.ctx, bad) == binding.ERR_INVALID_ARG
    a = binding.ddgs_adam(1.0, 0.01, 0.9, 0.999, 1e-8, 7)
    assert _status(binding.ddgs_set_pose_optimizer, R.ctx, a) == binding.ERR_INVALID_ARG
    # the fitting optimiser needs every parameter gradient in the captured step
    R.set_fit_optimizer(10.0)
    n = R.image_size()
    img, dl, loss = torch.empty(n, device="cuda"), torch.empty(n, device="cuda"), torch.empty(1, device="cuda")
    g = R.alloc_grads(("dmean", "dpose"))
    assert _status(binding.ddgs_step_capture, R.ctx, binding.LOSS_L1_DSSIM, img.data_ptr(), 0.2, img.data_ptr(),
                   dl.data_ptr(), loss.data_ptr(), R.grads_struct(g)) == binding.ERR_INVALID_ARG
    R.set_fit_optimizer(None)
    # still usable
    assert np.isfinite(R.render().cpu().numpy()).all()


def test_densify_and_sampling_out_of_order(R):
    sc = synth.random_scene(2, 40, k=4, L=1)
    p = R.set_scene(sc)
    noise = torch.zeros((40, 2, 3), device="cuda")
    o = binding.ddgs_densify_opts(2e-4, 1.0, 0.005, 0.0, 0.0, 1.6)
    # no statistics set
    assert _status(binding.ddgs_densify_plan, R.ctx, o, noise.data_ptr()) == binding.ERR_STATE
    R.set_densify_stats(R.new_densify_stats())
    # apply before plan
    out = binding.ddgs_params(*[p[k].data_ptr() for k in binding.PARAM_NAMES])
    assert _status(binding.ddgs_densify_apply, R.ctx, out) == binding.ERR_STATE
    bad = binding.ddgs_densify_opts(2e-4, 1.0, 0.005, 0.0, 0.0, 0.9)  # split factor must exceed 1
    assert _status(binding.ddgs_densify_plan, R.ctx, bad, noise.data_ptr()) == binding.ERR_INVALID_ARG
    # a plan is dropped by a new model
    binding.ddgs_densify_plan(R.ctx, o, noise.data_ptr())
    R.set_scene(sc)
    assert _status(binding.ddgs_densify_apply, R.ctx, out) == binding.ERR_STATE
    # dual sampling before prepare, and a degenerate volume
    assert _status(binding.ddgs_rads_sample, R.ctx, 0, None, 0, None, None, None) == binding.ERR_STATE
    hu = torch.zeros((2, 3, 4), device="cuda")
    f3 = ctypes.c_float * 3
    vol = binding.ddgs_volume(4, 3, 2, f3(1.0, 1.0, 0.0), f3(0.0, 0.0, 0.0), hu.data_ptr())
    assert _status(binding.ddgs_rads_prepare, R.ctx, vol) == binding.ERR_INVALID_ARG
    R.set_densify_stats(None)
