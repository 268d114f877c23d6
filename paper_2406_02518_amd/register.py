"""2D/3D pose registration on the GPU (Sec. 4.4): every view's pose is
refined by gradient descent on an image loss against its target, through the
renderer's pose-tangent gradient.

One captured step per iteration renders every view, scores it (global NCC by
default), back-propagates to each view's pose tangent (rho, omega) and takes
an Adam step that re-bases the device view table (R <- Exp(omega) R,
t <- Exp(omega) t + rho); the optimiser state never leaves the device.  The
loss is read back every ``check_every`` iterations to test convergence."""
import numpy as np

from . import binding


def register(R, targets, iters=200, lr_trans=1.0, lr_rot=0.01, beta1=0.9, beta2=0.999, eps=1e-8,
             loss=binding.LOSS_NCC, lam=0.0, check_every=10, rel_tol=1e-5):
    """Registers the views set on renderer R to ``targets`` (a float32 device
    tensor laid out like R's images).  Returns (poses, history): the final
    (3, 4) poses and a list of (iteration, per-view losses)."""
    import torch

    V = len(R.views)
    n = R.image_size()
    if targets.numel() != n:
        raise ValueError(f"targets hold {targets.numel()} floats, the views need {n}")
    images = torch.empty(n, device=R.device)
    dl = torch.empty_like(images)
    loss_out = torch.empty(V, device=R.device)
    grads = R.alloc_grads(("dpose",))
    R.set_pose_optimizer(lr_trans, lr_rot, beta1, beta2, eps)
    try:
        with torch.cuda.stream(R.stream):
            binding.ddgs_step_capture(R.ctx, loss, targets.data_ptr(), lam, images.data_ptr(), dl.data_ptr(),
                                      loss_out.data_ptr(), R.grads_struct(grads))
        history = []
        prev = None
        for it in range(1, iters + 1):
            binding.ddgs_step_launch(R.ctx)
            if it % check_every == 0 or it == iters:
                binding.ddgs_check(R.ctx)
                cur = loss_out.cpu().numpy().astype(np.float64)
                history.append((it, cur))
                if prev is not None and np.all(np.abs(prev - cur) <= rel_tol * np.maximum(np.abs(prev), 1e-12)):
                    break
                prev = cur
        return R.get_poses(), history
    finally:
        R.set_pose_optimizer(None)
