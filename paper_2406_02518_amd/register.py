"""2D/3D pose registration on the GPU (Sec. 4.3): every view's pose is
refined by gradient descent on an image loss against its target, through the
renderer's pose-tangent gradient.

One captured step per iteration renders every view, scores it (global NCC by
default), back-propagates to each view's pose tangent (rho, omega) and takes
an Adam step that re-bases the device view table; the optimiser state never
leaves the device.  By default the rotation turns about the isocentre (the
world origin): R <- Exp(omega) R, t <- t + rho.  Turning about the source
instead (``pivot=None``) moves the image almost as a sideways shift does, so
rotation and translation become nearly interchangeable and descent stalls in
the resulting valley.  The loss is read back every ``check_every``
iterations to test convergence.  A replay whose tile entries exceed the
captured capacity changes no pose; at the next check the capacity is raised,
the step captured again and the skipped iterations replayed."""
import numpy as np

from . import binding


def register(R, targets, iters=200, lr_trans=1.0, lr_rot=0.008, beta1=0.9, beta2=0.999, eps=1e-8,
             loss=binding.LOSS_NCC, lam=0.0, check_every=10, rel_tol=1e-5, abs_tol=1e-8, pivot=(0.0, 0.0, 0.0)):
    """Registers the views set on renderer R to ``targets`` (a float32 device
    tensor laid out like R's images).  Learning rates are per Adam step, in mm
    (translation) and rad (rotation).  Stops after ``iters`` iterations or
    when, between two checks, no view's loss changed by more than
    max(rel_tol * |loss|, abs_tol).  Returns (poses, history): the final
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
    R.set_pose_optimizer(lr_trans, lr_rot, beta1, beta2, eps, pivot=pivot)

    def capture():
        with torch.cuda.stream(R.stream):
            binding.ddgs_step_capture(R.ctx, loss, targets.data_ptr(), lam, images.data_ptr(), dl.data_ptr(),
                                      loss_out.data_ptr(), R.grads_struct(grads))

    try:
        capture()
        history = []
        prev = None
        for it in range(1, iters + 1):
            binding.ddgs_step_launch(R.ctx)
            if it % check_every == 0 or it == iters:
                # replays skipped by an overflow are the last ones: run them again
                skipped = R.check_step()
                while skipped:
                    capture()
                    for _ in range(skipped):
                        binding.ddgs_step_launch(R.ctx)
                    skipped = R.check_step()
                cur = loss_out.cpu().numpy().astype(np.float64)
                history.append((it, cur))
                if prev is not None and np.all(np.abs(prev - cur) <= np.maximum(rel_tol * np.abs(prev), abs_tol)):
                    break
                prev = cur
        return R.get_poses(), history
    finally:
        R.set_pose_optimizer(None)


def rotation_error_deg(pose, pose_ref):
    """Angle (degrees) of the relative rotation R R_ref^T."""
    Rr = np.asarray(pose, np.float64)[:, :3] @ np.asarray(pose_ref, np.float64)[:, :3].T
    return float(np.degrees(np.arccos(np.clip(0.5 * (np.trace(Rr) - 1.0), -1.0, 1.0))))


def source_error_mm(pose, pose_ref):
    """Distance (mm) between the source positions -R^T t of two poses."""
    a, b = np.asarray(pose, np.float64), np.asarray(pose_ref, np.float64)
    return float(np.linalg.norm(a[:, :3].T @ a[:, 3] - b[:, :3].T @ b[:, 3]))


def target_registration_error(pose, pose_ref, points):
    """Mean 3D distance (mm) between world points placed by the two poses
    (measured in the source frame, where both poses put them)."""
    X = np.asarray(points, np.float64).reshape(-1, 3)
    a, b = np.asarray(pose, np.float64), np.asarray(pose_ref, np.float64)
    return float(np.mean(np.linalg.norm(X @ (a[:, :3] - b[:, :3]).T + (a[:, 3] - b[:, 3]), axis=1)))


def projection_distance(pose, pose_ref, f_px, points):
    """Mean detector distance (px) between the projections of world points
    under two poses, pixel = f_px (x, y) / z in the source frame."""
    X = np.asarray(points, np.float64).reshape(-1, 3)
    out = []
    for P in (np.asarray(pose, np.float64), np.asarray(pose_ref, np.float64)):
        x = X @ P[:, :3].T + P[:, 3]
        out.append(f_px * x[:, :2] / x[:, 2:3])
    return float(np.mean(np.linalg.norm(out[0] - out[1], axis=1)))
