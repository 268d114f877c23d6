"""FP64 reference of one pose-optimiser step (test infrastructure, like the
rest of oracle/): an Adam step on a view's pose-tangent gradient (rho, omega)
followed by the re-basing the registration uses (Sec. 4.3): R <- Exp(omega) R,
t <- Exp(omega) t + rho, the left tangent at 0 that the backward
differentiates.  Only tests import this module."""
import numpy as np


def exp_so3(w):
    """Rotation matrix of the rotation vector w (Rodrigues' formula)."""
    w = np.asarray(w, dtype=np.float64)
    th = float(np.linalg.norm(w))
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + (np.sin(th) / th) * K + ((1.0 - np.cos(th)) / th ** 2) * (K @ K)


def adam_step(g, m, s, t, lr, beta1, beta2, eps):
    """Adam (Kingma & Ba) with bias correction, step t = 1, 2, ...: returns the
    update and the new first and second moments."""
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * m + (1.0 - beta1) * g
    s = beta2 * s + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    shat = s / (1.0 - beta2 ** t)
    return -np.asarray(lr, dtype=np.float64) * mhat / (np.sqrt(shat) + eps), m, s


def rebase(pose, delta):
    """[Exp(w) R | Exp(w) t + rho] for delta = (rho, w)."""
    P = np.asarray(pose, dtype=np.float64)
    E = exp_so3(delta[3:])
    return np.concatenate([E @ P[:, :3], (E @ P[:, 3] + np.asarray(delta[:3]))[:, None]], axis=1)


def rebase_about(pose, delta, pivot):
    """Rotation by Exp(w) about the world point ``pivot`` and a shift rho in
    the source frame: with p = R pivot + t, [Exp(w) R | Exp(w)(t - p) + p + rho]."""
    P = np.asarray(pose, dtype=np.float64)
    E = exp_so3(delta[3:])
    p = P[:, :3] @ np.asarray(pivot, np.float64) + P[:, 3]
    return np.concatenate([E @ P[:, :3], (E @ (P[:, 3] - p) + p + np.asarray(delta[:3]))[:, None]], axis=1)


def pivot_gradient(g, pose, pivot):
    """Gradient for the tangent of ``rebase_about`` from the left-tangent
    gradient g = (g_rho, g_omega): a camera point x moves by
    omega x (x - p) + rho, the left tangent (rho - omega x p, omega), so the
    chain rule gives (g_rho, g_omega + g_rho x p)."""
    g = np.asarray(g, np.float64)
    P = np.asarray(pose, np.float64)
    p = P[:, :3] @ np.asarray(pivot, np.float64) + P[:, 3]
    return np.concatenate([g[:3], g[3:] + np.cross(g[:3], p)])


def pose_errors(pose, pose_gt):
    """Rotation error (degrees, angle of R R_gt^T) and source-position error (mm)."""
    P, G = np.asarray(pose, np.float64), np.asarray(pose_gt, np.float64)
    Rd = P[:, :3] @ G[:, :3].T
    ang = np.degrees(np.arccos(np.clip((np.trace(Rd) - 1.0) / 2.0, -1.0, 1.0)))
    so, sg = -P[:, :3].T @ P[:, 3], -G[:, :3].T @ G[:, 3]
    return float(ang), float(np.linalg.norm(so - sg))


def projection_distance(pose, pose_gt, f, points):
    """Mean distance in detector pixels between the projections of world points
    under two poses (camera frame x = R X + t, pixel u = f x0/x2, v = f x1/x2
    with f = SDD / pitch; the principal point cancels in the difference)."""
    X = np.asarray(points, np.float64).reshape(-1, 3)
    P, G = np.asarray(pose, np.float64), np.asarray(pose_gt, np.float64)
    a = X @ P[:, :3].T + P[:, 3]
    b = X @ G[:, :3].T + G[:, 3]
    ua = f * a[:, :2] / a[:, 2:3]
    ub = f * b[:, :2] / b[:, 2:3]
    return float(np.mean(np.linalg.norm(ua - ub, axis=1)))
