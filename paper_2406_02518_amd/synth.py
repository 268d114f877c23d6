"""Seeded synthetic inputs for the DRR splatting path.

This module only draws inputs: Gaussian sets, detector views and poses.  It
holds none of the renderer's arithmetic (no projection, compositing, radiosity
or gradient), so both the GPU path and the FP64 oracle can consume its output.

The paper's data (CT scans of NAF-CT, CTPelvic1K and Ljubljana, Sec. 4.1) is
not available; a seeded nested-ellipsoid HU phantom stands in for it.
Gaussians are placed at phantom voxels above -500 HU with a per-axis std of
about one voxel, 20 % of them direction-dependent (the paper's initial split
of 15000 + 5000 isotropic to 5000 directional points, Sec. 3.3 and App. A.2).
"""
from dataclasses import dataclass, field, replace
from typing import List

import numpy as np
from scipy.spatial.transform import Rotation

K_DEFAULT = 16   # 16 feature coefficients per Gaussian
L_DEFAULT = 3    # degree-3 directional basis: k_L = 15


@dataclass
class Scene:
    """Structure-of-arrays Gaussian set (float32).  [0, n_iso) isotropic."""
    mean: np.ndarray           # (3, n) mm
    quat: np.ndarray           # (4, n) (w, x, y, z), unnormalised
    log_scale: np.ndarray      # (3, n) log std, mm
    opacity_logit: np.ndarray  # (n,)
    feat: np.ndarray           # (k, n)
    b_iso: np.ndarray          # (k,)
    B_dir: np.ndarray          # (k_L, k)
    n_iso: int
    L: int
    entangled: bool = False    # co-located ablation: both radiosity terms on every Gaussian (n_iso = 0)

    @property
    def n(self):
        return int(self.mean.shape[1])

    @property
    def k(self):
        return int(self.feat.shape[0])

    def arrays(self):
        return dict(mean=self.mean, quat=self.quat, log_scale=self.log_scale,
                    opacity_logit=self.opacity_logit, feat=self.feat, b_iso=self.b_iso,
                    B_dir=self.B_dir)

    def copy(self):
        return replace(self, **{k: np.array(v, copy=True) for k, v in self.arrays().items()})

    def subset(self, idx_iso, idx_dir):
        """Keeps the listed isotropic and directional Gaussians, iso first."""
        idx = np.concatenate([np.asarray(idx_iso, dtype=np.int64), np.asarray(idx_dir, dtype=np.int64)])
        a = self.arrays()
        out = {k: np.ascontiguousarray(v[..., idx]) for k, v in a.items() if k not in ("b_iso", "B_dir")}
        return Scene(b_iso=self.b_iso.copy(), B_dir=self.B_dir.copy(), n_iso=len(idx_iso), L=self.L, **out)


@dataclass
class View:
    """Cone-beam view: detector W x H pixels of ``pitch`` mm at ``sdd`` mm from
    the source; ``pose`` (3, 4) float32 world -> source frame [R | t]."""
    W: int
    H: int
    pitch: float
    sdd: float
    pose: np.ndarray
    sid: float = 0.0
    azimuth_deg: float = 0.0


@dataclass
class Config:
    name: str
    scene: Scene
    views: List[View]
    extra: dict = field(default_factory=dict)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def azimuth_pose(theta_deg, sid):
    """Source on a circle of radius ``sid`` about the world z axis, looking at
    the isocentre (world origin); detector rows run along world +z."""
    th = np.deg2rad(theta_deg)
    c, s = np.cos(th), np.sin(th)
    R = np.array([[s, -c, 0.0], [0.0, 0.0, 1.0], [-c, -s, 0.0]])
    src = sid * np.array([c, s, 0.0])
    t = -R @ src
    return np.concatenate([R, t[:, None]], axis=1)


def view(W, H, pitch, sdd, sid, azimuth_deg, pose=None):
    P = azimuth_pose(azimuth_deg, sid) if pose is None else pose
    return View(W=int(W), H=int(H), pitch=float(np.float32(pitch)), sdd=float(np.float32(sdd)),
                pose=_f32(P), sid=float(sid), azimuth_deg=float(azimuth_deg))


def perturbed_pose(pose0, rotvec, tau):
    """[R0 Exp(w) | R0 tau + t0]: the volume rotated about the isocentre by
    the rotation vector w and shifted by tau (world frame)."""
    P = np.asarray(pose0, dtype=np.float64)
    R0, t0 = P[:, :3], P[:, 3]
    Rw = Rotation.from_rotvec(np.asarray(rotvec, dtype=np.float64)).as_matrix()
    return np.concatenate([R0 @ Rw, (R0 @ np.asarray(tau, dtype=np.float64) + t0)[:, None]], axis=1)


def random_unit_quaternions(rng, n):
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _logit(p):
    p = np.asarray(p, dtype=np.float64)
    return np.log(p) - np.log1p(-p)


def encode_iso_features(rng, target_c, b, noise_std=0.05):
    """Features whose isotropic radiosity equals ``target_c``: the component
    along b carries logit(c), the orthogonal part is noise."""
    k = b.shape[0]
    bb = float(b @ b)
    zeta = rng.normal(0.0, noise_std, size=(k, target_c.shape[0]))
    zeta -= np.outer(b, b @ zeta) / bb
    return np.outer(b, _logit(target_c)) / bb + zeta


def random_scene(seed, n, k=K_DEFAULT, L=L_DEFAULT, iso_fraction=0.8, extent=32.0,
                 std_range=(0.5, 2.0), alpha_range=(0.02, 0.2), center=(0.0, 0.0, 0.0)):
    """Means uniform in a cube of half-size ``extent`` mm, per-axis std uniform
    in ``std_range``, random rotations; the first ``iso_fraction`` isotropic
    with target radiosity ~U(0,1); directional features ~N(0, 0.05^2)."""
    ss = np.random.SeedSequence(seed)
    r_geo, r_feat, r_basis = (np.random.default_rng(s) for s in ss.spawn(3))
    kl = L * (L + 2)
    n_iso = int(round(iso_fraction * n))
    mean = r_geo.uniform(-extent, extent, size=(3, n)) + np.asarray(center, dtype=np.float64)[:, None]
    log_scale = np.log(r_geo.uniform(std_range[0], std_range[1], size=(3, n)))
    quat = random_unit_quaternions(r_geo, n)
    alpha = r_geo.uniform(alpha_range[0], alpha_range[1], size=n)
    b = r_basis.normal(size=k)
    B = r_basis.normal(size=(kl, k))
    feat = np.zeros((k, n))
    c_target = np.clip(r_feat.uniform(0.0, 1.0, size=n_iso), 1e-3, 1 - 1e-3)
    feat[:, :n_iso] = encode_iso_features(r_feat, c_target, b)
    feat[:, n_iso:] = r_feat.normal(0.0, 0.05, size=(k, n - n_iso))
    return Scene(mean=_f32(mean), quat=_f32(quat), log_scale=_f32(log_scale),
                 opacity_logit=_f32(_logit(alpha)), feat=_f32(feat), b_iso=_f32(b), B_dir=_f32(B),
                 n_iso=n_iso, L=L)


def with_features(scene, seed, k, L, variant="disentangled"):
    """The geometry of ``scene`` with new seeded features and bases of size k
    and degree L, for the model variants of the ablations: "disentangled"
    keeps the isotropic / directional split, "iso_only" and "dir_only" make
    every Gaussian one kind, "entangled" gives every Gaussian both terms.
    Features ~N(0, 0.5^2), b_iso ~N(0, 1), B_dir ~N(0, 0.3^2)."""
    rng = np.random.default_rng(seed)
    n, kl = scene.n, L * (L + 2)
    n_iso = {"disentangled": scene.n_iso, "iso_only": n, "dir_only": 0, "entangled": 0}[variant]
    return replace(scene, feat=_f32(rng.normal(0.0, 0.5, size=(k, n))), b_iso=_f32(rng.normal(size=k)),
                   B_dir=_f32(rng.normal(0.0, 0.3, size=(kl, k))), n_iso=n_iso, L=L,
                   entangled=variant == "entangled")


def phantom(n, rng):
    """n^3 HU volume at 1 mm: air -1000, a soft-tissue body ellipsoid (0..80),
    three organ ellipsoids, two air-filled lungs, a spine cylinder with cortex
    (1000..1500) and marrow (300..600), and a pelvis-like shell (300..1500)."""
    ax = (np.arange(n) + 0.5) / n * 2.0 - 1.0
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    hu = np.full((n, n, n), -1000.0, dtype=np.float32)
    body = (X / 0.85) ** 2 + (Y / 0.65) ** 2 + (Z / 0.90) ** 2 <= 1.0
    hu[body] = rng.uniform(0.0, 80.0, size=int(body.sum()))
    for _ in range(3):
        c = rng.uniform(-0.35, 0.35, size=3) * np.array([1.0, 0.8, 1.0])
        r = rng.uniform(0.12, 0.25, size=3)
        organ = ((X - c[0]) / r[0]) ** 2 + ((Y - c[1]) / r[1]) ** 2 + ((Z - c[2]) / r[2]) ** 2 <= 1.0
        organ &= body
        hu[organ] = rng.uniform(0.0, 80.0) + rng.uniform(-5.0, 5.0, size=int(organ.sum()))
    for sx in (-1.0, 1.0):
        lung = ((X - 0.4 * sx) / 0.28) ** 2 + ((Y - 0.1) / 0.35) ** 2 + ((Z - 0.45) / 0.35) ** 2 <= 1.0
        hu[lung & body] = -1000.0
    rr = np.sqrt(X ** 2 + (Y + 0.35) ** 2)
    spine = (rr <= 0.10) & (np.abs(Z) <= 0.85)
    cortex = spine & (rr > 0.07)
    marrow = spine & (rr <= 0.07)
    hu[cortex] = rng.uniform(1000.0, 1500.0, size=int(cortex.sum()))
    hu[marrow] = rng.uniform(300.0, 600.0, size=int(marrow.sum()))
    outer = (X / 0.66) ** 2 + (Y / 0.50) ** 2 + (Z / 0.36) ** 2 <= 1.0
    inner = (X / 0.60) ** 2 + (Y / 0.45) ** 2 + (Z / 0.30) ** 2 <= 1.0
    pelvis = outer & ~inner & (np.abs(Z) < 0.25)
    hu[pelvis] = rng.uniform(300.0, 1500.0, size=int(pelvis.sum()))
    return hu


def scene_from_phantom(seed, nvox, n, opacity_scale, k=K_DEFAULT, L=L_DEFAULT, dir_fraction=0.2):
    """Gaussians at n distinct phantom voxels above -500 HU (centre plus
    U(-0.5, 0.5) mm jitter), std 1 mm x U(0.8, 1.25) per axis, random
    rotation.  Normalised density d = (HU + 1000) / 2500; isotropic target
    radiosity clip(d + N(0, 0.02^2), 0.01, 0.99); opacity
    clip(opacity_scale d, 1e-3, 0.99); directional features ~N(0, 0.05^2)."""
    ss = np.random.SeedSequence(seed)
    r_ph, r_samp, r_par, r_basis = (np.random.default_rng(s) for s in ss.spawn(4))
    hu = phantom(nvox, r_ph)
    cand = np.flatnonzero(hu.ravel() > -500.0)
    if cand.size < n:
        raise ValueError(f"phantom {nvox}^3 has only {cand.size} voxels above -500 HU (< {n})")
    pick = np.sort(r_samp.choice(cand, size=n, replace=False))
    ijk = np.stack(np.unravel_index(pick, hu.shape)).astype(np.float64)
    mean = ijk + 0.5 - nvox / 2.0 + r_samp.uniform(-0.5, 0.5, size=(3, n))
    dens = (hu.ravel()[pick].astype(np.float64) + 1000.0) / 2500.0
    order = r_samp.permutation(n)
    n_dir = int(round(dir_fraction * n))
    n_iso = n - n_dir
    mean, dens = mean[:, order], dens[order]
    kl = L * (L + 2)
    log_scale = np.log(r_par.uniform(0.8, 1.25, size=(3, n)))
    quat = random_unit_quaternions(r_par, n)
    alpha = np.clip(opacity_scale * dens, 1e-3, 0.99)
    b = r_basis.normal(size=k)
    B = r_basis.normal(size=(kl, k))
    feat = np.zeros((k, n))
    c_iso = np.clip(dens[:n_iso] + r_par.normal(0.0, 0.02, size=n_iso), 0.01, 0.99)
    feat[:, :n_iso] = encode_iso_features(r_par, c_iso, b)
    feat[:, n_iso:] = r_par.normal(0.0, 0.05, size=(k, n_dir))
    return Scene(mean=_f32(mean), quat=_f32(quat), log_scale=_f32(log_scale),
                 opacity_logit=_f32(_logit(alpha)), feat=_f32(feat), b_iso=_f32(b), B_dir=_f32(B),
                 n_iso=n_iso, L=L)


def perturb_scene(seed, scene, mean_std=0.5, log_scale_std=0.1, opacity_std=0.2, feat_std=0.05):
    """The model being fitted: the true model plus Gaussian noise."""
    rng = np.random.default_rng(seed)
    s = scene.copy()
    s.mean = _f32(s.mean + rng.normal(0.0, mean_std, size=s.mean.shape))
    s.log_scale = _f32(s.log_scale + rng.normal(0.0, log_scale_std, size=s.log_scale.shape))
    s.opacity_logit = _f32(s.opacity_logit + rng.normal(0.0, opacity_std, size=s.opacity_logit.shape))
    s.feat = _f32(s.feat + rng.normal(0.0, feat_std, size=s.feat.shape))
    return s


# Per-config opacity scale, chosen so that a typical body pixel ends with a
# transmittance of roughly 0.25: sum of s over a pixel ~ -ln 0.25 = 1.39 with
# about (pairs per pixel) x 0.22 x scale x 0.45 (mean of exp(-d2/2) over the
# 3-sigma disc is ~0.22, mean normalised density ~0.45).
OPACITY_SCALE = {"C2": 0.2, "C3": 0.055, "C4": 0.07, "C5": 0.03}

CONFIG_NAMES = ("C1", "C2", "C3", "C4", "C5")


def config(name, scale=1.0, det_scale=None):
    """Configurations of the measured workloads.  ``scale`` < 1 shrinks the
    Gaussian count and the phantom for quick tests; the detector shrinks by
    ``det_scale`` (default sqrt(scale)) with the pitch enlarged so that the
    field of view is kept."""
    if det_scale is None:
        det_scale = scale ** 0.5
    seed = 1000 + CONFIG_NAMES.index(name) + 1
    ss = np.random.SeedSequence(seed)
    r_pose = np.random.default_rng(ss.spawn(1)[0])

    def det(px):
        return max(8, int(round(px * det_scale)))

    if name == "C1":
        n = max(16, int(round(2000 * scale)))
        sc = random_scene(seed, n)
        W = det(64)
        return Config(name, sc, [view(W, W, 64.0 / W, 1000.0, 600.0, 0.0)])
    if name == "C2":
        nvox = max(16, int(round(128 * scale ** (1 / 3))))
        sc = scene_from_phantom(seed, nvox, max(16, int(round(100_000 * scale))), OPACITY_SCALE["C2"])
        W = det(256)
        return Config(name, sc, [view(W, W, 1.5 * 256 / W, 1000.0, 600.0, 0.0)])
    if name == "C3":
        nvox = max(16, int(round(256 * scale ** (1 / 3))))
        true = scene_from_phantom(seed, nvox, max(16, int(round(500_000 * scale))), OPACITY_SCALE["C3"])
        fit = perturb_scene(seed + 7, true)
        W = det(512)
        views = [view(W, W, 0.8 * 512 / W, 1000.0, 600.0, 10.0 * j) for j in range(36)]
        return Config(name, fit, views, dict(true_scene=true, lam=0.2))
    if name == "C4":
        nvox = max(16, int(round(192 * scale ** (1 / 3))))
        sc = scene_from_phantom(seed, nvox, max(16, int(round(300_000 * scale))), OPACITY_SCALE["C4"])
        W = det(256)
        az = float(r_pose.uniform(0.0, 360.0))
        gt = view(W, W, 1.5 * 256 / W, 1000.0, 600.0, az)
        views = []
        for _ in range(64):
            w = np.deg2rad(r_pose.uniform(-10.0, 10.0, size=3))
            tau = r_pose.uniform(-20.0, 20.0, size=3)
            views.append(view(W, W, gt.pitch, 1000.0, 600.0, az, pose=perturbed_pose(gt.pose, w, tau)))
        return Config(name, sc, views, dict(gt_view=gt))
    if name == "C5":
        nvox = max(16, int(round(256 * scale ** (1 / 3))))
        sc = scene_from_phantom(seed, nvox, max(16, int(round(1_000_000 * scale))), OPACITY_SCALE["C5"])
        sizes = np.array([256] * 6 + [512] * 6 + [1024] * 4)
        r_pose.shuffle(sizes)
        views = []
        for s in sizes:
            pitch = float(r_pose.uniform(0.4, 1.5))
            sid = float(r_pose.uniform(500.0, 700.0))
            az = float(r_pose.uniform(0.0, 360.0))
            W = det(int(s))
            views.append(view(W, W, pitch * s / W, 1000.0, sid, az))
        rng_w = np.random.default_rng(seed + 11)
        return Config(name, sc, views, dict(dl_seed=int(rng_w.integers(1 << 31))))
    raise KeyError(name)
