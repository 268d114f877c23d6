"""Radiodensity-aware dual sampling (Sec. 3.3) from a CT volume on the GPU:
interface points at the (min + max) / 2 level plus radiodensity-weighted voxel
centres, the paper's set sizes n1 = 15000 and n2 = 10000 (Sec. 4.1), and the
starting model built on them.  The random keys and draws come from a seeded
torch generator on the device and are handed to the library."""
import ctypes

import numpy as np

from . import binding


def sample(R, hu, spacing, origin, n1=15000, n2=10000, seed=0):
    """hu: float32 device tensor [nz][ny][nx] (HU).  Returns (points [3][N],
    log_scale [3][N], n_iso, info) on R's device."""
    import torch

    if hu.dtype != torch.float32 or not hu.is_contiguous() or hu.dim() != 3:
        raise ValueError("hu must be a contiguous float32 tensor [nz][ny][nx]")
    f3 = ctypes.c_float * 3
    vol = binding.ddgs_volume(hu.shape[2], hu.shape[1], hu.shape[0], f3(*spacing), f3(*origin), hu.data_ptr())
    with torch.cuda.stream(R.stream):
        level, M, W = binding.ddgs_rads_prepare(R.ctx, vol)
        gen = torch.Generator(device=R.device)
        gen.manual_seed(int(seed))
        keys = torch.randint(0, 1 << 32, (max(M, 1),), generator=gen, device=R.device, dtype=torch.int64)
        keys = (keys - (keys >= (1 << 31)).to(torch.int64) * (1 << 32)).to(torch.int32)  # same bits as u32
        draws = torch.randint(0, max(W, 1), (max(n2, 1),), generator=gen, device=R.device, dtype=torch.int64)
        N = min(n1, M) + n2
        pts = torch.empty((3, max(N, 1)), device=R.device)
        ls = torch.empty((3, max(N, 1)), device=R.device)
        n_iso = binding.ddgs_rads_sample(R.ctx, n1, keys.data_ptr(), n2, draws.data_ptr(), pts.data_ptr(),
                                         ls.data_ptr())
    return pts[:, :N], ls[:, :N], n_iso, {"level": level, "crossings": M, "total_weight": W}


def initial_model(points, log_scale, k, L, b_iso=None, B_dir=None, opacity=0.1):
    """Starting parameters on the sampled points, as 3D Gaussian splatting
    starts: identity rotations, the nearest-neighbour scales, opacity 0.1;
    features start at zero (Eq. 3 then gives c = 1/2) and the bases are the
    caller's (default zero)."""
    import torch

    dev = points.device
    N = points.shape[1]
    quat = torch.zeros((4, N), device=dev)
    quat[0] = 1.0
    kl = L * (L + 2)
    return {"mean": points.contiguous(), "quat": quat, "log_scale": log_scale.contiguous(),
            "opacity_logit": torch.full((N,), float(np.log(opacity) - np.log1p(-opacity)), device=dev),
            "feat": torch.zeros((k, N), device=dev),
            "b_iso": (b_iso if b_iso is not None else torch.zeros(k, device=dev)).contiguous(),
            "B_dir": (B_dir if B_dir is not None else torch.zeros((kl, k), device=dev)).contiguous()}
