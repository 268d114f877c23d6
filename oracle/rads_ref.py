"""FP64 reference of radiodensity-aware dual sampling (Sec. 3.3; Sec. 4.1 for
the iso-level and the set sizes).  Test infrastructure, like the rest of
oracle/; only tests and the benchmark's CPU leg import it.

* P^mc: marching-cubes points at the interface level (min + max) / 2 of the
  volume.  The vertices marching cubes places are the points where the level
  crosses a voxel edge, linearly interpolated between the two voxel centres
  (the case table only connects them into triangles), so the candidate set is
  every crossing of every edge between neighbouring voxel centres, in edge
  order ((z * ny + y) * nx + x) * 3 + axis (x, y, z axes 0, 1, 2).  An edge
  crosses when exactly one end is below the level.  n1 of them are kept:
  those with the smallest caller-supplied random keys (ties by edge order),
  in key order.
* P^dw: n2 voxel centres drawn independently with probability proportional
  to the voxel's radiodensity, normalised to [0, 1] over the volume and
  quantised to 16 bits: w = floor((hu - min) / (max - min) * 65535) in
  float32; draw j picks the first voxel whose inclusive weight sum exceeds
  the caller-supplied integer r_j in [0, sum w).
* All of P^mc and the first half of P^dw initialise isotropic Gaussians, the
  second half of P^dw directional ones (Sec. 3.3).
* Scales as in 3D Gaussian splatting's initialisation: every axis gets
  log sqrt(mean squared distance to the 3 nearest other points), the mean
  clamped below at 1e-7 mm^2.

Integer decisions (edge crossings, weights) are taken in float32 as the
kernels take them; positions are computed in FP64.
"""
import numpy as np


def iso_level(hu):
    hu = np.asarray(hu, np.float32)
    return np.float32((np.float32(hu.min()) + np.float32(hu.max())) * np.float32(0.5))


def crossings(hu, iso, spacing, origin):
    """Interface points (M, 3) in edge order; hu is [nz][ny][nx] float32."""
    hu = np.asarray(hu, np.float32)
    nz, ny, nx = hu.shape
    iso = np.float32(iso)
    ids, pts = [], []
    for axis, sl_a, sl_b in ((0, np.s_[:, :, :-1], np.s_[:, :, 1:]), (1, np.s_[:, :-1, :], np.s_[:, 1:, :]),
                             (2, np.s_[:-1, :, :], np.s_[1:, :, :])):
        a, b = hu[sl_a], hu[sl_b]
        cross = (a < iso) != (b < iso)
        z, y, x = np.nonzero(cross)
        av, bv = a[cross].astype(np.float64), b[cross].astype(np.float64)
        t = (float(iso) - av) / (bv - av)
        g = np.stack([x, y, z], axis=1).astype(np.float64)
        g[:, axis] += t
        pts.append(np.asarray(origin, np.float64) + g * np.asarray(spacing, np.float64))
        ids.append(((z.astype(np.int64) * ny + y) * nx + x) * 3 + axis)
    ids = np.concatenate(ids)
    order = np.argsort(ids, kind="stable")
    return np.concatenate(pts)[order], ids[order]


def weights(hu):
    hu = np.asarray(hu, np.float32)
    mn, mx = np.float32(hu.min()), np.float32(hu.max())
    if not mx > mn:
        return np.zeros(hu.size, np.uint32)
    return np.floor(((hu.ravel() - mn) / (mx - mn)) * np.float32(65535.0)).astype(np.uint32)


def weighted_draws(hu, draws, spacing, origin):
    """Voxel centres (n2, 3) picked by the integer draws."""
    nz, ny, nx = np.asarray(hu).shape
    cdf = np.cumsum(weights(hu).astype(np.uint64))
    idx = np.searchsorted(cdf, np.asarray(draws, np.uint64), side="right")
    idx = np.minimum(idx, cdf.size - 1)
    z, rem = np.divmod(idx, ny * nx)
    y, x = np.divmod(rem, nx)
    g = np.stack([x, y, z], axis=1).astype(np.float64)
    return np.asarray(origin, np.float64) + g * np.asarray(spacing, np.float64), idx


def knn_log_scale(points, k=3, rows=None):
    """log sqrt(mean squared distance to the k nearest other points), by brute
    force, for every point or the given rows."""
    P = np.asarray(points, np.float64)
    n = P.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    out = np.empty(len(rows))
    for lo in range(0, len(rows), 512):
        rr = rows[lo:lo + 512]
        d2 = ((P[rr, None, :] - P[None, :, :]) ** 2).sum(axis=2)
        d2[np.arange(len(rr)), rr] = np.inf
        kk = min(k, n - 1)
        near = np.sort(d2, axis=1)[:, :kk] if kk > 0 else np.zeros((d2.shape[0], 0))
        mean = near.mean(axis=1) if kk > 0 else np.zeros(d2.shape[0])
        out[lo:lo + 512] = 0.5 * np.log(np.maximum(mean, 1e-7))
    return out


def rads(hu, spacing, origin, n1, mc_keys, draws):
    """Initial points (N, 3), n_iso and per-point log-scale for the caller's
    keys (one per crossing) and integer draws."""
    iso = iso_level(hu)
    pmc, _ = crossings(hu, iso, spacing, origin)
    order = np.lexsort((np.arange(len(pmc)), np.asarray(mc_keys, np.uint32)))[:n1]
    pdw, _ = weighted_draws(hu, draws, spacing, origin)
    pts = np.concatenate([pmc[order], pdw])
    n_iso = len(order) + len(draws) // 2
    return pts, n_iso, knn_log_scale(pts)
