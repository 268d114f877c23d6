"""Shared helpers of the GPU tests (not collected by pytest)."""
import numpy as np

from paper_2406_02518_amd import synth


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


# Pixels near a hit decision of Eq. 1 (the kappa cutoff, the sigma_max clamp,
# the t_min stop) have two correct sets of contributors: the kernel decides in
# FP32, the oracle in FP64, and the two projected means and conics differ by
# rounding.  Worst case near the cutoff: the FP32 mean of a ~1000 px image is
# off by up to ~5e-4 px after the projection's roundings, and d2 moves by
# 2 sqrt(d2 lambda_max(A)) per pixel of mean, lambda_max <= 1 / 0.3 (the
# dilation), so d2 / kappa^2 is uncertain to ~6e-4.  Sampled-pixel parity
# compares only pixels whose decisions are unique at that band.
DECISION_BAND = 1e-3


def unique_pixels(scene, views, pix, opts=None, band=DECISION_BAND):
    """Rows of pix (M, 3) whose relative margin to every hit decision exceeds band."""
    from oracle import ref
    m = ref.pixel_margins(scene, views, pix, opts=opts)
    return pix[m > band]


def make_renderer(**opts):
    from paper_2406_02518_amd import binding
    r = binding.Renderer(0)
    if opts:
        r.set_options(**opts)
    return r


def small_scene(seed=5, n=600, k=16, L=3, extent=20.0, iso_fraction=0.8, std_range=(0.5, 2.0),
                alpha_range=(0.02, 0.3)):
    return synth.random_scene(seed, n, k=k, L=L, extent=extent, iso_fraction=iso_fraction,
                              std_range=std_range, alpha_range=alpha_range)


def kept_tiles(rect, mask):
    """The kept tiles of a rectangle (tx0, ty0, tx1, ty1) in row-major order:
    bit b of the mask is place b when the rectangle has at most 32 tiles,
    larger rectangles keep every tile."""
    tx0, ty0, tx1, ty1 = (int(x) for x in rect)
    area = (tx1 - tx0 + 1) * (ty1 - ty0 + 1)
    out, b = [], 0
    for ty in range(ty0, ty1 + 1):
        for tx in range(tx0, tx1 + 1):
            if area > 32 or (int(mask) >> b) & 1:
                out.append((tx, ty))
            b += 1
    return out


def box_min_d2(A00, A01, A11, xl, xh, yl, yh):
    """min of d^T A d over the box [xl, xh] x [yl, yh] of offsets (FP64): the
    vertices and the interior critical points of the four edges."""
    if xl <= 0 <= xh and yl <= 0 <= yh:
        return 0.0
    q = lambda x, y: A00 * x * x + 2 * A01 * x * y + A11 * y * y  # noqa: E731
    c = [q(x, y) for x in (xl, xh) for y in (yl, yh)]
    for x in (xl, xh):
        y = -A01 * x / A11
        if yl <= y <= yh:
            c.append(q(x, y))
    for y in (yl, yh):
        x = -A01 * y / A00
        if xl <= x <= xh:
            c.append(q(x, y))
    return min(c)


def expected_tile_lists(zkeys, counts, rects, tile_base, ntx_per_view, n, masks):
    """Host construction of the sorted tile lists: emit every (view, Gaussian)
    entry of its kept tiles in (depth key, index) order, then stable-sort by
    tile id."""
    VN = zkeys.size
    order = np.lexsort((np.arange(VN), zkeys))  # by zkey, ties by index
    keys, vals = [], []
    for vi in order:
        c = counts[vi]
        if c == 0:
            continue
        v, i = divmod(int(vi), n)
        tiles = kept_tiles(rects[vi], masks[vi])
        assert len(tiles) == c
        for tx, ty in tiles:
            keys.append(tile_base[v] + ty * ntx_per_view[v] + tx)
            vals.append(i)
    keys = np.asarray(keys, dtype=np.uint32)
    vals = np.asarray(vals, dtype=np.uint32)
    s = np.argsort(keys, kind="stable")
    return keys[s], vals[s]
