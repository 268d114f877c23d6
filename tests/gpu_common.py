"""Shared helpers of the GPU tests (not collected by pytest)."""
import numpy as np

from paper_2406_02518_amd import synth


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


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


def expected_tile_lists(zkeys, counts, rects, tile_base, ntx_per_view, n):
    """Host construction of the sorted tile lists: emit every (view, Gaussian)
    rectangle in (depth key, index) order, then stable-sort by tile id."""
    VN = zkeys.size
    order = np.lexsort((np.arange(VN), zkeys))  # by zkey, ties by index
    keys, vals = [], []
    for vi in order:
        c = counts[vi]
        if c == 0:
            continue
        v, i = divmod(int(vi), n)
        tx0, ty0, tx1, ty1 = (int(x) for x in rects[vi])
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                keys.append(tile_base[v] + ty * ntx_per_view[v] + tx)
                vals.append(i)
    keys = np.asarray(keys, dtype=np.uint32)
    vals = np.asarray(vals, dtype=np.uint32)
    s = np.argsort(keys, kind="stable")
    return keys[s], vals[s]
