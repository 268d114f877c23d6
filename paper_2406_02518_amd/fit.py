"""Fitting loop (Sec. 4.1 training; App., Gaussians that move, split and drop):
the model is fitted to target DRRs with the (1 - lambda) L1 + lambda D-SSIM
loss of Eq. 2, one view per iteration.

Every iteration is one replay of a captured step: render -> loss -> backward
-> Adam on every parameter group, updating the model tensors in place; the
densification statistics accumulate inside the same replay.  Densification
changes the number of Gaussians, which a captured graph cannot, so it runs
between replays (plan and apply on the device, then the step is captured
again for the new size); the optimiser moments are carried across.  The
schedule follows the 3D Gaussian splatting defaults the paper adopts for
everything but the bases and features: densify every 100 iterations from
500 to 15000, reset opacities to 0.01 every 3000, drop oversized Gaussians
(world bound 0.1 x extent, screen bound 20 px) after the first reset.

The captured step has a fixed tile-entry capacity.  A replay that needs more
changes nothing (its updates are skipped on the device); at the next check the
loop raises the capacity, captures the step again and replays the skipped
iterations, so the run is the same as one with ample capacity."""
from dataclasses import dataclass

import numpy as np

from . import binding


@dataclass
class FitSchedule:
    densify_from: int = 500
    densify_until: int = 15000
    densify_every: int = 100
    opacity_reset_every: int = 3000
    grad_threshold: float = 2e-4
    dense_fraction: float = 0.01      # dense scale = fraction x extent
    world_fraction: float = 0.1       # world bound = fraction x extent
    max_screen_radius: float = 20.0
    min_opacity: float = 0.005
    reset_alpha: float = 0.01


def fit(R, params, n_iso, L, views, targets, iters, extent, lam=0.2, schedule=None, seed=0, log_every=100,
        entangled=False, rates=None, on_log=None):
    """Fits ``params`` (dict of float32 device tensors, replaced on
    densification) to ``targets`` (one float32 device tensor per view, all of
    the same size) on renderer R.  Returns (params, n_iso, history) with
    history a list of (iteration, n, mean loss over the last ``log_every``
    iterations)."""
    import torch

    sch = schedule or FitSchedule()
    P = int(views[0].W) * int(views[0].H)
    if any(int(v.W) * int(v.H) != P for v in views):
        raise ValueError("the captured step needs views of one size")
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device=R.device)
    gen.manual_seed(int(seed))
    tgt = torch.empty(P, device=R.device)
    img = torch.empty(P, device=R.device)
    dl = torch.empty(P, device=R.device)
    tgts = [t.contiguous() for t in targets]
    loss = torch.empty(1, device=R.device)
    losses = torch.zeros(max(1, log_every), device=R.device)

    state = {}

    def capture():
        with torch.cuda.stream(R.stream):
            binding.ddgs_step_capture(R.ctx, binding.LOSS_L1_DSSIM, tgt.data_ptr(), lam, img.data_ptr(),
                                      dl.data_ptr(), loss.data_ptr(), R.grads_struct(state["grads"]))

    def setup(p, ni):
        R.set_model(p, ni, L, entangled)
        stats = R.new_densify_stats()
        R.set_densify_stats(stats)
        R.set_views([views[0]])
        state.update(params=p, n_iso=ni, stats=stats, grads=R.alloc_grads())
        capture()

    window = []   # (iteration, view) of the replays launched since the last check

    def launch(it, j):
        with torch.cuda.stream(R.stream):
            # (the step reads this view's target in place: no copy)
            binding.ddgs_step_set_target(R.ctx, tgts[j].data_ptr())
            R.set_views([views[j]])
            binding.ddgs_step_launch(R.ctx)
            losses[(it - 1) % len(losses)].copy_(loss[0], non_blocking=True)
        window.append((it, j))

    def check():
        # an overflowed replay changed nothing: grow, capture again, replay it
        while True:
            skipped = R.check_step()
            if skipped == 0:
                break
            redo = window[len(window) - skipped:]
            window.clear()
            capture()
            for it_j in redo:
                launch(*it_j)
        window.clear()

    R.set_model(params, n_iso, L, entangled)
    R.set_fit_optimizer(extent, **(rates or {}))
    setup(params, n_iso)
    history = []
    order = []
    try:
        for it in range(1, iters + 1):
            if not order:
                order = list(rng.permutation(len(views)))
            launch(it, int(order.pop()))
            if log_every and it % log_every == 0:
                check()
                history.append((it, R.n, float(losses.mean().item())))
                if on_log:
                    on_log(history[-1])
            if sch.densify_from <= it <= sch.densify_until and it % sch.densify_every == 0:
                check()
                late = sch.opacity_reset_every > 0 and it > sch.opacity_reset_every
                with torch.cuda.stream(R.stream):
                    noise = torch.randn((R.n, 2, 3), generator=gen, device=R.device)
                    new, ni = R.densify(noise, grad_threshold=sch.grad_threshold,
                                        dense_scale=sch.dense_fraction * extent, min_opacity=sch.min_opacity,
                                        max_world_scale=sch.world_fraction * extent if late else 0.0,
                                        max_screen_radius=sch.max_screen_radius if late else 0.0)
                setup(new, ni)
            if sch.opacity_reset_every and it % sch.opacity_reset_every == 0:
                check()
                R.reset_opacity(sch.reset_alpha)
        check()
        return state["params"], state["n_iso"], history
    finally:
        R.set_fit_optimizer(None)
        R.set_densify_stats(None)
