#!/usr/bin/env python3
"""Benchmark of the DDGS-CT DRR splatting hot path on one MI355X.

Headline: milliseconds per 512x512 DRR forward + backward at 500k Gaussians
(the fitting step: render -> (1-lambda) L1 + lambda D-SSIM against a target
-> backward to every Gaussian parameter and both bases), one view per step,
cycling over 36 azimuth poses 10 degrees apart.  Secondary: the speed-up of
the batched, graph-captured pose-scoring step (64 perturbed poses of a
300k-Gaussian model, 256x256 detector, forward + NCC + pose-only backward)
over 64 sequential plain calls, and a registration run that refines those 64
candidates towards the target image inside the captured step.

Inputs are synthetic and seeded (a nested-ellipsoid HU phantom stands in for
CT scans).  The fitting targets are renders of the unperturbed model made by
the same GPU renderer before timing; the timed work is the perturbed model's
fitting step.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

METRIC = "ms per 512² DRR fwd+bwd @500k Gaussians; batched-pose vs plain speedup"
ROOT = os.path.dirname(os.path.abspath(__file__))

# Algorithmic lane operations per contributing (pixel, Gaussian) pair: every
# add, multiply, fused multiply-add, compare, min, select, exp or reciprocal
# counts 1 (one VALU lane issue each):
#   forward  : offset 2, quadratic form d2 5 (3 multiplies, 2 fused), cut-off
#              compare 1, exp 1, alpha G 1, min with sigma_max 1, T s 1,
#              colour fma 1, 1 - s 1, T (1 - s) 1                         = 16
#   backward : the forward's transmittance recomputation 15 (everything but
#              the colour), tail update 1, dL/ds = g (c T - S / (1 - s)) 4
#              (reciprocal, multiply, fused, multiply), clamp subgradient
#              select 1, q = dL/ds G 1, dL/dc = g T s 1, the moments q dx,
#              q dy, q dx^2, q dx dy, q dy^2 5, and the reduction of the 7
#              gradient terms over the tile's pixels 7                    = 34
# Peak: 256 CU x 64 lanes x 2.4 GHz = 39.3 T lane-op/s (one non-packed
# VALU instruction per lane per cycle; packed FP32 is disabled).
LANE_OPS_FWD = 16
LANE_OPS_BWD = 34
PEAK_LANE_OPS = 39.3   # T lane-op/s
# The same work counted in floating-point operations with a fused multiply-add
# as 2 (forward 19, backward 52), against 78.6 TFLOP/s (256 CU x 4 SIMD x 16
# lanes x 2 x 2.4 GHz, no packed FP32): the FMA-weighted view of one roofline.
FLOPS_FWD = 19
FLOPS_BWD = 52
PEAK_ALU_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=36)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-rads", action="store_true")
    ap.add_argument("--fit-iters", type=int, default=720,
                    help="iterations of the fitting run on the 500k-Gaussian workload (0: skip)")
    ap.add_argument("--cpu-row-stride", type=int, default=2,
                    help="oracle baseline: every n-th detector row of one view")
    ap.add_argument("--batched-reps", type=int, default=5)
    ap.add_argument("--register-iters", type=int, default=200,
                    help="iterations of the registration run on the 64 pose candidates (0: skip)")
    ap.add_argument("--tile", default="auto", help="WxH, or auto: the built-in autotuner picks tile shape, "
                    "scheduling and chunk size on the live inputs")
    ap.add_argument("--split", type=int, default=None,
                    help="chunk size with a fixed --tile (default: the library's default)")
    ap.add_argument("--workload", default="all", choices=("all", "fitting", "batched", "uneven"),
                    help="run one workload only (for per-workload profiler runs); the JSON line then carries "
                         "the fitting step only when it ran")
    ap.add_argument("--cpu-extra-stride", type=int, default=32,
                    help="oracle timings of the 64-pose and uneven workloads: every n-th detector row (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (4 times); used to scale the HBM "
                         "byte counters of a profiler to known traffic")
    return ap.parse_args()


def host_cpu():
    """Model name and logical CPU count of the host the oracle runs on."""
    name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": name, "logical_cpus": os.cpu_count()}


def copy_calibration():
    import torch
    n = 64 << 20  # floats: 256 MiB
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 4}), flush=True)


def ordinal(k):
    """1st, 2nd, 3rd, 4th, ..., 11th, 12th, 13th, ..., 21st, 32nd."""
    suffix = "th" if 10 <= k % 100 <= 20 else {1: "st", 2: "nd", 3: "rd"}.get(k % 10, "th")
    return f"{k}{suffix}"


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch from a committed rocprofv3 counter summary, valid
    only while the kernel sources are unchanged."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        src = hashlib.sha256()
        for f in d["sources"]:
            src.update(open(os.path.join(ROOT, f), "rb").read())
        if src.hexdigest() != d["sources_sha256"]:
            return None
        return float(d["bytes_per_launch"])
    except Exception:  # noqa: BLE001 - a stale or unreadable summary means "not measured"
        return None


def valu_from_profiles(kernel, workload):
    """VALU instructions per launch and the issue fraction from the committed
    SQ counter summary, valid only while the kernel sources are unchanged."""
    path = os.path.join(ROOT, "profiles", f"valu_raster_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        src = hashlib.sha256()
        for f in d["sources"]:
            src.update(open(os.path.join(ROOT, f), "rb").read())
        if src.hexdigest() != d["sources_sha256"]:
            return None
        k = d["kernels"][kernel]
        return {"valu_insts_per_launch": int(k["valu_insts"]), "issue_frac": round(k["valu_issue_frac"], 3)}
    except Exception:  # noqa: BLE001 - a stale or unreadable summary means "not measured"
        return None


def lds_from_profiles(kernel, workload):
    """LDS utilisation of the kernel from the committed SQ counter summary:
    SQ_LDS_IDX_ACTIVE cycles over the CU-cycles of the kernel (the profiler's
    LdsUtil), with the bank-conflict share; valid only while the kernel
    sources are unchanged."""
    path = os.path.join(ROOT, "profiles", f"lds_raster_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        src = hashlib.sha256()
        for f in d["sources"]:
            src.update(open(os.path.join(ROOT, f), "rb").read())
        if src.hexdigest() != d["sources_sha256"]:
            return None
        k = d["kernels"][kernel]
        return {"lds_util": round(k["lds_util"], 4), "bank_conflict_frac": round(k["bank_conflict_frac"], 4)}
    except Exception:  # noqa: BLE001 - a stale or unreadable summary means "not measured"
        return None


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "this renderer has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2406_02518_amd import binding, fit, rads, register, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration()
        return
    fixed = None if args.tile == "auto" else tuple(int(x) for x in args.tile.split("x"))
    fixed_opts = {} if not fixed else dict(tile_w=fixed[0], tile_h=fixed[1],
                                           **({} if args.split is None else {"split": args.split}))
    stream = torch.cuda.Stream()

    run_fit = args.workload in ("all", "fitting")
    ms_per_step = stages = roofline = stage_roofline = step_dist = tuned = cfg = views = None
    variants = fitting = rads_info = None
    plain_ms = []
    if run_fit:
        # ------------------------------------------------------------ C3 setup
        log("generating the 500k-Gaussian fitting workload")
        cfg = synth.config("C3")
        views = cfg.views
        R = binding.Renderer(0, stream=stream)
        if fixed:
            R.set_options(**fixed_opts)
        with torch.cuda.stream(stream):
            R.set_scene(cfg.extra["true_scene"])
            R.set_views(views)
            targets_all = R.render().clone()
            P = views[0].W * views[0].H
            targets = [targets_all[j * P:(j + 1) * P] for j in range(len(views))]
            params = R.set_scene(cfg.scene)
            if not fixed:
                R.set_views([views[0]])
                binding.ddgs_autotune(R.ctx, None, 3)
            tuned = R.options()
            log("raster options:", json.dumps(tuned))
            # capacity of the captured step: the largest per-pose entry count + 25 %
            maxM = 0
            for v in views:
                R.set_views([v])
                R.render()
                maxM = max(maxM, R.num_rendered())
        stream.synchronize()
        R.set_options(capacity=int(maxM * 1.25) + 1024)
        R.set_views([views[0]])
        img = torch.empty(P, device="cuda")
        dl = torch.empty(P, device="cuda")
        loss = torch.empty(1, device="cuda")
        tgt = torch.empty(P, device="cuda")
        grads = R.alloc_grads()
        binding.ddgs_step_capture(R.ctx, binding.LOSS_L1_DSSIM, tgt.data_ptr(), 0.2, img.data_ptr(), dl.data_ptr(),
                                  loss.data_ptr(), R.grads_struct(grads))

        def step(j):
            with torch.cuda.stream(stream):
                binding.ddgs_step_set_target(R.ctx, targets[j % len(views)].data_ptr())
                R.set_views([views[j % len(views)]])
                binding.ddgs_step_launch(R.ctx)

        log(f"warmup {args.warmup}, timed {args.steps} steps")
        for j in range(args.warmup):
            step(j)
        binding.ddgs_check(R.ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(args.steps):
            step(j)
        stream.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        binding.ddgs_check(R.ctx)  # raises if any replay overflowed its capacity
        ms_per_step = (t1 - t0) * 1e3 / max(1, args.steps)
        log(f"captured fitting step: {ms_per_step:.3f} ms")

        # per-step distribution: event-timed replays, `reps` per pose
        reps = 20
        marks = []
        with torch.cuda.stream(stream):
            for j in range(len(views)):
                for _ in range(reps):
                    binding.ddgs_step_set_target(R.ctx, targets[j].data_ptr())
                    R.set_views([views[j]])
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    binding.ddgs_step_launch(R.ctx)
                    e1.record(stream)
                    marks.append((j, e0, e1))
        stream.synchronize()
        binding.ddgs_check(R.ctx)
        per = np.array([a.elapsed_time(b) for _, a, b in marks])
        pose_med = [float(np.median(per[[i for i, (j, _, _) in enumerate(marks) if j == p]])) for p in range(len(views))]
        step_dist = {"repeats_per_pose": reps, "poses": len(views), "median_ms": round(float(np.median(per)), 4),
                     "p10_ms": round(float(np.percentile(per, 10)), 4), "p90_ms": round(float(np.percentile(per, 90)), 4),
                     "pose_median_min_ms": round(min(pose_med), 4), "pose_median_max_ms": round(max(pose_med), 4)}
        log("step distribution:", json.dumps(step_dist))

        # ------------------------------ per-stage HIP-event timing + pair counts
        binding.ddgs_enable_timing(R.ctx, 1)
        R.set_options(capacity=0)
        stages = {k: 0.0 for k in binding.STAGES}
        ev_pairs = co_pairs = entries = 0
        plain_ms = []
        nst = min(len(views), max(1, args.steps))
        with torch.cuda.stream(stream):
            for j in range(nst):
                R.set_views([views[j]])
                stream.synchronize()
                a = time.perf_counter()
                im = R.render()
                lo, d = R.loss(binding.LOSS_L1_DSSIM, im, targets[j], 0.2)
                R.backward(d, grads=grads)
                stream.synchronize()
                plain_ms.append((time.perf_counter() - a) * 1e3)
                st = binding.ddgs_stage_times(R.ctx)
                for k in stages:
                    stages[k] += st[k] / nst
            # pair statistics in a separate, untimed render per pose (the
            # counters are same-address atomics that would perturb the timing)
            binding.ddgs_enable_timing(R.ctx, 0)
            binding.ddgs_debug_count_pairs(R.ctx, 1)
            for j in range(nst):
                R.set_views([views[j]])
                R.render()
                e, c = binding.ddgs_debug_pair_counts(R.ctx)
                ev_pairs += e / nst
                co_pairs += c / nst
                entries += R.num_rendered() / nst
            binding.ddgs_debug_count_pairs(R.ctx, 0)
        dominant = max(("raster_fwd", "raster_bwd"), key=lambda k: stages[k])
        bwd = dominant == "raster_bwd"
        lane_ops = co_pairs * (LANE_OPS_BWD if bwd else LANE_OPS_FWD)
        achieved = lane_ops / (stages[dominant] * 1e-3) / 1e12
        flops = co_pairs * (FLOPS_BWD if bwd else FLOPS_FWD)
        achieved_f = flops / (stages[dominant] * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": dominant, "achieved": round(achieved, 4), "peak": PEAK_LANE_OPS,
                    "unit": "T lane-op/s", "frac": round(achieved / PEAK_LANE_OPS, 5),
                    "traffic": traffic_from_profiles(dominant, "C3"),
                    "kernel_ms": round(stages[dominant], 4),
                    "contributing_pairs_per_launch": int(co_pairs), "evaluated_pairs_per_launch": int(ev_pairs),
                    "lane_ops_per_contributing_pair": LANE_OPS_BWD if bwd else LANE_OPS_FWD,
                    "fma_weighted": {"achieved": round(achieved_f, 4), "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                                     "frac": round(achieved_f / PEAK_ALU_TFLOPS, 5),
                                     "flops_per_contributing_pair": FLOPS_BWD if bwd else FLOPS_FWD},
                    "valu_issue": valu_from_profiles(dominant, "C3"),
                    "lds": lds_from_profiles(dominant, "C3")}
        # every stage against its own bound, from algorithmic work per launch:
        # parameters 4 (11 + k) B per Gaussian, a 28 B record or gradient slot per
        # (view, Gaussian) / tile entry, 8 B keys + values, 12 B per pixel
        n3, k3, P3 = cfg.scene.n, cfg.scene.k, int(views[0].W) * int(views[0].H)
        pbytes = 4 * (11 + k3)
        algo = {"project": ("hbm", (pbytes + 28) * n3), "sort": ("hbm", 16 * n3 + 16 * entries),
                "raster_fwd": ("alu", LANE_OPS_FWD * co_pairs), "loss": ("hbm", 12 * P3),
                "raster_bwd": ("alu", LANE_OPS_BWD * co_pairs), "project_bwd": ("hbm", 2 * pbytes * n3 + 28 * entries)}
        stage_roofline = []
        for k, (bound, work) in algo.items():
            t = stages[k] * 1e-3
            if bound == "alu":
                a = work / t / 1e12
                stage_roofline.append({"stage": k, "bound": "alu", "achieved": round(a, 3), "peak": PEAK_LANE_OPS,
                                       "unit": "T lane-op/s", "frac": round(a / PEAK_LANE_OPS, 4),
                                       "ms": round(stages[k], 4)})
            else:
                a = work / t / 1e9
                stage_roofline.append({"stage": k, "bound": "hbm", "achieved": round(a, 1), "peak": PEAK_HBM_GBS,
                                       "unit": "GB/s", "frac": round(a / PEAK_HBM_GBS, 4), "ms": round(stages[k], 4)})
        log("stages (ms):", json.dumps({k: round(v, 4) for k, v in stages.items()}))

        # ---------------- model variants of the ablations on the same geometry
        # (same Gaussians, poses, targets and raster options; new seeded features
        # and bases of each size), one captured fitting step per pose
        variants = None
        if not args.no_variants:
            variants = []
            R.set_options(capacity=int(maxM * 1.25) + 1024)
            for name, k_v, L_v, kind in (("disentangled L=3 k=16", 16, 3, "disentangled"),
                                         ("disentangled L=1 k=8", 8, 1, "disentangled"),
                                         ("disentangled L=3 k=8", 8, 3, "disentangled"),
                                         ("disentangled L=3 k=32", 32, 3, "disentangled"),
                                         ("disentangled L=3 k=1", 1, 3, "disentangled"),
                                         ("iso-only k=16", 16, 3, "iso_only"),
                                         ("dir-only L=3 k=16", 16, 3, "dir_only"),
                                         ("entangled L=3 k=16", 16, 3, "entangled")):
                sc_v = synth.with_features(cfg.scene, 5150 + len(variants), k_v, L_v, kind)
                with torch.cuda.stream(stream):
                    R.set_scene(sc_v)
                    R.set_views([views[0]])
                g_v = R.alloc_grads()
                binding.ddgs_step_capture(R.ctx, binding.LOSS_L1_DSSIM, tgt.data_ptr(), 0.2, img.data_ptr(),
                                          dl.data_ptr(), loss.data_ptr(), R.grads_struct(g_v))
                for j in range(3):
                    step(j)
                binding.ddgs_check(R.ctx)
                stream.synchronize()
                a = time.perf_counter()
                for j in range(len(views)):
                    step(j)
                stream.synchronize()
                t_v = (time.perf_counter() - a) * 1e3 / len(views)
                binding.ddgs_check(R.ctx)
                variants.append({"model": name, "n_iso": int(sc_v.n_iso), "ms_per_step": round(t_v, 4)})
                log("variant:", json.dumps(variants[-1]))

        # ------------- fitting run: captured step + Adam, densification between
        fitting = None
        if args.fit_iters > 0:
            R.set_options(capacity=0)  # every capture sizes itself (the model grows)
            with torch.cuda.stream(stream):
                p_fit = R.set_scene(cfg.scene)
            extent = float(np.abs(cfg.scene.mean).max())
            sched = fit.FitSchedule(densify_from=100, densify_until=600, densify_every=100, opacity_reset_every=0)
            stream.synchronize()
            a = time.perf_counter()
            _, _, hist = fit.fit(R, p_fit, cfg.scene.n_iso, cfg.scene.L, views, targets, iters=args.fit_iters,
                                 extent=extent, schedule=sched, log_every=72)
            stream.synchronize()
            t_fit = time.perf_counter() - a
            n_dens = len([i for i in range(1, args.fit_iters + 1)
                          if sched.densify_from <= i <= sched.densify_until and i % sched.densify_every == 0])
            fitting = {"workload": "fitting run on the same 500k-Gaussian model, poses and targets: one captured step "
                                   "(render, (1-0.2) L1 + 0.2 D-SSIM, backward, Adam on every group) per iteration, "
                                   "one pose per iteration in shuffled epochs, densification every 100 iterations "
                                   "from 100 to 600 followed by a new capture",
                       "iterations": args.fit_iters, "seconds": round(t_fit, 3),
                       "ms_per_iteration": round(t_fit * 1e3 / args.fit_iters, 4), "densifications": n_dens,
                       "gaussians": [int(cfg.scene.n), int(hist[-1][1]) if hist else int(cfg.scene.n)],
                       "loss_first_last_72": [round(hist[0][2], 7), round(hist[-1][2], 7)] if hist else None}
            log("fitting:", json.dumps(fitting))

        # ------------- initialisation by dual sampling of a 256^3 phantom volume
        rads_info = None
        if not args.no_rads:
            ph = synth.phantom(256, np.random.default_rng(1003))
            hu_t = torch.from_numpy(np.ascontiguousarray(ph.transpose(2, 1, 0))).cuda()
            torch.cuda.synchronize()
            ts = []
            for rep in range(4):
                a = time.perf_counter()
                pts_r, ls_r, n_iso_r, info = rads.sample(R, hu_t, (1.0, 1.0, 1.0), (-127.5, -127.5, -127.5), seed=rep)
                stream.synchronize()
                ts.append((time.perf_counter() - a) * 1e3)
            rads_info = {"workload": "radiodensity-aware dual sampling of a 256^3 HU phantom at 1 mm: level "
                                     "(min + max) / 2, interface points, n1 = 15000 of them, n2 = 10000 weighted "
                                     "voxel centres, 3-nearest-neighbour scales",
                         "ms": round(float(np.median(ts[1:])), 3), "crossings": int(info["crossings"]),
                         "points": int(pts_r.shape[1]), "n_iso": int(n_iso_r)}
            log("rads:", json.dumps(rads_info))
        R.close()

    # ------------------------------------------- C4 batched vs plain speed-up
    batched = None
    if not args.no_batched and args.workload in ("all", "batched"):
        log("pose-scoring workload: 64 poses x 300k Gaussians")
        c4 = synth.config("C4")
        R4 = binding.Renderer(0, stream=stream)
        if fixed:
            R4.set_options(**fixed_opts)
        with torch.cuda.stream(stream):
            R4.set_scene(c4.scene)
            R4.set_views([c4.extra["gt_view"]])
            target1 = R4.render().clone()
        P4 = target1.numel()
        V4 = len(c4.views)

        # the plain path: its own context on the same model, one view per call
        # (setting views drops a captured step, so the batched context keeps
        # its 64 views and its graph)
        Rp = binding.Renderer(0, stream=stream)

        def plain_once(keep=False):
            outs = []
            with torch.cuda.stream(stream):
                for v in c4.views:
                    Rp.set_views([v])
                    im = Rp.render()
                    _, d4 = Rp.loss(binding.LOSS_NCC, im, target1, 0.0)
                    Rp.backward(d4, which=("dpose",))
                    if keep:
                        outs.append(im.clone())
            return outs

        # one set of raster options for both paths (tuned on the 64-view batch)
        R4.set_views(c4.views)
        if not fixed:
            binding.ddgs_autotune(R4.ctx, None, 3)
        tuned4 = R4.options()
        log("batched raster options:", json.dumps(tuned4))
        with torch.cuda.stream(stream):
            Rp.set_scene(c4.scene)
        Rp.set_options(**{k: tuned4[k] for k in ("tile_w", "tile_h", "persistent", "split")})
        plain_imgs = plain_once(keep=True)
        stream.synchronize()
        target64 = target1.repeat(V4)
        img64 = torch.empty(P4 * V4, device="cuda")
        dl64 = torch.empty_like(img64)
        loss64 = torch.empty(V4, device="cuda")
        g64 = R4.alloc_grads(("dpose",))
        binding.ddgs_step_capture(R4.ctx, binding.LOSS_NCC, target64.data_ptr(), 0.0, img64.data_ptr(),
                                  dl64.data_ptr(), loss64.data_ptr(), R4.grads_struct(g64))
        binding.ddgs_step_launch(R4.ctx)
        binding.ddgs_check(R4.ctx)
        identical = all(torch.equal(img64[i * P4:(i + 1) * P4], plain_imgs[i]) for i in range(V4))
        # the timed plain calls run at their own best chunk size: the batch's
        # tuning times the batch only, and one 256x256 view has a sixty-fourth
        # of its tiles (chunks of 1024 then leave most tiles in one item)
        base4 = {k: tuned4[k] for k in ("tile_w", "tile_h", "persistent", "split")}
        plain_split, best = base4["split"], None
        for sp_ in sorted({base4["split"], 256, 1024}):
            Rp.set_options(**dict(base4, split=sp_))
            plain_once()
            ts = []
            for _ in range(2):
                stream.synchronize()
                a = time.perf_counter()
                plain_once()
                stream.synchronize()
                ts.append((time.perf_counter() - a) * 1e3)
            if best is None or min(ts) < best:
                best, plain_split = min(ts), sp_
        Rp.set_options(**dict(base4, split=plain_split))
        # paired repetitions: 64 plain calls, then one replay of the captured
        # step, each timed between synchronisations; the speed-up of every pair
        t_pl, t_ba = [], []
        for _ in range(max(3, args.batched_reps)):
            stream.synchronize()
            a = time.perf_counter()
            plain_once()
            stream.synchronize()
            t_pl.append((time.perf_counter() - a) * 1e3)
            stream.synchronize()
            a = time.perf_counter()
            binding.ddgs_step_launch(R4.ctx)
            stream.synchronize()
            t_ba.append((time.perf_counter() - a) * 1e3)
        binding.ddgs_check(R4.ctx)
        t_pl, t_ba = np.array(t_pl), np.array(t_ba)
        sp = t_pl / t_ba

        def spread(x):
            return {"median": round(float(np.median(x)), 3), "min": round(float(x.min()), 3),
                    "max": round(float(x.max()), 3)}

        batched = {"workload": "64 perturbed poses (rotation U(+-10 deg), translation U(+-20 mm)) of a 300k-Gaussian "
                               "192^3-phantom model, 256x256 at 1.5 mm, forward + NCC + pose-only backward",
                   "repetitions": int(len(sp)),
                   "plain_ms": round(float(np.median(t_pl)), 3), "batched_ms": round(float(np.median(t_ba)), 3),
                   "speedup": round(float(np.median(sp)), 3),
                   "spread": {"plain_ms": spread(t_pl), "batched_ms": spread(t_ba), "speedup": spread(sp)},
                   "images_bit_identical": bool(identical),
                   "raster_options": base4, "plain_raster_options": dict(base4, split=plain_split)}
        log("batched:", json.dumps(batched))

        # registration: every candidate pose refined towards the target image
        # (Adam on the pose tangent inside the captured step, rotation about the
        # isocentre), then the error measures against the true pose
        if args.register_iters > 0:
            gt4 = c4.extra["gt_view"]
            pts4 = c4.scene.mean.T[::16]
            f4 = gt4.sdd / gt4.pitch

            def errors(poses):
                return np.array([[register.rotation_error_deg(p, gt4.pose), register.source_error_mm(p, gt4.pose),
                                  register.target_registration_error(p, gt4.pose, pts4),
                                  register.projection_distance(p, gt4.pose, f4, pts4)] for p in poses])

            e0 = errors([v.pose for v in c4.views])
            R4.set_views(c4.views)
            stream.synchronize()
            a = time.perf_counter()
            poses, hist = register.register(R4, target64, iters=args.register_iters, check_every=25)
            stream.synchronize()
            t_reg = time.perf_counter() - a
            e1 = errors(poses)
            iters = hist[-1][0]

            def stats(e):
                return {"median": round(float(np.median(e)), 4), "max": round(float(np.max(e)), 4)}

            registration = {
                "workload": "the same 64 candidate poses registered to the target image: NCC, Adam (1 mm, 0.008 rad "
                            "per step) on the pose tangent with rotation about the isocentre, inside the captured step",
                "iterations": int(iters), "seconds": round(t_reg, 3), "ms_per_iteration": round(t_reg * 1e3 / iters, 3),
                "loss_median": [round(float(np.median(hist[0][1])), 6), round(float(np.median(hist[-1][1])), 8)],
                "start": {k: stats(e0[:, j]) for j, k in enumerate(("rot_deg", "source_mm", "tre_mm", "proj_px"))},
                "end": {k: stats(e1[:, j]) for j, k in enumerate(("rot_deg", "source_mm", "tre_mm", "proj_px"))},
                "frac_rot_below_1deg": round(float(np.mean(e1[:, 0] < 1.0)), 4),
                "frac_proj_below_1px": round(float(np.mean(e1[:, 3] < 1.0)), 4)}
            batched["registration"] = registration
            log("registration:", json.dumps(registration))
        Rp.close()
        R4.close()

    # ------------------------------------ uneven batch (1M Gaussians, 16 views)
    uneven = None
    if not args.no_uneven and args.workload in ("all", "uneven"):
        log("uneven batch: 1M Gaussians, 16 views of 256^2 / 512^2 / 1024^2")
        c5 = synth.config("C5")
        R5 = binding.Renderer(0, stream=stream)
        with torch.cuda.stream(stream):
            R5.set_scene(c5.scene)
            R5.set_views(c5.views)
            if fixed:
                R5.set_options(**fixed_opts)
            else:
                binding.ddgs_autotune(R5.ctx, None, 3)
            tuned5 = R5.options()
            log("uneven raster options:", json.dumps(tuned5))
            P5 = R5.image_size()
            w5 = torch.from_numpy(np.random.default_rng(c5.extra["dl_seed"]).normal(size=P5).astype(np.float32)).cuda()
            img5 = torch.empty(P5, device="cuda")
            dl5 = torch.empty(P5, device="cuda")
            loss5 = torch.empty(len(c5.views), device="cuda")
            g5 = R5.alloc_grads()
            binding.ddgs_step_capture(R5.ctx, binding.LOSS_LINEAR, w5.data_ptr(), 0.0, img5.data_ptr(),
                                      dl5.data_ptr(), loss5.data_ptr(), R5.grads_struct(g5))
            for _ in range(2):
                binding.ddgs_step_launch(R5.ctx)
        binding.ddgs_check(R5.ctx)
        ts = []
        for _ in range(args.batched_reps):
            stream.synchronize()
            a = time.perf_counter()
            binding.ddgs_step_launch(R5.ctx)
            stream.synchronize()
            ts.append((time.perf_counter() - a) * 1e3)
        binding.ddgs_check(R5.ctx)
        n5 = R5.num_rendered()
        uneven = {"workload": "1M Gaussians (256^3 phantom), 16 views in one captured step: 6 x 256^2, 6 x 512^2, "
                              "4 x 1024^2, pitch U(0.4, 1.5) mm, source-isocentre U(500, 700) mm; forward + "
                              "linear loss with fixed random weights + backward to all parameters and poses",
                  "ms_per_step": round(float(np.median(ts)), 3), "tile_entries": int(n5),
                  "raster_options": {k: tuned5[k] for k in ("tile_w", "tile_h", "persistent", "split")}}
        log("uneven:", json.dumps(uneven))
        R5.close()

    # ---------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu_baseline and run_fit:
        from oracle import ref
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        v = views[0]
        rows = np.arange(0, v.H, args.cpu_row_stride)
        uu, vv = np.meshgrid(np.arange(v.W), rows)
        pix = np.stack([np.zeros(uu.size, int), uu.ravel(), vv.ravel()], 1).astype(np.int32)
        gw = np.random.default_rng(0).normal(size=len(pix))
        log(f"oracle baseline: {len(rows)} of {v.H} rows, {threads} threads")
        a = time.perf_counter()
        ref.render_pixels(cfg.scene, [v], pix, threads=threads)
        ref.backward(cfg.scene, [v], pix, gw, threads=threads)
        dt = time.perf_counter() - a
        scale = v.H / len(rows)
        cpu = {"value": round(dt * scale * 1e3, 1), "unit": "ms", "cores": threads, "kind": "oracle", "host": host_cpu(),
               "sample": f"view 0 of the fitting workload, every {ordinal(args.cpu_row_stride)} detector row "
                         f"({len(rows)} of {v.H} rows = {len(pix)} pixels x 500k Gaussians), forward at those "
                         f"pixels + analytic FP64 backward of a linear loss on them; {dt:.1f} s measured, "
                         f"scaled by {scale:g} to one full 512x512 fwd+bwd"}
        # more oracle timings: pair tests per second (every pixel is tested
        # against every valid Gaussian), one thread on a smaller sample, and
        # the two small workloads in full
        pair_tests = len(pix) * cfg.scene.n
        cpu["pair_tests_per_s"] = round(pair_tests / dt, 1)
        rows1 = np.arange(0, v.H, 64)
        u1, v1 = np.meshgrid(np.arange(v.W), rows1)
        pix1 = np.stack([np.zeros(u1.size, int), u1.ravel(), v1.ravel()], 1).astype(np.int32)
        a = time.perf_counter()
        ref.render_pixels(cfg.scene, [v], pix1, threads=1)
        ref.backward(cfg.scene, [v], pix1, np.ones(len(pix1)), threads=1)
        dt1 = time.perf_counter() - a
        cpu["single_thread_pair_tests_per_s"] = round(len(pix1) * cfg.scene.n / dt1, 1)
        # the 64-pose and uneven workloads on every n-th detector row of every
        # view, forward at those pixels + backward of a linear loss on them,
        # scaled by the exact pixel ratio (extrapolated)
        if args.cpu_extra_stride > 0:
            for name, label in (("C4", "batched_64_poses"), ("C5", "uneven_16_views")):
                cs = synth.config(name)
                rows_all, full = [], 0
                for vi, vw in enumerate(cs.views):
                    rr = np.arange(0, vw.H, args.cpu_extra_stride)
                    uu_, vv_ = np.meshgrid(np.arange(vw.W), rr)
                    rows_all.append(np.stack([np.full(uu_.size, vi), uu_.ravel(), vv_.ravel()], 1))
                    full += vw.W * vw.H
                pix_x = np.concatenate(rows_all).astype(np.int32)
                a = time.perf_counter()
                ref.render_pixels(cs.scene, cs.views, pix_x, threads=threads)
                ref.backward(cs.scene, cs.views, pix_x, np.ones(len(pix_x)), threads=threads)
                dt_x = time.perf_counter() - a
                cpu[f"{label}_fwd_bwd_ms_extrapolated"] = round(dt_x * full / len(pix_x) * 1e3, 1)
                cpu[f"{label}_sample"] = (f"every {ordinal(args.cpu_extra_stride)} detector row of all {len(cs.views)} views "
                                          f"({len(pix_x)} of {full} pixels x {cs.scene.n} Gaussians), "
                                          f"{dt_x:.1f} s measured, scaled by {full / len(pix_x):.2f}")
        for name in ("C1", "C2"):
            cs = synth.config(name)
            a = time.perf_counter()
            ref.render(cs.scene, cs.views, threads=threads)
            t_f = time.perf_counter() - a
            allp = ref.all_pixels(cs.views)
            a = time.perf_counter()
            ref.backward(cs.scene, cs.views, allp, np.ones(len(allp)), threads=threads)
            t_b = time.perf_counter() - a
            cpu[f"{name}_full_fwd_ms"] = round(t_f * 1e3, 1)
            cpu[f"{name}_full_fwd_bwd_ms"] = round((t_f + t_b) * 1e3, 1)
        log("cpu:", json.dumps(cpu))

    config = {"workload": "fitting step: 500k Gaussians (256^3 phantom), 512x512 detector at 0.8 mm, "
                          "one of 36 azimuth poses per step, (1-0.2) L1 + 0.2 D-SSIM vs a target, "
                          "backward to all parameters and bases; one captured HIP graph per step"}
    if run_fit:
        config.update({"gaussians": cfg.scene.n, "detector": f"{views[0].W}x{views[0].H}", "poses": len(views),
                       "k": cfg.scene.k, "L": cfg.scene.L,
                       "raster_options": {k: tuned[k] for k in ("tile_w", "tile_h", "persistent", "split")},
                       "plain_path_ms_per_step": round(float(np.median(plain_ms)), 4)})
    else:
        config["workload"] = f"only the {args.workload} workload ran (--workload); no fitting-step figure"
    out = {
        "metric": METRIC, "value": round(ms_per_step, 4) if run_fit else None, "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4) if run_fit else None,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": config,
        "stages_ms": {k: round(v, 4) for k, v in stages.items()} if run_fit else None,
        "roofline": roofline,
        "stage_roofline": stage_roofline,
        "step_distribution": step_dist,
        "variants": variants,
        "fitting": fitting,
        "rads": rads_info,
        "batched": batched,
        "uneven_batch": uneven,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
