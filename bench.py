"""Benchmark of the lookback ray-marching hot path on one MI355X.

Default workload (``--workload jet``): the jet-like single-render case.
  Grid 256 x 256 x 512 unit cells, 16 epochs t_m = -L/2 + m L/15 (L = grid
  diagonal), FP32 records (j, beta), seeded jet (radius 12, Lorentz factor 5 on
  the spine falling to 1.2 at the edge, lognormal sigma 0.5 turbulence, 4 knots
  at beta 0.98), alpha = 0.6, t_obs = 0, four 512 x 512 views at theta = 10,
  30, 60 and 90 deg (phi = 0), pixel scale L / 512 (the bounding sphere fills
  the image).
One step = one batched render of the four views (one persistent tile-queue
launch, replayed from a captured hipGraph) with the stack resident in HBM.
The plain kernel (one launch per image, one thread per pixel) is timed on the
same stack and views for comparison.

Other workloads: ``batch`` (384^3, 32 epochs, FP16 or BF16, 64 isotropic views
with sides from {128, 256, 512, 1024}), ``serve`` (Poisson request stream on
resident 128^3..512^3 FP16 stacks) and ``large`` (512 x 512 x 2048, 40 epochs,
BF16, 1024^2 views).

Prints one JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q))


# --------------------------------------------------------------------------- helpers

def make_jet_stack(dart, torch, dims, n_epochs, seed, gamma, knots, storage, keep_host):
    import synth
    t0 = time.time()
    j, b, times = synth.jet_torch(dims, n_epochs, seed, gamma_spine=gamma, n_knots=knots)
    torch.cuda.synchronize()
    host = None
    if keep_host:
        host = (j.cpu().numpy(), b.cpu().numpy())
    st = dart.dart_load_epochs(dims, (1.0, 1.0, 1.0), times, j, b, storage)
    torch.cuda.synchronize()
    del j, b
    torch.cuda.empty_cache()
    log(f"stack {dims} x {n_epochs} epochs generated and loaded in {time.time() - t0:.1f} s")
    return st, times, host


def time_steps(torch, stream, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in evs]
    return wall, per


def bandwidth_probe(dart, torch, stream, nbytes=4 << 30, reps=10):
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dart.dart_bandwidth_probe(dst, src, nbytes, 2, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        a.record(stream)
        dart.dart_bandwidth_probe(dst, src, nbytes, reps, stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes * reps / (ms * 1e-3) / 1e9


def oracle_sample(host, times, views, n_rays, seed, threads):
    """Runs the FP64 oracle on n_rays random pixels spread over the views.
    Returns (per-view list of (pixels, values), total cell-steps, seconds)."""
    import oracle
    j, b = host
    ost = oracle.Stack(j, b, times)
    rng = np.random.default_rng(seed)
    out, steps, secs = [], 0, 0.0
    per_view = max(1, n_rays // len(views))
    for v in views:
        pix = np.stack([rng.integers(0, v.width, per_view), rng.integers(0, v.height, per_view)],
                       axis=1).astype(np.int32)
        ov = oracle.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, v.t_obs,
                         v.alpha, v.flags & 7)
        t0 = time.perf_counter()
        val, n = oracle.render(ost, ov, pixels=pix, threads=threads)
        secs += time.perf_counter() - t0
        steps += n
        out.append((pix, val))
    return out, steps, secs


def pix_err(got, ref, img_max):
    floor = 1e-3 * img_max
    return np.abs(got - ref) / np.maximum(np.abs(ref), floor)


# --------------------------------------------------------------------------- workloads

def run_render_workload(args, dart, torch, name, dims, n_epochs, storage, views_spec, gamma,
                        knots, seed, rec_bytes, dtype_name):
    stream = torch.cuda.Stream()
    keep_host = not args.no_cpu_baseline or args.check
    st, times, host = make_jet_stack(dart, torch, dims, n_epochs, seed, gamma, knots, storage,
                                     keep_host)
    L = math.sqrt(sum(float(d) ** 2 for d in dims))
    views = [dart.View(th, ph, P, P, L / P, 0.0, alpha) for th, ph, P, alpha in views_spec]
    imgs = [torch.zeros((v.height, v.width), dtype=torch.float32, device="cuda") for v in views]
    stacks = [st] * len(views)
    n_img = len(views)

    tuning = None
    if args.tuning:
        tw, th_, w, order, orient, bx, by, bz = [int(x) for x in args.tuning.split(",")]
        dart.dart_stack_rebrick(st, (bx, by, bz), stream)
        dart.dart_set_tuning(tw, th_, w, order, orient)
        tuning = {"tile": [tw, th_], "waves_per_cu": w, "order": order, "orient": orient,
                  "brick": [bx, by, bz], "fixed": True}
        log(f"fixed tuning: {tuning}")
    elif args.autotune:
        t0 = time.time()
        best, ms = dart.dart_autotune(stacks, views, rebrick=args.rebrick, stream=stream)
        info = dart.dart_stack_get_info(st)
        tuning = {"tile": [best.tile_w, best.tile_h], "waves_per_cu": best.waves_per_cu,
                  "order": best.order, "orient": best.orient, "brick": list(info.brick),
                  "best_ms": ms, "tune_s": time.time() - t0}
        log(f"autotune ({time.time() - t0:.1f} s): {tuning}")

    # untimed: cell-steps and flux of every image, compulsory samples
    with torch.cuda.stream(stream):
        flux, steps = dart.dart_render_batch(stacks, views, imgs, stream=stream)
    cell_steps = int(np.sum(steps))
    samples = [dart.dart_count_samples(st, v, stream) for v in views] if not args.profile else []
    out_bytes = sum(4 * v.width * v.height for v in views)
    compulsory = (sum(samples) * rec_bytes + out_bytes) if samples else None
    log(f"{n_img} images, {cell_steps:.4e} cell-steps per step, samples {sum(samples) if samples else 'n/a'}")

    def batched():
        dart.dart_render_batch(stacks, views, imgs, stream=stream, stats=False)

    wall, per = time_steps(torch, stream, batched, args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    kernel_ms = float(np.mean(per))
    log(f"batched: {ms_step:.3f} ms/step wall, {kernel_ms:.3f} ms/step events")

    plain_imgs = [torch.zeros_like(im) for im in imgs]

    def plain():
        for v, im in zip(views, plain_imgs):
            dart.dart_render(st, v, im, stream=stream, stats=False)

    res = {}
    if not args.profile:
        pwall, pper = time_steps(torch, stream, plain, args.steps, args.warmup)
        pms = 1e3 * pwall / args.steps
        log(f"plain: {pms:.3f} ms/step")
        torch.cuda.synchronize()
        same = all(torch.equal(a, b) for a, b in zip(imgs, plain_imgs))
        res["plain"] = {"ms_per_step": pms, "images_per_s": n_img / (pms * 1e-3),
                        "cell_steps_per_s": cell_steps / (pms * 1e-3),
                        "identical_to_batched": bool(same)}

    # accuracy on sampled pixels against the FP64 oracle (dequantised inputs)
    if args.check and host is not None:
        jq, bq = dequantised(host, dtype_name)
        samp, _, _ = oracle_sample((jq, bq), times, views, args.check_rays, 7, None)
        errs = []
        for (pix, val), im in zip(samp, imgs):
            g = im.cpu().numpy()
            got = g[pix[:, 1], pix[:, 0]].astype(np.float64)
            errs.append(pix_err(got, val, float(np.abs(g).max())).max())
        res["accuracy"] = {"max_pixel_rel_err": float(max(errs)), "sampled_pixels": int(args.check_rays),
                           "tolerance": 1e-5 if dtype_name == "f32" else 2e-3}
        log(f"accuracy: max per-pixel rel err {max(errs):.3e} over {args.check_rays} sampled pixels")

    cpu = None
    if not args.no_cpu_baseline and host is not None:
        jq, bq = dequantised(host, dtype_name)
        threads = os.cpu_count() or 1
        # calibrate on a small sample, then size the sample for ~10-20 s
        _, n0, s0 = oracle_sample((jq, bq), times, views, 256 * n_img, 11, threads)
        rays = int(min(1 << 20, max(256 * n_img, 256 * n_img * 12.0 / max(s0, 1e-3))))
        _, n1, s1 = oracle_sample((jq, bq), times, views, rays, 12, threads)
        cpu = {"value": n1 / s1, "unit": "cell-steps/s", "cores": threads, "kind": "oracle",
               "sample": f"{rays} random pixels over the {n_img} views ({n1} cell-steps, {s1:.1f} s)",
               "images_per_s_equiv": (n1 / s1) / (cell_steps / n_img)}
        log(f"cpu oracle: {n1 / s1:.3e} cell-steps/s on {threads} threads")

    # in profile mode a 1 GiB copy (2 launches) runs as the counter calibration kernel
    bw = bandwidth_probe(dart, torch, stream, nbytes=(1 << 30) if args.profile else (4 << 30),
                         reps=2 if args.profile else 10)
    achieved = compulsory / (kernel_ms * 1e-3) / 1e9 if compulsory else None
    roof = None
    if achieved is not None:
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": "k_batch (persistent tile-queue render)",
                "bytes_per_launch": compulsory,
                "bytes_definition": "distinct (cell, epoch) records with positive weight x record "
                                    "bytes + image bytes",
                "measured_copy_gbs": bw,
                "frac_of_measured_copy": (achieved / bw) if bw else None,
                "gather_bytes_gbs": cell_steps * 2 * rec_bytes / (kernel_ms * 1e-3) / 1e9}
    value = cell_steps / (ms_step * 1e-3)
    line = {
        "metric": "cell-steps/s & images/s (batched vs plain kernel) at 1e-5 rel; p50/p99 ms",
        "value": value, "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype_name, "data": "synthetic",
        "config": {"workload": name, "grid": list(dims), "epochs": n_epochs,
                   "images_per_step": n_img, "pixels_per_step": sum(v.width * v.height for v in views),
                   "cell_steps_per_step": cell_steps, "storage": dtype_name},
        "images_per_s": n_img / (ms_step * 1e-3),
        "p50_ms": pct(per, 50), "p99_ms": pct(per, 99),
        "roofline": roof, "cpu_baseline": cpu,
    }
    if "plain" in res:
        line["plain"] = res["plain"]
        line["speedup_images_per_s_vs_plain"] = line["images_per_s"] / res["plain"]["images_per_s"]
    if "accuracy" in res:
        line["accuracy"] = res["accuracy"]
    if tuning:
        line["tuning"] = tuning
    return line


def dequantised(host, dtype_name):
    import synth
    j, b = host
    if dtype_name == "f32":
        return j, b
    f = synth.round_f16 if dtype_name == "f16" else synth.round_bf16
    return f(j), f(b)


# --------------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="jet", choices=["jet"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check", action="store_true", default=True)
    ap.add_argument("--no-check", dest="check", action="store_false")
    ap.add_argument("--check-rays", type=int, default=2048)
    ap.add_argument("--no-autotune", dest="autotune", action="store_false", default=True,
                    help="skip the (untimed) tile / occupancy / brick-shape tuning")
    ap.add_argument("--no-rebrick", dest="rebrick", action="store_false", default=True)
    ap.add_argument("--tuning", default=None,
                    help="fixed launch shape instead of autotuning: "
                         "tile_w,tile_h,waves_per_cu,order,orient,brick_x,brick_y,brick_z")
    ap.add_argument("--profile", action="store_true",
                    help="timed batched loop only (for rocprofv3 runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)
    if args.profile:
        args.no_cpu_baseline = True
        args.check = False

    import torch
    import paper_2609_09322_amd as dart
    torch.cuda.set_device(0)

    if args.workload == "jet":
        views = [(th, 0.0, 512, 0.6) for th in (10.0, 30.0, 60.0, 90.0)]
        line = run_render_workload(
            args, dart, torch, "jet 256x256x512, 16 epochs, FP32, 4 views 512^2 (theta 10/30/60/90)",
            (256, 256, 512), 16, dart.DART_F32, views, 5.0, 4, 2, 16, "f32")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
