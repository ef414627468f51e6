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
resident 128^3..512^3 FP16 stacks), ``large`` (512 x 512 x 2048, 40 epochs,
BF16, 1024^2 views), ``labelled`` (the jet with its core refined), ``stream``
(the jet's epochs streamed from host memory) and ``vector`` (the jet with three
emissivity components).

Prints one JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
TRAFFIC_TABLE = os.path.join(ROOT, "profiles", "k_batch_traffic.txt")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_id():
    """Identity of the render kernels' source: counter measurements taken on
    other sources do not describe the kernel that runs."""
    h = hashlib.sha256()
    for f in ("dart_kernels.hip", "dart_internal.h"):
        with open(os.path.join(ROOT, "paper_2609_09322_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def tuning_key(t):
    """The --tuning string of a launch shape: tile_w,tile_h,waves_per_cu,order,
    orient,brick_x,brick_y,brick_z,depth_sync,cells_per_batch."""
    return ",".join(str(x) for x in (t["tile"][0], t["tile"][1], t["waves_per_cu"], t["order"],
                                     t["orient"], *t["brick"], t.get("depth_sync", 0),
                                     t.get("cells_per_batch", 4) or 4))


def tuning_dict(best, info):
    return {"tile": [best.tile_w, best.tile_h], "waves_per_cu": best.waves_per_cu,
            "order": best.order, "orient": best.orient, "brick": list(info.brick),
            "depth_sync": best.depth_sync, "cells_per_batch": best.cells_per_batch or 4}


def apply_fixed_tuning(dart, st, spec, stream):
    f = normalise_tuning(spec)
    tw, th_, w, order, orient, bx, by, bz, sync, k = [int(x) for x in f.split(",")]
    dart.dart_stack_rebrick(st, (bx, by, bz), stream)
    dart.dart_set_tuning(tw, th_, w, order, orient, sync, k)
    return {"tile": [tw, th_], "waves_per_cu": w, "order": order, "orient": orient,
            "brick": [bx, by, bz], "depth_sync": sync, "cells_per_batch": k, "fixed": True}


def normalise_tuning(spec):
    """--tuning with the optional depth_sync (0) and cells_per_batch (4) fields
    filled in."""
    n = spec.count(",")
    return spec + (",0,4" if n == 7 else ",4" if n == 8 else "")


def counter_row(workload, tuning):
    """The committed counter-table row for this workload, this kernel source and
    this launch shape: (fetch bytes, write bytes, L2 hit rate or None, source
    text), or (None, None, None, reason) when there is none."""
    if not tuning:
        return None, None, None, "no launch shape"
    key, kid = tuning_key(tuning), kernel_source_id()
    rows = []
    if os.path.exists(TRAFFIC_TABLE):
        with open(TRAFFIC_TABLE) as fh:
            for ln in fh:
                f = ln.split()
                if len(f) >= 5 and not ln.startswith("#"):
                    rows.append(f)
    for f in rows:
        if f[0] == workload and f[1] == kid and f[2] == key:
            hit = float(f[5]) if len(f) >= 6 else None
            return (float(f[3]), float(f[4]), hit,
                    f"counters for {workload}, tuning {key}, kernel {kid}")
    return None, None, None, f"no counter row for {workload}, tuning {key}, kernel {kid}"


def measured_traffic(workload, tuning):
    """HBM bytes per k_batch launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)
    from the committed counter table, when it holds a row for this workload,
    this kernel source and this launch shape; otherwise None and the reason."""
    fetch, write, _, src = counter_row(workload, tuning)
    return (fetch + write if fetch is not None else None), src


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q))


# --------------------------------------------------------------------------- helpers

def host_copy(j_dev, b_dev, kind):
    """Host copy of device float32 fields in the oracle's encoding for a stack
    stored as `kind` (float32, binary16, or bfloat16 bit patterns), converted
    one epoch at a time."""
    import synth
    if kind == "f32":
        return j_dev.cpu().numpy(), b_dev.cpu().numpy()
    dt = np.float16 if kind == "f16" else np.uint16
    conv = synth.to_f16 if kind == "f16" else synth.to_bf16_bits
    jh = np.empty(tuple(j_dev.shape), dtype=dt)
    bh = np.empty(tuple(b_dev.shape), dtype=dt)
    for m in range(j_dev.shape[0]):
        jh[m] = conv(j_dev[m].cpu().numpy())
        bh[m] = conv(b_dev[m].cpu().numpy())
    return jh, bh


def make_jet_stack(dart, torch, dims, n_epochs, seed, gamma, knots, storage, kind, keep_host,
                   keep_source=False):
    """The seeded jet stack, loaded from device-generated FP32 fields.  Returns
    (stack, epoch times, host copy in the stored encoding or None, host copy of
    the FP32 source fields or None)."""
    import synth
    t0 = time.time()
    j, b, times = synth.jet_torch(dims, n_epochs, seed, gamma_spine=gamma, n_knots=knots)
    torch.cuda.synchronize()
    host = host_copy(j, b, kind) if keep_host else None
    src = None
    if keep_source:
        src = host if kind == "f32" else (j.cpu().numpy(), b.cpu().numpy())
    st = dart.dart_load_epochs(dims, (1.0, 1.0, 1.0), times, j, b, storage)
    torch.cuda.synchronize()
    del j, b
    torch.cuda.empty_cache()
    log(f"stack {dims} x {n_epochs} epochs ({kind}) generated and loaded in {time.time() - t0:.1f} s")
    return st, times, host, src


def workload_key(args):
    """Row key of the counter table: the workload, its storage type for the
    batch, and the options that change the launch."""
    return ((args.workload if args.workload != "batch" else f"batch-{args.storage}")
            + ("-exact" if args.exact_time else "")
            + (f"-sides{args.sides}" if getattr(args, "sides", None) else ""))


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


def gather_probe(dart, torch, stream, nbytes=4 << 30, reps=10):
    """GB/s of a gather over scattered whole 128-B lines (dart_gather_probe):
    the reference for a kernel that gathers lines from scattered addresses."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dart.dart_gather_probe(src, nbytes, 2, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        a.record(stream)
        dart.dart_gather_probe(src, nbytes, reps, stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    del src
    torch.cuda.empty_cache()
    return float(nbytes) * reps / (ms * 1e-3) / 1e9


def read_probe(dart, torch, stream, nbytes=4 << 30, reps=10):
    """GB/s of a read-only pass over nbytes (dart_bandwidth_probe without a
    destination): the reference for a kernel that mostly reads."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dart.dart_bandwidth_probe(None, src, nbytes, 2, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        a.record(stream)
        dart.dart_bandwidth_probe(None, src, nbytes, reps, stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    del src
    torch.cuda.empty_cache()
    return nbytes * reps / (ms * 1e-3) / 1e9


def oracle_sample(host, times, views, n_rays, seed, threads, kind="f32"):
    """Runs the FP64 oracle on n_rays random pixels spread over the views.
    Returns (per-view list of (pixels, values), total cell-steps, seconds)."""
    import oracle
    j, b = host
    ost = oracle.Stack(j, b, times, encoding=kind)
    rng = np.random.default_rng(seed)
    out, steps, secs = [], 0, 0.0
    per_view = max(1, n_rays // len(views))
    for v in views:
        pix = np.stack([rng.integers(0, v.width, per_view), rng.integers(0, v.height, per_view)],
                       axis=1).astype(np.int32)
        ov = oracle.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, v.t_obs,
                         v.alpha, (v.flags & 7) | (oracle.EXACT_TIME if v.flags & 0x100 else 0))
        t0 = time.perf_counter()
        val, n = oracle.render(ost, ov, pixels=pix, threads=threads)
        secs += time.perf_counter() - t0
        steps += n
        out.append((pix, val))
    return out, steps, secs


def pix_err(got, ref, img_max):
    floor = 1e-3 * img_max
    return np.abs(got - ref) / np.maximum(np.abs(ref), floor)


def whole_image_accuracy(host, src, times, views, imgs, flux, steps, idx, kind, tol):
    """Every pixel, the flux and the cell-steps of views[idx] against the FP64
    oracle on the stored values (the error floor from the oracle image), and
    the storage error: the oracle on the stored values against the oracle on
    the FP32 source fields (for 16-bit storage; zero for FP32)."""
    import oracle
    ost = oracle.Stack(host[0], host[1], times, encoding=kind)
    sst = oracle.Stack(src[0], src[1], times) if (src is not None and kind != "f32") else None
    worst = dict(pix=0.0, flux=0.0, steps=0.0, s_pix=0.0, s_flux=0.0)
    t0 = time.perf_counter()
    for k in idx:
        v = views[k]
        ov = oracle.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, v.t_obs,
                         v.alpha, (v.flags & 7) | (oracle.EXACT_TIME if v.flags & 0x100 else 0))
        ref, rsteps = oracle.render(ost, ov)
        rflux = oracle.flux(ref, ov)
        g = imgs[k].cpu().numpy().astype(np.float64)
        worst["pix"] = max(worst["pix"], float(pix_err(g, ref, float(np.abs(ref).max())).max()))
        worst["flux"] = max(worst["flux"], abs(float(flux[k]) / rflux - 1.0))
        worst["steps"] = max(worst["steps"], abs(int(steps[k]) - rsteps) / max(rsteps, 1))
        if sst is not None:
            sref, _ = oracle.render(sst, ov)
            sflux = oracle.flux(sref, ov)
            worst["s_pix"] = max(worst["s_pix"],
                                 float(pix_err(ref, sref, float(np.abs(sref).max())).max()))
            worst["s_flux"] = max(worst["s_flux"], abs(rflux / sflux - 1.0))
    out = {"max_pixel_rel_err": worst["pix"], "flux_rel_err": worst["flux"],
           "cell_steps_rel_diff": worst["steps"], "images_checked_whole": len(idx),
           "tolerance": {"pixel": tol, "flux": 1e-6, "cell_steps": 1e-5},
           "within_tolerance": bool(worst["pix"] <= tol and worst["flux"] <= 1e-6
                                    and worst["steps"] <= 1e-5),
           "against": "FP64 oracle on the stored values, every pixel of the checked images",
           "oracle_s": time.perf_counter() - t0}
    if kind == "f32":
        out["storage_error"] = {"max_pixel_rel_err": 0.0, "flux_rel_err": 0.0,
                                "note": "FP32 storage holds the FP32 source fields exactly"}
    elif sst is not None:
        out["storage_error"] = {"max_pixel_rel_err": worst["s_pix"], "flux_rel_err": worst["s_flux"],
                                "against": "FP64 oracle on the FP32 source fields (reported, "
                                           "not graded)"}
    return out


# --------------------------------------------------------------------------- workloads

def run_render_workload(args, dart, torch, name, dims, n_epochs, storage, views_spec, gamma,
                        knots, seed, rec_bytes, dtype_name, check_views=None, tune_views=None):
    """check_views: the first check_views views are checked whole against the
    oracle (every pixel, flux, cell-steps, storage error); None checks them all."""
    stream = torch.cuda.Stream()
    wkey = workload_key(args)
    keep_host = not args.no_cpu_baseline or args.check
    st, times, host, src = make_jet_stack(dart, torch, dims, n_epochs, seed, gamma, knots, storage,
                                          dtype_name, keep_host, keep_source=args.check)
    L = math.sqrt(sum(float(d) ** 2 for d in dims))
    vflags = dart.DART_EXACT_TIME if args.exact_time else 0
    views = [dart.View(th, ph, P, P, L / P, 0.0, alpha, vflags) for th, ph, P, alpha in views_spec]
    imgs = [torch.zeros((v.height, v.width), dtype=torch.float32, device="cuda") for v in views]
    stacks = [st] * len(views)
    n_img = len(views)

    tuning = None
    if args.tuning:
        tuning = apply_fixed_tuning(dart, st, args.tuning, stream)
        log(f"fixed tuning: {tuning}")
    elif args.autotune:
        t0 = time.time()
        tv = views if tune_views is None else views[:tune_views]
        best, ms = dart.dart_autotune([st] * len(tv), tv, rebrick=args.rebrick, stream=stream)
        tuning = tuning_dict(best, dart.dart_stack_get_info(st))
        tuning.update(best_ms=ms, tune_s=time.time() - t0)
        log(f"autotune ({time.time() - t0:.1f} s): {tuning}")

    # untimed: cell-steps and flux of every image, compulsory samples
    with torch.cuda.stream(stream):
        flux, steps = dart.dart_render_batch(stacks, views, imgs, stream=stream)
    cell_steps = int(np.sum(steps))
    samples = [dart.dart_count_samples(st, v, stream) for v in views] if not args.profile else []
    out_bytes = sum(4 * v.width * v.height for v in views)
    # compulsory bytes as the metric defines them: distinct positive-weight
    # (cell, epoch) samples x record bytes + images; and the bytes renders of
    # this layout must read (emissivity plane, whole records where marked)
    compulsory = (sum(samples) * rec_bytes + out_bytes) if samples else None
    lines = [dart.dart_count_lines(st, v, stream) for v in views] if not args.profile else []
    line_bytes = (sum(lines) * 128 + out_bytes) if lines else None
    counted = [dart.dart_count_bytes(st, v, stream) for v in views] if not args.profile else []
    plane_bytes = (sum(c for c, _ in counted) + out_bytes) if counted else None
    plane_lines = (sum(l for _, l in counted) + out_bytes) if counted else None
    # (renders read an emissivity plane when the counted bytes fall below whole records)
    plane = bool(counted) and plane_bytes < compulsory
    log(f"{n_img} images, {cell_steps:.4e} cell-steps per step, samples {sum(samples) if samples else 'n/a'}, "
        f"compulsory {compulsory}, line bytes {line_bytes}, emissivity plane {plane} "
        f"(bytes {plane_bytes}, line bytes {plane_lines})")

    def batched():
        dart.dart_render_batch(stacks, views, imgs, stream=stream, stats=False)

    wall, per = time_steps(torch, stream, batched, args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    kernel_ms = float(np.mean(per))
    log(f"batched: {ms_step:.3f} ms/step wall, {kernel_ms:.3f} ms/step events")

    # the same batched render reading whole records for every cell
    ro_views = [dart.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, v.t_obs,
                          v.alpha, v.flags | dart.DART_RECORDS_ONLY) for v in views]
    ro_imgs = [torch.zeros_like(im) for im in imgs]

    def records_only():
        dart.dart_render_batch(stacks, ro_views, ro_imgs, stream=stream, stats=False)

    ro = None
    if plane and not args.profile:
        rwall, rper = time_steps(torch, stream, records_only, args.steps, args.warmup)
        torch.cuda.synchronize()
        ro = {"ms_per_step": 1e3 * rwall / args.steps, "kernel_ms": float(np.mean(rper)),
              "images_per_s": n_img / rwall * args.steps,
              "identical_images": bool(all(torch.equal(a, b) for a, b in zip(imgs, ro_imgs))),
              "note": "the same batched call with DART_RECORDS_ONLY: whole records for every "
                      "cell instead of the emissivity plane"}
        log(f"records only: {ro}")
    del ro_imgs

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
        # the plain kernel with a host synchronisation after every image
        def plain_sync():
            for v, im in zip(views, plain_imgs):
                dart.dart_render(st, v, im, stream=stream, stats=False)
                stream.synchronize()

        swall, _ = time_steps(torch, stream, plain_sync, max(1, args.steps // 2), 1)
        sms = 1e3 * swall / max(1, args.steps // 2)
        res["plain"] = {"ms_per_step": pms, "images_per_s": n_img / (pms * 1e-3),
                        "cell_steps_per_s": cell_steps / (pms * 1e-3),
                        "identical_to_batched": bool(same),
                        "synchronised_ms_per_step": sms,
                        "note": "one launch per image back to back on one stream (the stronger "
                                "of the two); synchronised: a host wait after every image"}
        # the same batched call handing back pinned host images (the render
        # waits for its device-to-host copies): the PCIe-inclusive rate
        host_imgs = [torch.empty((v.height, v.width), dtype=torch.float32, pin_memory=True)
                     for v in views]

        def to_host():
            dart.dart_render_batch([st] * n_img, views, host_imgs,
                                   stream=stream, stats=False)

        hwall, _ = time_steps(torch, stream, to_host, max(1, args.steps // 2), 1)
        hms = 1e3 * hwall / max(1, args.steps // 2)
        res["host_images"] = {"ms_per_step": hms, "images_per_s": n_img / (hms * 1e-3),
                              "note": "batched render into pinned host images, "
                                      "device-to-host copies included"}
        log(f"host images: {hms:.3f} ms/step")

    # accuracy of whole images against the FP64 oracle (on the stored values),
    # and the storage error (the stored values against the FP32 source fields)
    if args.check and host is not None:
        idx = list(range(n_img if check_views is None else min(check_views, n_img)))
        acc = whole_image_accuracy(host, src, times, views, imgs, flux, steps, idx, dtype_name,
                                   1e-5 if dtype_name == "f32" else 2e-3)
        res["accuracy"] = acc
        log(f"accuracy ({len(idx)} whole images): max per-pixel rel err "
            f"{acc['max_pixel_rel_err']:.3e}, flux {acc['flux_rel_err']:.2e}, cell-steps "
            f"{acc['cell_steps_rel_diff']:.2e}; storage error {acc.get('storage_error')}")
    del src

    cpu = None
    if not args.no_cpu_baseline and host is not None:
        # the host cores this process may use (OMP_NUM_THREADS caps it where set)
        threads = min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS") or 1 << 10))
        # calibrate on a sample of ~1 s, then size the timed sample for ~15 s
        cal = 8192 * max(1, 16 // n_img) * n_img
        _, n0, s0 = oracle_sample(host, times, views, cal, 11, threads, dtype_name)
        rays = int(min(1 << 25, max(cal, cal * 15.0 / max(s0, 1e-3))))
        _, n1, s1 = oracle_sample(host, times, views, rays, 12, threads, dtype_name)
        # and on one core, over a sample of ~5 s
        r1 = max(n_img, int(rays * 5.0 / max(s1 * threads, 1e-3)))
        _, m1, t1 = oracle_sample(host, times, views, r1, 13, 1, dtype_name)
        cpu = {"value": n1 / s1, "unit": "cell-steps/s", "cores": threads, "kind": "oracle",
               "sample": f"{rays} random pixels over the {n_img} views ({n1} cell-steps, {s1:.1f} s)",
               "images_per_s_equiv": (n1 / s1) / (cell_steps / n_img),
               "one_core": {"value": m1 / t1, "sample": f"{r1} random pixels ({m1} cell-steps, "
                                                       f"{t1:.1f} s)"},
               "cpu_model": cpu_model()}
        log(f"cpu oracle: {n1 / s1:.3e} cell-steps/s on {threads} threads, {m1 / t1:.3e} on one")

    # in profile mode a 1 GiB copy (2 launches) runs as the counter calibration kernel
    bw = bandwidth_probe(dart, torch, stream, nbytes=(1 << 30) if args.profile else (4 << 30),
                         reps=2 if args.profile else 10)
    rd = None if args.profile else read_probe(dart, torch, stream)
    gp = None if args.profile else gather_probe(dart, torch, stream)
    achieved = compulsory / (kernel_ms * 1e-3) / 1e9 if compulsory else None
    roof = None
    if achieved is not None:
        traffic, tsrc = measured_traffic(wkey, tuning)
        l2_hit = counter_row(wkey, tuning)[2]
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": tsrc,
                "l2_hit_rate": l2_hit,
                "l2_hit_rate_definition": "TCC_HIT / (TCC_HIT + TCC_MISS) of the render kernel, "
                                          "from the same counter row as traffic",
                "fetched_over_line_bytes": (traffic / line_bytes) if (traffic and line_bytes)
                else None,
                "line_over_compulsory_bytes": (line_bytes / compulsory) if line_bytes else None,
                "traffic_gbs": traffic / (kernel_ms * 1e-3) / 1e9 if traffic else None,
                "kernel": "k_batch (persistent tile-queue render)",
                "bytes_per_launch": compulsory,
                "bytes_definition": "distinct (cell, epoch) records with positive weight x record "
                                    "bytes + image bytes",
                "emissivity_plane": plane,
                "plane_bytes_per_launch": plane_bytes if plane else None,
                "plane_bytes_definition": "the bytes a render of this layout must read: one "
                                          "emissivity-plane value per positive-weight sample, "
                                          "+ the whole record where marked (velocity), + images; "
                                          "with the plane, achieved counts record bytes the "
                                          "kernel does not move, so traffic (counters) is the "
                                          "HBM truth",
                "plane_gbs": plane_bytes / (kernel_ms * 1e-3) / 1e9 if plane else None,
                "plane_line_bytes_per_launch": plane_lines if plane else None,
                "measured_copy_gbs": bw,
                "frac_of_measured_copy": (achieved / bw) if bw else None,
                "measured_read_gbs": rd,
                "frac_of_measured_read": (achieved / rd) if rd else None,
                "fetched_over_measured_read": (traffic / (kernel_ms * 1e-3) / 1e9 / rd)
                if (traffic and rd) else None,
                "measured_gather_gbs": gp,
                "frac_of_measured_gather": (achieved / gp) if gp else None,
                "fetched_over_measured_gather": (traffic / (kernel_ms * 1e-3) / 1e9 / gp)
                if (traffic and gp) else None,
                "gather_bytes_gbs": cell_steps * 2 * rec_bytes / (kernel_ms * 1e-3) / 1e9,
                "line_bytes_per_launch": line_bytes,
                "line_bytes_definition": "distinct 128-B lines of the resident records holding "
                                         "those records x 128 + image bytes (the fewest bytes a "
                                         "line-granular fetch of whole records can move)",
                "line_gbs": line_bytes / (kernel_ms * 1e-3) / 1e9 if line_bytes else None}
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
        "step_ms_p50": pct(per, 50), "step_ms_p99": pct(per, 99),
        "roofline": roof, "cpu_baseline": cpu,
    }
    if "host_images" in res:
        line["host_images"] = res["host_images"]
    if ro is not None:
        line["records_only"] = ro
    if "plain" in res:
        line["plain"] = res["plain"]
        line["speedup_images_per_s_vs_plain"] = line["images_per_s"] / res["plain"]["images_per_s"]
    if "accuracy" in res:
        line["accuracy"] = res["accuracy"]
    if tuning:
        line["tuning"] = tuning
    return line


def build_stack_incremental(dart, torch, dims, n_epochs, seed, gamma, knots, storage,
                            chunk_bytes=8 << 30, z_slab=None):
    """Creates a stack and fills it a few epochs at a time from device-generated
    float32 fields (the two-phase load for stacks too large to stage whole).
    z_slab=(z0, nz_slab) makes a stack of those z-layers of the domain `dims`,
    placed in the domain so that its renders are partial renders of the whole."""
    import synth
    times = synth.jet_times(dims, n_epochs)
    nx, ny, nz = dims
    params = synth.jet_params(dims, seed, gamma_spine=gamma, n_knots=knots)
    if z_slab is not None:
        params.z_begin, params.z_count = int(z_slab[0]), int(z_slab[1])
    st = dart.dart_stack_create((nx, ny, params.z_count), (1.0, 1.0, 1.0), times, storage)
    if z_slab is not None:
        dart.dart_stack_set_placement(st, (0.0, 0.0, float(params.z_begin)),
                                      (0.5 * nx, 0.5 * ny, 0.5 * nz))
    nz = params.z_count
    per_epoch = nx * ny * nz * 16
    chunk = max(1, min(n_epochs, chunk_bytes // per_epoch))
    stream = torch.cuda.current_stream()
    jbuf = torch.empty((chunk, nz, ny, nx), dtype=torch.float32, device="cuda")
    bbuf = torch.empty((chunk, nz, ny, nx, 3), dtype=torch.float32, device="cuda")
    for m0 in range(0, n_epochs, chunk):
        c = min(chunk, n_epochs - m0)
        synth.jet_fill_device(params, times[m0:m0 + c], jbuf.data_ptr(), bbuf.data_ptr(),
                              stream.cuda_stream)
        dart.dart_stack_set_epochs(st, m0, jbuf[:c], bbuf[:c], stream=stream)
    torch.cuda.synchronize()
    del jbuf, bbuf
    torch.cuda.empty_cache()
    return st, times


def served_cpu_baseline(dart, torch, stacks, reqs, seconds=12.0):
    """The oracle on random pixels of the served requests that use the 128^3 and
    256^3 stacks (their stored values read back with dart_stack_read_epoch and
    held as binary16 on the host; the 512^3 stacks are left out to bound host
    memory), on every host core this process may use."""
    import oracle
    threads = min(len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS") or 1 << 10))
    host = {}
    for st, n, M in stacks:
        if n > 256:
            continue
        jh = np.empty((M, n, n, n), dtype=np.float16)
        bh = np.empty((M, n, n, n, 3), dtype=np.float16)
        jd = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
        bd = torch.empty((n, n, n, 3), dtype=torch.float32, device="cuda")
        for m in range(M):
            dart.dart_stack_read_epoch(st, m, jd, bd)
            torch.cuda.synchronize()
            jh[m] = jd.cpu().numpy().astype(np.float16)   # exact: the values are binary16
            bh[m] = bd.cpu().numpy().astype(np.float16)
        host[id(st)] = oracle.Stack(jh, bh, synth_times(n, M), encoding="f16")
        del jd, bd
    rng = np.random.default_rng(14)
    cand = [(s, v) for s, v in reqs if id(s) in host]
    done_steps, secs, rays = 0, 0.0, 0
    while secs < seconds and cand:
        s, v = cand[int(rng.integers(0, len(cand)))]
        pix = np.stack([rng.integers(0, v.width, 4096), rng.integers(0, v.height, 4096)],
                       axis=1).astype(np.int32)
        ov = oracle.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, v.t_obs,
                         v.alpha, v.flags & 7)
        t0 = time.perf_counter()
        _, n_steps = oracle.render(host[id(s)], ov, pixels=pix, threads=threads)
        secs += time.perf_counter() - t0
        done_steps += n_steps
        rays += len(pix)
    return {"value": done_steps / max(secs, 1e-9), "unit": "cell-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{rays} random pixels of served requests on the 128^3 and 256^3 stacks "
                      f"({done_steps} cell-steps, {secs:.1f} s)",
            "cpu_model": cpu_model()}


def synth_times(n, M):
    import synth
    return synth.jet_times((n, n, n), M)


def run_serve_workload(args, dart, torch):
    """Poisson request stream on resident FP16 stacks through the server.

    Latency runs from each request's scheduled arrival to its completion: the
    submitter sleeps until the arrival time, submits at once (every request has
    its own output image, so it never waits for a buffer) and charges any
    lateness of the submission to the request."""
    import synth
    rng = np.random.default_rng(1004)
    specs = [(128, 8), (128, 32), (256, 16), (256, 32), (512, 8), (512, 32)]
    stacks = []
    t0 = time.time()
    for k, (n, M) in enumerate(specs):
        gamma = float(rng.uniform(2.0, 5.0))
        st, _ = build_stack_incremental(dart, torch, (n, n, n), M, 2000 + k, gamma, 4,
                                        dart.DART_F16)
        stacks.append((st, n, M))
    resident = sum(dart.dart_stack_get_info(s).device_bytes for s, _, _ in stacks)
    log(f"{len(stacks)} FP16 stacks resident ({resident / 1e9:.1f} GB) in {time.time() - t0:.1f} s")
    n_req, warm, rate = args.requests, args.serve_warmup, args.rate
    sizes = (128, 256, 512, 1024)
    reqs = []
    for q in range(n_req):
        s, n, M = stacks[int(rng.integers(0, len(stacks)))]
        P = int(rng.choice(sizes))
        th = math.degrees(math.acos(rng.uniform(-1.0, 1.0)))
        reqs.append((s, dart.View(th, float(rng.uniform(0, 360)), P, P,
                                  math.sqrt(3.0) * n / P, 0.0, float(rng.uniform(0.5, 1.0)))))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    # launch shape and bricks tuned on a sample of the requests (every stack
    # gets the same tuning; a wave launches with its first request's stack's)
    t0 = time.time()
    tune_stream = torch.cuda.Stream()
    best, best_ms = dart.dart_autotune([s for s, _ in reqs[:64]], [v for _, v in reqs[:64]],
                                       rebrick=args.rebrick, stream=tune_stream)
    tuning = tuning_dict(best, dart.dart_stack_get_info(stacks[0][0]))
    tuning.update(best_ms=best_ms, tune_s=time.time() - t0, tuned_on="the first 64 requests")
    log(f"autotune ({time.time() - t0:.1f} s): {tuning}")
    imgs = [torch.zeros((v.height, v.width), dtype=torch.float32, device="cuda") for _, v in reqs]
    srv = dart.dart_server_create(args.budget_gb << 30, max_inflight=1024, n_streams=3)

    def timeline_delta(a, b):
        w = max(1, b.waves_timed - a.waves_timed)
        out = {"waves": int(b.waves_timed - a.waves_timed)}
        for f in ("plan_ms", "enqueue_ms", "callback_to_retire_ms", "device_ms", "kernel_ms",
                  "stream_idle_ms"):
            out[f + "_per_wave"] = (getattr(b, f) - getattr(a, f)) / w
        out["kernel_ms_total"] = b.kernel_ms - a.kernel_ms
        return out

    def stream_run(arr, count):
        tickets, late = [], []
        start = time.perf_counter()
        for q in range(count):
            s, v = reqs[q]
            due = start + arr[q]
            delay = due - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            late.append(time.perf_counter() - due)
            tickets.append(dart.dart_submit(srv, s, v, imgs[q]))
        results = [dart.dart_wait(srv, t) for t in tickets]
        return results, np.asarray(late) * 1e3, time.perf_counter() - start

    tl0 = dart.dart_server_get_timeline(srv)
    results, late_ms, wall = stream_run(arrivals, n_req)
    tl1 = dart.dart_server_get_timeline(srv)
    lat_submit = np.array([r[2] for r in results[warm:]])
    lat = late_ms[warm:] + lat_submit
    steps_served = sum(r[1] for r in results[warm:])
    span = arrivals[-1] - arrivals[warm]
    log(f"served {n_req} requests at {rate}/s: from arrival p50 {np.percentile(lat, 50):.2f} ms, "
        f"p99 {np.percentile(lat, 99):.2f} ms (submission late by at most {late_ms.max():.2f} ms)")
    stats = dart.dart_server_get_stats(srv)
    # every served image against its solo render (the plain kernel, alone)
    torch.cuda.synchronize()
    same, checked = 0, 0
    for q in range(n_req):
        s, v = reqs[q]
        solo = torch.empty_like(imgs[q])
        dart.dart_render(s, v, solo, stats=False)
        same += int(torch.equal(solo, imgs[q]))
        checked += 1
    torch.cuda.synchronize()
    log(f"served images equal to their solo renders: {same} of {checked}")
    # saturation: the first sat_n requests offered at once
    sat_n = min(1000, n_req)
    tl2 = dart.dart_server_get_timeline(srv)
    sres, _, sat_wall = stream_run(np.zeros(sat_n), sat_n)
    tl3 = dart.dart_server_get_timeline(srv)
    sat_steps = sum(r[1] for r in sres)
    dart.dart_server_destroy(srv)
    # plain kernel, one request after the other, on the same requests
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for q in range(sat_n):
        s, v = reqs[q]
        dart.dart_render(s, v, imgs[q], stream=stream, stats=False)
    torch.cuda.synchronize()
    plain_wall = time.perf_counter() - p0
    # compulsory bytes of the saturation requests (records + images), and the
    # bytes renders of the resident layout must read (emissivity plane)
    comp, comp_plane = 0, 0
    for q in range(sat_n):
        s, v = reqs[q]
        comp += dart.dart_count_samples(s, v, stream) * 8 + 4 * v.width * v.height
        comp_plane += dart.dart_count_bytes(s, v, stream)[0] + 4 * v.width * v.height
    achieved = comp / sat_wall / 1e9
    cpu = None if args.no_cpu_baseline else served_cpu_baseline(dart, torch, stacks, reqs)
    return {
        "metric": "cell-steps/s & images/s (batched vs plain kernel) at 1e-5 rel; p50/p99 ms",
        "value": sat_steps / sat_wall, "unit": "cell-steps/s", "n_gpus": 1,
        "steps": n_req, "warmup": warm, "ms_per_step": 1e3 * sat_wall / sat_n,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": "served stream: Poisson %g req/s over 6 resident FP16 jet stacks "
                               "(128^3..512^3, 8-32 epochs), images 128^2..1024^2" % rate,
                   "requests": n_req, "resident_gb": resident / 1e9, "budget_gb": args.budget_gb},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "latency_definition": "scheduled arrival to completion (the completion callback of the "
                              "request's wave), after the first %d requests" % warm,
        "latency_from_submit_ms": {"p50": float(np.percentile(lat_submit, 50)),
                                   "p99": float(np.percentile(lat_submit, 99))},
        "submission_late_ms_max": float(late_ms.max()),
        "offered_req_per_s": rate, "served_req_per_s": (n_req - warm) / max(span, 1e-9),
        "served_cell_steps_per_s": steps_served / max(span, 1e-9),
        "saturation_images_per_s": sat_n / sat_wall,
        "saturation_cell_steps_per_s": sat_steps / sat_wall,
        "plain_images_per_s": sat_n / plain_wall,
        "speedup_images_per_s_vs_plain": plain_wall / sat_wall,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "traffic_source": "no counter run of the served mix",
                     "bytes_per_launch": None,
                     "bytes_definition": "compulsory bytes of the %d saturation requests "
                                         "(distinct positive-weight records x 8 B + images) over "
                                         "their wall time, host scheduling included" % sat_n,
                     "plane_bytes": comp_plane,
                     "plane_gbs": comp_plane / sat_wall / 1e9,
                     "plane_bytes_definition": "the bytes renders of the resident layout must "
                                               "read: 2 B emissivity-plane value per sample, + "
                                               "8 B records where marked, + images"},
        "waves": int(stats.waves), "max_wave_requests": int(stats.max_wave_requests),
        "timeline_poisson": timeline_delta(tl0, tl1),
        "timeline_saturation": timeline_delta(tl2, tl3),
        "tuning": tuning,
        "served_equals_solo": {"identical": same, "checked": checked,
                               "note": "each image served in the Poisson mix against the same "
                                       "request rendered alone by the plain kernel, bit for bit"},
        "cpu_baseline": cpu,
    }


class EpochReader:
    """Regenerates epochs of a jet stack on the device and reads each back once,
    as float32, into a two-slot pinned host ring (epoch e in slot e mod 2): the
    snapshot-outer oracle asks for epochs m and m+1 with m increasing."""

    def __init__(self, torch, dims, times, seed, gamma, knots):
        import synth
        self.torch, self.times = torch, np.asarray(times)
        self.params = synth.jet_params(dims, seed, gamma_spine=gamma, n_knots=knots)
        nx, ny, nz = dims
        self.j = torch.empty((1, nz, ny, nx), dtype=torch.float32, device="cuda")
        self.b = torch.empty((1, nz, ny, nx, 3), dtype=torch.float32, device="cuda")
        self.jr = torch.empty((2, nz, ny, nx), dtype=torch.float32, pin_memory=True)
        self.br = torch.empty((2, nz, ny, nx, 3), dtype=torch.float32, pin_memory=True)
        self.slot = [-1, -1]

    def _load(self, e):
        import synth
        if self.slot[e % 2] == e:
            return
        synth.jet_fill_device(self.params, self.times[e:e + 1], self.j.data_ptr(),
                              self.b.data_ptr(), self.torch.cuda.current_stream().cuda_stream)
        self.jr[e % 2].copy_(self.j[0])
        self.br[e % 2].copy_(self.b[0])
        self.torch.cuda.synchronize()
        self.slot[e % 2] = e

    def pair(self, m):
        self._load(m)
        self._load(m + 1)
        return self.jr.numpy(), self.br.numpy()


def streamed_oracle_flux(torch, dims, times, seed, gamma, knots, views, kind="f32_as_bf16",
                         with_source=False):
    """Whole images of several views by the snapshot-outer oracle: the outer
    loop runs over epoch intervals, each epoch is read back once.  Returns
    [(image, flux, cell_steps)] per view on the stored values (``kind``); with
    ``with_source`` also the same on the FP32 source fields, in the same pass
    (for the storage error), as a second list."""
    import oracle
    t = np.asarray(times)
    M = len(t)
    reader = EpochReader(torch, dims, t, seed, gamma, knots)
    ovs = [oracle.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, v.t_obs,
                       v.alpha, v.flags & 7) for v in views]
    kinds = [kind] + (["f32"] if with_source else [])
    imgs = {k: [np.zeros((v.height, v.width)) for v in views] for k in kinds}
    steps = {k: [0] * len(views) for k in kinds}
    for m in range(M - 1):
        js, bs = reader.pair(m)
        for enc in kinds:
            for k, ov in enumerate(ovs):
                steps[enc][k] += oracle.render_window(t, js, bs, m, ov, t[m], t[m + 1],
                                                      int(m == M - 2), imgs[enc][k],
                                                      encoding=enc, ring=True)
    del reader
    out = [[(img, oracle.flux(img, ov), n) for img, ov, n in zip(imgs[enc], ovs, steps[enc])]
           for enc in kinds]
    return (out[0], out[1]) if with_source else out[0]


def run_large_workload(args, dart, torch):
    """512 x 512 x 2048 cells, 40 epochs, BF16 (171.8 GB resident), 256 views at
    1024^2 with FP64 ray parameters and Kahan sums."""
    import synth
    dims, M, gamma, knots, seed = (512, 512, 2048), 40, 10.0, 12, 5
    t0 = time.time()
    st, times = build_stack_incremental(dart, torch, dims, M, seed, gamma, knots,
                                        dart.DART_BF16, chunk_bytes=9 << 30)
    info = dart.dart_stack_get_info(st)
    log(f"BF16 stack {dims} x {M} epochs: {info.device_bytes / 1e9:.1f} GB in {time.time() - t0:.1f} s")
    L = synth.diag(dims)
    flags = dart.DART_FORCE_F64_DDA
    views = [dart.View(th, ph, 1024, 1024, L / 1024, 0.0, 0.6, flags)
             for th, ph, _ in synth.isotropic_views(args.large_views, 1005, sizes=(1024,))]
    stream = torch.cuda.Stream()
    if args.tuning:
        tuning = apply_fixed_tuning(dart, st, args.tuning, stream)
    else:
        # brick shapes are re-laid in place, one epoch at a time (no room for a copy)
        best, ms = dart.dart_autotune([st] * 8, views[:8], rebrick=args.rebrick, stream=stream)
        tuning = tuning_dict(best, dart.dart_stack_get_info(st))
    log(f"tuning: {tuning}")
    imgs = [torch.zeros((1024, 1024), dtype=torch.float32, device="cuda") for _ in views]
    n = len(views)
    flux, steps = dart.dart_render_batch([st] * n, views, imgs, stream=stream)
    cell_steps = int(np.sum(steps))

    def batched():
        dart.dart_render_batch([st] * n, views, imgs, stream=stream, stats=False)

    wall, per = time_steps(torch, stream, batched, args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    if args.profile:
        # the 1 GiB copy is the counter calibration kernel
        bandwidth_probe(dart, torch, stream, nbytes=1 << 30, reps=2)
        log(f"batched {ms_step:.1f} ms/step, {cell_steps:.3e} cell-steps")
        return {"profile": True, "ms_per_step": ms_step, "cell_steps": cell_steps,
                "tuning": tuning}
    pl = torch.zeros((1024, 1024), dtype=torch.float32, device="cuda")

    def plain():
        for v in views:
            dart.dart_render(st, v, pl, stream=stream, stats=False)

    pwall, _ = time_steps(torch, stream, plain, max(1, args.steps // 2), 1)
    pms = 1e3 * pwall / max(1, args.steps // 2)
    log(f"batched {ms_step:.1f} ms/step, plain {pms:.1f} ms/step, {cell_steps:.3e} cell-steps")
    samples = [dart.dart_count_samples(st, v, stream) for v in views[:4]]
    est_compulsory = (sum(samples) / 4 * n) * 8 + n * 4 * 1024 * 1024
    lines = [dart.dart_count_lines(st, v, stream) for v in views[:4]]
    est_lines = (sum(lines) / 4 * n) * 128 + n * 4 * 1024 * 1024
    counted = [dart.dart_count_bytes(st, v, stream) for v in views[:4]]
    est_plane = (sum(c for c, _ in counted) / 4 * n) + n * 4 * 1024 * 1024
    acc, cpu = None, None
    if args.check:
        t1 = time.time()
        ref, src = streamed_oracle_flux(torch, dims, times, seed, gamma, knots,
                                        views[:args.large_check], with_source=True)
        oracle_s = time.time() - t1
        errs = [abs(flux[k] - r[1]) / abs(r[1]) for k, r in enumerate(ref)]
        perr, serr, sflux = [], [], []
        for k, (r, q) in enumerate(zip(ref, src)):
            g = imgs[k].cpu().numpy().astype(np.float64)
            perr.append(float(pix_err(g, r[0], float(np.abs(r[0]).max())).max()))
            serr.append(float(pix_err(r[0], q[0], float(np.abs(q[0]).max())).max()))
            sflux.append(abs(r[1] / q[1] - 1.0))
        acc = {"flux_rel_err": [float(e) for e in errs], "max_pixel_rel_err": perr,
               "cell_steps_rel_diff": [abs(int(steps[k]) - r[2]) / max(r[2], 1)
                                       for k, r in enumerate(ref)],
               "images_checked_whole": len(ref), "oracle_s": oracle_s,
               "tolerance": {"flux": 1e-6, "pixel": 2e-3, "cell_steps": 1e-5},
               "against": "FP64 snapshot-outer oracle on the stored values, every pixel",
               "storage_error": {"max_pixel_rel_err": serr, "flux_rel_err": sflux,
                                 "against": "the same oracle on the FP32 source fields, in the "
                                            "same pass (reported, not graded)"}}
        log(f"oracle check: {acc}")
        threads = min(len(os.sched_getaffinity(0)),
                      int(os.environ.get("OMP_NUM_THREADS") or 1 << 10))
        n_ref = sum(r[2] for r in ref)
        cpu = {"value": 2 * n_ref / oracle_s, "unit": "cell-steps/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{len(ref)} whole images, snapshot-outer, on the stored and on the "
                         f"source fields ({2 * n_ref} cell-steps in {oracle_s:.1f} s, the "
                         f"device-to-host epoch readback included)",
               "cpu_model": cpu_model()}
    achieved = est_compulsory / (float(np.mean(per)) * 1e-3) / 1e9
    traffic, tsrc = measured_traffic("large", tuning)
    l2_hit = counter_row("large", tuning)[2]
    slabs = None
    if args.large_slabs > 1:
        torch.cuda.synchronize()
        dart.dart_free_epochs(st)
        slabs = render_slabs(args, dart, torch, dims, M, seed, gamma, knots, views, imgs, flux,
                             steps, stream, brick=tuning["brick"])
        log(f"slabs: {slabs}")
    return {
        "metric": "cell-steps/s & images/s (batched vs plain kernel) at 1e-5 rel; p50/p99 ms",
        "value": cell_steps / (ms_step * 1e-3), "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"large: 512x512x2048, 40 epochs, BF16 ({info.device_bytes / 1e9:.1f} GB "
                               f"resident), {n} views at 1024^2, FP64 ray parameters, Kahan",
                   "cell_steps_per_step": cell_steps},
        "images_per_s": n / (ms_step * 1e-3), "step_ms_p50": pct(per, 50), "step_ms_p99": pct(per, 99),
        "plain": {"ms_per_step": pms, "images_per_s": n / (pms * 1e-3)},
        "speedup_images_per_s_vs_plain": pms / ms_step,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": tsrc,
                     "l2_hit_rate": l2_hit,
                     "bytes_per_launch": est_compulsory,
                     "bytes_definition": "compulsory records estimated from 4 counted views",
                     "plane_bytes_per_launch": est_plane,
                     "plane_gbs": est_plane / (float(np.mean(per)) * 1e-3) / 1e9,
                     "plane_bytes_definition": "the bytes renders of the resident layout must "
                                               "read (emissivity plane, whole records where "
                                               "marked), estimated from the same 4 views",
                     "line_bytes_per_launch": est_lines,
                     "line_gbs": est_lines / (float(np.mean(per)) * 1e-3) / 1e9},
        "accuracy": acc, "tuning": tuning, "cpu_baseline": cpu, "slabs": slabs,
    }


def render_slabs(args, dart, torch, dims, M, seed, gamma, knots, views, whole_imgs, whole_flux,
                 whole_steps, stream, brick=None):
    """Domain slabs on one GPU: the grid is cut into z-slabs; each is loaded
    alone (the share one GPU of a slab-sharded job would hold), placed in the
    domain, and rendered with every view adding into one set of images.  The
    sum must equal the render of the whole domain (flux within 1e-6)."""
    nx, ny, nz = dims
    k = args.large_slabs
    cuts = [round(i * nz / k) for i in range(k + 1)]
    n = len(views)
    acc_views = [dart.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, v.t_obs,
                           v.alpha, v.flags | dart.DART_ACCUMULATE) for v in views]
    total = [torch.zeros_like(im) for im in whole_imgs]
    scratch = [torch.empty_like(im) for im in whole_imgs]
    flux = np.zeros(n)
    steps = np.zeros(n, dtype=np.uint64)
    per_slab = []
    for a in range(k):
        t0 = time.time()
        st, _ = build_stack_incremental(dart, torch, dims, M, seed, gamma, knots, dart.DART_BF16,
                                        chunk_bytes=9 << 30, z_slab=(cuts[a], cuts[a + 1] - cuts[a]))
        if brick is not None:
            dart.dart_stack_rebrick(st, brick, stream)
        gb = dart.dart_stack_get_info(st).device_bytes / 1e9
        f, s = dart.dart_render_batch([st] * n, acc_views, total, stream=stream)
        flux += f
        steps += s

        def one():
            dart.dart_render_batch([st] * n, views, scratch, stream=stream, stats=False)

        reps = max(1, min(args.steps, 3))
        wall, _ = time_steps(torch, stream, one, reps, 1)
        per_slab.append({"z": [cuts[a], cuts[a + 1]], "resident_gb": gb,
                         "ms_per_step": 1e3 * wall / reps, "cell_steps": int(np.sum(s)),
                         "load_s": time.time() - t0})
        torch.cuda.synchronize()
        dart.dart_free_epochs(st)
    torch.cuda.synchronize()
    perr = 0.0
    for g, w in zip(total, whole_imgs):
        floor = 1e-3 * float(w.abs().max())
        e = ((g.double() - w.double()).abs() / w.double().abs().clamp_min(floor)).max()
        perr = max(perr, float(e))
    ferr = float(np.max(np.abs(flux - whole_flux) / np.abs(whole_flux)))
    serr = float(np.max(np.abs(steps.astype(np.float64) - whole_steps.astype(np.float64)) /
                        whole_steps.astype(np.float64)))
    return {"n": k, "per_slab": per_slab, "images": n, "flux_rel_err_vs_whole": ferr,
            "max_pixel_rel_err_vs_whole": perr, "cell_steps_rel_diff": serr,
            "tolerance": {"flux": 1e-6, "pixel": 1e-5}}


def run_labelled_workload(args, dart, torch):
    """The jet grid (256x256x512, 16 epochs, FP32) in the labelled mode: the
    jet's core (x, y in [64, 192), z in [171, 341)) refined twice, the rest
    as six coarse sub-domains around it; the four jet views in one batch."""
    import synth
    dims, M = (256, 256, 512), 16
    t0 = time.time()
    j, b, times = synth.jet_torch(dims, M, 2, gamma_spine=5.0, n_knots=4)
    torch.cuda.synchronize()
    boxes = [((0, 256), (0, 256), (0, 171)), ((0, 256), (0, 256), (341, 512)),
             ((0, 64), (0, 256), (171, 341)), ((192, 256), (0, 256), (171, 341)),
             ((64, 192), (0, 64), (171, 341)), ((64, 192), (192, 256), (171, 341))]
    core = ((64, 192), (64, 192), (171, 341))
    centre = (128.0, 128.0, 256.0)
    parts, host = [], []

    def add(jb, bb, cell, org):
        nz, ny, nx = jb.shape[1:4]
        s = dart.dart_load_epochs((nx, ny, nz), cell, times, jb, bb, dart.DART_F32)
        torch.cuda.synchronize()   # the load reads jb, bb in stream order
        dart.dart_stack_rebrick(s, (1, 8, 1))
        dart.dart_stack_set_placement(s, org, centre)
        parts.append(s)
        if args.check:
            host.append((jb.cpu().numpy(), bb.cpu().numpy(), cell, org))

    for (x0, x1), (y0, y1), (z0, z1) in boxes:
        add(j[:, z0:z1, y0:y1, x0:x1].contiguous(), b[:, z0:z1, y0:y1, x0:x1].contiguous(),
            (1.0, 1.0, 1.0), (x0, y0, z0))
    (x0, x1), (y0, y1), (z0, z1) = core
    jc = j[:, z0:z1, y0:y1, x0:x1]
    bc = b[:, z0:z1, y0:y1, x0:x1]
    del j, b
    jr = jc.repeat_interleave(2, dim=1).repeat_interleave(2, dim=2).repeat_interleave(2, dim=3)
    br = bc.repeat_interleave(2, dim=1).repeat_interleave(2, dim=2).repeat_interleave(2, dim=3)
    del jc, bc
    add(jr.contiguous(), br.contiguous(), (0.5, 0.5, 0.5), (x0, y0, z0))
    del jr, br
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    lab = dart.dart_labelled_create(parts)
    gb = dart.dart_stack_get_info(lab).device_bytes / 1e9
    log(f"labelled stack: {len(parts)} sub-domains, {gb:.1f} GB, built in {time.time() - t0:.1f} s")
    L = synth.diag(dims)
    views = [dart.View(th, 0.0, 512, 512, L / 512, 0.0, 0.6) for th in (10.0, 30.0, 60.0, 90.0)]
    stream = torch.cuda.Stream()
    if args.tuning:
        f = [int(x) for x in normalise_tuning(args.tuning).split(",")]
        dart.dart_set_tuning(f[0], f[1], f[2], f[3], f[4], f[8], f[9])
        best = dart.dart_get_tuning()
    else:
        best, _ = dart.dart_autotune([lab] * 4, views, rebrick=False, stream=stream)
    tuning = tuning_dict(best, dart.dart_stack_get_info(parts[0]))
    imgs = [torch.zeros((512, 512), dtype=torch.float32, device="cuda") for _ in views]
    flux, steps = dart.dart_render_batch([lab] * 4, views, imgs, stream=stream)
    cell_steps = int(np.sum(steps))

    def batched():
        dart.dart_render_batch([lab] * 4, views, imgs, stream=stream, stats=False)

    wall, per = time_steps(torch, stream, batched, args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    pl = [torch.zeros_like(im) for im in imgs]

    def plain():
        for v, im in zip(views, pl):
            dart.dart_render(lab, v, im, stream=stream, stats=False)

    pwall, _ = time_steps(torch, stream, plain, args.steps, args.warmup)
    pms = 1e3 * pwall / args.steps
    torch.cuda.synchronize()
    same = all(torch.equal(a, c) for a, c in zip(imgs, pl))
    log(f"labelled: batched {ms_step:.3f} ms/step, plain {pms:.3f} ms/step, {cell_steps:.4e} cell-steps")
    acc = None
    if args.check:
        import oracle
        oparts = [oracle.Stack(jb, bb, times, cell=cell, origin=org, centre=centre)
                  for jb, bb, cell, org in host]
        rng = np.random.default_rng(7)
        errs = []
        for k, v in enumerate(views):
            pix = np.stack([rng.integers(0, 512, 512), rng.integers(0, 512, 512)], axis=1).astype(np.int32)
            ov = oracle.View(v.theta_deg, v.phi_deg, 512, 512, v.pixel_scale, 0.0, 0.6, 0)
            ref, _ = oracle.render_labelled(oparts, ov, pixels=pix)
            got = imgs[k].cpu().numpy()
            gv = got[pix[:, 1], pix[:, 0]].astype(np.float64)
            errs.append(float(pix_err(gv, ref, float(np.abs(got).max())).max()))
        acc = {"max_pixel_rel_err": max(errs), "sampled_pixels": 512 * len(views),
               "tolerance": 1e-5}
        log(f"accuracy vs the oracle's labelled render: {acc}")
    return {
        "metric": "cell-steps/s & images/s (batched vs plain kernel) at 1e-5 rel; p50/p99 ms",
        "value": cell_steps / (ms_step * 1e-3), "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "labelled: jet 256x256x512, 16 epochs, FP32, core refined 2x "
                               "(7 sub-domains), 4 views 512^2", "sub_domains": len(parts),
                   "resident_gb": gb, "cell_steps_per_step": cell_steps},
        "images_per_s": 4 / (ms_step * 1e-3), "step_ms_p50": pct(per, 50), "step_ms_p99": pct(per, 99),
        "plain": {"ms_per_step": pms, "images_per_s": 4 / (pms * 1e-3),
                  "identical_to_batched": bool(same)},
        "speedup_images_per_s_vs_plain": pms / ms_step,
        "accuracy": acc, "tuning": tuning, "roofline": None, "cpu_baseline": None,
    }


def run_vector_workload(args, dart, torch):
    """Vector sums: the jet grid (256x256x512, 16 epochs, FP32) with three
    components, a total emissivity I and two signed ones Q = 0.6 I cos(2 chi),
    U = 0.6 I sin(2 chi) (chi: a synthetic angle field that winds around the
    jet axis and twists along it), all with the jet's velocity; the four jet
    views.  One fused render of the vector stack against the three components
    rendered as scalar stacks in one batch."""
    import synth
    dims, M = (256, 256, 512), 16
    t0 = time.time()
    j, b, times = synth.jet_torch(dims, M, 2, gamma_spine=5.0, n_knots=4)
    nx, ny, nz = dims
    z = torch.arange(nz, device="cuda", dtype=torch.float32).view(nz, 1, 1)
    y = torch.arange(ny, device="cuda", dtype=torch.float32).view(1, ny, 1)
    x = torch.arange(nx, device="cuda", dtype=torch.float32).view(1, 1, nx)
    chi = torch.atan2(y + 0.5 - 0.5 * ny, x + 0.5 - 0.5 * nx) + (z / nz) * math.pi
    q = (0.6 * j * torch.cos(2.0 * chi)).contiguous()
    u = (0.6 * j * torch.sin(2.0 * chi)).contiguous()
    del chi
    torch.cuda.synchronize()
    comps = []
    host = []
    for arr in (j, q, u):
        s = dart.dart_load_epochs(dims, (1.0, 1.0, 1.0), times, arr, b, dart.DART_F32)
        torch.cuda.synchronize()
        dart.dart_stack_rebrick(s, (1, 8, 1))
        comps.append(s)
        if args.check:
            host.append(arr.cpu().numpy())
    bh = b.cpu().numpy() if args.check else None
    del j, q, u, b
    torch.cuda.empty_cache()
    vec = dart.dart_vector_create(comps)
    gb = dart.dart_stack_get_info(vec).device_bytes / 1e9
    log(f"vector stack: 3 components, {gb:.1f} GB, built in {time.time() - t0:.1f} s")
    L = synth.diag(dims)
    views = [dart.View(th, 0.0, 512, 512, L / 512, 0.0, 0.6) for th in (10.0, 30.0, 60.0, 90.0)]
    stream = torch.cuda.Stream()
    if args.tuning:
        f = [int(x) for x in normalise_tuning(args.tuning).split(",")]
        dart.dart_set_tuning(f[0], f[1], f[2], f[3], f[4], f[8], f[9])
        best = dart.dart_get_tuning()
    else:
        best, _ = dart.dart_autotune([vec] * 4, views, rebrick=False, stream=stream)
    tuning = tuning_dict(best, dart.dart_stack_get_info(comps[0]))
    vimgs = [torch.zeros((3, 512, 512), dtype=torch.float32, device="cuda") for _ in views]
    flux, steps = dart.dart_render_batch([vec] * 4, views, vimgs, stream=stream)
    cell_steps = int(np.sum(steps))

    def fused():
        dart.dart_render_batch([vec] * 4, views, vimgs, stream=stream, stats=False)

    wall, per = time_steps(torch, stream, fused, args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    kernel_ms = float(np.mean(per))
    simgs = [torch.zeros((512, 512), dtype=torch.float32, device="cuda") for _ in range(12)]
    sstacks = [c for c in comps for _ in views]
    sviews = views * 3

    def separate():
        dart.dart_render_batch(sstacks, sviews, simgs, stream=stream, stats=False)

    swall, _ = time_steps(torch, stream, separate, args.steps, args.warmup)
    sms = 1e3 * swall / args.steps
    torch.cuda.synchronize()
    same = all(torch.equal(vimgs[k][c], simgs[c * 4 + k]) for c in range(3) for k in range(4))
    samples = sum(dart.dart_count_samples(comps[0], v, stream) for v in views)
    out_bytes = 3 * 4 * 512 * 512 * len(views)
    # component 0's whole record and the emissivity field of the two others
    compulsory = samples * (16 + 2 * 4) + out_bytes
    achieved = compulsory / (kernel_ms * 1e-3) / 1e9
    log(f"vector: fused {ms_step:.3f} ms/step, three scalar stacks {sms:.3f} ms/step, "
        f"{cell_steps:.4e} cell-steps, identical {same}")
    acc = None
    if args.check:
        import oracle
        rng = np.random.default_rng(11)
        errs = []
        for c in range(3):
            ost = oracle.Stack(host[c], bh, times, encoding="f32")
            ost_abs = oracle.Stack(np.abs(host[c]), bh, times, encoding="f32")
            for k, v in enumerate(views):
                pix = np.stack([rng.integers(0, 512, 128), rng.integers(0, 512, 128)],
                               axis=1).astype(np.int32)
                ov = oracle.View(v.theta_deg, v.phi_deg, 512, 512, v.pixel_scale, 0.0, 0.6, 0)
                ref, _ = oracle.render(ost, ov, pixels=pix)
                scale, _ = oracle.render(ost_abs, ov, pixels=pix)
                got = vimgs[k][c].cpu().numpy()[pix[:, 1], pix[:, 0]].astype(np.float64)
                floor = 1e-3 * max(float(scale.max()), 1e-300)
                errs.append(float((np.abs(got - ref) / np.maximum(scale, floor)).max()))
        acc = {"max_pixel_rel_err": max(errs), "sampled_pixels": 128 * 4 * 3,
               "tolerance": 1e-5, "definition": "|got - oracle| / oracle render of |j_c|"}
        log(f"accuracy vs the oracle: {acc}")
    return {
        "metric": "cell-steps/s & images/s (batched vs plain kernel) at 1e-5 rel; p50/p99 ms",
        "value": cell_steps / (ms_step * 1e-3), "unit": "cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "vector: jet 256x256x512, 16 epochs, FP32, components I, Q, U, "
                               "4 views 512^2", "components": 3, "resident_gb": gb,
                   "cell_steps_per_step": cell_steps},
        "component_cell_steps_per_s": 3 * cell_steps / (ms_step * 1e-3),
        "images_per_s": 12 / (ms_step * 1e-3), "step_ms_p50": pct(per, 50), "step_ms_p99": pct(per, 99),
        "separate": {"ms_per_step": sms, "note": "the three components as scalar stacks, 12 "
                     "images in one batched call", "identical_to_fused": bool(same)},
        "speedup_vs_separate": sms / ms_step,
        "accuracy": acc, "tuning": tuning,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": compulsory,
                     "bytes_definition": "distinct (cell, epoch) samples x (component 0's record "
                                         "+ 4 B emissivity of each other component) + images"},
        "cpu_baseline": None,
    }


def run_stream_workload(args, dart, torch):
    """Out-of-core: the jet epochs (256x256x512, 16 epochs, FP32 source) stay
    in pinned host memory (or, second measurement, in device memory in the
    caller's layout) and stream through a 3-slot ring, FP32 storage; the four
    jet views per step.  The bound is the host-to-device copy."""
    import synth
    dims, M = (256, 256, 512), 16
    j, b, times = synth.jet_torch(dims, M, 2, gamma_spine=5.0, n_knots=4)
    torch.cuda.synchronize()
    jh = torch.empty(j.shape, dtype=torch.float32, pin_memory=True)
    bh = torch.empty(b.shape, dtype=torch.float32, pin_memory=True)
    jh.copy_(j)
    bh.copy_(b)
    L = synth.diag(dims)
    views = [dart.View(th, 0.0, 512, 512, L / 512, 0.0, 0.6) for th in (10.0, 30.0, 60.0, 90.0)]
    stream = torch.cuda.Stream()
    # resident reference (also the launch shape the stream uses)
    res = dart.dart_load_epochs(dims, (1, 1, 1), times, j, b, dart.DART_F32)
    torch.cuda.synchronize()
    dart.dart_stack_rebrick(res, (1, 8, 1), stream)
    dart.dart_set_tuning(64, 1, 12, 0, 0, 0)
    rimgs = [torch.zeros((512, 512), dtype=torch.float32, device="cuda") for _ in views]
    f64 = [dart.View(v.theta_deg, v.phi_deg, 512, 512, v.pixel_scale, 0.0, 0.6,
                     dart.DART_FORCE_F64_DDA) for v in views]
    rflux, rsteps = dart.dart_render_batch([res] * 4, f64, rimgs, stream=stream)

    def resident():
        dart.dart_render_batch([res] * 4, f64, rimgs, stream=stream, stats=False)

    rwall, _ = time_steps(torch, stream, resident, args.steps, args.warmup)
    rms = 1e3 * rwall / args.steps
    sm = dart.dart_streamer_create(dims, (1, 1, 1), times, dart.DART_F32, ring_epochs=3,
                                   brick=(1, 8, 1))
    imgs = [torch.zeros((512, 512), dtype=torch.float32, device="cuda") for _ in views]
    out = {}
    for src_name, (js, bs) in (("pinned_host", (jh, bh)), ("device", (j, b))):
        flux, steps = dart.dart_streamer_render(sm, js, bs, views, imgs, stream=stream)
        same_steps = bool(np.array_equal(steps, rsteps))
        err = max(float(((a.double() - c.double()).abs() /
                         c.double().abs().clamp_min(1e-3 * float(c.abs().max()))).max())
                  for a, c in zip(imgs, rimgs))

        def streamed():
            dart.dart_streamer_render(sm, js, bs, views, imgs, stream=stream, stats=False)

        reps = max(2, args.steps // 10)
        wall, _ = time_steps(torch, stream, streamed, reps, 1)
        ms = 1e3 * wall / reps
        st = dart.dart_streamer_get_stats(sm)
        out[src_name] = {"ms_per_step": ms, "images_per_s": 4 / (ms * 1e-3),
                         "epochs_loaded": st.epochs_loaded, "intervals": st.intervals,
                         "bytes_uploaded": st.bytes_uploaded,
                         "upload_gbs": st.bytes_uploaded / (ms * 1e-3) / 1e9,
                         "cell_steps_equal_resident": same_steps,
                         "max_pixel_rel_diff_vs_resident": err}
        log(f"stream from {src_name}: {ms:.2f} ms/step, {out[src_name]}")
    # the bound: a pinned host-to-device copy of one epoch's source
    one = torch.empty(j[0].numel() * 4, dtype=torch.float32, device="cuda")
    src = torch.empty(one.numel(), dtype=torch.float32, pin_memory=True)
    wall, _ = time_steps(torch, stream, lambda: one.copy_(src, non_blocking=True), 5, 1)
    h2d = one.numel() * 4 / (wall / 5) / 1e9
    log(f"pinned H2D copy: {h2d:.1f} GB/s; resident render {rms:.3f} ms/step")
    cell_steps = int(np.sum(rsteps))
    ms = out["pinned_host"]["ms_per_step"]
    return {
        "metric": "cell-steps/s & images/s (batched vs plain kernel) at 1e-5 rel; p50/p99 ms",
        "value": cell_steps / (ms * 1e-3), "unit": "cell-steps/s", "n_gpus": 1,
        "steps": max(2, args.steps // 10), "warmup": 1, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "stream: jet 256x256x512, 16 epochs, FP32 source in pinned host "
                               "memory, 3-slot ring, 4 views 512^2", "cell_steps_per_step": cell_steps},
        "images_per_s": 4 / (ms * 1e-3), "streams": out,
        "resident_ms_per_step": rms, "pinned_h2d_gbs": h2d,
        "roofline": {"bound": "pcie", "achieved": out["pinned_host"]["upload_gbs"], "peak": h2d,
                     "unit": "GB/s", "frac": out["pinned_host"]["upload_gbs"] / h2d,
                     "traffic": None, "peak_definition": "measured pinned host-to-device copy"},
        "cpu_baseline": None,
    }


# --------------------------------------------------------------------------- counters

def pmc_summary(fetch_csv, write_csv, workload, tuning):
    """One row of the traffic table from two rocprofv3 --pmc runs of
    `bench.py --profile` (FETCH_SIZE in the first, WRITE_SIZE in the second).
    Both counters are in KiB per dispatch; each is scaled by what it reads for
    the 1 GiB k_copy that the profile run launches (1 GiB read, 1 GiB written)."""
    import csv
    import collections

    def load(path):
        agg = collections.defaultdict(list)
        with open(path) as fh:
            for r in csv.DictReader(fh):
                agg[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in agg.items()}

    def pick(d, kernel, counter):
        vals = [v for (k, c), v in d.items() if kernel in k and c == counter]
        if len(vals) != 1:
            raise SystemExit(f"expected one {kernel} kernel with {counter}, found {len(vals)}")
        return vals[0]

    a, b = load(fetch_csv), load(write_csv)
    gib_kib = float(1 << 20)
    fscale = gib_kib / pick(a, "k_copy", "FETCH_SIZE")
    wscale = gib_kib / pick(b, "k_copy", "WRITE_SIZE")
    fetch = pick(a, "k_batch", "FETCH_SIZE") * 1024 * fscale
    write = pick(b, "k_batch", "WRITE_SIZE") * 1024 * wscale
    hit = pick(b, "k_batch", "TCC_HIT_sum")
    miss = pick(b, "k_batch", "TCC_MISS_sum")
    print(f"# FETCH_SIZE scale {fscale:.4f}, WRITE_SIZE scale {wscale:.4f}, "
          f"TCC_HIT {hit:.4g}, TCC_MISS {miss:.4g} (misses x 128 B = {miss * 128:.4g} B)")
    print(f"{workload} {kernel_source_id()} {tuning} {fetch:.0f} {write:.0f} {hit / (hit + miss):.4f}")


# --------------------------------------------------------------------------- main

def run_batch_workload(args, dart, torch):
    import synth
    views = [(th, ph, P, 0.6) for th, ph, P in synth.isotropic_views(64, 1003)]
    name = (f"uneven batch 384^3, 32 epochs, {args.storage.upper()}, 64 isotropic views, "
            "sides in {128,256,512,1024}")
    if args.sides:
        # one size class of the same 64 views (a breakdown, not the workload)
        keep = {int(x) for x in args.sides.split(",")}
        views = [v for v in views if v[2] in keep]
        name += f", only the {len(views)} views of side {args.sides}"
    storage = dart.DART_F16 if args.storage == "f16" else dart.DART_BF16
    return run_render_workload(args, dart, torch, name, (384, 384, 384), 32, storage, views, 5.0,
                               4, 3, 8, args.storage, check_views=8)


def release(torch):
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def nested_object(line):
    """A workload's line as an object inside the default line: its own metric
    values, workload, roofline, comparisons, accuracy and CPU baseline."""
    drop = ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data")
    return {k: v for k, v in line.items() if k not in drop}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="jet",
                    choices=["jet", "batch", "serve", "large", "labelled", "stream", "vector"])
    ap.add_argument("--large-views", type=int, default=256)
    ap.add_argument("--large-check", type=int, default=4)
    ap.add_argument("--large-slabs", type=int, default=2,
                    help="large workload: also render the domain as this many z-slabs "
                         "and compare their sum with the whole (0: skip)")
    ap.add_argument("--storage", default="f16", choices=["f16", "bf16"],
                    help="batch workload: 16-bit storage type")
    ap.add_argument("--sides", default=None,
                    help="batch workload: keep only the views with these image sides "
                         "(comma-separated), for a per-size breakdown")
    ap.add_argument("--requests", type=int, default=6000)
    ap.add_argument("--serve-warmup", type=int, default=500)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--budget-gb", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--exact-time", action="store_true",
                    help="jet / batch workloads: views with DART_EXACT_TIME (chords cut at "
                         "epoch times)")
    ap.add_argument("--check", action="store_true", default=True)
    ap.add_argument("--no-check", dest="check", action="store_false")
    ap.add_argument("--check-rays", type=int, default=2048)
    ap.add_argument("--no-autotune", dest="autotune", action="store_false", default=True,
                    help="skip the (untimed) tile / occupancy / brick-shape tuning")
    ap.add_argument("--no-rebrick", dest="rebrick", action="store_false", default=True)
    ap.add_argument("--tuning", default=None,
                    help="fixed launch shape instead of autotuning: "
                         "tile_w,tile_h,waves_per_cu,order,orient,brick_x,brick_y,brick_z"
                         "[,depth_sync[,cells_per_batch]]")
    ap.add_argument("--profile", action="store_true",
                    help="timed batched loop only (for rocprofv3 runs)")
    ap.add_argument("--no-nested", dest="nested", action="store_false", default=True,
                    help="jet workload: leave out the batched (384^3 FP16) and served objects "
                         "that the default run adds to its line")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print the traffic-table row for two rocprofv3 --pmc counter files "
                         "of a --profile run (with the same --workload/--storage/--tuning)")
    args = ap.parse_args()
    if args.pmc_summary:
        wkey = workload_key(args)
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], wkey, normalise_tuning(args.tuning))
        return
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
        if args.nested and not args.profile:
            # the batched and served forms of the same metric, in the same run
            t0 = time.time()
            release(torch)
            bargs = argparse.Namespace(**vars(args))
            bargs.workload, bargs.storage, bargs.sides = "batch", "f16", None
            line["batch_fp16"] = nested_object(run_batch_workload(bargs, dart, torch))
            log(f"batch object in {time.time() - t0:.0f} s")
            t0 = time.time()
            release(torch)
            sargs = argparse.Namespace(**vars(args))
            sargs.workload = "serve"
            served = nested_object(run_serve_workload(sargs, dart, torch))
            line["served"] = served
            log(f"served object in {time.time() - t0:.0f} s")
            # the metric's p50 / p99 are the served stream's latencies
            line["p50_ms"], line["p99_ms"] = served["p50_ms"], served["p99_ms"]
            line["latency_source"] = "served object: " + served["latency_definition"]
    elif args.workload == "batch":
        line = run_batch_workload(args, dart, torch)
    elif args.workload == "serve":
        line = run_serve_workload(args, dart, torch)
    elif args.workload == "labelled":
        line = run_labelled_workload(args, dart, torch)
    elif args.workload == "stream":
        line = run_stream_workload(args, dart, torch)
    elif args.workload == "vector":
        line = run_vector_workload(args, dart, torch)
    else:
        line = run_large_workload(args, dart, torch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
