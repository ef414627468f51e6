"""GPU parity at the workloads' full sizes, in the launch configuration the
bench times (autotuned tile / occupancy / brick shape, persistent batched
kernel replayed from a captured graph).

* jet, 256 x 256 x 512, 16 epochs, FP32, four 512^2 views: every pixel of
  the four images against the FP64 oracle (<= 1e-5), total flux (<= 1e-6).
* uneven batch, 384^3, 32 epochs, FP16 and BF16, 64 isotropic views with
  sides in {128, 256, 512, 1024} rendered by one batched call: the first 8
  views and the first 1024^2 view checked whole (every pixel <= 2e-3, flux
  <= 1e-6, cell-steps) against the oracle on the stored (rounded) values,
  with the storage error against the FP32 source fields printed beside.
* served mix: requests on several resident FP16 stacks submitted to the
  continuous-batching server under a tight memory budget; every served image
  is bit-identical to a solo render of the same request.
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2609_09322_amd as d
    return d, torch


def pix_err(got, ref):
    floor = 1e-3 * max(np.abs(ref).max(), 1e-300)
    return np.abs(np.asarray(got, np.float64) - ref) / np.maximum(np.abs(ref), floor)


def _host_16bit(j_dev, b_dev, kind):
    """Epoch-by-epoch rounding of device float32 fields to the host 16-bit
    encoding the oracle reads (numpy's own rounding, not the kernels')."""
    M = j_dev.shape[0]
    if kind == "f16":
        jh = np.empty(tuple(j_dev.shape), dtype=np.float16)
        bh = np.empty(tuple(b_dev.shape), dtype=np.float16)
        conv = synth.to_f16
    else:
        jh = np.empty(tuple(j_dev.shape), dtype=np.uint16)
        bh = np.empty(tuple(b_dev.shape), dtype=np.uint16)
        conv = synth.to_bf16_bits
    for m in range(M):
        jh[m] = conv(j_dev[m].cpu().numpy())
        bh[m] = conv(b_dev[m].cpu().numpy())
    return jh, bh


def test_jet_workload_every_pixel(env):
    dart, torch = env
    dims, M = (256, 256, 512), 16
    j, b, times = synth.jet_torch(dims, M, 2, gamma_spine=5.0, n_knots=4)
    torch.cuda.synchronize()
    jh, bh = j.cpu().numpy(), b.cpu().numpy()
    st = dart.dart_load_epochs(dims, (1, 1, 1), times, j, b, dart.DART_F32)
    del j, b
    torch.cuda.empty_cache()
    L = synth.diag(dims)
    views = [dart.View(th, 0.0, 512, 512, L / 512, 0.0, 0.6) for th in (10.0, 30.0, 60.0, 90.0)]
    stream = torch.cuda.Stream()
    dart.dart_autotune([st] * 4, views, rebrick=True, stream=stream)
    imgs = [torch.zeros((512, 512), dtype=torch.float32, device="cuda") for _ in views]
    flux, steps = dart.dart_render_batch([st] * 4, views, imgs, stream=stream)
    ost = oracle.Stack(jh, bh, times)
    for k, v in enumerate(views):
        ov = oracle.View(v.theta_deg, v.phi_deg, 512, 512, v.pixel_scale, 0.0, 0.6, 0)
        ref, rsteps = oracle.render(ost, ov)
        got = imgs[k].cpu().numpy()
        e = pix_err(got, ref)
        print(f"jet theta {v.theta_deg}: max per-pixel err {e.max():.3e}, flux "
              f"{flux[k]:.9e} vs {oracle.flux(ref, ov):.9e}, steps {steps[k]} vs {rsteps}", flush=True)
        assert e.max() <= 1e-5
        assert flux[k] == pytest.approx(oracle.flux(ref, ov), rel=1e-6)
        assert abs(int(steps[k]) - rsteps) <= 1e-5 * rsteps


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_uneven_batch_checked_images(env, kind):
    """The 64-view batch in one call; the first 8 views (the seeded sample)
    and the first 1024^2 view are checked whole: every pixel within 2e-3 of
    the oracle on the stored values, flux within 1e-6, cell-steps within 1e-5.
    The storage error (the oracle on the stored values against the oracle on
    the FP32 source fields) is printed for each, not graded."""
    dart, torch = env
    dims, M = (384, 384, 384), 32
    j, b, times = synth.jet_torch(dims, M, 3, gamma_spine=5.0, n_knots=4)
    torch.cuda.synchronize()
    storage = dart.DART_F16 if kind == "f16" else dart.DART_BF16
    st = dart.dart_load_epochs(dims, (1, 1, 1), times, j, b, storage)
    jh, bh = _host_16bit(j, b, kind)
    js, bs = j.cpu().numpy(), b.cpu().numpy()
    del j, b
    torch.cuda.empty_cache()
    L = synth.diag(dims)
    spec = synth.isotropic_views(64, 1003)
    views = [dart.View(th, ph, P, P, L / P, 0.0, 0.6) for th, ph, P in spec]
    stream = torch.cuda.Stream()
    dart.dart_autotune([st] * 8, views[:8], rebrick=True, stream=stream)
    imgs = [torch.zeros((v.height, v.width), dtype=torch.float32, device="cuda") for v in views]
    flux, steps = dart.dart_render_batch([st] * 64, views, imgs, stream=stream)
    ost = oracle.Stack(jh, bh, times, encoding=kind)
    src = oracle.Stack(js, bs, times)
    checked = list(range(8)) + [next(k for k, v in enumerate(views) if v.width == 1024)]
    for k in checked:
        v = views[k]
        ov = oracle.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, 0.0, 0.6, 0)
        got = imgs[k].cpu().numpy()
        ref, rsteps = oracle.render(ost, ov)
        e = pix_err(got, ref).max()
        rflux = oracle.flux(ref, ov)
        sref, _ = oracle.render(src, ov)
        sflux = oracle.flux(sref, ov)
        print(f"{kind} view {k} ({v.width}^2, theta {v.theta_deg:.1f}): max per-pixel err "
              f"{e:.3e}, flux {flux[k]:.9e} vs {rflux:.9e} ({abs(flux[k] / rflux - 1):.2e}), "
              f"steps {steps[k]} vs {rsteps}; storage error: per pixel "
              f"{pix_err(ref, sref).max():.3e}, flux {abs(rflux / sflux - 1):.3e}", flush=True)
        assert e <= 2e-3
        assert flux[k] == pytest.approx(rflux, rel=1e-6)
        assert abs(int(steps[k]) - rsteps) <= 1e-5 * rsteps


def test_server_mix_equals_solo(env):
    dart, torch = env
    stacks, dims_l = [], [(64, 64, 64), (96, 96, 128), (128, 128, 128)]
    for k, dims in enumerate(dims_l):
        M = (8, 16, 12)[k]
        j, b, times = synth.jet_torch(dims, M, 40 + k, gamma_spine=3.0 + k, n_knots=4)
        stacks.append((dart.dart_load_epochs(dims, (1, 1, 1), times, j, b, dart.DART_F16), dims))
        del j, b
    torch.cuda.empty_cache()
    rng = np.random.default_rng(4)
    reqs = []
    for q in range(60):
        s, dims = stacks[int(rng.integers(0, 3))]
        P = int(rng.choice([64, 128, 256, 512]))
        th = math.degrees(math.acos(rng.uniform(-1, 1)))
        v = dart.View(th, float(rng.uniform(0, 360)), P, P, synth.diag(dims) / P, 0.0,
                      float(rng.uniform(0.5, 1.0)))
        reqs.append((s, v, torch.full((P, P), -1.0, dtype=torch.float32, device="cuda")))
    # The whole mix arrives as one burst; a 3 MiB budget (a 512^2 image is
    # 1 MiB) makes later requests wait for memory held by earlier ones.
    budget = 3 << 20
    srv = dart.dart_server_create(budget, max_inflight=64, n_streams=3)
    tickets = [dart.dart_submit(srv, s, v, im) for s, v, im in reqs]
    results = [dart.dart_wait(srv, t) for t in tickets]
    stats = dart.dart_server_get_stats(srv)
    tl = dart.dart_server_get_timeline(srv)
    dart.dart_server_destroy(srv)
    # every retired wave is timed; its render kernels are part of its device work
    assert tl.waves_timed == stats.waves
    assert 0.0 < tl.kernel_ms <= tl.device_ms
    assert tl.plan_ms > 0.0 and tl.enqueue_ms > 0.0 and tl.stream_idle_ms >= 0.0
    assert stats.completed == len(reqs)
    assert stats.admission_waits > 0
    assert stats.waves > 1
    assert stats.bytes_peak <= budget
    torch.cuda.synchronize()
    for (s, v, im), (flux, nsteps, lat) in zip(reqs, results):
        solo = torch.zeros_like(im)
        f, n = dart.dart_render_batch([s], [v], [solo])
        assert torch.equal(im, solo)
        assert flux == pytest.approx(float(f[0]), rel=1e-12)
        assert nsteps == int(n[0])
        assert lat > 0.0
    print(f"server: {stats.waves} waves, largest {stats.max_wave_requests} requests, "
          f"{stats.admission_waits} admission waits, peak {stats.bytes_peak} B", flush=True)
