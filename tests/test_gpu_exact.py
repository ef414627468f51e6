"""Exact temporal integration (DART_EXACT_TIME): chords cut at the epoch
times and window ends, each piece weighted at its own midpoint.  GPU against
the oracle in the same mode (pins P16 tie the oracle's exact mode to the
continuous integral), batched against plain, with depth-synchronous marching,
and against the midpoint mode where the two must agree (fields linear in time).
"""
import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import labelled_refinement_case

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 2e-3, "bf16": 2e-3}


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2609_09322_amd as d
    return d, torch


def pix_err(gpu, ref):
    floor = 1e-3 * max(np.abs(ref).max(), 1e-300)
    return np.abs(np.asarray(gpu, np.float64) - ref) / np.maximum(np.abs(ref), floor)


def _store(d, name):
    return {"f64": d.DART_F64, "f32": d.DART_F32, "f16": d.DART_F16, "bf16": d.DART_BF16}[name]


@pytest.mark.parametrize("store", ["f64", "f32", "f16", "bf16"])
def test_exact_time_matches_oracle(env, store):
    dart, torch = env
    dims = (14, 11, 17)
    t = np.linspace(-9.0, 9.0, 7)       # cadence 3: most chords are cut
    j, b, _ = synth.random_stack(dims, len(t), seed=61, beta_max=0.8, times=t)
    src = np.float64 if store == "f64" else np.float32
    st = dart.dart_load_epochs(dims, (1, 1, 1), t, j.astype(src), b.astype(src), _store(dart, store))
    enc = {"f64": "f64", "f32": "f32", "f16": "f32_as_f16", "bf16": "f32_as_bf16"}[store]
    ost = oracle.Stack(j.astype(src), b.astype(src), t, encoding=enc)
    out64 = store == "f64"
    for th, ph, fl in [(37.0, 211.0, 0), (90.0, 0.0, 0), (123.0, 300.0, dart.DART_NO_BEAMING),
                       (8.0, 45.0, 0)]:
        flags = fl | dart.DART_EXACT_TIME
        v = dart.View(th, ph, 40, 36, 0.6, 0.5, 0.7, flags, dart.DART_F64 if out64 else dart.DART_F32)
        img = torch.zeros((36, 40), dtype=torch.float64 if out64 else torch.float32, device="cuda")
        (f,), (n,) = dart.dart_render_batch([st], [v], [img])
        ov = oracle.View(th, ph, 40, 36, 0.6, 0.5, 0.7, (fl & 7) | oracle.EXACT_TIME)
        ref, rn = oracle.render(ost, ov)
        mid, _ = oracle.render(ost, oracle.View(th, ph, 40, 36, 0.6, 0.5, 0.7, fl & 7))
        e = pix_err(img.cpu().numpy(), ref).max()
        print(f"exact {store} ({th}, {ph}): err {e:.2e}, steps {n} vs {rn}, "
              f"midpoint mode differs by {pix_err(mid, ref).max():.2e}", flush=True)
        assert e <= TOL[store]
        assert abs(int(n) - rn) <= (0 if store == "f64" else 2)
        assert f == pytest.approx(oracle.flux(ref, ov), rel=1e-6)
        # the mode matters here: the midpoint sampling is measurably different
        if store == "f64":
            assert pix_err(mid, ref).max() > 1e-6


@pytest.mark.parametrize("sync", [0, 2])
def test_exact_time_batch_equals_plain(env, sync):
    dart, torch = env
    dims = (24, 20, 28)
    t = np.linspace(-20.0, 20.0, 9)
    j, b, _ = synth.random_stack(dims, len(t), seed=62, beta_max=0.8, times=t)
    st = dart.dart_load_epochs(dims, (1, 1, 1), t, j.astype(np.float32), b.astype(np.float32),
                               dart.DART_F32)
    saved = dart.dart_get_tuning()
    dart.dart_set_tuning(16, 4, 8, 0, 1, sync)
    try:
        views = [dart.View(th, ph, W, H, 0.7, 1.0, 0.6, dart.DART_EXACT_TIME)
                 for th, ph, W, H in [(33.0, 12.0, 47, 31), (99.0, 250.0, 64, 64), (150.0, 80.0, 9, 70)]]
        imgs = [torch.zeros((v.height, v.width), dtype=torch.float32, device="cuda") for v in views]
        flux, steps = dart.dart_render_batch([st] * 3, views, imgs)
    finally:
        dart.dart_set_tuning(saved.tile_w, saved.tile_h, saved.waves_per_cu, saved.order,
                             saved.orient, saved.depth_sync)
    ost = oracle.Stack(j.astype(np.float32), b.astype(np.float32), t)
    for k, v in enumerate(views):
        plain = np.zeros((v.height, v.width), np.float32)
        pf, ps = dart.dart_render(st, v, plain)
        np.testing.assert_array_equal(imgs[k].cpu().numpy(), plain)
        assert int(steps[k]) == ps
        ref, _ = oracle.render(ost, oracle.View(v.theta_deg, v.phi_deg, v.width, v.height,
                                                v.pixel_scale, 1.0, 0.6, oracle.EXACT_TIME))
        assert pix_err(plain, ref).max() <= 1e-5


def test_exact_equals_midpoint_for_linear_fields_and_flag_rules(env):
    dart, torch = env
    (j, b), _, t, _ = labelled_refinement_case()
    nz, ny, nx = j.shape[1:4]
    st = dart.dart_load_epochs((nx, ny, nz), (1, 1, 1), t, j, b, dart.DART_F64)
    for th, ph in [(35.0, 20.0), (128.0, 300.0)]:
        a = np.zeros((28, 30))
        c = np.zeros((28, 30))
        dart.dart_render(st, dart.View(th, ph, 30, 28, 0.5, 0.0, 0.7, 0, dart.DART_F64), a)
        dart.dart_render(st, dart.View(th, ph, 30, 28, 0.5, 0.0, 0.7, dart.DART_EXACT_TIME,
                                       dart.DART_F64), c)
        assert np.abs(a - c).max() <= 1e-12 * np.abs(a).max()
    v = dart.View(30.0, 0.0, 8, 8, 1.0, 0.0, 0.7, dart.DART_EXACT_TIME | dart.DART_NEAREST_EPOCH)
    with pytest.raises(dart.DartError) as ei:
        dart.dart_render(st, v, np.zeros((8, 8), np.float32))
    assert ei.value.status == dart.DART_E_INVAL
    sm = dart.dart_streamer_create((nx, ny, nz), (1, 1, 1), t, dart.DART_F32)
    with pytest.raises(dart.DartError) as ei:
        dart.dart_streamer_render(sm, j.astype(np.float32), b.astype(np.float32),
                                  [dart.View(30.0, 0.0, 8, 8, 1.0, 0.0, 0.7, dart.DART_EXACT_TIME)],
                                  [np.zeros((8, 8), np.float32)])
    assert ei.value.status == dart.DART_E_INVAL
