"""Out-of-core rendering through a device ring of epochs (dart_streamer_*):
the streamed lookback sum equals the resident one (identical cell steps,
flux and pixels within 1e-6 of the resident render with FP64 ray parameters,
and within the storage tolerance of the FP64 oracle), with host and device
sources, rings of 3 and
5 slots, routines A/B/C and nearest-epoch views in one call, intervals no view
sees skipped unread, and bad source values reported with their epoch.
"""
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


def pix_err(gpu, ref):
    floor = 1e-3 * max(np.abs(ref).max(), 1e-300)
    return np.abs(np.asarray(gpu, np.float64) - ref) / np.maximum(np.abs(ref), floor)


@pytest.fixture(scope="module")
def jet(env):
    dart, torch = env
    dims, M = (64, 48, 128), 9
    jd, bd, t = synth.jet_torch(dims, M, 31, gamma_spine=4.0, n_knots=3)
    torch.cuda.synchronize()
    return dims, t, jd, bd


@pytest.mark.parametrize("store,ring,src", [("f32", 3, "host"), ("f32", 5, "device"),
                                             ("f16", 3, "device")])
def test_streamed_equals_resident(env, jet, store, ring, src):
    dart, torch = env
    dims, t, jd, bd = jet
    storage = dart.DART_F32 if store == "f32" else dart.DART_F16
    L = synth.diag(dims)
    views = [dart.View(th, ph, 80, 64, 1.05 * L / 80, 0.0, 0.6, fl)
             for th, ph, fl in [(10.0, 0.0, 0), (60.0, 30.0, 0), (90.0, 90.0, dart.DART_NO_LOOKBACK),
                                (135.0, 200.0, dart.DART_NO_BEAMING),
                                (75.0, 300.0, dart.DART_NEAREST_EPOCH)]]
    res = dart.dart_load_epochs(dims, (1, 1, 1), t, jd, bd, storage)
    ref_imgs = [torch.zeros((64, 80), dtype=torch.float32, device="cuda") for _ in views]
    # streamed renders march with FP64 ray parameters; so does the reference
    f64 = [dart.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, v.t_obs, v.alpha,
                     v.flags | dart.DART_FORCE_F64_DDA) for v in views]
    rflux, rsteps = dart.dart_render_batch([res] * len(views), f64, ref_imgs)
    sm = dart.dart_streamer_create(dims, (1, 1, 1), t, storage, ring_epochs=ring)
    if src == "host":
        jh, bh = jd.cpu().numpy(), bd.cpu().numpy()
        imgs = [np.full((64, 80), -1.0, dtype=np.float32) for _ in views]
        flux, steps = dart.dart_streamer_render(sm, jh, bh, views, imgs)
        got = imgs
    else:
        imgs = [torch.full((64, 80), -1.0, dtype=torch.float32, device="cuda") for _ in views]
        flux, steps = dart.dart_streamer_render(sm, jd, bd, views, imgs)
        got = [im.cpu().numpy() for im in imgs]
    st = dart.dart_streamer_get_stats(sm)
    assert st.intervals >= 1 and st.epochs_loaded + st.epochs_skipped == len(t)
    enc = "f32" if store == "f32" else "f32_as_f16"
    ost = oracle.Stack(jd.cpu().numpy(), bd.cpu().numpy(), t, encoding=enc)
    tol = 1e-5 if store == "f32" else 2e-3
    for k, v in enumerate(views):
        r = ref_imgs[k].cpu().numpy()
        e_res = pix_err(got[k], r.astype(np.float64)).max()
        ov = oracle.View(v.theta_deg, v.phi_deg, 80, 64, v.pixel_scale, 0.0, 0.6, v.flags & 7)
        o, os_ = oracle.render(ost, ov)
        e_orc = pix_err(got[k], o).max()
        print(f"streamed {store} ring {ring} {src} view {k}: vs resident {e_res:.2e}, vs oracle "
              f"{e_orc:.2e}, steps {steps[k]} vs {rsteps[k]}", flush=True)
        assert int(steps[k]) == int(rsteps[k])
        assert e_res <= 1e-6
        assert e_orc <= tol
        assert flux[k] == pytest.approx(rflux[k], rel=1e-6)
    dart.dart_streamer_destroy(sm)


def test_flexload_skips_unseen_epochs(env):
    """A long series seen over a short stretch: only the epochs whose
    intervals the views can reach are read; the image equals the resident one."""
    dart, torch = env
    dims = (32, 32, 32)
    L = synth.diag(dims)
    t = np.linspace(-4 * L, 4 * L, 17)           # cadence L / 2: the grid spans ~2 intervals
    j, b, _ = synth.random_stack(dims, len(t), seed=8, beta_max=0.7, times=t, dtype=np.float32)
    views = [dart.View(40.0, 10.0, 48, 48, 1.1 * L / 48, 0.3 * L, 0.7),
             dart.View(120.0, 70.0, 48, 48, 1.1 * L / 48, 0.1 * L, 0.7)]
    res = dart.dart_load_epochs(dims, (1, 1, 1), t, j, b, dart.DART_F32)
    ref = [np.zeros((48, 48), np.float32) for _ in views]
    rflux, rsteps = dart.dart_render_batch([res] * 2, views, ref)
    sm = dart.dart_streamer_create(dims, (1, 1, 1), t, dart.DART_F32, ring_epochs=3)
    got = [np.zeros((48, 48), np.float32) for _ in views]
    flux, steps = dart.dart_streamer_render(sm, j, b, views, got)
    st = dart.dart_streamer_get_stats(sm)
    print(f"flexload: {st.epochs_loaded} epochs read, {st.epochs_skipped} skipped, "
          f"{st.intervals} intervals", flush=True)
    assert st.epochs_skipped >= 10
    assert st.bytes_uploaded == st.epochs_loaded * 32 ** 3 * 16
    for k in range(2):
        assert int(steps[k]) == int(rsteps[k])
        assert pix_err(got[k], ref[k].astype(np.float64)).max() <= 1e-6
    # a view whose window misses the series entirely gives a zero image
    far = dart.View(40.0, 10.0, 16, 16, 3.0, 100 * L, 0.7)
    z = np.full((16, 16), 7.0, np.float32)
    f2, s2 = dart.dart_streamer_render(sm, j, b, [far], [z])
    assert not z.any() and int(s2[0]) == 0


def test_stream_reports_bad_epoch(env):
    dart, torch = env
    dims = (8, 8, 8)
    j, b, t = synth.random_stack(dims, 5, seed=9, beta_max=0.5, dtype=np.float32)
    b[3, 2, 1, 4, 2] = 1.5          # |beta| > 1 in epoch 3, cell (4, 1, 2)
    sm = dart.dart_streamer_create(dims, (1, 1, 1), t, dart.DART_F32)
    v = dart.View(30.0, 0.0, 16, 16, 1.0, float(t.mean()), 0.6)
    with pytest.raises(dart.DartError) as ei:
        dart.dart_streamer_render(sm, j, b, [v], [np.zeros((16, 16), np.float32)])
    assert ei.value.status == dart.DART_E_RANGE
    assert "epoch 3" in str(ei.value) and "x=4" in str(ei.value)
    with pytest.raises(dart.DartError):
        dart.dart_streamer_create(dims, (1, 1, 1), t, dart.DART_F32, ring_epochs=2)
