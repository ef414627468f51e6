"""Labelled mode (Sec. 4): a domain given as non-overlapping placed
sub-domains, each with its own resolution, rendered in one pass through the
C ABI (dart_labelled_create) and compared with the FP64 oracle's labelled
render (the sum of its placed sub-domains), and, for fields linear in time,
with the oracle's render of the unrefined grid (pin P15).
"""
import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import labelled_refinement_case, refine

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


def _parts(dart, blocks, t, centre, storage, src):
    out = []
    for jb, bb, cell, org in blocks:
        nz, ny, nx = jb.shape[1:4]
        s = dart.dart_load_epochs((nx, ny, nz), cell, t, np.ascontiguousarray(jb, dtype=src),
                                  np.ascontiguousarray(bb, dtype=src), storage)
        dart.dart_stack_set_placement(s, org, centre)
        out.append(s)
    return out


@pytest.mark.parametrize("sync", [0, 2])
def test_refined_subdomain_equals_coarse_fp64(env, sync):
    dart, torch = env
    (j, beta), blocks, t, centre = labelled_refinement_case()
    lab = dart.dart_labelled_create(_parts(dart, blocks, t, centre, dart.DART_F64, np.float64))
    coarse = oracle.Stack(j, beta, t)
    oparts = [oracle.Stack(jb, bb, t, cell=cell, origin=org, centre=centre)
              for jb, bb, cell, org in blocks]
    saved = dart.dart_get_tuning()
    dart.dart_set_tuning(16, 4, 8, 0, 1, sync)
    try:
        views = [dart.View(th, ph, 40, 36, 0.45, 0.0, 0.7, 0, dart.DART_F64)
                 for th, ph in [(35.0, 20.0), (90.0, 0.0), (128.0, 300.0)]]
        imgs = [torch.zeros((36, 40), dtype=torch.float64, device="cuda") for _ in views]
        flux, steps = dart.dart_render_batch([lab] * 3, views, imgs)
    finally:
        dart.dart_set_tuning(saved.tile_w, saved.tile_h, saved.waves_per_cu, saved.order,
                             saved.orient, saved.depth_sync)
    for k, v in enumerate(views):
        ov = oracle.View(v.theta_deg, v.phi_deg, 40, 36, 0.45, 0.0, 0.7, 0)
        ref, _ = oracle.render(coarse, ov)
        lref, lsteps = oracle.render_labelled(oparts, ov)
        got = imgs[k].cpu().numpy()
        assert pix_err(got, ref).max() <= 1e-12
        assert pix_err(got, lref).max() <= 1e-12
        assert flux[k] == pytest.approx(oracle.flux(lref, ov), rel=1e-12)
        assert abs(int(steps[k]) - lsteps) <= 2


def _jet_blocks(dims, M, seed):
    """A jet grid as three z-sub-domains, the middle one refined twice."""
    import torch
    jd, bd, t = synth.jet_torch(dims, M, seed, gamma_spine=4.0, n_knots=3)
    torch.cuda.synchronize()
    j, b = jd.cpu().numpy(), bd.cpu().numpy()
    nx, ny, nz = dims
    z1, z2 = 40, 88
    blocks = [(j[:, :z1], b[:, :z1], (1.0, 1.0, 1.0), (0.0, 0.0, 0.0)),
              (refine(j[:, z1:z2], 2), refine(b[:, z1:z2], 2), (0.5, 0.5, 0.5), (0.0, 0.0, float(z1))),
              (j[:, z2:], b[:, z2:], (1.0, 1.0, 1.0), (0.0, 0.0, float(z2)))]
    return blocks, t, (0.5 * nx, 0.5 * ny, 0.5 * nz)


@pytest.mark.parametrize("store", ["f32", "f16"])
def test_labelled_jet_batch_and_server(env, store):
    """Three sub-domains (one refined) of a jet grid, rendered in one batch
    with a plain stack beside them, and through the server; every image
    against the oracle's labelled render."""
    dart, torch = env
    dims = (48, 40, 128)
    blocks, t, centre = _jet_blocks(dims, 6, 23)
    storage = dart.DART_F32 if store == "f32" else dart.DART_F16
    parts = _parts(dart, blocks, t, centre, storage, np.float32)
    lab = dart.dart_labelled_create(parts)
    info = dart.dart_stack_get_info(lab)
    assert info.device_bytes == sum(dart.dart_stack_get_info(p).device_bytes for p in parts)
    plain = parts[0]
    L = synth.diag(dims)
    views = [dart.View(th, ph, 64, 48, 1.05 * L / 64, 0.0, 0.6)
             for th, ph in [(10.0, 0.0), (60.0, 45.0), (90.0, 90.0), (140.0, 200.0)]]
    imgs = [torch.zeros((48, 64), dtype=torch.float32, device="cuda") for _ in range(5)]
    flux, steps = dart.dart_render_batch([lab] * 4 + [plain], views + [views[1]], imgs)
    enc = "f32" if store == "f32" else "f32_as_f16"
    oparts = [oracle.Stack(jb, bb, t, cell=cell, encoding=enc, origin=org, centre=centre)
              for jb, bb, cell, org in blocks]
    tol = 1e-5 if store == "f32" else 2e-3
    for k, v in enumerate(views):
        ov = oracle.View(v.theta_deg, v.phi_deg, 64, 48, v.pixel_scale, 0.0, 0.6, 0)
        ref, rs = oracle.render_labelled(oparts, ov)
        got = imgs[k].cpu().numpy()
        e = pix_err(got, ref).max()
        print(f"labelled {store} view {k}: max per-pixel err {e:.3e}", flush=True)
        assert e <= tol
        assert flux[k] == pytest.approx(oracle.flux(ref, ov), rel=1e-6)
        assert abs(int(steps[k]) - rs) <= 1e-5 * rs + 2
    ref0, _ = oracle.render(oparts[0], oracle.View(60.0, 45.0, 64, 48, views[1].pixel_scale, 0.0,
                                                    0.6, 0))
    assert pix_err(imgs[4].cpu().numpy(), ref0).max() <= tol
    # the same labelled renders through the server, bit-identical to the batch
    srv = dart.dart_server_create(64 << 20, max_inflight=8, n_streams=2)
    try:
        outs = [torch.full((48, 64), -1.0, dtype=torch.float32, device="cuda") for _ in views]
        tickets = [dart.dart_submit(srv, lab, v, o) for v, o in zip(views, outs)]
        for tk in tickets:
            dart.dart_wait(srv, tk)
    finally:
        dart.dart_server_destroy(srv)
    torch.cuda.synchronize()
    for k in range(4):
        assert torch.equal(outs[k], imgs[k])


def test_labelled_errors_and_ownership(env):
    dart, torch = env
    dims = (8, 8, 8)
    j, b, t = synth.random_stack(dims, 3, seed=5, beta_max=0.5, dtype=np.float32)
    a = dart.dart_load_epochs(dims, (1, 1, 1), t, j, b, dart.DART_F32)
    c = dart.dart_load_epochs(dims, (1, 1, 1), t, j, b, dart.DART_F32)
    # unplaced sub-domains cannot be joined (more than one)
    with pytest.raises(dart.DartError) as ei:
        dart.dart_labelled_create([a, c])
    assert ei.value.status == dart.DART_E_INVAL
    dart.dart_stack_set_placement(a, (0, 0, 0), (8, 4, 4))
    dart.dart_stack_set_placement(c, (8, 0, 0), (8, 4, 4))
    # other epoch times
    d = dart.dart_load_epochs(dims, (1, 1, 1), t + 1.0, j, b, dart.DART_F32)
    dart.dart_stack_set_placement(d, (0, 8, 0), (8, 4, 4))
    with pytest.raises(dart.DartError) as ei:
        dart.dart_labelled_create([a, d])
    assert ei.value.status == dart.DART_E_INVAL
    lab = dart.dart_labelled_create([a, c])
    for call in (lambda: dart.dart_free_epochs(a), lambda: dart.dart_stack_rebrick(c, (2, 2, 2)),
                 lambda: dart.dart_stack_set_placement(a, (0, 0, 0), (8, 4, 4))):
        with pytest.raises(dart.DartError) as ei:
            call()
        assert ei.value.status == dart.DART_E_BUSY
    v = dart.View(30.0, 0.0, 16, 16, 1.0, float(t.mean()), 0.6)
    for call in (lambda: dart.dart_count_samples(lab, v), lambda: dart.dart_stack_rebrick(lab, (2, 2, 2)),
                 lambda: dart.dart_labelled_create([lab])):
        with pytest.raises(dart.DartError) as ei:
            call()
        assert ei.value.status == dart.DART_E_INVAL
    img = torch.zeros((16, 16), dtype=torch.float32, device="cuda")
    dart.dart_render(lab, v, img)
    one = torch.zeros_like(img)
    dart.dart_render(a, v, one)
    two = torch.zeros_like(img)
    dart.dart_render(c, v, two)
    assert torch.allclose(img, one + two, rtol=1e-6, atol=1e-30)
    torch.cuda.synchronize()
    dart.dart_free_epochs(lab)
    dart.dart_free_epochs(a)   # released by the labelled stack
