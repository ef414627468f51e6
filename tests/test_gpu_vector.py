"""Vector sums through the C ABI (dart_vector_create).

A vector stack joins component stacks that share grid, layout and epoch times.
One march per ray integrates every component's emissivity with the same
chords, epoch weights and the Doppler factor of component 0's velocity, so
component c of every pixel must equal, bit for bit, the scalar render of the
stack (j_c, beta_0), through the plain and the batched kernel, and match the
FP64 oracle's render of (j_c, beta_0) within the storage type's tolerance.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

DIMS = (26, 21, 30)
TIMES = np.linspace(-30.0, 32.0, 6)
TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 2e-3}


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2609_09322_amd as d
    j0, b0, _ = synth.random_stack(DIMS, len(TIMES), seed=61, beta_max=0.85, times=TIMES)
    rng = np.random.default_rng(62)
    # components 1 and 2 signed, like the linear-polarisation Stokes parameters
    extra = [j0 * rng.uniform(-0.8, 0.8, size=j0.shape) for _ in range(2)]
    return d, torch, [j0] + extra, b0


def _sto(d, store):
    return {"f64": d.DART_F64, "f32": d.DART_F32, "f16": d.DART_F16}[store]


def _stacks(d, js, b0, store):
    src = np.float64 if store == "f64" else np.float32
    return [d.dart_load_epochs(DIMS, (1, 1, 1), TIMES, np.ascontiguousarray(j, dtype=src),
                               np.ascontiguousarray(b0, dtype=src), _sto(d, store)) for j in js]


def _views(d, store, flags=0):
    out = d.DART_F64 if store == "f64" else d.DART_F32
    L = synth.diag(DIMS)
    return [d.View(th, ph, W, H, 1.1 * L / max(W, H), 1.5, 0.7, flags, out)
            for th, ph, W, H in [(25.0, 40.0, 37, 29), (90.0, 0.0, 16, 45), (140.0, 250.0, 50, 33)]]


def _host(store, shape):
    return np.zeros(shape, dtype=np.float64 if store == "f64" else np.float32)


@pytest.mark.parametrize("store", ["f64", "f32", "f16"])
@pytest.mark.parametrize("n", [2, 3])
def test_vector_equals_scalar_renders_and_oracle(env, store, n):
    d, torch, js, b0 = env
    comps = _stacks(d, js[:n], b0, store)
    vec = d.dart_vector_create(comps)
    info = d.dart_stack_get_info(vec)
    # the components, and a packed copy of the others' emissivity (a quarter of
    # a record each)
    cb = [d.dart_stack_get_info(c).device_bytes for c in comps]
    assert info.device_bytes == sum(cb) + (n - 1) * cb[0] // 4
    views = _views(d, store)
    dt = torch.float64 if store == "f64" else torch.float32
    # batched: vector views mixed with scalar views of component 0
    vimgs = [torch.zeros((n, v.height, v.width), dtype=dt, device="cuda") for v in views]
    simgs = [torch.zeros((v.height, v.width), dtype=dt, device="cuda") for v in views]
    flux, steps = d.dart_render_batch([vec] * len(views) + [comps[0]] * len(views),
                                      views + views, vimgs + simgs)
    enc = {"f64": None, "f32": "f32", "f16": "f32_as_f16"}[store]
    for k, v in enumerate(views):
        got_b = vimgs[k].cpu().numpy()
        got_p = _host(store, (n, v.height, v.width))
        pf, ps_ = d.dart_render(vec, v, got_p)
        np.testing.assert_array_equal(got_b, got_p)
        assert int(steps[k]) == ps_ == int(steps[len(views) + k])
        np.testing.assert_array_equal(got_b[0], simgs[k].cpu().numpy())
        ov = oracle.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, v.t_obs,
                         v.alpha, 0)
        for c in range(n):
            sc = _host(store, (v.height, v.width))
            d.dart_render(comps[c], v, sc)
            np.testing.assert_array_equal(got_b[c], sc)
            refs = []
            for jj in (js[c], np.abs(js[c])):
                if enc is None:
                    ost = oracle.Stack(jj, b0, TIMES)
                else:
                    ost = oracle.Stack(jj.astype(np.float32), b0.astype(np.float32), TIMES,
                                       encoding=enc)
                refs.append(oracle.render(ost, ov)[0])
            ref, scale = refs
            # signed components cancel along a ray: rounding scales with the
            # sum of |terms|, the render of |j_c| (equal to ref for c = 0)
            floor = 1e-3 * max(scale.max(), 1e-300)
            e = (np.abs(got_b[c].astype(np.float64) - ref) / np.maximum(scale, floor)).max()
            assert e <= TOL[store], (store, n, k, c, e)
        assert flux[k] == pytest.approx(pf, rel=1e-12)
    d.dart_free_epochs(vec)
    for c in comps:
        d.dart_free_epochs(c)


@pytest.mark.parametrize("tuning", [(64, 1, 8, 3, 0, 0, 8), (16, 4, 16, 4, 1, 3, 4)])
def test_vector_batched_launch_shapes_and_accumulate(env, tuning):
    d, torch, js, b0 = env
    # FP64 images: the kernel adds each FP64 pixel sum to the stored value
    comps = _stacks(d, js, b0, "f64")
    vec = d.dart_vector_create(comps)
    views = _views(d, "f64")
    saved = d.dart_get_tuning()
    d.dart_set_tuning(*tuning)
    try:
        imgs = [torch.full((3, v.height, v.width), 0.25, dtype=torch.float64, device="cuda")
                for v in views]
        acc = [d.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, v.t_obs, v.alpha,
                      d.DART_ACCUMULATE | d.DART_DEVICE_PTRS, d.DART_F64) for v in views]
        d.dart_render_batch([vec] * len(views), acc, imgs)
    finally:
        d.dart_set_tuning(saved.tile_w, saved.tile_h, saved.waves_per_cu, saved.order,
                          saved.orient, saved.depth_sync, saved.cells_per_batch or 4)
    for k, v in enumerate(views):
        plain = _host("f64", (3, v.height, v.width))
        d.dart_render(vec, v, plain)
        np.testing.assert_array_equal(imgs[k].cpu().numpy(), 0.25 + plain)


def test_vector_rules(env):
    d, torch, js, b0 = env
    comps = _stacks(d, js, b0, "f32")
    other = d.dart_load_epochs((10, 10, 10), (1, 1, 1), TIMES,
                               np.zeros((len(TIMES), 10, 10, 10), np.float32),
                               np.zeros((len(TIMES), 10, 10, 10, 3), np.float32), d.DART_F32)
    for bad in ([comps[0]], comps + [comps[0], comps[1]], [comps[0], comps[0]], [comps[0], other]):
        with pytest.raises(d.DartError) as ei:
            d.dart_vector_create(bad)
        assert ei.value.status == d.DART_E_INVAL
    d.dart_stack_rebrick(comps[2], (1, 8, 1))
    with pytest.raises(d.DartError):   # another brick shape than component 0
        d.dart_vector_create(comps)
    d.dart_stack_rebrick(comps[2], tuple(d.dart_stack_get_info(comps[0]).brick))
    vec = d.dart_vector_create(comps)
    v = _views(d, "f32")[0]
    img = np.zeros((3, v.height, v.width), np.float32)
    for call in (lambda: d.dart_render(vec, d.View(v.theta_deg, v.phi_deg, v.width, v.height,
                                                   v.pixel_scale, v.t_obs, v.alpha,
                                                   d.DART_EXACT_TIME), img),
                 lambda: d.dart_stack_rebrick(vec, (2, 2, 2)),
                 lambda: d.dart_labelled_create([vec]),
                 lambda: d.dart_vector_create([vec, comps[0]])):
        with pytest.raises(d.DartError) as ei:
            call()
        assert ei.value.status == d.DART_E_INVAL
    with pytest.raises(d.DartError) as ei:
        d.dart_free_epochs(comps[1])
    assert ei.value.status == d.DART_E_BUSY
    srv = d.dart_server_create(16 << 20, max_inflight=4, n_streams=1)
    try:
        out = torch.zeros((3, v.height, v.width), dtype=torch.float32, device="cuda")
        with pytest.raises(d.DartError) as ei:
            d.dart_submit(srv, vec, v, out)
        assert ei.value.status == d.DART_E_INVAL
    finally:
        d.dart_server_destroy(srv)
    # refilling a component is allowed and shows in the next render
    d.dart_render(vec, v, img)
    before = img.copy()
    src = np.ascontiguousarray(2.0 * js[1], dtype=np.float32)
    d.dart_stack_set_epochs(comps[1], 0, src, np.ascontiguousarray(b0, dtype=np.float32))
    d.dart_render(vec, v, img)
    np.testing.assert_array_equal(img[0], before[0])
    np.testing.assert_array_equal(img[2], before[2])
    assert not np.array_equal(img[1], before[1])
    d.dart_free_epochs(vec)
    for c in comps:
        d.dart_free_epochs(c)
