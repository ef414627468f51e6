"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Per-pixel error is |gpu - oracle| / max(|oracle|, 1e-3 max|oracle|) (a floor
for grazing rays with tiny chords); the bars are 1e-12 for FP64 stacks, 1e-5
for FP32 stacks and 2e-3 for FP16/BF16 stacks, total flux within 1e-6 (1e-12
for FP64).  16-bit parity compares with the oracle run on the dequantised
stored values (rounded on the host by numpy, independently of the kernels).
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 2e-3, "bf16": 2e-3}
FLUX_TOL = {"f64": 1e-12, "f32": 1e-6, "f16": 1e-6, "bf16": 1e-6}


@pytest.fixture(scope="module")
def dart():
    import torch
    assert torch.cuda.is_available()
    import paper_2609_09322_amd as d
    return d


def _store(d, name):
    return {"f64": d.DART_F64, "f32": d.DART_F32, "f16": d.DART_F16, "bf16": d.DART_BF16}[name]


def _dequant(x, name):
    if name == "f64":
        return np.asarray(x, dtype=np.float64)
    x32 = np.asarray(x, dtype=np.float32)
    if name == "f32":
        return x32
    return synth.round_f16(x32) if name == "f16" else synth.round_bf16(x32)


def pix_err(gpu, ref):
    floor = 1e-3 * max(np.abs(ref).max(), 1e-300)
    return np.abs(np.asarray(gpu, np.float64) - ref) / np.maximum(np.abs(ref), floor)


def _render_both(dart, j, beta, times, store, view_args, flags=0, dims=None, cell=(1, 1, 1),
                 batch=False):
    nz, ny, nx = j.shape[1:4]
    dims = dims or (nx, ny, nz)
    src = np.float64 if store == "f64" else np.float32
    st = dart.dart_load_epochs(dims, cell, times, np.ascontiguousarray(j, dtype=src),
                               np.ascontiguousarray(beta, dtype=src), _store(dart, store))
    th, ph, W, H, ps, t_obs, alpha = view_args
    out64 = store == "f64"
    v = dart.View(th, ph, W, H, ps, t_obs, alpha, flags, dart.DART_F64 if out64 else dart.DART_F32)
    img = np.zeros((H, W), dtype=np.float64 if out64 else np.float32)
    if batch:
        f, s = dart.dart_render_batch([st], [v], [img])
        flux, steps = float(f[0]), int(s[0])
    else:
        flux, steps = dart.dart_render(st, v, img)
    ostack = oracle.Stack(_dequant(j, store).astype(np.float64), _dequant(beta, store).astype(np.float64),
                          times, cell=cell)
    ov = oracle.View(th, ph, W, H, ps, t_obs, alpha, flags & 7)
    ref, ref_steps = oracle.render(ostack, ov)
    return img, flux, steps, ref, oracle.flux(ref, ov), ref_steps


def test_config1_blobs_fp64(dart):
    """64^3 three-blob stack, FP64, theta 30, 128^2 at 0.5 cell/px, t_obs 1.5."""
    j, beta, t = synth.blobs(seed=1)
    img, flux, steps, ref, rflux, rsteps = _render_both(
        dart, j, beta, t, "f64", (30.0, 0.0, 128, 128, 0.5, 1.5, 0.7))
    print("config1 max err", pix_err(img, ref).max(), "steps", steps, rsteps)
    assert pix_err(img, ref).max() <= TOL["f64"]
    assert flux == pytest.approx(rflux, rel=FLUX_TOL["f64"])
    assert abs(steps - rsteps) <= max(2, 1e-5 * rsteps)


def test_config1b_full_window_fp64(dart):
    """Epoch times x64 and t_obs = 96: the window covers the whole grid."""
    j, beta, t = synth.blobs(seed=1, times=(0.0, 64.0, 128.0, 192.0), speed=0.6 / 64)
    img, flux, steps, ref, rflux, rsteps = _render_both(
        dart, j, beta, t, "f64", (30.0, 0.0, 128, 128, 0.5, 96.0, 0.7))
    assert rsteps > 1_000_000
    assert pix_err(img, ref).max() <= TOL["f64"]
    assert flux == pytest.approx(rflux, rel=FLUX_TOL["f64"])
    assert abs(steps - rsteps) <= max(2, 1e-5 * rsteps)


VIEWS = [(90.0, 0.0), (0.0, 0.0), (180.0, 0.0), (90.0, 90.0), (37.0, 211.0), (89.5, 0.3),
         (1e-3, 45.0), (123.0, 300.0)]


@pytest.mark.parametrize("store", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("flags", [0, 1, 2, 4])
def test_random_grids_all_storage(dart, store, flags):
    """Random fields on a small ragged grid, cardinal, grazing and oblique
    views, every storage type and routine (lookback, no lookback, no beaming,
    nearest epoch)."""
    dims = (13, 9, 11)
    j, beta, t = synth.random_stack(dims, 6, seed=7, beta_max=0.9, j_range=(0.1, 1.0))
    L = synth.diag(dims)
    t_obs = float(0.5 * (t[0] + t[-1]))
    for th, ph in VIEWS:
        img, flux, steps, ref, rflux, rsteps = _render_both(
            dart, j, beta, t, store, (th, ph, 37, 29, 1.05 * L / 33, t_obs, 0.6), flags=flags,
            cell=(1.0, 0.9, 1.2))
        e = pix_err(img, ref).max()
        assert e <= TOL[store], (store, flags, th, ph, e)
        if rflux:
            assert flux == pytest.approx(rflux, rel=max(FLUX_TOL[store], 1e-12)), (store, th, ph)


@pytest.mark.parametrize("store", ["f32", "f16"])
@pytest.mark.parametrize("sync", [0, 1, 3])
def test_batch_equals_plain_and_oracle(dart, store, sync):
    """The persistent batched kernel gives the same pixels as the plain kernel
    and as the oracle, with images of ragged sizes and mixed stacks; also with
    depth-synchronous marching (sync > 0), which changes only the order in
    which a wavefront's rays take their cells."""
    import torch
    saved = dart.dart_get_tuning()
    dart.dart_set_tuning(32, 2, 8, 0, 1, sync)
    try:
        _batch_equals_plain_and_oracle(dart, store, torch)
    finally:
        dart.dart_set_tuning(saved.tile_w, saved.tile_h, saved.waves_per_cu, saved.order,
                             saved.orient, saved.depth_sync)


@pytest.mark.parametrize("sync", [0, 2])
def test_eight_cells_per_batch_keeps_pixels(dart, sync):
    """Walking 8 cells per batch instead of 4 changes when records are
    requested, not what is summed: the plain kernel's pixels bit for bit."""
    import torch
    saved = dart.dart_get_tuning()
    dart.dart_set_tuning(32, 2, 8, 3, 1, sync, 8)
    try:
        assert dart.dart_get_tuning().cells_per_batch == 8
        for store in ("f32", "f16"):
            _batch_equals_plain_and_oracle(dart, store, torch)
    finally:
        dart.dart_set_tuning(saved.tile_w, saved.tile_h, saved.waves_per_cu, saved.order,
                             saved.orient, saved.depth_sync, saved.cells_per_batch or 4)


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_tile_orders_keep_pixels(dart, order):
    """Every tile queue order (longest first, Z-order, rows from the middle
    outward, heavy rows dealt to the queues) gives the plain kernel's pixels
    bit for bit."""
    import torch
    saved = dart.dart_get_tuning()
    dart.dart_set_tuning(16, 4, 8, order, 1, 0)
    try:
        _batch_equals_plain_and_oracle(dart, "f32", torch)
    finally:
        dart.dart_set_tuning(saved.tile_w, saved.tile_h, saved.waves_per_cu, saved.order,
                             saved.orient, saved.depth_sync)


def _batch_equals_plain_and_oracle(dart, store, torch):
    dims_a, dims_b = (24, 20, 28), (16, 16, 16)
    ja, ba, ta = synth.random_stack(dims_a, 5, seed=1, beta_max=0.8)
    jb, bb, tb = synth.random_stack(dims_b, 3, seed=2, beta_max=0.8)
    src = np.float32
    sa = dart.dart_load_epochs(dims_a, (1, 1, 1), ta, ja.astype(src), ba.astype(src), _store(dart, store))
    sb = dart.dart_load_epochs(dims_b, (1, 1, 1), tb, jb.astype(src), bb.astype(src), _store(dart, store))
    views, stacks, host = [], [], []
    rng = np.random.default_rng(5)
    for k in range(7):
        s, t, dims = (sa, ta, dims_a) if k % 2 == 0 else (sb, tb, dims_b)
        W, H = int(rng.integers(5, 90)), int(rng.integers(3, 70))
        v = dart.View(float(rng.uniform(0, 180)), float(rng.uniform(0, 360)), W, H,
                      1.1 * synth.diag(dims) / max(W, H), float(t.mean()), 0.7)
        views.append(v)
        stacks.append(s)
        host.append((dims, t, (ja, ba) if k % 2 == 0 else (jb, bb)))
    imgs = [torch.zeros((v.height, v.width), dtype=torch.float32, device="cuda") for v in views]
    flux, steps = dart.dart_render_batch(stacks, views, imgs)
    for k, v in enumerate(views):
        plain = np.zeros((v.height, v.width), dtype=np.float32)
        pf, ps_ = dart.dart_render(stacks[k], v, plain)
        got = imgs[k].cpu().numpy()
        np.testing.assert_array_equal(got, plain)
        assert int(steps[k]) == ps_
        assert flux[k] == pytest.approx(pf, rel=1e-12)
        dims, t, (jj, bb_) = host[k]
        ost = oracle.Stack(_dequant(jj, store).astype(np.float64), _dequant(bb_, store).astype(np.float64), t)
        ref, rs = oracle.render(ost, oracle.View(v.theta_deg, v.phi_deg, v.width, v.height,
                                                 v.pixel_scale, v.t_obs, v.alpha, 0))
        assert pix_err(got, ref).max() <= TOL[store]


@pytest.mark.parametrize("store", ["f32", "f16"])
@pytest.mark.parametrize("sync", [0, 2])
def test_one_epoch_walks_mixed_in_a_batch(dart, store, sync):
    """Views that take one epoch per cell (nearest-epoch mode, a one-epoch
    stack) and views that interpolate run in one batched launch; each wave
    picks its walk from its view.  Pixels equal the plain kernel's bit for bit
    and match the oracle."""
    import torch
    dims = (21, 17, 19)
    j, b, t = synth.random_stack(dims, 5, seed=23, beta_max=0.8)
    src = np.float32
    s5 = dart.dart_load_epochs(dims, (1, 1, 1), t, j.astype(src), b.astype(src), _store(dart, store))
    s1 = dart.dart_load_epochs(dims, (1, 1, 1), t[:1], j[:1].astype(src), b[:1].astype(src),
                               _store(dart, store))
    L = synth.diag(dims)
    tm = float(t.mean())
    spec = [(s5, 0, 40.0, 30.0, tm), (s5, dart.DART_NEAREST_EPOCH, 40.0, 30.0, tm),
            (s5, dart.DART_NEAREST_EPOCH | dart.DART_NO_LOOKBACK, 75.0, 200.0, tm),
            (s1, dart.DART_NO_LOOKBACK, 120.0, 10.0, float(t[0])), (s5, dart.DART_NO_LOOKBACK, 10.0, 80.0, tm),
            (s1, dart.DART_NEAREST_EPOCH | dart.DART_NO_LOOKBACK, 90.0, 45.0, float(t[0]))]
    stacks, views = [], []
    for k, (st, fl, th, ph, to) in enumerate(spec):
        W, H = 23 + 5 * k, 19 + 3 * k
        stacks.append(st)
        views.append(dart.View(th, ph, W, H, 1.1 * L / max(W, H), to, 0.6, fl))
    saved = dart.dart_get_tuning()
    dart.dart_set_tuning(16, 4, 8, 3, 1, sync, 8)
    try:
        imgs = [torch.zeros((v.height, v.width), dtype=torch.float32, device="cuda") for v in views]
        flux, steps = dart.dart_render_batch(stacks, views, imgs)
    finally:
        dart.dart_set_tuning(saved.tile_w, saved.tile_h, saved.waves_per_cu, saved.order,
                             saved.orient, saved.depth_sync, saved.cells_per_batch or 4)
    for k, v in enumerate(views):
        plain = np.zeros((v.height, v.width), dtype=np.float32)
        pf, ps_ = dart.dart_render(stacks[k], v, plain)
        got = imgs[k].cpu().numpy()
        np.testing.assert_array_equal(got, plain)
        assert int(steps[k]) == ps_
        M = 1 if stacks[k] is s1 else 5
        ost = oracle.Stack(_dequant(j[:M], store).astype(np.float64),
                           _dequant(b[:M], store).astype(np.float64), t[:M])
        ref, rs = oracle.render(ost, oracle.View(v.theta_deg, v.phi_deg, v.width, v.height,
                                                 v.pixel_scale, v.t_obs, v.alpha, v.flags & 7))
        assert ref.max() > 0, k
        assert pix_err(got, ref).max() <= TOL[store], (store, sync, k)
    dart.dart_free_epochs(s1)
    dart.dart_free_epochs(s5)


@pytest.mark.parametrize("on_stream", [False, True])
def test_replay_follows_a_new_stack(dart, on_stream):
    """A batched call repeated with the same arguments replays its cached plan;
    a stack freed and replaced (often at the same host address) must not be
    taken for the old one: the images follow the new stack's data."""
    import torch
    dims = (20, 18, 22)
    views = [dart.View(35.0, 40.0, 33, 27, 1.1 * synth.diag(dims) / 33, 0.0, 0.7)]
    img = [torch.zeros((27, 33), dtype=torch.float32, device="cuda")]
    stream = torch.cuda.Stream() if on_stream else None
    for seed in (3, 4, 5):
        j, b, t = synth.random_stack(dims, 4, seed=seed, beta_max=0.7,
                                     times=np.linspace(-20.0, 20.0, 4))
        st = dart.dart_load_epochs(dims, (1, 1, 1), t, j.astype(np.float32), b.astype(np.float32),
                                   dart.DART_F32)
        for _ in range(2):
            dart.dart_render_batch([st], views, img, stream=stream)
        torch.cuda.synchronize()
        plain = np.zeros((27, 33), dtype=np.float32)
        dart.dart_render(st, views[0], plain)
        np.testing.assert_array_equal(img[0].cpu().numpy(), plain)
        dart.dart_free_epochs(st)
        del st


def test_graph_replay_is_stable(dart):
    """Repeated identical batch calls replay a captured graph: every replay
    must reproduce the first result exactly."""
    import torch
    dims = (32, 32, 32)
    j, b, t = synth.random_stack(dims, 4, seed=3, beta_max=0.9)
    s = dart.dart_load_epochs(dims, (1, 1, 1), t, j.astype(np.float32), b.astype(np.float32), dart.DART_F32)
    views = [dart.View(th, 20.0, 96, 80, 0.6, float(t.mean()), 0.6) for th in (15.0, 70.0, 130.0)]
    imgs = [torch.zeros((v.height, v.width), dtype=torch.float32, device="cuda") for v in views]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        f0, s0 = dart.dart_render_batch([s] * 3, views, imgs, stream=stream)
        first = [im.clone() for im in imgs]
        for rep in range(4):
            for im in imgs:
                im.fill_(-1.0)
            torch.cuda.synchronize()
            f, st = dart.dart_render_batch([s] * 3, views, imgs, stream=stream)
            torch.cuda.synchronize()
            for a, b_ in zip(imgs, first):
                assert torch.equal(a, b_)
            np.testing.assert_array_equal(st, s0)
            np.testing.assert_allclose(f, f0, rtol=1e-12)


def test_count_samples_matches_oracle(dart):
    dims = (12, 10, 14)
    j, b, t = synth.random_stack(dims, 5, seed=9, beta_max=0.5)
    s = dart.dart_load_epochs(dims, (1, 1, 1), t, j, b, dart.DART_F64)
    for th, ph, ps in [(40.0, 30.0, 0.7), (90.0, 0.0, 0.5), (120.0, 200.0, 1.6)]:
        v = dart.View(th, ph, 40, 36, ps, float(t.mean()), 0.7)
        got = dart.dart_count_samples(s, v)
        want = oracle.count_samples(oracle.Stack(j, b, t), oracle.View(th, ph, 40, 36, ps, float(t.mean()), 0.7, 0))
        assert abs(got - want) <= max(2, 1e-4 * want), (got, want)


@pytest.mark.parametrize("store,brick", [("f32", (1, 8, 1)), ("f32", (2, 2, 2)), ("f16", (4, 2, 2)),
                                         ("bf16", (1, 1, 16))])
def test_count_lines_matches_oracle_blocks(dart, store, brick):
    """With a brick of exactly one 128-byte line of records, the distinct lines
    a view reads are the distinct (brick, epoch) pairs the oracle counts from
    the geometry alone."""
    dims = (16, 16, 32)
    j, b, t = synth.random_stack(dims, 5, seed=19, beta_max=0.5, dtype=np.float32)
    s = dart.dart_load_epochs(dims, (1, 1, 1), t, j, b, _store(dart, store))
    dart.dart_stack_rebrick(s, brick)
    for th, ph, ps in [(40.0, 30.0, 0.7), (90.0, 0.0, 1.3), (120.0, 200.0, 2.6)]:
        v = dart.View(th, ph, 48, 40, ps, float(t.mean()), 0.7)
        got = dart.dart_count_lines(s, v)
        want = oracle.count_blocks(dims, t, oracle.View(th, ph, 48, 40, ps, float(t.mean()), 0.7, 0),
                                   brick)
        assert abs(got - want) <= max(2, 1e-4 * want), (got, want)


def test_edge_cases(dart):
    dims = (9, 9, 9)
    j, b, t = synth.random_stack(dims, 3, seed=4, beta_max=0.6)
    s = dart.dart_load_epochs(dims, (1, 1, 1), t, j.astype(np.float32), b.astype(np.float32), dart.DART_F32)
    # every ray misses (pixel centres 50-150 cells off the grid): zeros written
    img = np.full((4, 4), 7.0, dtype=np.float32)
    f, n = dart.dart_render(s, dart.View(30.0, 0.0, 4, 4, 100.0, float(t.mean()), 0.6), img)
    assert n == 0 and f == 0.0 and not img.any()
    img = np.full((3, 5), 7.0, dtype=np.float32)
    # t_obs outside the epoch coverage without lookback: zero image
    f, n = dart.dart_render(s, dart.View(30.0, 0.0, 5, 3, 1.0, float(t[-1] + 100), 0.6,
                                         dart.DART_NO_LOOKBACK), img)
    assert n == 0 and f == 0.0 and not img.any()
    # a 1x1 image
    one = np.zeros((1, 1), dtype=np.float32)
    f, n = dart.dart_render(s, dart.View(45.0, 45.0, 1, 1, 0.3, float(t.mean()), 0.6), one)
    ref, _ = oracle.render(oracle.Stack(j.astype(np.float32).astype(np.float64),
                                        b.astype(np.float32).astype(np.float64), t),
                           oracle.View(45.0, 45.0, 1, 1, 0.3, float(t.mean()), 0.6, 0))
    assert pix_err(one, ref).max() <= 1e-5
    # single epoch with NO_LOOKBACK at exactly t_0
    s1 = dart.dart_load_epochs(dims, (1, 1, 1), t[:1], j[:1].astype(np.float32), b[:1].astype(np.float32), dart.DART_F32)
    im1 = np.zeros((10, 10), dtype=np.float32)
    dart.dart_render(s1, dart.View(60.0, 10.0, 10, 10, 1.4, float(t[0]), 0.6, dart.DART_NO_LOOKBACK), im1)
    ref1, _ = oracle.render(oracle.Stack(j[:1].astype(np.float32).astype(np.float64),
                                         b[:1].astype(np.float32).astype(np.float64), t[:1]),
                            oracle.View(60.0, 10.0, 10, 10, 1.4, float(t[0]), 0.6, 1))
    assert pix_err(im1, ref1).max() <= 1e-5


def test_long_rays_fp64_dda(dart):
    """A 4608 x 8 x 8 grid lets rays cross > 4096 cells: the ray parameters
    switch to FP64 by themselves; the result matches the oracle."""
    dims = (4608, 8, 8)
    rng = np.random.default_rng(12)
    M = 3
    jf = rng.uniform(0.5, 1.0, size=(M, 8, 8, 4608)).astype(np.float32)
    bf = np.zeros((M, 8, 8, 4608, 3), dtype=np.float32)
    bf[..., 0] = rng.uniform(-0.5, 0.5, size=(M, 8, 8, 4608))
    t = np.array([-5000.0, 0.0, 5000.0])
    s = dart.dart_load_epochs(dims, (1, 1, 1), t, jf, bf, dart.DART_F32)
    ost = oracle.Stack(jf.astype(np.float64), bf.astype(np.float64), t)
    for th, ph in [(89.985, 0.01), (90.0, 0.02)]:
        v = dart.View(th, ph, 12, 12, 0.6, 0.0, 0.6)
        img = np.zeros((12, 12), dtype=np.float32)
        f, n = dart.dart_render(s, v, img)
        ref, rn = oracle.render(ost, oracle.View(th, ph, 12, 12, 0.6, 0.0, 0.6, 0))
        assert rn > 12 * 12 * 4096
        assert pix_err(img, ref).max() <= 1e-5


def test_validation_errors(dart):
    dims = (4, 4, 4)
    j = np.ones((2, 4, 4, 4))
    b = np.zeros((2, 4, 4, 4, 3))
    t = np.array([0.0, 1.0])
    bad = b.copy()
    bad[1, 2, 3, 1, 2] = 1.0
    with pytest.raises(dart.DartError) as e:
        dart.dart_load_epochs(dims, (1, 1, 1), t, j, bad, dart.DART_F64)
    assert e.value.status == dart.DART_E_RANGE and "x=1, y=3, z=2" in str(e.value)
    nan = j.copy()
    nan[0, 0, 0, 0] = np.nan
    with pytest.raises(dart.DartError) as e:
        dart.dart_load_epochs(dims, (1, 1, 1), t, nan, b, dart.DART_F64)
    assert e.value.status == dart.DART_E_RANGE
    # rounds to |beta| = 1 in bfloat16 although it is < 1 in FP32
    near = b.copy().astype(np.float32)
    near[..., 2] = 0.999
    with pytest.raises(dart.DartError) as e:
        dart.dart_load_epochs(dims, (1, 1, 1), t, j.astype(np.float32), near, dart.DART_BF16)
    assert e.value.status == dart.DART_E_RANGE
    big = j.astype(np.float32) * 1e6
    with pytest.raises(dart.DartError) as e:
        dart.dart_load_epochs(dims, (1, 1, 1), t, big, b.astype(np.float32), dart.DART_F16)
    assert e.value.status == dart.DART_E_RANGE
    with pytest.raises(dart.DartError) as e:
        dart.dart_load_epochs(dims, (1, 1, 1), np.array([1.0, 1.0]), j, b, dart.DART_F64)
    assert e.value.status == dart.DART_E_INVAL
    s = dart.dart_load_epochs(dims, (1, 1, 1), t, j, b, dart.DART_F64)
    img = np.zeros((4, 4))
    for vv in [dart.View(0, 0, 0, 4, 1.0, 0.5, 0.6, 0, dart.DART_F64),
               dart.View(0, 0, 4, 4, -1.0, 0.5, 0.6, 0, dart.DART_F64),
               dart.View(float("nan"), 0, 4, 4, 1.0, 0.5, 0.6, 0, dart.DART_F64)]:
        with pytest.raises(dart.DartError) as e:
            dart.dart_render(s, vv, img)
        assert e.value.status == dart.DART_E_INVAL
    s32 = dart.dart_load_epochs(dims, (1, 1, 1), t, j.astype(np.float32), b.astype(np.float32), dart.DART_F32)
    with pytest.raises(dart.DartError):
        dart.dart_render(s32, dart.View(0, 0, 4, 4, 1.0, 0.5, 0.6, 0, dart.DART_F64), img)


def test_bandwidth_probes(dart):
    """The measurement probes: the copy writes an exact copy, the read-only and
    gather passes run over a buffer whose size is not a multiple of their grid
    (and the gather probe rejects a line count that is not a power of two)."""
    import torch
    n = (1 << 20) + 16 * 37  # bytes: a ragged tail for the copy and the read pass
    src = torch.arange(n // 4, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    dart.dart_bandwidth_probe(dst, src, n, 2)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    dart.dart_bandwidth_probe(None, src, n, 3)
    g = torch.ones((128 << 12) // 4, dtype=torch.float32, device="cuda")
    dart.dart_gather_probe(g, 128 << 12, 3)
    torch.cuda.synchronize()
    with pytest.raises(dart.DartError) as ei:
        dart.dart_gather_probe(g, 128 * 3000, 1)
    assert ei.value.status == dart.DART_E_INVAL
    assert float(g.sum()) == g.numel()
