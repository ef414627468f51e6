"""The emissivity plane: renders that read a stack's packed emissivity (and
whole records only where a contributing record is marked) against renders of
the same views that read whole records for every cell (DART_RECORDS_ONLY).

The two are the same computation of Eq. 19 on the same stored values, so the
images and cell-steps must agree bit for bit; flux totals are FP64 atomics
whose order varies, so they agree to 1e-12.  Cases: FP32, FP16 and BF16
stacks; the batched kernel with and without depth synchronisation, four and
eight cells per batch and exact temporal integration; the plain kernel; the
plane read through 32-bit offsets (planes up to 4 GiB, the default here) and
through 64-bit addresses (DART_PLANE_ADDR64, the form of larger planes); a
stack with negative and -0 emissivity and -0 velocity components (records
the plane must send to the whole-record path), checked against the FP64
oracle as well; a refill of some epochs (the plane is packed again); and the
byte counts of dart_count_bytes against dart_count_samples.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

DIMS = (96, 80, 160)
M = 8


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    import paper_2609_09322_amd as d
    return d, torch


def _views(d, flags=0):
    L = synth.diag(DIMS)
    out = []
    for th, ph, side in ((10.0, 0.0, 96), (37.0, 21.0, 128), (64.0, 200.0, 80), (90.0, 90.0, 112)):
        out.append(d.View(th, ph, side, side, L / side, 0.0, 0.6, flags))
    return out


def _ro(d, views):
    return [d.View(v.theta_deg, v.phi_deg, v.width, v.height, v.pixel_scale, v.t_obs, v.alpha,
                   v.flags | d.DART_RECORDS_ONLY) for v in views]


def _render_pair(d, torch, st, views, batched=True):
    """Images, flux and steps with the plane and with whole records."""
    out = []
    for vs in (views, _ro(d, views)):
        imgs = [torch.zeros((v.height, v.width), dtype=torch.float32, device="cuda") for v in vs]
        if batched:
            flux, steps = d.dart_render_batch([st] * len(vs), vs, imgs)
        else:
            flux, steps = [], []
            for v, im in zip(vs, imgs):
                f, s = d.dart_render(st, v, im)
                flux.append(f)
                steps.append(s)
        torch.cuda.synchronize()
        out.append(([im.cpu().numpy() for im in imgs], np.asarray(flux, np.float64),
                    np.asarray(steps, np.uint64)))
    return out


def _assert_same(pair, what):
    (ia, fa, sa), (ib, fb, sb) = pair
    for k, (a, b) in enumerate(zip(ia, ib)):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"{what}: image {k} differs"
    assert np.array_equal(sa, sb), f"{what}: cell-steps {sa} vs {sb}"
    assert np.allclose(fa, fb, rtol=1e-12, atol=0), f"{what}: flux {fa} vs {fb}"
    assert np.all(sa > 0)


def _plane_bytes(d, st):
    return d.dart_stack_get_info(st).device_bytes


@pytest.fixture()
def keep_tuning(env):
    d, _ = env
    t = d.dart_get_tuning()
    yield
    d.dart_set_tuning(t.tile_w, t.tile_h, t.waves_per_cu, t.order, t.orient, t.depth_sync,
                      t.cells_per_batch)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_plane_equals_records(env, keep_tuning, storage):
    d, torch = env
    j, b, times = synth.jet_torch(DIMS, M, 11, gamma_spine=5.0, n_knots=4)
    kind = {"f32": d.DART_F32, "f16": d.DART_F16, "bf16": d.DART_BF16}[storage]
    st = d.dart_load_epochs(DIMS, (1, 1, 1), times, j, b, kind)
    del j, b
    before = _plane_bytes(d, st)
    views = _views(d)
    try:
        for sync, k in ((0, 4), (6, 8), (3, 4), (0, 8)):
            d.dart_set_tuning(16, 4, 12, 4, 1, sync, k)
            _assert_same(_render_pair(d, torch, st, views), f"{storage} sync {sync} k {k}")
            print(f"{storage} sync {sync} k {k}: identical", flush=True)
        ex = _views(d, d.DART_EXACT_TIME)
        _assert_same(_render_pair(d, torch, st, ex), f"{storage} exact time")
        _assert_same(_render_pair(d, torch, st, views[:2], batched=False), f"{storage} plain")
        # the plane through 64-bit addresses
        wide = _views(d, d.DART_PLANE_ADDR64)
        for sync, k in ((0, 4), (6, 8)):
            d.dart_set_tuning(16, 4, 12, 4, 1, sync, k)
            _assert_same(_render_pair(d, torch, st, wide), f"{storage} 64-bit sync {sync} k {k}")
        wex = _views(d, d.DART_EXACT_TIME | d.DART_PLANE_ADDR64)
        _assert_same(_render_pair(d, torch, st, wex), f"{storage} 64-bit exact time")
        _assert_same(_render_pair(d, torch, st, wide[:2], batched=False), f"{storage} 64-bit plain")
        print(f"{storage} 64-bit plane addresses: identical", flush=True)
        # the plane is a quarter of the record bytes
        after = _plane_bytes(d, st)
        assert after - before == before // 4, (before, after)
    finally:
        d.dart_free_epochs(st)


def test_marked_records_and_refill(env, keep_tuning):
    """Negative and -0 emissivity, -0 velocity components: the plane marks those
    records to be read whole; the images equal the whole-record render and the
    FP64 oracle.  A refill of two epochs repacks the plane."""
    d, torch = env
    dims = (48, 40, 64)
    j, b, times = synth.jet_torch(dims, 4, 5, gamma_spine=4.0, n_knots=2)
    torch.cuda.synchronize()
    jh, bh = j.cpu().numpy(), b.cpu().numpy()
    rng = np.random.default_rng(3)
    for m in range(4):
        cells = rng.choice(jh[m].size, size=jh[m].size // 50, replace=False)
        jf = jh[m].reshape(-1)
        jf[cells[: len(cells) // 2]] *= -1.0                  # negative emissivity
        jf[cells[len(cells) // 2: len(cells) // 2 + 20]] = -0.0
        bf = bh[m].reshape(-1, 3)
        bf[cells[-40:], 1] = -0.0                             # -0 velocity component
    st = d.dart_load_epochs(dims, (1, 1, 1), times, jh, bh, d.DART_F32)
    L = synth.diag(dims)
    views = [d.View(th, ph, 64, 64, L / 64, 0.0, 0.7) for th, ph in ((15.0, 5.0), (75.0, 130.0))]
    try:
        d.dart_set_tuning(16, 4, 12, 4, 1, 6, 8)
        pair = _render_pair(d, torch, st, views)
        _assert_same(pair, "marked records")
        ost = oracle.Stack(jh, bh, times)
        for k, v in enumerate(views):
            ov = oracle.View(v.theta_deg, v.phi_deg, 64, 64, v.pixel_scale, 0.0, 0.7, 0)
            ref, _ = oracle.render(ost, ov)
            got = pair[0][0][k].astype(np.float64)
            floor = 1e-3 * np.abs(ref).max()
            err = np.abs(got - ref) / np.maximum(np.abs(ref), floor)
            assert err.max() <= 1e-5, err.max()
        # refill epochs 1 and 2 with other values: the next render repacks
        j2, b2, _ = synth.jet_torch(dims, 4, 9, gamma_spine=3.0, n_knots=1, times=times)
        torch.cuda.synchronize()
        d.dart_stack_set_epochs(st, 1, j2[1:3].contiguous(), b2[1:3].contiguous())
        pair2 = _render_pair(d, torch, st, views)
        _assert_same(pair2, "after refill")
        assert not np.array_equal(pair2[0][0][0], pair[0][0][0])
    finally:
        d.dart_free_epochs(st)


def test_count_bytes(env):
    """Plane-aware byte counts: with the plane every sample costs a quarter
    record and marked samples a record more; DART_RECORDS_ONLY counts records."""
    d, torch = env
    j, b, times = synth.jet_torch(DIMS, M, 11, gamma_spine=5.0, n_knots=4)
    st = d.dart_load_epochs(DIMS, (1, 1, 1), times, j, b, d.DART_F16)
    del j, b
    try:
        for v in _views(d):
            samples = d.dart_count_samples(st, v)
            lines = d.dart_count_lines(st, v)
            comp, lb = d.dart_count_bytes(st, v)
            rv = _ro(d, [v])[0]
            rcomp, rlb = d.dart_count_bytes(st, rv)
            assert rcomp == samples * 8 and rlb == lines * 128
            # at least one plane value per sample, at most plane + record each
            assert samples * 2 <= comp <= samples * 10
            assert (comp - samples * 2) % 8 == 0
            assert comp < rcomp, (comp, rcomp)   # the jet's volume is mostly at rest
            assert lb > 0
            print(f"view {v.theta_deg}: samples {samples}, plane bytes {comp} vs records {rcomp}, "
                  f"lines {lb} vs {rlb}", flush=True)
    finally:
        d.dart_free_epochs(st)


def test_batched_writes_every_pixel(env, keep_tuning):
    """Tiles whose rays all miss the grid are not marched: a fill kernel
    writes their zeros.  Images prefilled with NaN must come out equal, bit for
    bit, to the plain kernel's (which writes every pixel), for FP32 and FP64
    images; an adding view (DART_ACCUMULATE) keeps its prior values there."""
    d, torch = env
    dims = (40, 48, 56)
    j, b, times = synth.jet_torch(dims, 3, 21, gamma_spine=3.0, n_knots=1)
    torch.cuda.synchronize()
    jh, bh = j.cpu().numpy(), b.cpu().numpy()
    s32 = d.dart_load_epochs(dims, (1, 1, 1), times, j, b, d.DART_F32)
    s64 = d.dart_load_epochs(dims, (1, 1, 1), times, jh.astype(np.float64), bh.astype(np.float64),
                             d.DART_F64)
    L = synth.diag(dims)
    try:
        for tile in ((64, 1, 0), (16, 4, 6), (8, 8, 0)):
            d.dart_set_tuning(tile[0], tile[1], 8, 4, 1, tile[2], 8)
            for st, dt, npdt in ((s32, d.DART_F32, np.float32), (s64, d.DART_F64, np.float64)):
                # images twice the grid's extent: most tiles miss it
                # (axis-aligned views see edges end-on; the others cut corners
                # off the projection's bounding rectangle)
                views = [d.View(th, ph, 100, 72, 2.0 * L / 100, 1.0, 0.6, 0, dt)
                         for th, ph in ((20.0, 10.0), (75.0, 240.0), (0.0, 0.0), (90.0, 0.0),
                                        (90.0, 90.0), (54.7, 45.0), (123.0, 301.0),
                                        (170.0, 77.0))]
                tdt = torch.float32 if npdt == np.float32 else torch.float64
                got = [torch.full((v.height, v.width), float("nan"), dtype=tdt, device="cuda")
                       for v in views]
                ref = [torch.zeros((v.height, v.width), dtype=tdt, device="cuda") for v in views]
                d.dart_render_batch([st] * len(views), views, got)
                for v, im in zip(views, ref):
                    d.dart_render(st, v, im)
                torch.cuda.synchronize()
                for a, r in zip(got, ref):
                    an, rn = a.cpu().numpy(), r.cpu().numpy()
                    assert not np.isnan(an).any(), f"unwritten pixels, tile {tile}"
                    assert np.array_equal(an, rn), f"tile {tile}"
                    assert (rn == 0).mean() > 0.3      # the views are mostly sky
        # adding views keep their values where no ray reaches the grid
        d.dart_set_tuning(16, 4, 8, 4, 1, 0, 8)
        views = [d.View(30.0, 50.0, 100, 72, 2.0 * L / 100, 1.0, 0.6, d.DART_ACCUMULATE)]
        got = [torch.full((72, 100), 1.5, dtype=torch.float32, device="cuda")]
        ref = [torch.full((72, 100), 1.5, dtype=torch.float32, device="cuda")]
        d.dart_render_batch([s32], views, got)
        d.dart_render(s32, views[0], ref[0])
        torch.cuda.synchronize()
        assert np.array_equal(got[0].cpu().numpy(), ref[0].cpu().numpy())
    finally:
        d.dart_free_epochs(s32)
        d.dart_free_epochs(s64)
