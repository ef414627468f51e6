"""Bit-exact checks of the device-side 16-bit store (the load step: caller
fields -> resident records, round to nearest even, Sec. 2.5's inputs j' and
beta), of the 32-bit offset and tile-coordinate guards, and of the epoch
read-back.

The expected 16-bit values come from an exact rounding written here from the
definition of the two formats (the value as a rational number, scaled to the
format's quantum at its exponent, rounded half to even by Python's exact
integer arithmetic), not from any library routine the kernels use; numpy's
binary16 conversion is a second, independent reference for FP16.  Inputs
cover exact ties, values one source ulp beside a tie, FP64 values whose
rounding through FP32 would tie (double rounding), subnormals of both
formats, the largest finite values, and velocities that round to 1 (which
the load must refuse).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# (significand bits incl. the implicit one, smallest normal exponent, largest finite)
FORMATS = {"f16": (11, -14, 65504.0), "bf16": (8, -126, float.fromhex("0x1.fep127"))}


def round16(x, kind):
    """Nearest value of the 16-bit format to the finite float x (ties to even),
    as a Python float; +-inf when it overflows."""
    bits, emin, big = FORMATS[kind]
    if x == 0.0:
        return x
    fx = Fraction(x)
    ax = abs(fx)
    e = math.frexp(abs(x))[1] - 1            # 2^e <= |x| < 2^(e+1)
    q = Fraction(2) ** (max(e, emin) - (bits - 1))   # quantum at that exponent
    n = round(ax / q)                        # Fraction.__round__: half to even
    v = n * q
    # overflow: beyond the largest finite value plus half its quantum
    top = Fraction(big) + Fraction(2) ** (math.frexp(big)[1] - 1 - bits)
    if v > Fraction(big) or ax >= top:
        return math.copysign(math.inf, x)
    return math.copysign(float(v), x)


def _cases(kind):
    bits, emin, big = FORMATS[kind]
    u = 2.0 ** (1 - bits)                    # ulp of the format at 1
    sub = 2.0 ** (emin - bits + 1)           # smallest subnormal
    vals = [0.0, 1.0, -1.0, 1.0 + u / 2, 1.0 + 3 * u / 2, 1.0 + u / 2 + 2.0 ** -40,
            1.0 + u / 2 - 2.0 ** -40, 1.0 + 3 * u / 2 - 2.0 ** -40, 2.0 - u / 4,
            sub, sub / 2, 3 * sub / 2, 5 * sub / 2, 3.7 * sub, 2.0 ** emin - sub / 2,
            2.0 ** emin, 2.0 ** emin * (1 + u / 2), big, -big, 0.1, 1.0 / 3.0, 7.25e-3,
            123.456, 1e-30 if kind == "bf16" else 1e-6]
    if kind == "f16":
        vals += [65519.0, 65519.99, 2047.5, 2049.0, 2051.0, 6.1e-5, 5.96e-8, 2.98e-8, 4.0e-8]
    else:
        vals += [3.0e38, 1.0 + 2.0 ** -8 + 2.0 ** -30, 2.0 ** -133, 2.0 ** -134,
                 1.5 * 2.0 ** -134, 3.0 * 2.0 ** -135]
    return vals


def _fields(vals, src):
    """One epoch of an nx x 2 x 1 grid: row y = 0 holds the values as j, row
    y = 1 holds their negatives; beta components take scaled copies that stay
    below 1 in magnitude."""
    n = len(vals)
    j = np.zeros((1, 1, 2, n), dtype=np.float64)
    j[0, 0, 0] = vals
    j[0, 0, 1] = [-v for v in vals]
    b = np.zeros((1, 1, 2, n, 3), dtype=np.float64)
    small = [v if abs(v) < 0.5 else v / (2.0 ** math.ceil(math.log2(abs(v)) + 2)) for v in vals]
    b[0, 0, 0, :, 0] = small
    b[0, 0, 1, :, 1] = small
    b[0, 0, 0, :, 2] = [-s for s in small]
    if src == "f32":
        # the test values are FP32 values already where that is the source
        j, b = j.astype(np.float32), b.astype(np.float32)
    return j, b


@pytest.mark.parametrize("src", ["f32", "f64"])
@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_store_is_round_to_nearest_even(kind, src):
    import torch
    import paper_2609_09322_amd as dart
    vals = [v for v in _cases(kind) if math.isfinite(round16(v, kind))]
    if src == "f32":
        vals = [float(np.float32(v)) for v in vals]
        vals = [v for v in vals if math.isfinite(round16(v, kind))]
    j, b = _fields(vals, src)
    storage = dart.DART_F16 if kind == "f16" else dart.DART_BF16
    n = len(vals)
    st = dart.dart_load_epochs((n, 2, 1), (1, 1, 1), [0.0], j, b, storage)
    jr = np.zeros((1, 2, n), dtype=np.float32)
    br = np.zeros((1, 2, n, 3), dtype=np.float32)
    dart.dart_stack_read_epoch(st, 0, jr, br)
    want_j = np.array([round16(float(x), kind) for x in j.reshape(-1)], dtype=np.float64)
    want_b = np.array([round16(float(x), kind) for x in b.reshape(-1)], dtype=np.float64)
    got_j = jr.reshape(-1).astype(np.float64)
    got_b = br.reshape(-1).astype(np.float64)
    bad = np.nonzero(got_j.view(np.uint64) != want_j.view(np.uint64))[0]
    assert bad.size == 0, [(float(j.reshape(-1)[k]).hex(), got_j[k], want_j[k]) for k in bad[:5]]
    bad = np.nonzero(got_b.view(np.uint64) != want_b.view(np.uint64))[0]
    assert bad.size == 0, [(float(b.reshape(-1)[k]).hex(), got_b[k], want_b[k]) for k in bad[:5]]
    if kind == "f16":
        # numpy's binary16 conversion, from the source type directly
        assert np.array_equal(jr.reshape(-1), j.reshape(-1).astype(np.float16).astype(np.float32))
        assert np.array_equal(br.reshape(-1), b.reshape(-1).astype(np.float16).astype(np.float32))
    # the double-rounding cases really differ from rounding through FP32
    if src == "f64":
        tie = 1.0 + 2.0 ** (-FORMATS[kind][0]) + 2.0 ** -40
        k = vals.index(tie)
        assert jr[0, 0, k] == round16(tie, kind) != round16(float(np.float32(tie)), kind)

    # the render reads the same values: one epoch, no lookback, no beaming, a
    # cardinal view down the one-cell-thick z axis, unit chords, so each pixel
    # is the stored emissivity (a view at theta = 0, phi = 0 puts x on the
    # rows, reversed, and y on the columns).  FP32 subnormals excluded: the
    # render multiplies, the read-back only widens.
    v = dart.View(0.0, 0.0, 2, n, 1.0, 0.0, 0.6, dart.DART_NO_LOOKBACK | dart.DART_NO_BEAMING)
    img = np.zeros((n, 2), dtype=np.float32)
    dart.dart_render(st, v, img)
    ref = jr[0].T[::-1]          # image row r = cell x = n - 1 - r, column = y
    normal = np.abs(ref) >= np.float32(2.0 ** -126)
    assert np.array_equal(img[normal | (ref == 0)], ref[normal | (ref == 0)])


@pytest.mark.parametrize("kind", ["f16", "bf16"])
def test_velocity_rounding_to_one_is_refused(kind):
    import paper_2609_09322_amd as dart
    storage = dart.DART_F16 if kind == "f16" else dart.DART_BF16
    bits = FORMATS[kind][0]
    below = 1.0 - 2.0 ** -bits               # largest format value below 1
    ok = below                               # exact: stays
    bad = 1.0 - 2.0 ** -(bits + 2)           # nearer to 1 than to `below`: rounds to 1
    assert round16(ok, kind) == ok and round16(bad, kind) == 1.0
    for vz, accepted in ((ok, True), (bad, False)):
        j = np.ones((1, 1, 1, 4), dtype=np.float64)
        b = np.zeros((1, 1, 1, 4, 3), dtype=np.float64)
        b[0, 0, 0, 2, 2] = vz
        if accepted:
            st = dart.dart_load_epochs((4, 1, 1), (1, 1, 1), [0.0], j, b, storage)
            br = np.zeros((1, 1, 4, 3), dtype=np.float32)
            dart.dart_stack_read_epoch(st, 0, np.zeros((1, 1, 4), np.float32), br)
            assert br[0, 0, 2, 2] == np.float32(ok)
        else:
            with pytest.raises(dart.DartError) as ei:
                dart.dart_load_epochs((4, 1, 1), (1, 1, 1), [0.0], j, b, storage)
            assert ei.value.status == dart.DART_E_RANGE
            assert "x=2" in str(ei.value)


def test_read_epoch_fp32_and_fp64_are_exact():
    import torch
    import paper_2609_09322_amd as dart
    rng = np.random.default_rng(8)
    dims = (13, 7, 5)
    j = rng.uniform(-2, 2, size=(3, 5, 7, 13))
    b = rng.uniform(-0.5, 0.5, size=(3, 5, 7, 13, 3))
    for storage, dt in ((dart.DART_F64, np.float64), (dart.DART_F32, np.float32)):
        st = dart.dart_load_epochs(dims, (1, 1, 1), [0.0, 1.0, 2.0], j, b, storage)
        for m in range(3):
            jr = np.zeros((5, 7, 13), dtype=dt)
            br = np.zeros((5, 7, 13, 3), dtype=dt)
            dart.dart_stack_read_epoch(st, m, jr, br)
            assert np.array_equal(jr, j[m].astype(dt))
            assert np.array_equal(br, b[m].astype(dt))
        # device arrays, after a re-lay of the stack
        dart.dart_stack_rebrick(st, (4, 1, 2))
        jd = torch.zeros((5, 7, 13), dtype=torch.float64 if dt is np.float64 else torch.float32,
                         device="cuda")
        bd = torch.zeros((5, 7, 13, 3), dtype=jd.dtype, device="cuda")
        dart.dart_stack_read_epoch(st, 2, jd, bd)
        torch.cuda.synchronize()
        assert np.array_equal(jd.cpu().numpy(), j[2].astype(dt))
        assert np.array_equal(bd.cpu().numpy(), b[2].astype(dt))
        with pytest.raises(dart.DartError):
            dart.dart_stack_read_epoch(st, 3, jr, br)
        with pytest.raises(ValueError):
            dart.dart_stack_read_epoch(st, 0, jr[:2], br)


def test_rebrick_past_32_bit_offsets_is_refused_before_allocating():
    """An x extent of one cell in 4x2x2 bricks: 2^29 cells pad to 2^31 records
    (17 GB, allocated but not filled); re-laid as 16x1x1 bricks they would be
    2^33 records, beyond the 32-bit offsets: refused at once, nothing
    allocated, the stack unchanged."""
    import torch
    import paper_2609_09322_amd as dart
    free, _ = torch.cuda.mem_get_info()
    if free < 40e9:
        pytest.skip("needs 17 GB of device memory")
    st = dart.dart_stack_create((1, 1 << 9, 1 << 20), (1, 1, 1), [0.0], dart.DART_F16)
    before = dart.dart_stack_get_info(st)
    assert tuple(before.brick) == (4, 2, 2) and before.device_bytes == (1 << 31) * 8
    free0, _ = torch.cuda.mem_get_info()
    with pytest.raises(dart.DartError) as ei:
        dart.dart_stack_rebrick(st, (16, 1, 1))
    assert ei.value.status == dart.DART_E_INVAL and "2^32" in str(ei.value)
    free1, _ = torch.cuda.mem_get_info()
    assert abs(free1 - free0) < (64 << 20)
    after = dart.dart_stack_get_info(st)
    assert tuple(after.brick) == (4, 2, 2) and after.device_bytes == before.device_bytes
    dart.dart_free_epochs(st)


def test_tile_coordinates_beyond_16_bits_are_refused():
    """Tile coordinates are 16-bit: with 1 x 64 tiles a 70000-pixel-wide image
    needs 70000 tiles per row, which the batched planner refuses; the same view
    renders with 64 x 1 tiles."""
    import torch
    import paper_2609_09322_amd as dart
    j = np.ones((1, 2, 2, 2), dtype=np.float32)
    b = np.zeros((1, 2, 2, 2, 3), dtype=np.float32)
    st = dart.dart_load_epochs((2, 2, 2), (1, 1, 1), [0.0], j, b, dart.DART_F32)
    saved = dart.dart_get_tuning()
    v = dart.View(90.0, 0.0, 70000, 1, 1e-4, 0.0, 0.6, dart.DART_NO_LOOKBACK)
    img = torch.zeros((1, 70000), dtype=torch.float32, device="cuda")
    try:
        dart.dart_set_tuning(1, 64, 8, 0, 0, 0, 4)
        with pytest.raises(dart.DartError) as ei:
            dart.dart_render_batch([st], [v], [img])
        assert ei.value.status == dart.DART_E_INVAL and "65536" in str(ei.value)
        dart.dart_set_tuning(64, 1, 8, 0, 0, 0, 4)
        flux, steps = dart.dart_render_batch([st], [v], [img])
        ref = torch.zeros_like(img)
        dart.dart_render(st, v, ref)
        torch.cuda.synchronize()
        assert torch.equal(img, ref) and steps[0] > 0
    finally:
        dart.dart_set_tuning(saved.tile_w, saved.tile_h, saved.waves_per_cu, saved.order,
                             saved.orient, saved.depth_sync, saved.cells_per_batch)
