"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every symbol include/dart.h declares, and the Python binding mirrors them."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dart.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dart_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["dart_load_epochs", "dart_free_epochs", "dart_render", "dart_render_batch",
                 "dart_server_create", "dart_submit", "dart_poll", "dart_wait",
                 "dart_server_destroy", "dart_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2609_09322_amd.dart as b
    lib = b.LIB_PATH
    assert os.path.exists(lib), "run __graft_entry__.build() first"
    out = subprocess.check_output(["nm", "-D", "--defined-only", lib], text=True)
    exported = set(re.findall(r" T (dart_[a-z_]+)$", out, flags=re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_2609_09322_amd as d
    for n in _declared():
        assert hasattr(d, n), n
    assert sorted(d.EXPORTS) == _declared()


def test_library_loads_and_reports_errors_without_gpu():
    import ctypes
    import paper_2609_09322_amd as d
    assert "gfx950" in d.dart_version()
    lib = d.dart._load()
    # argument validation runs before any device call
    rc = lib.dart_render(None, None, None, None, None, None)
    assert rc == d.DART_E_INVAL
    assert "NULL" in d.dart_last_error() or "null" in d.dart_last_error().lower()
    rc = lib.dart_server_create(ctypes.c_size_t(10), 1, 1, None)
    assert rc == d.DART_E_INVAL
    # the entry points added for sub-domains, labelled stacks and streaming
    # also check their arguments before touching a device
    origin = (ctypes.c_double * 3)(0, 0, 0)
    assert lib.dart_stack_set_placement(None, origin, origin) == d.DART_E_INVAL
    out = ctypes.c_void_p(1)
    assert lib.dart_labelled_create(None, 0, ctypes.byref(out)) == d.DART_E_INVAL
    assert out.value is None
    dims = (ctypes.c_int32 * 3)(4, 4, 4)
    cell = (ctypes.c_double * 3)(1, 1, 1)
    t = (ctypes.c_double * 2)(0.0, 1.0)
    out = ctypes.c_void_p(1)
    assert lib.dart_streamer_create(dims, cell, 2, t, d.DART_F32, 2, None,
                                    ctypes.byref(out)) == d.DART_E_INVAL
    assert "ring_epochs" in d.dart_last_error()
    assert out.value is None
    assert lib.dart_streamer_render(None, d.DART_F32, None, None, 0, None, 0, None, None, None,
                                    None) == d.DART_E_INVAL
    assert lib.dart_streamer_destroy(None) == d.DART_E_INVAL
    assert lib.dart_count_lines(None, None, None, None) == d.DART_E_INVAL
    # probes: sizes checked before any device call
    assert lib.dart_gather_probe(None, ctypes.c_uint64(1 << 20), 1, None) == d.DART_E_INVAL
    for nbytes in (0, 100, 128 * 3, 128 * 1000):
        assert lib.dart_gather_probe(ctypes.c_void_p(16), ctypes.c_uint64(nbytes), 1,
                                     None) == d.DART_E_INVAL
    assert "power of two" in d.dart_last_error()
    assert lib.dart_bandwidth_probe(None, None, ctypes.c_uint64(16), 1, None) == d.DART_E_INVAL
    # vector stacks: 2 to 4 components
    out = ctypes.c_void_p(1)
    assert lib.dart_vector_create(None, 2, ctypes.byref(out)) == d.DART_E_INVAL
    assert out.value is None
    comps = (ctypes.c_void_p * 5)()
    for n in (0, 1, 5):
        assert lib.dart_vector_create(comps, n, ctypes.byref(out)) == d.DART_E_INVAL
    assert "2 to 4" in d.dart_last_error()


def test_record_offsets_fit_32_bits_checked_before_allocation():
    """Record offsets inside an epoch are 32-bit: a stack whose padded epoch
    would hold more than 2^32 records is refused before any device call (so
    here, without a GPU, with DART_E_INVAL rather than a device error)."""
    import ctypes
    import paper_2609_09322_amd as d
    lib = d.dart._load()
    cell = (ctypes.c_double * 3)(1, 1, 1)
    t = (ctypes.c_double * 1)(0.0)
    out = ctypes.c_void_p(1)
    # 2^31 cells; 16-bit records in 4x2x2 bricks pad x from 1 to 4: 2^33 records
    dims = (ctypes.c_int32 * 3)(1, 1 << 11, 1 << 20)
    assert lib.dart_stack_create(dims, cell, 1, t, d.DART_F16, 0, ctypes.byref(out)) == d.DART_E_INVAL
    assert "2^32" in d.dart_last_error()
    assert out.value is None
    # the same grid as FP32 records (2x2x2 bricks): 2^32 records, the most allowed,
    # passes the check and reaches the device (none here)
    out = ctypes.c_void_p(1)
    rc = lib.dart_stack_create(dims, cell, 1, t, d.DART_F32, 0, ctypes.byref(out))
    assert rc != d.DART_OK and "2^32" not in d.dart_last_error()
    assert out.value is None


def test_tuning_checks_without_gpu():
    """dart_set_tuning validates every field on the host; a rejected tuning
    leaves the current one in place."""
    import paper_2609_09322_amd as d
    saved = d.dart_get_tuning()
    for bad in (dict(cells_per_batch=5), dict(cells_per_batch=16), dict(order=5),
                dict(order=-1), dict(depth_sync=65)):
        args = dict(order=3, orient=0, depth_sync=0, cells_per_batch=8)
        args.update(bad)
        with pytest.raises(d.DartError) as ei:
            d.dart_set_tuning(64, 1, 8, **args)
        assert ei.value.status == d.DART_E_INVAL
    with pytest.raises(d.DartError):
        d.dart_set_tuning(48, 1, 8)          # not 64 pixels per tile
    with pytest.raises(d.DartError):
        d.dart_set_tuning(64, 1, 6)          # waves per CU not a multiple of 4
    got = d.dart_get_tuning()
    assert (got.tile_w, got.tile_h, got.waves_per_cu, got.order, got.cells_per_batch) == \
        (saved.tile_w, saved.tile_h, saved.waves_per_cu, saved.order, saved.cells_per_batch)
    for k in (0, 4, 8):
        d.dart_set_tuning(64, 1, 8, 4, 0, 2, k)
        assert d.dart_get_tuning().cells_per_batch == k
    d.dart_set_tuning(saved.tile_w, saved.tile_h, saved.waves_per_cu, saved.order,
                      saved.orient, saved.depth_sync, saved.cells_per_batch)


def test_structs_match_header_layout():
    import ctypes
    import paper_2609_09322_amd as d
    # dart_view: 2 doubles, 2 int32, 3 doubles, uint32 flags, 4-byte enum -> 56 bytes
    assert ctypes.sizeof(d.dart_view) == 56
    assert ctypes.sizeof(d.dart_tuning) == 28
    assert ctypes.sizeof(d.dart.dart_stream_stats) == 24
    # dart_server_timeline: one uint64 and six doubles
    assert ctypes.sizeof(d.dart.dart_server_timeline) == 56


def test_product_does_not_reach_the_oracle():
    """The product package and its sources never name the oracle or load it."""
    pkg = os.path.join(ROOT, "paper_2609_09322_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower(), f
                assert "liborc" not in txt, f
