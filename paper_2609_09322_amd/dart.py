"""ctypes binding of libdart.so (include/dart.h): argument marshalling only.

Every call maps one-to-one onto a C entry point of the same name; all work
runs in the HIP library.  Host arrays are numpy arrays; device arrays are
torch tensors on a ROCm device (their ``data_ptr()`` is passed with
``DART_DEVICE_PTRS``).  A non-OK status raises :class:`DartError`.
If the library is missing the import fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdart.so")

DART_OK, DART_E_INVAL, DART_E_RANGE, DART_E_NOMEM = 0, -1, -2, -3
DART_E_DEVICE, DART_E_BUSY, DART_E_INTERNAL = -4, -5, -6
DART_F64, DART_F32, DART_F16, DART_BF16 = 0, 1, 2, 3
DART_NO_LOOKBACK = 0x1
DART_NO_BEAMING = 0x2
DART_NEAREST_EPOCH = 0x4
DART_NO_KAHAN = 0x8
DART_FORCE_F64_DDA = 0x10
DART_DEVICE_PTRS = 0x20
DART_KERNEL_PLAIN = 0x40
DART_ACCUMULATE = 0x80
DART_EXACT_TIME = 0x100
DART_RECORDS_ONLY = 0x200
DART_PLANE_ADDR64 = 0x400

EXPORTS = ["dart_load_epochs", "dart_stack_create", "dart_stack_set_epochs", "dart_free_epochs",
           "dart_stack_get_info", "dart_stack_read_epoch", "dart_stack_rebrick", "dart_stack_set_placement",
           "dart_labelled_create", "dart_vector_create", "dart_streamer_create",
           "dart_streamer_render",
           "dart_streamer_get_stats", "dart_streamer_destroy", "dart_render", "dart_render_batch",
           "dart_render_batch_noalloc", "dart_autotune", "dart_set_tuning", "dart_get_tuning", "dart_count_samples", "dart_count_lines",
           "dart_count_bytes",
           "dart_record_bytes", "dart_bandwidth_probe", "dart_gather_probe", "dart_server_create", "dart_submit",
           "dart_poll", "dart_wait", "dart_server_destroy", "dart_server_get_stats",
           "dart_server_get_timeline",
           "dart_last_error", "dart_version"]


class DartError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"dart status {status}: {message}")
        self.status = status


class dart_view(ctypes.Structure):
    _fields_ = [("theta_deg", ctypes.c_double), ("phi_deg", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("pixel_scale", ctypes.c_double), ("t_obs", ctypes.c_double),
                ("alpha", ctypes.c_double), ("flags", ctypes.c_uint32),
                ("out_dtype", ctypes.c_int)]


class dart_stack_info(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("n_epochs", ctypes.c_int32),
                ("storage", ctypes.c_int), ("brick", ctypes.c_int32 * 3),
                ("device_bytes", ctypes.c_uint64)]


class dart_tuning(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("order", ctypes.c_int32),
                ("orient", ctypes.c_int32), ("depth_sync", ctypes.c_int32),
                ("cells_per_batch", ctypes.c_int32)]


class dart_server_timeline(ctypes.Structure):
    _fields_ = [("waves_timed", ctypes.c_uint64), ("plan_ms", ctypes.c_double),
                ("enqueue_ms", ctypes.c_double), ("callback_to_retire_ms", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("stream_idle_ms", ctypes.c_double)]


class dart_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("waves", ctypes.c_uint64), ("max_wave_requests", ctypes.c_uint64),
                ("bytes_in_use", ctypes.c_uint64), ("bytes_peak", ctypes.c_uint64),
                ("admission_waits", ctypes.c_uint64)]


@dataclass
class View:
    theta_deg: float
    phi_deg: float
    width: int
    height: int
    pixel_scale: float
    t_obs: float
    alpha: float
    flags: int = 0
    out_dtype: int = DART_F32

    def c(self) -> dart_view:
        return dart_view(float(self.theta_deg), float(self.phi_deg), int(self.width),
                         int(self.height), float(self.pixel_scale), float(self.t_obs),
                         float(self.alpha), int(self.flags), int(self.out_dtype))


_P = ctypes.c_void_p
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    I32, U32, U64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "dart_load_epochs": [_P, _P, I32, _P, ctypes.c_int, ctypes.c_int, _P, _P, U32, _P, _P],
        "dart_stack_create": [_P, _P, I32, _P, ctypes.c_int, U32, _P],
        "dart_stack_set_epochs": [_P, I32, I32, ctypes.c_int, _P, _P, U32, _P],
        "dart_free_epochs": [_P],
        "dart_stack_get_info": [_P, _P],
        "dart_stack_read_epoch": [_P, I32, _P, _P, U32, _P],
        "dart_stack_rebrick": [_P, _P, _P],
        "dart_stack_set_placement": [_P, _P, _P],
        "dart_labelled_create": [_P, I32, _P],
        "dart_vector_create": [_P, I32, _P],
        "dart_streamer_create": [_P, _P, I32, _P, ctypes.c_int, I32, _P, _P],
        "dart_streamer_render": [_P, ctypes.c_int, _P, _P, U32, _P, I32, _P, _P, _P, _P],
        "dart_streamer_get_stats": [_P, _P],
        "dart_streamer_destroy": [_P],
        "dart_render": [_P, _P, _P, _P, _P, _P],
        "dart_render_batch": [_P, _P, I32, _P, _P, _P, _P],
        "dart_render_batch_noalloc": [_P, _P, I32, _P, _P, _P, _P],
        "dart_autotune": [_P, _P, I32, I32, _P, _P, _P],
        "dart_set_tuning": [_P],
        "dart_get_tuning": [_P],
        "dart_count_samples": [_P, _P, _P, _P],
        "dart_count_lines": [_P, _P, _P, _P],
        "dart_count_bytes": [_P, _P, _P, _P, _P],
        "dart_record_bytes": [_P, _P],
        "dart_bandwidth_probe": [_P, _P, U64, I32, _P],
        "dart_gather_probe": [_P, U64, I32, _P],
        "dart_server_create": [ctypes.c_size_t, I32, I32, _P],
        "dart_submit": [_P, _P, _P, _P, _P],
        "dart_poll": [_P, U64, _P, _P, _P, _P],
        "dart_wait": [_P, U64, _P, _P, _P],
        "dart_server_destroy": [_P],
        "dart_server_get_stats": [_P, _P],
        "dart_server_get_timeline": [_P, _P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.dart_last_error.restype = ctypes.c_char_p
    lib.dart_last_error.argtypes = []
    lib.dart_version.restype = ctypes.c_char_p
    lib.dart_version.argtypes = []
    _lib = lib
    return lib


def _check(status):
    if status != DART_OK:
        raise DartError(status, _load().dart_last_error().decode())


def _ptr(x):
    """(address, is_device) of a numpy array, torch tensor or raw int address."""
    if x is None:
        return None, False
    if isinstance(x, int):
        return x, False
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("arrays must be C-contiguous")
        return x.ctypes.data, False
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return x.data_ptr(), x.device.type != "cpu"
    raise TypeError(f"unsupported buffer type {type(x)}")


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dtype_code(x):
    name = str(getattr(x, "dtype", ""))
    if "float64" in name:
        return DART_F64
    if "float32" in name:
        return DART_F32
    raise TypeError(f"fields must be float32 or float64, got {name}")


def dart_last_error() -> str:
    return _load().dart_last_error().decode()


def dart_version() -> str:
    return _load().dart_version().decode()


class Stack:
    """Owning handle of a resident stack (freed by dart_free_epochs or on GC)."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            try:
                _lib.dart_free_epochs(self.handle)
            except Exception:
                pass
            self.handle = None


def dart_load_epochs(dims, cell, epoch_times, emissivity, velocity, storage,
                     flags=0, stream=None) -> Stack:
    lib = _load()
    d = (ctypes.c_int32 * 3)(*[int(v) for v in dims])
    c = (ctypes.c_double * 3)(*[float(v) for v in cell])
    t = np.ascontiguousarray(epoch_times, dtype=np.float64)
    jp, jdev = _ptr(emissivity)
    bp, bdev = _ptr(velocity)
    if jdev != bdev:
        raise ValueError("emissivity and velocity must both be host or both be device arrays")
    if jdev:
        flags |= DART_DEVICE_PTRS
    out = ctypes.c_void_p()
    _check(lib.dart_load_epochs(d, c, len(t), t.ctypes.data, _dtype_code(emissivity), storage,
                                jp, bp, flags, _stream(stream), ctypes.byref(out)))
    return Stack(out.value)


def dart_stack_create(dims, cell, epoch_times, storage, flags=0) -> Stack:
    lib = _load()
    d = (ctypes.c_int32 * 3)(*[int(v) for v in dims])
    c = (ctypes.c_double * 3)(*[float(v) for v in cell])
    t = np.ascontiguousarray(epoch_times, dtype=np.float64)
    out = ctypes.c_void_p()
    _check(lib.dart_stack_create(d, c, len(t), t.ctypes.data, storage, flags, ctypes.byref(out)))
    return Stack(out.value)


def dart_stack_set_epochs(stack: Stack, m0, emissivity, velocity, flags=0, stream=None):
    jp, jdev = _ptr(emissivity)
    bp, _ = _ptr(velocity)
    if jdev:
        flags |= DART_DEVICE_PTRS
    count = int(emissivity.shape[0])
    _check(_load().dart_stack_set_epochs(stack.handle, int(m0), count, _dtype_code(emissivity),
                                         jp, bp, flags, _stream(stream)))


def dart_free_epochs(stack: Stack):
    _check(_load().dart_free_epochs(stack.handle))
    stack.handle = None


def dart_stack_get_info(stack: Stack) -> dart_stack_info:
    info = dart_stack_info()
    _check(_load().dart_stack_get_info(stack.handle, ctypes.byref(info)))
    return info


def dart_stack_read_epoch(stack: Stack, m, emissivity, velocity, stream=None):
    """Epoch m as stored, widened exactly, into ``emissivity`` ([nz][ny][nx]) and
    ``velocity`` ([nz][ny][nx][3]): float64 arrays for FP64 stacks, float32 for
    the others; both numpy arrays or both device tensors."""
    info = dart_stack_get_info(stack)
    nx, ny, nz = info.dims
    esz = 8 if info.storage == DART_F64 else 4
    for arr, per in ((emissivity, 1), (velocity, 3)):
        if isinstance(arr, np.ndarray):
            count, item = arr.size, arr.itemsize
        else:
            count, item = arr.numel(), arr.element_size()
        if count != nx * ny * nz * per or item != esz:
            raise ValueError(f"read_epoch arrays: {nx * ny * nz * per} values of {esz} bytes "
                             f"expected, got {count} of {item}")
    jp, jdev = _ptr(emissivity)
    bp, bdev = _ptr(velocity)
    if jdev != bdev:
        raise ValueError("emissivity and velocity must both be host or both be device arrays")
    _check(_load().dart_stack_read_epoch(stack.handle, int(m), jp, bp,
                                         DART_DEVICE_PTRS if jdev else 0, _stream(stream)))


def dart_stack_rebrick(stack: Stack, brick, stream=None):
    b = (ctypes.c_int32 * 3)(*[int(v) for v in brick])
    _check(_load().dart_stack_rebrick(stack.handle, b, _stream(stream)))


def dart_stack_set_placement(stack: Stack, origin, centre):
    o = (ctypes.c_double * 3)(*[float(v) for v in origin])
    c = (ctypes.c_double * 3)(*[float(v) for v in centre])
    _check(_load().dart_stack_set_placement(stack.handle, o, c))


def dart_labelled_create(blocks) -> Stack:
    """A labelled stack over placed sub-domain stacks (which it keeps alive)."""
    arr = (ctypes.c_void_p * len(blocks))(*[b.handle for b in blocks])
    out = ctypes.c_void_p()
    _check(_load().dart_labelled_create(arr, len(blocks), ctypes.byref(out)))
    s = Stack(out.value)
    s.parts = list(blocks)
    return s


def dart_vector_create(components) -> Stack:
    """A vector stack over 2-4 component stacks (which it keeps alive); its
    renders fill images of shape [n_components, height, width]."""
    arr = (ctypes.c_void_p * len(components))(*[c.handle for c in components])
    out = ctypes.c_void_p()
    _check(_load().dart_vector_create(arr, len(components), ctypes.byref(out)))
    s = Stack(out.value)
    s.parts = list(components)
    return s


def dart_record_bytes(stack: Stack) -> int:
    v = ctypes.c_uint32()
    _check(_load().dart_record_bytes(stack.handle, ctypes.byref(v)))
    return v.value


def _view_for(view: View, image):
    ip, idev = _ptr(image)
    cv = view.c()
    if idev:
        cv.flags |= DART_DEVICE_PTRS
    return cv, ip


def dart_render(stack: Stack, view: View, image, stream=None, stats=True):
    """Renders into ``image`` ([height][width] float32/float64 numpy array or
    device tensor).  Returns (flux, cell_steps) when ``stats`` is set (this
    waits for the stream), else (None, None)."""
    cv, ip = _view_for(view, image)
    f = ctypes.c_double(0.0)
    s = ctypes.c_uint64(0)
    _check(_load().dart_render(stack.handle, ctypes.byref(cv), ip,
                               ctypes.byref(f) if stats else None,
                               ctypes.byref(s) if stats else None, _stream(stream)))
    return (f.value, s.value) if stats else (None, None)


def dart_render_batch(stacks, views, images, stream=None, stats=True):
    n = len(views)
    st = (ctypes.c_void_p * n)(*[s.handle for s in stacks])
    vs = (dart_view * n)()
    ims = (ctypes.c_void_p * n)()
    for i, (v, im) in enumerate(zip(views, images)):
        cv, ip = _view_for(v, im)
        vs[i] = cv
        ims[i] = ip
    flux = np.zeros(n, dtype=np.float64)
    steps = np.zeros(n, dtype=np.uint64)
    _check(_load().dart_render_batch(st, vs, n, ims, flux.ctypes.data if stats else None,
                                     steps.ctypes.data if stats else None, _stream(stream)))
    return (flux, steps) if stats else (None, None)


def dart_render_batch_noalloc(stacks, views, images, stream=None, stats=True):
    """dart_render_batch with its scratch in the library's fixed device array
    (no allocation); images must be device tensors."""
    n = len(views)
    st = (ctypes.c_void_p * n)(*[s.handle for s in stacks])
    vs = (dart_view * n)()
    ims = (ctypes.c_void_p * n)()
    for i, (v, im) in enumerate(zip(views, images)):
        cv, ip = _view_for(v, im)
        vs[i] = cv
        ims[i] = ip
    flux = np.zeros(n, dtype=np.float64)
    steps = np.zeros(n, dtype=np.uint64)
    _check(_load().dart_render_batch_noalloc(st, vs, n, ims, flux.ctypes.data if stats else None,
                                             steps.ctypes.data if stats else None,
                                             _stream(stream)))
    return (flux, steps) if stats else (None, None)


def dart_autotune(stacks, views, rebrick=False, stream=None):
    n = len(views)
    st = (ctypes.c_void_p * n)(*[s.handle for s in stacks])
    vs = (dart_view * n)(*[v.c() for v in views])
    best = dart_tuning()
    ms = ctypes.c_double(0)
    _check(_load().dart_autotune(st, vs, n, 1 if rebrick else 0, ctypes.byref(best),
                                 ctypes.byref(ms), _stream(stream)))
    return best, ms.value


def dart_set_tuning(tile_w, tile_h, waves_per_cu, order=0, orient=1, depth_sync=0,
                    cells_per_batch=4):
    t = dart_tuning(tile_w, tile_h, waves_per_cu, order, orient, depth_sync, cells_per_batch)
    _check(_load().dart_set_tuning(ctypes.byref(t)))


def dart_get_tuning() -> dart_tuning:
    t = dart_tuning()
    _check(_load().dart_get_tuning(ctypes.byref(t)))
    return t


def dart_count_samples(stack: Stack, view: View, stream=None) -> int:
    n = ctypes.c_uint64(0)
    _check(_load().dart_count_samples(stack.handle, ctypes.byref(view.c()), ctypes.byref(n),
                                      _stream(stream)))
    return n.value


def dart_count_bytes(stack: Stack, view: View, stream=None):
    """(compulsory bytes, line bytes) of a render of the view as renders read
    the stack (its emissivity plane when it has one), images excluded."""
    c, l = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(_load().dart_count_bytes(stack.handle, ctypes.byref(view.c()), ctypes.byref(c),
                                    ctypes.byref(l), _stream(stream)))
    return c.value, l.value


def dart_count_lines(stack: Stack, view: View, stream=None) -> int:
    n = ctypes.c_uint64(0)
    _check(_load().dart_count_lines(stack.handle, ctypes.byref(view.c()), ctypes.byref(n),
                                    _stream(stream)))
    return n.value


def dart_bandwidth_probe(dst, src, nbytes, reps=1, stream=None):
    dp, _ = _ptr(dst)
    sp, _ = _ptr(src)
    _check(_load().dart_bandwidth_probe(dp, sp, int(nbytes), int(reps), _stream(stream)))


def dart_gather_probe(src, nbytes, reps=1, stream=None):
    sp, _ = _ptr(src)
    _check(_load().dart_gather_probe(sp, int(nbytes), int(reps), _stream(stream)))


class Server:
    def __init__(self, handle):
        self.handle = handle


class dart_stream_stats(ctypes.Structure):
    _fields_ = [("epochs_loaded", ctypes.c_int32), ("epochs_skipped", ctypes.c_int32),
                ("intervals", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("bytes_uploaded", ctypes.c_uint64)]


class Streamer:
    """Owning handle of an out-of-core streamer (destroyed on GC)."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            try:
                _lib.dart_streamer_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def dart_streamer_create(dims, cell, epoch_times, storage, ring_epochs=3, brick=None) -> Streamer:
    d = (ctypes.c_int32 * 3)(*[int(v) for v in dims])
    c = (ctypes.c_double * 3)(*[float(v) for v in cell])
    t = np.ascontiguousarray(epoch_times, dtype=np.float64)
    b = (ctypes.c_int32 * 3)(*[int(v) for v in brick]) if brick is not None else None
    out = ctypes.c_void_p()
    _check(_load().dart_streamer_create(d, c, len(t), t.ctypes.data, storage, int(ring_epochs), b,
                                        ctypes.byref(out)))
    return Streamer(out.value)


def dart_streamer_render(streamer: Streamer, emissivity, velocity, views, images, stream=None,
                         stats=True):
    """Out-of-core render of `views` from the epoch series in `emissivity` /
    `velocity` (host numpy / CPU tensors, or device tensors)."""
    jp, jdev = _ptr(emissivity)
    bp, bdev = _ptr(velocity)
    if jdev != bdev:
        raise ValueError("emissivity and velocity must both be host or both be device arrays")
    n = len(views)
    vs = (dart_view * n)()
    ims = (ctypes.c_void_p * n)()
    for i, (v, im) in enumerate(zip(views, images)):
        cv, ip = _view_for(v, im)
        vs[i] = cv
        ims[i] = ip
    flux = np.zeros(n, dtype=np.float64)
    steps = np.zeros(n, dtype=np.uint64)
    _check(_load().dart_streamer_render(streamer.handle, _dtype_code(emissivity), jp, bp,
                                        DART_DEVICE_PTRS if jdev else 0, vs, n, ims,
                                        flux.ctypes.data if stats else None,
                                        steps.ctypes.data if stats else None, _stream(stream)))
    return (flux, steps) if stats else (None, None)


def dart_streamer_get_stats(streamer: Streamer) -> dart_stream_stats:
    st = dart_stream_stats()
    _check(_load().dart_streamer_get_stats(streamer.handle, ctypes.byref(st)))
    return st


def dart_streamer_destroy(streamer: Streamer):
    _check(_load().dart_streamer_destroy(streamer.handle))
    streamer.handle = None


def dart_server_create(hbm_budget_bytes, max_inflight=256, n_streams=3) -> Server:
    out = ctypes.c_void_p()
    _check(_load().dart_server_create(int(hbm_budget_bytes), int(max_inflight), int(n_streams),
                                      ctypes.byref(out)))
    return Server(out.value)


def dart_submit(srv: Server, stack: Stack, view: View, image) -> int:
    cv, ip = _view_for(view, image)
    t = ctypes.c_uint64(0)
    _check(_load().dart_submit(srv.handle, stack.handle, ctypes.byref(cv), ip, ctypes.byref(t)))
    return t.value


def dart_poll(srv: Server, ticket):
    """(done, flux, cell_steps, latency_ms); a done ticket is retired."""
    done = ctypes.c_int32(0)
    f = ctypes.c_double(0)
    n = ctypes.c_uint64(0)
    lat = ctypes.c_double(0)
    _check(_load().dart_poll(srv.handle, int(ticket), ctypes.byref(done), ctypes.byref(f),
                             ctypes.byref(n), ctypes.byref(lat)))
    return bool(done.value), f.value, n.value, lat.value


def dart_wait(srv: Server, ticket):
    """Blocks until the request is done: (flux, cell_steps, latency_ms)."""
    f = ctypes.c_double(0)
    n = ctypes.c_uint64(0)
    lat = ctypes.c_double(0)
    _check(_load().dart_wait(srv.handle, int(ticket), ctypes.byref(f), ctypes.byref(n),
                             ctypes.byref(lat)))
    return f.value, n.value, lat.value


def dart_server_get_stats(srv: Server) -> dart_server_stats:
    st = dart_server_stats()
    _check(_load().dart_server_get_stats(srv.handle, ctypes.byref(st)))
    return st


def dart_server_get_timeline(srv: Server) -> dart_server_timeline:
    tl = dart_server_timeline()
    _check(_load().dart_server_get_timeline(srv.handle, ctypes.byref(tl)))
    return tl


def dart_server_destroy(srv: Server):
    _check(_load().dart_server_destroy(srv.handle))
    srv.handle = None
