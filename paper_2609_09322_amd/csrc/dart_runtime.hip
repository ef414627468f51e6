// dart_runtime.hip -- host runtime behind the C ABI (include/dart.h):
// resident stacks, view resolution, the plain and batched render paths
// (planner, tile queue, hipGraph replay), tuning, sample counting and the
// bandwidth probe.  The render server lives in dart_server.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dart.h"
#include "dart_internal.h"
#include "dart_runtime.h"

using namespace dart;

// ------------------------------------------------------------------ errors

static thread_local std::string g_err;

dart_status dart::fail(dart_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

dart_status dart::hip_fail(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(DART_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(DART_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char *dart_last_error(void) { return g_err.c_str(); }
extern "C" const char *dart_version(void) { return "dart-mi355x 0.1 (gfx950)"; }

#define HIP_TRY(call, what)                         \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// ------------------------------------------------------------------ devices

int dart::device_cus(int dev) {
    static std::mutex mu;
    static std::map<int, int> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        cus = 256;
    cache[dev] = cus;
    return cus;
}

// ------------------------------------------------------------------ stacks

static int store_of(dart_dtype d) {
    switch (d) {
        case DART_F64: return ST_F64;
        case DART_F32: return ST_F32;
        case DART_F16: return ST_F16;
        case DART_BF16: return ST_BF16;
    }
    return -1;
}
uint64_t dart::next_generation() {
    static std::atomic<uint64_t> counter{0};
    return ++counter;
}

uint32_t dart::record_bytes(int store) {
    return store == ST_F64 ? 32u : store == ST_F32 ? 16u : 8u;
}

static int ilog2_exact(int v) {
    int l = 0;
    while ((1 << l) < v) l++;
    return (1 << l) == v ? l : -1;
}

// Records per epoch of dims padded to whole bricks of 2^lb cells.
static uint64_t padded_records(const int32_t dims[3], const int lb[3]) {
    uint64_t per = 1;
    for (int a = 0; a < 3; a++)
        per *= (((uint64_t)dims[a] + (1u << lb[a]) - 1) >> lb[a]) << lb[a];
    return per;
}

// The kernels address a record inside its epoch with a 32-bit offset
// (brick index and cell in brick): the padded epoch must hold at most 2^32
// records.  Checked before anything is allocated.
static dart_status check_offsets(const int32_t dims[3], const int lb[3]) {
    const uint64_t per = padded_records(dims, lb);
    if (per > (1ull << 32))
        return fail(DART_E_INVAL,
                    "%llu records per epoch once padded to %dx%dx%d bricks: more than the 2^32 "
                    "that 32-bit record offsets address",
                    (unsigned long long)per, 1 << lb[0], 1 << lb[1], 1 << lb[2]);
    return DART_OK;
}

static void layout(dart_stack *s, const int lb[3]) {
    for (int a = 0; a < 3; a++) {
        s->dev.lb[a] = lb[a];
        s->dev.nb[a] = (s->dev.n[a] + (1 << lb[a]) - 1) >> lb[a];
    }
    s->dev.epoch_stride = (int64_t)padded_records(s->dev.n, lb);
}

static void default_brick(int store, int lb[3]) {
    // Bricks of about one 128-B cache line: 2x2x2 FP32 records (16 B each) or
    // 4x2x2 16-bit records (8 B); FP64 records (32 B) use 2x2x2 (two lines).
    // A cube-like line serves neighbouring rays of any orientation.
    lb[0] = store == ST_F16 || store == ST_BF16 ? 2 : 1;
    lb[1] = 1;
    lb[2] = 1;
}

static dart_status check_geometry(const int32_t dims[3], const double cell[3], int32_t M,
                                  const double *times) {
    if (!dims || !cell || !times) return fail(DART_E_INVAL, "null dims/cell/epoch_times");
    for (int a = 0; a < 3; a++) {
        if (dims[a] < 1 || dims[a] > (1 << 20))
            return fail(DART_E_INVAL, "dims[%d]=%d out of range", a, dims[a]);
        if (!(cell[a] > 0.0) || !isfinite(cell[a]))
            return fail(DART_E_INVAL, "cell[%d]=%g must be finite and > 0", a, cell[a]);
    }
    const uint64_t ncell = (uint64_t)dims[0] * dims[1] * dims[2];
    if (ncell > (1ull << 31)) return fail(DART_E_INVAL, "more than 2^31 cells per epoch");
    if (M < 1 || M > 65536) return fail(DART_E_INVAL, "n_epochs=%d out of range", M);
    for (int m = 0; m < M; m++)
        if (!isfinite(times[m])) return fail(DART_E_INVAL, "epoch_times[%d] not finite", m);
    for (int m = 0; m + 1 < M; m++)
        if (!(times[m + 1] > times[m]))
            return fail(DART_E_INVAL, "epoch_times not strictly increasing at %d", m + 1);
    return DART_OK;
}

extern "C" dart_status dart_stack_create(const int32_t dims[3], const double cell[3],
                                         int32_t n_epochs, const double *epoch_times,
                                         dart_dtype storage, uint32_t flags, dart_stack **out) {
    (void)flags;
    if (!out) return fail(DART_E_INVAL, "out is NULL");
    *out = nullptr;
    dart_status st = check_geometry(dims, cell, n_epochs, epoch_times);
    if (st != DART_OK) return st;
    const int store = store_of(storage);
    if (store < 0) return fail(DART_E_INVAL, "unknown storage dtype %d", (int)storage);
    int lb[3];
    default_brick(store, lb);
    st = check_offsets(dims, lb);
    if (st != DART_OK) return st;
    std::unique_ptr<dart_stack> s(new dart_stack());
    HIP_TRY(hipGetDevice(&s->device), "hipGetDevice");
    for (int a = 0; a < 3; a++) {
        s->dev.n[a] = dims[a];
        s->dev.cell[a] = cell[a];
    }
    s->dev.n_epochs = n_epochs;
    s->dev.store = store;
    s->storage = storage;
    s->times.assign(epoch_times, epoch_times + n_epochs);
    s->filled.assign(n_epochs, 0);
    layout(s.get(), lb);
    s->bytes = s->dev.epoch_stride * n_epochs * record_bytes(store);
    void *data = nullptr, *t = nullptr;
    hipError_t e = hipMalloc(&data, s->bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(stack)");
    // epoch times followed by 1 / (t_{m+1} - t_m) (0 for the last epoch)
    std::vector<double> tab(2 * (size_t)n_epochs, 0.0);
    for (int32_t m = 0; m < n_epochs; m++) {
        tab[m] = epoch_times[m];
        if (m + 1 < n_epochs) tab[n_epochs + m] = 1.0 / (epoch_times[m + 1] - epoch_times[m]);
    }
    e = hipMalloc(&t, sizeof(double) * tab.size());
    if (e != hipSuccess) {
        (void)hipFree(data);
        return hip_fail(e, "hipMalloc(times)");
    }
    e = hipMemcpy(t, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(data);
        (void)hipFree(t);
        return hip_fail(e, "hipMemcpy(times)");
    }
    s->dev.data = data;
    s->dev.times = (const double *)t;
    s->dev.inv_dt = (const double *)t + n_epochs;
    *out = s.release();
    return DART_OK;
}

static dart_status set_epochs_impl(dart_stack *s, int32_t m0, int32_t count, dart_dtype src,
                                   const void *j, const void *beta, uint32_t flags,
                                   hipStream_t stream) {
    if (!s) return fail(DART_E_INVAL, "stack is NULL");
    if (s->labelled()) return fail(DART_E_INVAL, "fill the sub-domains of a labelled stack instead");
    if (s->vector()) return fail(DART_E_INVAL, "fill the components of a vector stack instead");
    if (!j || !beta) return fail(DART_E_INVAL, "emissivity/velocity is NULL");
    if (m0 < 0 || count < 1 || m0 + count > s->dev.n_epochs)
        return fail(DART_E_INVAL, "epoch range [%d, %d) outside [0, %d)", m0, m0 + count,
                    s->dev.n_epochs);
    if (src != DART_F64 && src != DART_F32)
        return fail(DART_E_INVAL, "src_dtype must be DART_F64 or DART_F32");
    const int src_f64 = src == DART_F64;
    const size_t esz = src_f64 ? 8 : 4;
    const uint64_t ncell = (uint64_t)s->dev.n[0] * s->dev.n[1] * s->dev.n[2];
    unsigned long long *err = nullptr;
    HIP_TRY(hipMalloc(&err, sizeof(unsigned long long)), "hipMalloc(err)");
    struct Guard {
        void *p[3] = {nullptr, nullptr, nullptr};
        ~Guard() { for (void *q : p) if (q) (void)hipFree(q); }
    } guard;
    guard.p[0] = err;
    hipError_t e = launch_fill_u64(err, 1, ~0ull, stream);
    if (e != hipSuccess) return hip_fail(e, "clear error flag");
    if (flags & F_DEVICE_PTRS) {
        e = launch_convert(src_f64, s->dev.store, j, beta, m0, count, s->dev, (void *)s->dev.data,
                           err, stream);
        if (e != hipSuccess) return hip_fail(e, "convert kernel");
    } else {
        // host arrays: one epoch at a time through device staging
        void *dj = nullptr, *db = nullptr;
        HIP_TRY(hipMalloc(&dj, ncell * esz), "hipMalloc(staging)");
        guard.p[1] = dj;
        HIP_TRY(hipMalloc(&db, ncell * esz * 3), "hipMalloc(staging)");
        guard.p[2] = db;
        for (int32_t q = 0; q < count; q++) {
            const char *hj = (const char *)j + (size_t)q * ncell * esz;
            const char *hb = (const char *)beta + (size_t)q * ncell * esz * 3;
            HIP_TRY(hipMemcpyAsync(dj, hj, ncell * esz, hipMemcpyHostToDevice, stream), "H2D j");
            HIP_TRY(hipMemcpyAsync(db, hb, ncell * esz * 3, hipMemcpyHostToDevice, stream),
                    "H2D beta");
            e = launch_convert(src_f64, s->dev.store, dj, db, m0 + q, 1, s->dev,
                               (void *)s->dev.data, err, stream);
            if (e != hipSuccess) return hip_fail(e, "convert kernel");
            HIP_TRY(hipStreamSynchronize(stream), "sync");
        }
    }
    unsigned long long bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, err, sizeof(bad), hipMemcpyDeviceToHost, stream), "D2H err");
    HIP_TRY(hipStreamSynchronize(stream), "sync");
    if (bad != ~0ull) {
        const uint64_t m = bad / ncell, c = bad % ncell;
        const uint64_t x = c % s->dev.n[0], y = (c / s->dev.n[0]) % s->dev.n[1],
                       z = c / ((uint64_t)s->dev.n[0] * s->dev.n[1]);
        return fail(DART_E_RANGE,
                    "non-finite value or |beta| >= 1 (in the source or after rounding to the "
                    "storage type) at epoch %llu, cell (x=%llu, y=%llu, z=%llu)",
                    (unsigned long long)m, (unsigned long long)x, (unsigned long long)y,
                    (unsigned long long)z);
    }
    for (int32_t q = 0; q < count; q++) s->filled[m0 + q] = 1;
    s->generation = next_generation();
    return DART_OK;
}

extern "C" dart_status dart_stack_set_epochs(dart_stack *s, int32_t m0, int32_t count,
                                             dart_dtype src_dtype, const void *emissivity,
                                             const void *velocity, uint32_t flags,
                                             void *hip_stream) {
    return set_epochs_impl(s, m0, count, src_dtype, emissivity, velocity, flags,
                           (hipStream_t)hip_stream);
}

extern "C" dart_status dart_load_epochs(const int32_t dims[3], const double cell[3],
                                        int32_t n_epochs, const double *epoch_times,
                                        dart_dtype src_dtype, dart_dtype storage,
                                        const void *emissivity, const void *velocity,
                                        uint32_t flags, void *hip_stream, dart_stack **out) {
    if (!out) return fail(DART_E_INVAL, "out is NULL");
    *out = nullptr;
    dart_stack *s = nullptr;
    dart_status st = dart_stack_create(dims, cell, n_epochs, epoch_times, storage, flags, &s);
    if (st != DART_OK) return st;
    st = set_epochs_impl(s, 0, n_epochs, src_dtype, emissivity, velocity, flags,
                         (hipStream_t)hip_stream);
    if (st != DART_OK) {
        std::string keep = g_err;
        (void)hipFree((void *)s->dev.data);
        (void)hipFree((void *)s->dev.times);
        delete s;
        g_err = keep;
        return st;
    }
    *out = s;
    return DART_OK;
}

void dart::note_use(const dart_stack *cs, hipStream_t stream) {
    dart_stack *s = const_cast<dart_stack *>(cs);
    std::lock_guard<std::mutex> g(s->mu);
    for (auto &u : s->uses)
        if (u.first == stream) {
            (void)hipEventRecord(u.second, stream);
            return;
        }
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return;
    (void)hipEventRecord(ev, stream);
    s->uses.emplace_back(stream, ev);
}

bool dart::stack_busy(const dart_stack *cs) {
    dart_stack *s = const_cast<dart_stack *>(cs);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->pinned.load() > 0) return true;
    for (auto &u : s->uses)
        if (hipEventQuery(u.second) == hipErrorNotReady) return true;
    return false;
}

extern "C" dart_status dart_free_epochs(dart_stack *s) {
    if (!s) return fail(DART_E_INVAL, "stack is NULL");
    if (stack_busy(s)) return fail(DART_E_BUSY, "renders that read this stack are in flight");
    if (s->refs.load() > 0)
        return fail(DART_E_BUSY, "the stack is held by %d labelled or vector stack(s)",
                    s->refs.load());
    for (auto &u : s->uses) (void)hipEventDestroy(u.second);
    if (s->labelled()) {
        // the grids belong to the sub-domains
        (void)hipFree(s->dev_blocks);
        for (dart_stack *p : s->parts) p->refs--;
    } else if (s->vector()) {
        (void)hipFree(s->packed);
        for (dart_stack *c : s->comps) c->refs--;
    } else {
        (void)hipFree((void *)s->dev.data);
        (void)hipFree((void *)s->dev.times);
        if (s->jplane) (void)hipFree(s->jplane);
    }
    delete s;
    return DART_OK;
}

extern "C" dart_status dart_labelled_create(dart_stack *const *blocks, int32_t n_blocks,
                                            dart_stack **out) {
    if (out) *out = nullptr;
    if (!blocks || !out || n_blocks < 1) return fail(DART_E_INVAL, "bad labelled-stack arguments");
    if (n_blocks > 65536) return fail(DART_E_INVAL, "at most 65536 sub-domains");
    const dart_stack *b0 = blocks[0];
    for (int32_t i = 0; i < n_blocks; i++) {
        const dart_stack *b = blocks[i];
        if (!b) return fail(DART_E_INVAL, "blocks[%d] is NULL", i);
        if (b->labelled() || b->vector())
            return fail(DART_E_INVAL, "blocks[%d] is itself a labelled or vector stack", i);
        for (int32_t k = 0; k < i; k++)
            if (blocks[k] == b) return fail(DART_E_INVAL, "blocks[%d] repeats blocks[%d]", i, k);
        if (b->storage != b0->storage) return fail(DART_E_INVAL, "blocks[%d]: another storage type", i);
        if (b->device != b0->device) return fail(DART_E_INVAL, "blocks[%d]: another device", i);
        if (b->times != b0->times) return fail(DART_E_INVAL, "blocks[%d]: other epoch times", i);
        for (size_t m = 0; m < b->filled.size(); m++)
            if (!b->filled[m]) return fail(DART_E_INVAL, "blocks[%d]: epoch %zu never filled", i, m);
        if (n_blocks > 1 && !b->placed)
            return fail(DART_E_INVAL, "blocks[%d] is not placed (dart_stack_set_placement)", i);
        for (int a = 0; a < 3; a++)
            if (b->placed && b->centre[a] != b0->centre[a])
                return fail(DART_E_INVAL, "blocks[%d]: another domain centre", i);
    }
    std::vector<Block> hb(n_blocks);
    for (int32_t i = 0; i < n_blocks; i++) {
        const dart_stack *b = blocks[i];
        hb[i].st = b->dev;
        for (int a = 0; a < 3; a++)
            hb[i].centre[a] = b->placed ? b->centre[a] - b->origin[a] : 0.5 * b->dev.n[a] * b->dev.cell[a];
    }
    HIP_TRY(hipSetDevice(b0->device), "hipSetDevice");
    Block *d = nullptr;
    HIP_TRY(hipMalloc(&d, hb.size() * sizeof(Block)), "hipMalloc(blocks)");
    hipError_t e = hipMemcpy(d, hb.data(), hb.size() * sizeof(Block), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "upload blocks");
    }
    dart_stack *s = new dart_stack;
    s->dev = b0->dev;
    s->storage = b0->storage;
    s->times = b0->times;
    s->filled.assign(b0->filled.size(), 1);
    s->device = b0->device;
    s->dev_blocks = d;
    for (int32_t i = 0; i < n_blocks; i++) {
        s->parts.push_back(blocks[i]);
        s->bytes += blocks[i]->bytes;
        blocks[i]->refs++;
    }
    *out = s;
    return DART_OK;
}

// Bytes of one packed emissivity value, and of one component's packed array.
static uint64_t packed_bytes(const dart_stack *s) {
    return (uint64_t)s->dev.epoch_stride * s->dev.n_epochs * (record_bytes(s->dev.store) / 4);
}

static hipError_t pack_components(dart_stack *s, hipStream_t stream) {
    const uint64_t n = (uint64_t)s->dev.epoch_stride * s->dev.n_epochs;
    for (size_t c = 1; c < s->comps.size(); c++) {
        hipError_t e = launch_pack_j(s->dev.store, s->comps[c]->dev.data,
                                     (char *)s->packed + (c - 1) * packed_bytes(s), n, stream);
        if (e != hipSuccess) return e;
    }
    s->packed_gen.clear();
    for (dart_stack *c : s->comps) s->packed_gen.push_back(c->generation);
    return hipSuccess;
}

extern "C" dart_status dart_vector_create(dart_stack *const *components, int32_t n,
                                          dart_stack **out) {
    if (out) *out = nullptr;
    if (!components || !out) return fail(DART_E_INVAL, "bad vector-stack arguments");
    if (n < 2 || n > 4) return fail(DART_E_INVAL, "a vector stack has 2 to 4 components, not %d", n);
    const dart_stack *c0 = components[0];
    for (int32_t i = 0; i < n; i++) {
        const dart_stack *c = components[i];
        if (!c) return fail(DART_E_INVAL, "components[%d] is NULL", i);
        if (c->labelled() || c->vector())
            return fail(DART_E_INVAL, "components[%d] is a labelled or vector stack", i);
        for (int32_t k = 0; k < i; k++)
            if (components[k] == c) return fail(DART_E_INVAL, "components[%d] repeats components[%d]", i, k);
        if (c->storage != c0->storage) return fail(DART_E_INVAL, "components[%d]: another storage type", i);
        if (c->device != c0->device) return fail(DART_E_INVAL, "components[%d]: another device", i);
        if (c->times != c0->times) return fail(DART_E_INVAL, "components[%d]: other epoch times", i);
        for (int a = 0; a < 3; a++)
            if (c->dev.n[a] != c0->dev.n[a] || c->dev.cell[a] != c0->dev.cell[a] ||
                c->dev.lb[a] != c0->dev.lb[a])
                return fail(DART_E_INVAL, "components[%d]: another grid or brick shape", i);
        if (c->dev.epoch_stride != c0->dev.epoch_stride)
            return fail(DART_E_INVAL, "components[%d]: another layout", i);
        if (c->placed != c0->placed)
            return fail(DART_E_INVAL, "components[%d]: another placement", i);
        for (int a = 0; a < 3; a++)
            if (c->placed && (c->origin[a] != c0->origin[a] || c->centre[a] != c0->centre[a]))
                return fail(DART_E_INVAL, "components[%d]: another placement", i);
        for (size_t m = 0; m < c->filled.size(); m++)
            if (!c->filled[m]) return fail(DART_E_INVAL, "components[%d]: epoch %zu never filled", i, m);
    }
    dart_stack *s = new dart_stack;
    s->dev = c0->dev;
    s->storage = c0->storage;
    s->times = c0->times;
    s->filled.assign(c0->filled.size(), 1);
    s->device = c0->device;
    s->placed = c0->placed;
    for (int a = 0; a < 3; a++) {
        s->origin[a] = c0->origin[a];
        s->centre[a] = c0->centre[a];
    }
    for (int32_t i = 0; i < n; i++) s->comps.push_back(components[i]);
    // the other components' emissivity, packed one value per record index
    HIP_TRY(hipSetDevice(c0->device), "hipSetDevice");
    hipError_t e = hipMalloc(&s->packed, (n - 1) * packed_bytes(s));
    if (e == hipSuccess) e = pack_components(s, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        (void)hipFree(s->packed);
        delete s;
        return hip_fail(e, "pack vector components");
    }
    s->bytes = (n - 1) * packed_bytes(s);
    for (int32_t i = 0; i < n; i++) {
        s->bytes += components[i]->bytes;
        components[i]->refs++;
    }
    *out = s;
    return DART_OK;
}

extern "C" dart_status dart_stack_get_info(const dart_stack *s, dart_stack_info *info) {
    if (!s || !info) return fail(DART_E_INVAL, "NULL argument");
    for (int a = 0; a < 3; a++) {
        info->dims[a] = s->dev.n[a];
        info->brick[a] = 1 << s->dev.lb[a];
    }
    info->n_epochs = s->dev.n_epochs;
    info->storage = s->storage;
    info->device_bytes = s->bytes + s->jplane_bytes;
    return DART_OK;
}

extern "C" dart_status dart_stack_read_epoch(const dart_stack *s, int32_t m, void *emissivity,
                                             void *velocity, uint32_t flags, void *hip_stream) {
    if (!s || !emissivity || !velocity) return fail(DART_E_INVAL, "NULL argument");
    if (s->labelled() || s->vector())
        return fail(DART_E_INVAL, "read the epochs of the sub-domains or components instead");
    if (m < 0 || m >= s->dev.n_epochs)
        return fail(DART_E_INVAL, "epoch %d outside [0, %d)", m, s->dev.n_epochs);
    if (!s->filled[m]) return fail(DART_E_INVAL, "epoch %d was never filled", m);
    if (flags & ~(uint32_t)DART_DEVICE_PTRS) return fail(DART_E_INVAL, "unknown flags 0x%x", flags);
    hipStream_t stream = (hipStream_t)hip_stream;
    const uint64_t ncell = (uint64_t)s->dev.n[0] * s->dev.n[1] * s->dev.n[2];
    const size_t esz = s->dev.store == ST_F64 ? 8 : 4;
    if (flags & DART_DEVICE_PTRS) {
        HIP_TRY(launch_read_epoch(s->dev, m, emissivity, velocity, stream), "read kernel");
        note_use(s, stream);
        return DART_OK;
    }
    void *buf = nullptr;
    HIP_TRY(hipMalloc(&buf, ncell * esz * 4), "hipMalloc(read staging)");
    struct Free {
        void *p;
        ~Free() { (void)hipFree(p); }
    } guard{buf};
    void *dj = buf, *db = (char *)buf + ncell * esz;
    HIP_TRY(launch_read_epoch(s->dev, m, dj, db, stream), "read kernel");
    HIP_TRY(hipMemcpyAsync(emissivity, dj, ncell * esz, hipMemcpyDeviceToHost, stream), "D2H j");
    HIP_TRY(hipMemcpyAsync(velocity, db, 3 * ncell * esz, hipMemcpyDeviceToHost, stream), "D2H beta");
    HIP_TRY(hipStreamSynchronize(stream), "sync");
    return DART_OK;
}

extern "C" dart_status dart_record_bytes(const dart_stack *s, uint32_t *bytes_out) {
    if (!s || !bytes_out) return fail(DART_E_INVAL, "NULL argument");
    *bytes_out = record_bytes(s->dev.store);
    return DART_OK;
}

extern "C" dart_status dart_stack_set_placement(dart_stack *s, const double origin[3],
                                                const double centre[3]) {
    if (!s || !origin || !centre) return fail(DART_E_INVAL, "NULL argument");
    if (s->labelled()) return fail(DART_E_INVAL, "a labelled stack is placed by its sub-domains");
    if (s->vector()) return fail(DART_E_INVAL, "a vector stack is placed by its components");
    if (s->refs.load() > 0) return fail(DART_E_BUSY, "the stack is held by a labelled or vector stack");
    for (int a = 0; a < 3; a++)
        if (!isfinite(origin[a]) || !isfinite(centre[a]))
            return fail(DART_E_INVAL, "origin and centre must be finite");
    for (int a = 0; a < 3; a++) {
        s->origin[a] = origin[a];
        s->centre[a] = centre[a];
    }
    s->placed = true;
    s->generation = next_generation();
    return DART_OK;
}

extern "C" dart_status dart_stack_rebrick(dart_stack *s, const int32_t brick[3],
                                          void *hip_stream) {
    if (!s || !brick) return fail(DART_E_INVAL, "NULL argument");
    int lb[3], cells = 1;
    for (int a = 0; a < 3; a++) {
        lb[a] = ilog2_exact(brick[a]);
        if (lb[a] < 0 || brick[a] > 16) return fail(DART_E_INVAL, "brick[%d]=%d", a, brick[a]);
        cells *= brick[a];
    }
    if (cells > 4096) return fail(DART_E_INVAL, "brick larger than 4096 cells");
    {
        dart_status so = check_offsets(s->dev.n, lb);
        if (so != DART_OK) return so;
    }
    if (s->labelled()) return fail(DART_E_INVAL, "re-lay the sub-domains of a labelled stack before joining them");
    if (s->vector()) return fail(DART_E_INVAL, "re-lay the components of a vector stack before joining them");
    if (s->refs.load() > 0) return fail(DART_E_BUSY, "the stack is held by a labelled or vector stack");
    if (stack_busy(s)) return fail(DART_E_BUSY, "renders that read this stack are in flight");
    if (lb[0] == s->dev.lb[0] && lb[1] == s->dev.lb[1] && lb[2] == s->dev.lb[2]) return DART_OK;
    hipStream_t stream = (hipStream_t)hip_stream;
    dart_stack tmp;
    tmp.dev = s->dev;
    layout(&tmp, lb);
    const uint64_t rb = record_bytes(s->dev.store);
    const uint64_t bytes = tmp.dev.epoch_stride * s->dev.n_epochs * rb;
    void *data = nullptr;
    hipError_t em = hipMalloc(&data, bytes);
    if (em == hipErrorOutOfMemory && tmp.dev.epoch_stride == s->dev.epoch_stride &&
        s->dev.n_epochs > 1) {
        // No room for a second copy: re-lay one epoch at a time through a
        // one-epoch buffer and copy it back in place (same epoch size).
        (void)hipGetLastError();
        const uint64_t eb = s->dev.epoch_stride * rb;
        void *one = nullptr;
        HIP_TRY(hipMalloc(&one, eb), "hipMalloc(rebrick epoch)");
        hipError_t e = hipSuccess;
        for (int32_t m = 0; m < s->dev.n_epochs && e == hipSuccess; m++) {
            StackDev from = s->dev, to = tmp.dev;
            from.data = (const char *)s->dev.data + (uint64_t)m * eb;
            from.n_epochs = to.n_epochs = 1;
            to.data = one;
            e = launch_rebrick(s->dev.store, from, to, one, stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync((char *)s->dev.data + (uint64_t)m * eb, one, eb,
                                   hipMemcpyDeviceToDevice, stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        (void)hipFree(one);
        // a failure part-way leaves epochs in mixed layouts: the stack is unusable
        if (e != hipSuccess) {
            for (int32_t m = 0; m < s->dev.n_epochs; m++) s->filled[m] = false;
            s->generation = next_generation();
            return hip_fail(e, "rebrick in place (the stack's epochs must be loaded again)");
        }
        tmp.dev.data = s->dev.data;
        s->dev = tmp.dev;
        s->generation = next_generation();
        return DART_OK;
    }
    HIP_TRY(em, "hipMalloc(rebrick)");
    tmp.dev.data = data;
    hipError_t e = launch_rebrick(s->dev.store, s->dev, tmp.dev, data, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        (void)hipFree(data);
        return hip_fail(e, "rebrick");
    }
    (void)hipFree((void *)s->dev.data);
    s->dev = tmp.dev;
    s->bytes = bytes;
    s->generation = next_generation();
    return DART_OK;
}

// ------------------------------------------------------------------ views

// sin and cos of an angle in degrees.  The angle is split exactly (IEEE
// remainder) into a quarter-turn count q and a rest r in [-45, 45] degrees;
// sin and cos of r are rotated by q quarter turns, so multiples of 90 degrees
// give exact 0 and +-1 and the rest keeps full precision for any angle.
static void sincos_deg(double deg, double *s, double *c) {
    int q = 0;
    const double r = remquo(deg, 90.0, &q);
    const double rad = r * (M_PI / 180.0);
    const double sr = r == 0.0 ? 0.0 : sin(rad), cr = r == 0.0 ? 1.0 : cos(rad);
    double so, co;
    switch (q & 3) {
        case 0: so = sr; co = cr; break;
        case 1: so = cr; co = -sr; break;
        case 2: so = -sr; co = -cr; break;
        default: so = -cr; co = sr; break;
    }
    // (+0.0 instead of -0.0, so that signs of zero components never differ)
    *s = so + 0.0;
    *c = co + 0.0;
}

dart_status dart::resolve_view(const dart_stack *s, const dart_view *v, RayView *rv) {
    if (!s || !v || !rv) return fail(DART_E_INVAL, "NULL stack or view");
    for (int32_t m = 0; m < s->dev.n_epochs; m++)
        if (!s->filled[m]) return fail(DART_E_INVAL, "epoch %d of the stack was never filled", m);
    if (v->width < 1 || v->height < 1 || (int64_t)v->width * v->height > (1ll << 31))
        return fail(DART_E_INVAL, "image %dx%d out of range", v->width, v->height);
    if (v->width > 65535 * 64 || v->height > 65535 * 64)
        return fail(DART_E_INVAL, "image side too large");
    if (!(v->pixel_scale > 0.0) || !isfinite(v->pixel_scale))
        return fail(DART_E_INVAL, "pixel_scale must be finite and > 0");
    if (!isfinite(v->theta_deg) || !isfinite(v->phi_deg) || !isfinite(v->t_obs) ||
        !isfinite(v->alpha))
        return fail(DART_E_INVAL, "theta, phi, t_obs and alpha must be finite");
    if (v->out_dtype != DART_F32 && v->out_dtype != DART_F64)
        return fail(DART_E_INVAL, "out_dtype must be DART_F32 or DART_F64");
    if (v->out_dtype == DART_F64 && s->storage != DART_F64)
        return fail(DART_E_INVAL, "FP64 images need an FP64 stack");
    if (v->flags & ~(uint32_t)(DART_NO_LOOKBACK | DART_NO_BEAMING | DART_NEAREST_EPOCH |
                               DART_NO_KAHAN | DART_FORCE_F64_DDA | DART_DEVICE_PTRS |
                               DART_ACCUMULATE | DART_EXACT_TIME | DART_RECORDS_ONLY |
                               DART_PLANE_ADDR64))
        return fail(DART_E_INVAL, "unknown view flags 0x%x", v->flags);
    if ((v->flags & DART_EXACT_TIME) && (v->flags & DART_NEAREST_EPOCH))
        return fail(DART_E_INVAL, "DART_EXACT_TIME integrates the linear interpolation; "
                                  "it does not combine with DART_NEAREST_EPOCH");
    if ((v->flags & DART_ACCUMULATE) && !(v->flags & DART_DEVICE_PTRS))
        return fail(DART_E_INVAL, "DART_ACCUMULATE needs a device image (DART_DEVICE_PTRS)");
    if (s->vector() && (v->flags & DART_EXACT_TIME))
        return fail(DART_E_INVAL, "DART_EXACT_TIME is not available for vector stacks");
    memset(rv, 0, sizeof(*rv));
    const dart_stack *geo = s->labelled() ? s->parts[0] : s;  // camera centre, tile costs
    double st, ct, sp, cp;
    sincos_deg(v->theta_deg, &st, &ct);
    sincos_deg(v->phi_deg, &sp, &cp);
    const double nhat[3] = {st * cp, st * sp, ct};
    for (int a = 0; a < 3; a++) {
        rv->shat[a] = -nhat[a];
        rv->inv_shat[a] = rv->shat[a] != 0.0 ? 1.0 / rv->shat[a] : 0.0;
        rv->shat_hi[a] = (float)rv->shat[a];
        rv->shat_lo[a] = (float)(rv->shat[a] - (double)rv->shat_hi[a]);
        // kernels work in grid-local coordinates: the camera centre relative
        // to the grid's lower corner
        rv->centre[a] = geo->placed ? geo->centre[a] - geo->origin[a]
                                    : 0.5 * geo->dev.n[a] * geo->dev.cell[a];
    }
    rv->eu[0] = -sp; rv->eu[1] = cp; rv->eu[2] = 0.0;
    rv->ev[0] = -ct * cp; rv->ev[1] = -ct * sp; rv->ev[2] = st;
    rv->ps = v->pixel_scale;
    rv->t_obs = v->t_obs;
    rv->p = 2.0 + v->alpha;
    rv->flags = v->flags & (F_NO_LOOKBACK | F_NO_BEAMING | F_NEAREST | F_NO_KAHAN | F_F64_DDA |
                            F_ACCUMULATE);
    // exact temporal integration only changes anything with lookback and
    // more than one epoch
    if ((v->flags & DART_EXACT_TIME) && !(v->flags & DART_NO_LOOKBACK) && s->dev.n_epochs > 1)
        rv->flags |= F_EXACT;
    // FP64 ray parameters (plane crossings, chord midpoints) when a ray may
    // cross more than ~4k cells, and for FP32 stacks: FP32 crossings of
    // magnitude ~L/2 carry ~1e-5 absolute rounding, which chords at jumps of
    // the emissivity (a jet surface) turn into ~1e-5 relative pixel errors,
    // the size of the FP32 tolerance.  16-bit stacks keep FP32 crossings.
    int64_t most_cells = (int64_t)s->dev.n[0] + s->dev.n[1] + s->dev.n[2];
    for (const dart_stack *p : s->parts)
        most_cells = std::max(most_cells, (int64_t)p->dev.n[0] + p->dev.n[1] + p->dev.n[2]);
    if (most_cells > 4096 || s->dev.store == ST_F32) rv->flags |= F_F64_DDA;
    rv->width = v->width;
    rv->height = v->height;
    rv->out_f64 = v->out_dtype == DART_F64;
    rv->st = s->dev;
    // (the plane kernels always compensate their sums: views without
    // compensation read whole records)
    rv->st.jplane = (!(v->flags & (DART_RECORDS_ONLY | DART_NO_KAHAN)) && jplane_ready(s))
                        ? s->jplane
                        : nullptr;
    // a plane of at most 4 GiB is read through 32-bit byte offsets
    if (rv->st.jplane && s->jplane_bytes <= (1ull << 32) && !(v->flags & DART_PLANE_ADDR64))
        rv->flags |= F_PLANE32;
    rv->blocks = s->dev_blocks;
    rv->n_blocks = (int32_t)s->parts.size();
    rv->n_chan = s->channels();
    for (int c = 1; c < rv->n_chan; c++)
        rv->chan_data[c - 1] = (const char *)s->packed + (c - 1) * packed_bytes(s);
    const std::vector<double> &t = s->times;
    const int M = (int)t.size();
    if (v->flags & DART_NO_LOOKBACK) {
        rv->s_lo = -INFINITY;
        rv->s_hi = INFINITY;
        if (v->t_obs >= t[0] && v->t_obs <= t[M - 1]) {
            int m = 0;
            while (m + 1 < M - 1 && t[m + 1] <= v->t_obs) m++;
            rv->fixed_m = m;
            rv->fixed_w = M >= 2 ? (v->t_obs - t[m]) / (t[m + 1] - t[m]) : 0.0;
        } else {
            rv->fixed_m = -1;
            rv->fixed_w = 0.0;
        }
    } else {
        rv->s_lo = v->t_obs - t[M - 1];
        rv->s_hi = v->t_obs - t[0];
        rv->fixed_m = 0;
        rv->fixed_w = 0.0;
    }
    rv->fixed_wf = (float)rv->fixed_w;
    return DART_OK;
}

// ------------------------------------------------------------------ workspaces

Workspace *dart::get_workspace(hipStream_t stream) {
    static std::mutex mu;
    static std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> all;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(mu);
    auto &slot = all[{dev, stream}];
    if (!slot) {
        slot.reset(new Workspace());
        slot->stream = stream;
        slot->device = dev;
    }
    return slot.get();
}

template <typename T>
static hipError_t grow_dev(T *&p, size_t &cap, size_t need) {
    if (need <= cap && p) return hipSuccess;
    if (p) {
        hipError_t e = hipFree(p);
        if (e != hipSuccess) return e;
        p = nullptr;
        cap = 0;
    }
    size_t n = std::max(need, (size_t)1);
    hipError_t e = hipMalloc((void **)&p, n * sizeof(T));
    if (e == hipSuccess) cap = n;
    return e;
}

static hipError_t grow_host(void *&p, size_t &cap, size_t need) {
    if (need <= cap && p) return hipSuccess;
    if (p) {
        (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
    hipError_t e = hipHostMalloc(&p, std::max(need, (size_t)64), hipHostMallocDefault);
    if (e == hipSuccess) cap = std::max(need, (size_t)64);
    return e;
}

static void drop_graph(Workspace *ws) {
    if (ws->graph_exec) (void)hipGraphExecDestroy(ws->graph_exec);
    ws->graph_exec = nullptr;
    ws->graph_key.clear();
    ws->plan_ready = false;
    ws->plan_key.clear();
    ws->plan_groups.clear();
}

hipError_t dart::ws_reserve(Workspace *ws, size_t n_views, size_t n_tiles, size_t img_bytes,
                            size_t n_queues) {
    hipError_t e;
    // a captured graph holds these pointers: any reallocation invalidates it
    const void *before[4] = {ws->acc, ws->views, ws->tiles, ws->img};
    if (ws->stage_ready) {
        e = hipEventSynchronize(ws->stage_done);
        if (e != hipSuccess) return e;
    }
    if ((e = grow_dev(ws->acc, ws->acc_cap, 2 * std::max(n_views, (size_t)1) + n_queues)) != hipSuccess)
        return e;
    if ((e = grow_dev(ws->views, ws->views_cap, std::max(n_views, (size_t)1))) != hipSuccess) return e;
    if ((e = grow_dev(ws->tiles, ws->tiles_cap, std::max(n_tiles, (size_t)1))) != hipSuccess) return e;
    if (img_bytes && (e = grow_dev(ws->img, ws->img_cap, img_bytes)) != hipSuccess) return e;
    const size_t stage = n_views * sizeof(RayView) + n_tiles * sizeof(Tile) + 64;
    if ((e = grow_host(ws->stage, ws->stage_cap, stage)) != hipSuccess) return e;
    if (!ws->stage_ready) {
        if ((e = hipEventCreateWithFlags(&ws->stage_done, hipEventDisableTiming)) != hipSuccess)
            return e;
        ws->stage_ready = true;
    }
    const void *after[4] = {ws->acc, ws->views, ws->tiles, ws->img};
    if (memcmp(before, after, sizeof(before)) != 0) drop_graph(ws);
    return hipSuccess;
}

// ------------------------------------------------------------------ plain render

extern "C" dart_status dart_render(const dart_stack *s, const dart_view *v, void *image,
                                   double *flux_out, uint64_t *steps_out, void *hip_stream) {
    if (!image) return fail(DART_E_INVAL, "image is NULL");
    hipStream_t stream = (hipStream_t)hip_stream;
    dart_status st = refresh_jplane(s, stream, true);
    if (st != DART_OK) return st;
    RayView rv;
    st = resolve_view(s, v, &rv);
    if (st != DART_OK) return st;
    st = refresh_vector(s, stream);
    if (st != DART_OK) return st;
    Workspace *ws = get_workspace(stream);
    std::lock_guard<std::mutex> g(ws->mu);
    const bool dev_img = (v->flags & DART_DEVICE_PTRS) != 0;
    const size_t img_bytes = (size_t)rv.n_chan * v->width * v->height * (rv.out_f64 ? 8 : 4);
    HIP_TRY(ws_reserve(ws, 1, 0, dev_img ? 0 : img_bytes / 8 + 1, 0), "workspace");
    rv.image = dev_img ? image : (void *)ws->img;
    rv.acc_index = 0;
    double *flux_acc = (double *)ws->acc;
    unsigned long long *step_acc = ws->acc + 1;
    HIP_TRY(launch_fill_u64(ws->acc, 2, 0ull, stream), "clear accumulators");
    HIP_TRY(launch_plain(rv, flux_acc, step_acc, stream), "render kernel");
    note_use(s, stream);
    if (!dev_img)
        HIP_TRY(hipMemcpyAsync(image, ws->img, img_bytes, hipMemcpyDeviceToHost, stream), "D2H image");
    if (flux_out || steps_out || !dev_img) {
        unsigned long long acc[2];
        HIP_TRY(hipMemcpyAsync(acc, ws->acc, sizeof(acc), hipMemcpyDeviceToHost, stream), "D2H acc");
        HIP_TRY(hipStreamSynchronize(stream), "sync");
        double f;
        memcpy(&f, &acc[0], sizeof(f));
        if (flux_out) *flux_out = f;
        if (steps_out) *steps_out = acc[1];
    }
    return DART_OK;
}

// ------------------------------------------------------------------ tuning

static std::mutex g_tune_mu;
static dart_tuning g_tuning = {32, 2, 8, 0, 1, 0, 4};

static dart_status check_tuning(const dart_tuning *t) {
    if (!t) return fail(DART_E_INVAL, "tuning is NULL");
    const int lw = ilog2_exact(t->tile_w), lh = ilog2_exact(t->tile_h);
    if (lw < 0 || lh < 0 || t->tile_w * t->tile_h != 64)
        return fail(DART_E_INVAL, "tile %dx%d must be powers of two with 64 pixels", t->tile_w,
                    t->tile_h);
    if (t->waves_per_cu < 4 || t->waves_per_cu > 64 || t->waves_per_cu % 4)
        return fail(DART_E_INVAL, "waves_per_cu must be a multiple of 4 in [4, 64]");
    if (t->order < 0 || t->order > 4) return fail(DART_E_INVAL, "order must be in [0, 4]");
    if (t->orient != 0 && t->orient != 1) return fail(DART_E_INVAL, "orient must be 0 or 1");
    if (t->depth_sync < 0 || t->depth_sync > 64)
        return fail(DART_E_INVAL, "depth_sync must be in [0, 64]");
    if (t->cells_per_batch != 0 && t->cells_per_batch != 4 && t->cells_per_batch != 8)
        return fail(DART_E_INVAL, "cells_per_batch must be 4 or 8 (0 means 4)");

    return DART_OK;
}

extern "C" dart_status dart_set_tuning(const dart_tuning *t) {
    dart_status st = check_tuning(t);
    if (st != DART_OK) return st;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuning = *t;
    return DART_OK;
}

extern "C" dart_status dart_get_tuning(dart_tuning *t) {
    if (!t) return fail(DART_E_INVAL, "tuning is NULL");
    std::lock_guard<std::mutex> g(g_tune_mu);
    *t = g_tuning;
    return DART_OK;
}

dart_status dart::refresh_vector(const dart_stack *cs, hipStream_t stream) {
    if (!cs || !cs->vector()) return DART_OK;
    dart_stack *s = const_cast<dart_stack *>(cs);
    // one check-and-repack at a time per vector stack
    std::lock_guard<std::mutex> g(s->mu);
    bool stale = false;
    for (size_t c = 0; c < s->comps.size(); c++)
        stale = stale || s->comps[c]->generation != s->packed_gen[c];
    if (!stale) return DART_OK;
    // renders still reading the packed copy must finish first
    for (auto &u : s->uses) HIP_TRY(hipEventSynchronize(u.second), "wait for renders");
    HIP_TRY(pack_components(s, stream), "pack vector components");
    return DART_OK;
}

// The emissivity plane serves plain stacks with FP32 or 16-bit records (FP64
// records stay whole; labelled and vector stacks read their parts' records;
// streamed windows have no plane).
static bool jplane_eligible(const dart_stack *s) {
    return s && !s->labelled() && !s->vector() && s->dev.store != ST_F64 &&
           s->dev.epoch_stride > 0;
}

bool dart::jplane_ready(const dart_stack *s) {
    return jplane_eligible(s) && s->jplane_gen.load(std::memory_order_acquire) == s->generation;
}

dart_status dart::refresh_jplane(const dart_stack *cs, hipStream_t stream, bool may_alloc) {
    if (!jplane_eligible(cs)) return DART_OK;
    dart_stack *s = const_cast<dart_stack *>(cs);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->jplane_gen.load(std::memory_order_relaxed) == s->generation) return DART_OK;
    // (no second attempt to allocate for records that have not changed)
    if (s->jplane_no_room == s->generation) return DART_OK;
    for (char f : s->filled)
        if (!f) return DART_OK;  // (such a stack is not rendered)
    // nothing is packed into a graph the caller is capturing: its renders read
    // whole records until a render outside capture packs the plane
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(stream, &cap), "hipStreamIsCapturing");
    if (cap != hipStreamCaptureStatusNone) return DART_OK;
    const uint64_t n = (uint64_t)s->dev.epoch_stride * s->dev.n_epochs;
    const uint64_t need = n * (record_bytes(s->dev.store) / 4);
    if (s->jplane_bytes != need && !may_alloc) return DART_OK;
    // renders still reading the old plane must finish first
    for (auto &u : s->uses) HIP_TRY(hipEventSynchronize(u.second), "wait for renders");
    s->jplane_gen.store(0, std::memory_order_release);
    if (s->jplane_bytes != need) {
        if (s->jplane) (void)hipFree(s->jplane);
        s->jplane = nullptr;
        s->jplane_bytes = 0;
        void *p = nullptr;
        if (hipMalloc(&p, need) != hipSuccess) {
            (void)hipGetLastError();  // no room: renders read whole records
            s->jplane_no_room = s->generation;
            return DART_OK;
        }
        s->jplane = p;
        s->jplane_bytes = need;
    }
    HIP_TRY(launch_pack_jplane(s->dev.store, s->dev.data, s->jplane, n, stream),
            "pack emissivity plane");
    // complete before a render on any stream reads it
    HIP_TRY(hipStreamSynchronize(stream), "sync");
    s->jplane_gen.store(s->generation, std::memory_order_release);
    return DART_OK;
}

dart_tuning dart::tuning_for(const dart_stack *s) {
    if (s && s->tuned) return s->tuning;
    std::lock_guard<std::mutex> g(g_tune_mu);
    return g_tuning;
}

// ------------------------------------------------------------------ batch planner

// Estimated cell-steps of the ray through the tile centre, times 64 rays.
// Orientation of a view's tiles (tuning.orient): the tile's long side follows
// the image-plane projection of the bricks' long axis, so that the lanes of one
// wave read neighbouring cells of the same cache lines.  True when that turns
// the tile (tile_w and tile_h swap) for this view.
static bool orient_flips(const RayView &rv, const dart_tuning &tun) {
    if (!tun.orient) return false;
    int a = 0;
    for (int k = 1; k < 3; k++)
        if (rv.st.lb[k] > rv.st.lb[a]) a = k;
    const bool elongated = rv.st.lb[a] > std::min(rv.st.lb[0], std::min(rv.st.lb[1], rv.st.lb[2]));
    const bool long_u = tun.tile_w >= tun.tile_h;
    const bool axis_u = fabs(rv.eu[a]) >= fabs(rv.ev[a]);
    return elongated && long_u != axis_u;
}

// Rays of a view are parallel: the pixel ray at image-plane coordinates (u, w)
// can meet the grid box only if (u, w) lies in the box's projection, the
// convex hull of its 8 projected corners.  A row of tiles covers a band of w;
// the hull's part in that band spans an interval of u, found on the hull's
// edges (a convex region reaches its extremes on its boundary).  A tile whose
// u-interval misses it, both widened by a pixel, has no ray that reaches a
// cell: its pixels are 0 and it need not be marched.  Per view the planner
// builds the hull once and per row clips its edges to the band, so the test
// costs a few compares per tile (the server plans every wave).
struct Footprint {
    std::vector<std::pair<double, double>> hull;  // (u, w), counter-clockwise
    double margin;
};

static Footprint footprint(const RayView &rv) {
    Footprint f;
    std::vector<std::pair<double, double>> pts(8);
    double scale = 1.0;
    for (int c = 0; c < 8; c++) {
        double d[3];
        for (int a = 0; a < 3; a++)
            d[a] = ((c >> a) & 1 ? rv.st.n[a] * rv.st.cell[a] : 0.0) - rv.centre[a];
        pts[c].first = d[0] * rv.eu[0] + d[1] * rv.eu[1] + d[2] * rv.eu[2];
        pts[c].second = d[0] * rv.ev[0] + d[1] * rv.ev[1] + d[2] * rv.ev[2];
        scale = std::max({scale, fabs(pts[c].first), fabs(pts[c].second)});
    }
    // a pixel's width plus a relative margin: rounding never drops a tile
    // that a ray of it could reach
    f.margin = rv.ps + 1e-9 * scale;
    // convex hull (monotone chain)
    std::sort(pts.begin(), pts.end());
    auto cross = [](const std::pair<double, double> &o, const std::pair<double, double> &p,
                    const std::pair<double, double> &q) {
        return (p.first - o.first) * (q.second - o.second) -
               (p.second - o.second) * (q.first - o.first);
    };
    std::vector<std::pair<double, double>> h(16);
    int k = 0;
    for (int i = 0; i < 8; i++) {
        while (k >= 2 && cross(h[k - 2], h[k - 1], pts[i]) <= 0) k--;
        h[k++] = pts[i];
    }
    for (int i = 6, t = k + 1; i >= 0; i--) {
        while (k >= t && cross(h[k - 2], h[k - 1], pts[i]) <= 0) k--;
        h[k++] = pts[i];
    }
    h.resize(k > 1 ? k - 1 : k);
    f.hull = h;
    return f;
}

// The u-interval of the hull's part with w in [w0, w1] (widened by the
// margin); false when that part is empty.
static bool band_span(const Footprint &f, double w0, double w1, double *u_lo, double *u_hi) {
    w0 -= f.margin;
    w1 += f.margin;
    double lo = INFINITY, hi = -INFINITY;
    const size_t n = f.hull.size();
    if (n < 3) {  // degenerate: keep the tiles
        *u_lo = -INFINITY;
        *u_hi = INFINITY;
        return true;
    }
    for (size_t i = 0; i < n; i++) {
        const auto &p = f.hull[i], &q = f.hull[(i + 1) % n];
        // the part of edge p -> q with w in [w0, w1]
        double ta = 0.0, tb = 1.0;
        const double dw = q.second - p.second;
        if (dw == 0.0) {
            if (p.second < w0 || p.second > w1) continue;
        } else {
            double t0 = (w0 - p.second) / dw, t1 = (w1 - p.second) / dw;
            if (t0 > t1) std::swap(t0, t1);
            ta = std::max(ta, t0);
            tb = std::min(tb, t1);
            if (ta > tb) continue;
        }
        const double ua = p.first + ta * (q.first - p.first);
        const double ub = p.first + tb * (q.first - p.first);
        lo = std::min({lo, ua, ub});
        hi = std::max({hi, ua, ub});
    }
    if (!(lo <= hi)) return false;
    *u_lo = lo - f.margin;
    *u_hi = hi + f.margin;
    return true;
}

static double tile_cost(const RayView &rv, int tx, int ty, int tw, int th) {
    const double u = ((tx + 0.5) * tw - 0.5 * rv.width) * rv.ps;
    const double w = ((ty + 0.5) * th - 0.5 * rv.height) * rv.ps;
    double s_in = -INFINITY, s_out = INFINITY, per_len = 0.0;
    for (int a = 0; a < 3; a++) {
        const double o = rv.centre[a] + u * rv.eu[a] + w * rv.ev[a];
        const double d = rv.shat[a], hi = rv.st.n[a] * rv.st.cell[a];
        per_len += fabs(d) / rv.st.cell[a];
        if (d == 0.0) {
            if (o < 0 || o >= hi) return 1.0;
            continue;
        }
        double t0 = -o / d, t1 = (hi - o) / d;
        s_in = std::max(s_in, std::min(t0, t1));
        s_out = std::min(s_out, std::max(t0, t1));
    }
    s_in = std::max(s_in, rv.s_lo);
    s_out = std::min(s_out, rv.s_hi);
    if (!(s_out > s_in)) return 1.0;
    return 1.0 + 64.0 * (s_out - s_in) * per_len;
}

dart_status dart::plan_batch(const dart_stack *const *stacks, const dart_view *views, int32_t n,
                             void *const *images, const dart_tuning &tun,
                             std::vector<Group> &groups) {
    groups.clear();
    const int lw0 = ilog2_exact(tun.tile_w);
    std::map<int, size_t> gindex;
    for (int32_t i = 0; i < n; i++) {
        RayView rv;
        dart_status st = resolve_view(stacks[i], &views[i], &rv);
        if (st != DART_OK) return fail(st, "view %d: %s", i, dart_last_error());
        if (!images[i]) return fail(DART_E_INVAL, "images[%d] is NULL", i);
        rv.image = images[i];
        rv.acc_index = i;
        const int key = ((rv.flags & F_PLANE32) ? 128 : 0) + (rv.st.jplane ? 64 : 0) +
                        rv.st.store * 16 + (rv.n_chan > 1 ? 8 : 0) +
                        ((rv.flags & F_F64_DDA) ? 4 : 0) + (rv.n_blocks > 0 ? 2 : 0) +
                        ((rv.flags & F_EXACT) ? 1 : 0);
        auto it = gindex.find(key);
        if (it == gindex.end()) {
            it = gindex.emplace(key, groups.size()).first;
            groups.emplace_back();
            groups.back().store = rv.st.store;
            groups.back().f64 = (rv.flags & F_F64_DDA) != 0;
            groups.back().labelled = rv.n_blocks > 0;
            groups.back().exact = (rv.flags & F_EXACT) != 0;
            groups.back().vec = rv.n_chan > 1;
            groups.back().jp = rv.st.jplane != nullptr;
            groups.back().jp32 = (rv.flags & F_PLANE32) != 0;
        }
        Group &g = groups[it->second];
        const uint32_t vi = (uint32_t)g.views.size();
        const int lw = orient_flips(rv, tun) ? 6 - lw0 : lw0;
        rv.tile_w_log2 = lw;
        rv.sync_gap = tun.depth_sync > 0
                          ? tun.depth_sync * std::max(rv.st.cell[0], std::max(rv.st.cell[1], rv.st.cell[2]))
                          : 0.0;
        g.views.push_back(rv);
        const int tw = 1 << lw, th = 64 >> lw;
        const int ntx = (rv.width + tw - 1) / tw, nty = (rv.height + th - 1) / th;
        // tile coordinates are 16-bit in the descriptors
        if (ntx > 65536 || nty > 65536)
            return fail(DART_E_INVAL,
                        "view %d: %dx%d image in %dx%d tiles needs more than 65536 tiles per "
                        "side", i, rv.width, rv.height, tw, th);
        // (labelled stacks: the first sub-domain's box is not the domain's)
        const bool skip = rv.n_blocks == 0;
        const Footprint fp = footprint(rv);
        for (int ty = 0; ty < nty; ty++) {
            double u_lo = -INFINITY, u_hi = INFINITY;
            bool row_hits = true;
            if (skip) {
                const double w0 = (ty * th + 0.5 - 0.5 * rv.height) * rv.ps;
                const double w1 = ((ty + 1) * th - 0.5 - 0.5 * rv.height) * rv.ps;
                row_hits = band_span(fp, w0, w1, &u_lo, &u_hi);
            }
            for (int tx = 0; tx < ntx; tx++) {
                Tile t;
                t.view = vi;
                t.tx = (uint16_t)tx;
                t.ty = (uint16_t)ty;
                const double u0 = (tx * tw + 0.5 - 0.5 * rv.width) * rv.ps;
                const double u1 = ((tx + 1) * tw - 0.5 - 0.5 * rv.width) * rv.ps;
                if (skip && (!row_hits || u1 < u_lo || u0 > u_hi)) {
                    // cleared by a fill kernel; an adding view keeps its values
                    if (!(rv.flags & F_ACCUMULATE)) g.clear.push_back(t);
                } else {
                    g.tiles.push_back(t);
                }
            }
        }
    }
    for (Group &g : groups) {
        const size_t nq = MAX_QUEUES;
        bool bounds_set = false;
        if (tun.order == 4) {
            // whole tile rows, the row with the longest estimated tile first,
            // dealt round robin to the queue chunks: every chunk starts on
            // heavy rows and ends on light ones, and a row's tiles stay
            // together
            struct Row { double cost; uint32_t view; uint16_t ty; std::vector<Tile> tiles; };
            std::vector<Row> rows;
            std::map<std::pair<uint32_t, uint16_t>, size_t> at;
            for (const Tile &t : g.tiles) {
                auto key = std::make_pair(t.view, t.ty);
                auto it = at.find(key);
                if (it == at.end()) {
                    it = at.emplace(key, rows.size()).first;
                    rows.push_back(Row{0.0, t.view, t.ty, {}});
                }
                const RayView &tv = g.views[t.view];
                Row &r = rows[it->second];
                r.cost = std::max(r.cost, tile_cost(tv, t.tx, t.ty, 1 << tv.tile_w_log2,
                                                    64 >> tv.tile_w_log2));
                r.tiles.push_back(t);
            }
            std::stable_sort(rows.begin(), rows.end(),
                             [](const Row &a, const Row &b) { return a.cost > b.cost; });
            std::vector<std::vector<Tile>> chunk(nq);
            std::vector<size_t> load(nq, 0);
            for (const Row &r : rows) {
                // the chunk with the fewest tiles so far (ties: the lowest index)
                size_t q = 0;
                for (size_t k = 1; k < nq; k++)
                    if (load[k] < load[q]) q = k;
                chunk[q].insert(chunk[q].end(), r.tiles.begin(), r.tiles.end());
                load[q] += r.tiles.size();
            }
            g.tiles.clear();
            for (size_t q = 0; q < nq; q++) {
                g.q_begin[q] = (uint32_t)g.tiles.size();
                g.tiles.insert(g.tiles.end(), chunk[q].begin(), chunk[q].end());
            }
            g.q_begin[nq] = (uint32_t)g.tiles.size();
            bounds_set = true;
        } else if (tun.order == 3) {
            // rows from the middle outward: the upper half from its last row
            // up, then the lower half down.  Rows stay whole and in sequence
            // (neighbouring tiles still run together), but the rows through
            // the middle of the grid, whose rays are longest, start first and
            // each queue chunk ends with short or empty rows.
            auto row_key = [&g](const Tile &t) {
                const RayView &tv = g.views[t.view];
                const int th = 64 >> tv.tile_w_log2;
                const int nty = (tv.height + th - 1) / th, half = nty / 2;
                return t.ty < half ? half - 1 - t.ty : t.ty;
            };
            std::stable_sort(g.tiles.begin(), g.tiles.end(), [&](const Tile &a, const Tile &b) {
                if (a.view != b.view) return a.view < b.view;
                return row_key(a) < row_key(b);
            });
        } else if (tun.order == 2) {
            // Z-order (Morton) of the tile coordinates inside each view: tiles
            // that are close in the queue form compact 2D patches
            auto morton = [](uint32_t x, uint32_t y) {
                uint64_t k = 0;
                for (int b = 0; b < 16; b++)
                    k |= (uint64_t)((x >> b) & 1u) << (2 * b) | (uint64_t)((y >> b) & 1u) << (2 * b + 1);
                return k;
            };
            std::stable_sort(g.tiles.begin(), g.tiles.end(), [&](const Tile &a, const Tile &b) {
                if (a.view != b.view) return a.view < b.view;
                return morton(a.tx, a.ty) < morton(b.tx, b.ty);
            });
        } else if (tun.order == 1) {
            // longest estimated tile first; the queue chunks interleave so each
            // XCD's chunk also runs longest first
            std::vector<std::pair<double, uint32_t>> cost(g.tiles.size());
            for (size_t k = 0; k < g.tiles.size(); k++) {
                const Tile &t = g.tiles[k];
                const RayView &tv = g.views[t.view];
                cost[k] = {tile_cost(tv, t.tx, t.ty, 1 << tv.tile_w_log2, 64 >> tv.tile_w_log2),
                           (uint32_t)k};
            }
            std::stable_sort(cost.begin(), cost.end(),
                             [](const std::pair<double, uint32_t> &a,
                                const std::pair<double, uint32_t> &b) { return a.first > b.first; });
            const size_t nt = g.tiles.size();
            std::vector<Tile> out(nt);
            // rank r goes to chunk r % nq, position r / nq inside it
            std::vector<size_t> chunk_begin(nq + 1);
            for (size_t q = 0; q <= nq; q++) chunk_begin[q] = nt * q / nq;
            std::vector<size_t> fill(nq, 0);
            size_t q = 0;
            for (size_t r = 0; r < nt; r++) {
                // next chunk with room, round robin
                for (size_t tries = 0; tries < nq; tries++) {
                    if (chunk_begin[q] + fill[q] < chunk_begin[q + 1]) break;
                    q = (q + 1) % nq;
                }
                out[chunk_begin[q] + fill[q]++] = g.tiles[cost[r].second];
                q = (q + 1) % nq;
            }
            g.tiles.swap(out);
        }
        g.n_queues = (uint32_t)nq;
        if (!bounds_set)
            for (size_t q = 0; q <= nq; q++)
                g.q_begin[q] = (uint32_t)(((uint64_t)g.tiles.size() * q) / nq);
        // the tiles to clear follow the queued ones in the same array
        g.n_clear = (uint32_t)g.clear.size();
        g.tiles.insert(g.tiles.end(), g.clear.begin(), g.clear.end());
        g.clear.clear();
    }
    return DART_OK;
}

// Enqueues clear + persistent kernels of every group.  Accumulator layout:
// flux[n] (double bits), steps[n], then 4 slots (8 x uint32 queue heads) per
// group; dviews / dtiles hold the groups' descriptors at their offsets.
hipError_t dart::enqueue_plan(const std::vector<Group> &groups, int32_t n,
                              unsigned long long *acc, const RayView *dviews, const Tile *dtiles,
                              const dart_tuning &tun, int device, hipStream_t stream) {
    hipError_t e = launch_fill_u64(acc, 2 * (size_t)n + 4 * groups.size(), 0ull, stream);
    if (e != hipSuccess) return e;
    const int cus = device_cus(device);
    const int blocks = std::max(1, cus * tun.waves_per_cu / 4);
    for (size_t gi = 0; gi < groups.size(); gi++) {
        const Group &g = groups[gi];
        if (g.n_clear > 0) {
            e = launch_clear_tiles(dviews + g.view_off, dtiles + g.tile_off + g.q_begin[g.n_queues],
                                   g.n_clear, stream);
            if (e != hipSuccess) return e;
        }
        BatchLaunch bl;
        bl.views = dviews + g.view_off;
        bl.tiles = dtiles + g.tile_off;
        bl.n_tiles = (uint32_t)g.q_begin[g.n_queues];
        bl.head = (uint32_t *)(acc + 2 * (size_t)n + 4 * gi);
        bl.n_queues = g.n_queues;
        for (uint32_t q = 0; q <= g.n_queues; q++) bl.q_begin[q] = g.q_begin[q];
        bl.flux_acc = (double *)acc;
        bl.step_acc = acc + n;
        const int variant = g.vec ? (KV_VEC | (tun.cells_per_batch == 8 ? KV_K8 : 0))
                                  : (tun.depth_sync > 0 ? KV_SYNC : 0) |
                                        (g.labelled ? KV_LABELLED : 0) | (g.exact ? KV_EXACT : 0) |
                                        (g.jp ? KV_JP : 0) | (g.jp32 ? KV_JP32 : 0) |
                                        (tun.cells_per_batch == 8 ? KV_K8 : 0);
        // no more wavefronts than queued tiles: a small batch (one served
        // request of a few hundred tiles) launches only the workgroups its
        // tiles keep busy, instead of a full grid whose idle waves each visit
        // every queue head
        const int grid = std::max(1, std::min(blocks, (int)((bl.n_tiles + 3) / 4)));
        e = launch_batch(g.store, g.f64, variant, bl, grid, stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void dart::assign_offsets(std::vector<Group> &groups, size_t *n_views, size_t *n_tiles) {
    size_t nv = 0, nt = 0;
    for (Group &gr : groups) {
        gr.view_off = nv;
        gr.tile_off = nt;
        nv += gr.views.size();
        nt += gr.tiles.size();
    }
    *n_views = nv;
    *n_tiles = nt;
}

void dart::pack_descriptors(const std::vector<Group> &groups, size_t n_views, void *dst) {
    char *h = (char *)dst;
    char *ht = h + n_views * sizeof(RayView);
    for (const Group &gr : groups) {
        memcpy(h + gr.view_off * sizeof(RayView), gr.views.data(), gr.views.size() * sizeof(RayView));
        memcpy(ht + gr.tile_off * sizeof(Tile), gr.tiles.data(), gr.tiles.size() * sizeof(Tile));
    }
}

extern "C" dart_status dart_render_batch(const dart_stack *const *stacks, const dart_view *views,
                                         int32_t n, void *const *images, double *flux_out,
                                         uint64_t *steps_out, void *hip_stream) {
    if (n < 0 || (n > 0 && (!stacks || !views || !images)))
        return fail(DART_E_INVAL, "bad batch arguments");
    if (n == 0) return DART_OK;
    for (int32_t i = 0; i < n; i++)
        if (!stacks[i]) return fail(DART_E_INVAL, "stacks[%d] is NULL", i);
    {
        // two views of one call writing the same device image would race
        std::vector<std::pair<const void *, int32_t>> dst;
        for (int32_t i = 0; i < n; i++)
            if (views[i].flags & DART_DEVICE_PTRS) dst.emplace_back(images[i], i);
        std::sort(dst.begin(), dst.end());
        for (size_t k = 1; k < dst.size(); k++)
            if (dst[k].first == dst[k - 1].first)
                return fail(DART_E_INVAL, "views %d and %d write the same image", dst[k - 1].second,
                            dst[k].second);
    }
    bool force_plain = false;
    for (int32_t i = 0; i < n; i++)
        if (views[i].flags & DART_KERNEL_PLAIN) force_plain = true;
    hipStream_t stream = (hipStream_t)hip_stream;
    if (force_plain) {
        for (int32_t i = 0; i < n; i++) {
            dart_view v = views[i];
            v.flags &= ~DART_KERNEL_PLAIN;
            dart_status st = dart_render(stacks[i], &v, images[i], flux_out ? flux_out + i : nullptr,
                                         steps_out ? steps_out + i : nullptr, hip_stream);
            if (st != DART_OK) return st;
        }
        return DART_OK;
    }
    for (int32_t i = 0; i < n; i++) {
        dart_status st = refresh_vector(stacks[i], stream);
        if (st == DART_OK) st = refresh_jplane(stacks[i], stream, true);
        if (st != DART_OK) return st;
    }
    const dart_tuning tun = tuning_for(stacks[0]);
    Workspace *ws = get_workspace(stream);
    std::lock_guard<std::mutex> g(ws->mu);

    // replay key: everything the plan depends on
    std::vector<uint8_t> key;
    auto put = [&key](const void *p, size_t b) {
        const uint8_t *c = (const uint8_t *)p;
        key.insert(key.end(), c, c + b);
    };
    put(&n, sizeof(n));
    put(&tun, sizeof(tun));
    for (int32_t i = 0; i < n; i++) {
        put(&stacks[i], sizeof(void *));
        put(&stacks[i]->generation, sizeof(stacks[i]->generation));
        const uint8_t jp = jplane_ready(stacks[i]) ? 1 : 0;
        put(&jp, 1);
        put(&views[i], sizeof(dart_view));
        put(&images[i], sizeof(void *));
    }

    // host images render into workspace staging
    std::vector<void *> dev_images(images, images + n);
    std::vector<size_t> img_off(n, 0);
    size_t img_bytes = 0;
    for (int32_t i = 0; i < n; i++) {
        if (!(views[i].flags & DART_DEVICE_PTRS)) {
            img_off[i] = img_bytes;
            const size_t b = (size_t)stacks[i]->channels() * views[i].width * views[i].height *
                             (views[i].out_dtype == DART_F64 ? 8 : 4);
            img_bytes += (b + 255) & ~(size_t)255;
        }
    }
#ifndef DART_USE_GRAPH
#define DART_USE_GRAPH 1
#endif
    const bool use_graph = DART_USE_GRAPH && stream != nullptr;
    const bool replay = ws->plan_ready && key == ws->plan_key;
    if (!replay) {
        std::vector<Group> groups;
        // the plan needs image pointers; host ones are patched after reserve
        std::vector<void *> tmp_images(n);
        for (int32_t i = 0; i < n; i++)
            tmp_images[i] = images[i];
        dart_status st = plan_batch(stacks, views, n, tmp_images.data(), tun, groups);
        if (st != DART_OK) return st;
        size_t nv = 0, nt = 0;
        assign_offsets(groups, &nv, &nt);
        HIP_TRY(ws_reserve(ws, std::max(nv, (size_t)n), nt, img_bytes / 8 + 1, groups.size() * 4),
                "workspace");
        for (Group &gr : groups)
            for (RayView &rv : gr.views)
                if (!(views[rv.acc_index].flags & DART_DEVICE_PTRS))
                    rv.image = (char *)ws->img + img_off[rv.acc_index];
        // stage descriptors and upload
        char *h = (char *)ws->stage;
        pack_descriptors(groups, nv, h);
        char *ht = h + nv * sizeof(RayView);
        HIP_TRY(hipMemcpyAsync(ws->views, h, nv * sizeof(RayView), hipMemcpyHostToDevice, stream),
                "H2D views");
        HIP_TRY(hipMemcpyAsync(ws->tiles, ht, nt * sizeof(Tile), hipMemcpyHostToDevice, stream),
                "H2D tiles");
        HIP_TRY(hipEventRecord(ws->stage_done, stream), "event");
        drop_graph(ws);
        ws->plan_groups = groups;
        ws->plan_key = key;
        ws->plan_ready = true;
        if (use_graph) {
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal), "begin capture");
            hipError_t e = enqueue_plan(groups, n, ws->acc, ws->views, ws->tiles, tun, ws->device, stream);
            hipError_t e2 = hipStreamEndCapture(stream, &graph);
            if (e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return hip_fail(e, "capture batch");
            }
            if (e2 != hipSuccess) return hip_fail(e2, "end capture");
            hipGraphExec_t exec = nullptr;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return hip_fail(e, "instantiate graph");
            ws->graph_exec = exec;
            ws->graph_key = key;
        }
    }
    if (use_graph && ws->graph_exec)
        HIP_TRY(hipGraphLaunch(ws->graph_exec, stream), "graph launch");
    else
        HIP_TRY(enqueue_plan(ws->plan_groups, n, ws->acc, ws->views, ws->tiles, tun, ws->device,
                             stream),
                "batch kernels");
    for (int32_t i = 0; i < n; i++) note_use(stacks[i], stream);
    bool any_host = false;
    for (int32_t i = 0; i < n; i++) {
        if (!(views[i].flags & DART_DEVICE_PTRS)) {
            any_host = true;
            const size_t b = (size_t)stacks[i]->channels() * views[i].width * views[i].height *
                             (views[i].out_dtype == DART_F64 ? 8 : 4);
            HIP_TRY(hipMemcpyAsync(images[i], (char *)ws->img + img_off[i], b,
                                   hipMemcpyDeviceToHost, stream),
                    "D2H image");
        }
    }
    if (flux_out || steps_out || any_host) {
        std::vector<unsigned long long> acc(2 * (size_t)n);
        HIP_TRY(hipMemcpyAsync(acc.data(), ws->acc, acc.size() * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, stream),
                "D2H acc");
        HIP_TRY(hipStreamSynchronize(stream), "sync");
        for (int32_t i = 0; i < n; i++) {
            if (flux_out) memcpy(&flux_out[i], &acc[i], sizeof(double));
            if (steps_out) steps_out[i] = acc[n + i];
        }
    }
    return DART_OK;
}

// ------------------------------------------------------------------ autotune

extern "C" dart_status dart_autotune(dart_stack *const *stacks, const dart_view *views, int32_t n,
                                     int32_t rebrick, dart_tuning *best_out, double *best_ms_out,
                                     void *hip_stream) {
    if (n < 1 || !stacks || !views) return fail(DART_E_INVAL, "bad autotune arguments");
    for (int32_t i = 0; i < n; i++)
        if (!stacks[i] || (rebrick && (stacks[i]->labelled() || stacks[i]->vector())))
            return fail(DART_E_INVAL, "stacks[%d]: NULL, or labelled with rebrick != 0", i);
    hipStream_t stream = (hipStream_t)hip_stream;
    // scratch device images
    std::vector<dart_view> vv(views, views + n);
    size_t total = 0;
    std::vector<size_t> off(n);
    for (int32_t i = 0; i < n; i++) {
        vv[i].flags |= DART_DEVICE_PTRS;
        vv[i].flags &= ~(DART_KERNEL_PLAIN | DART_ACCUMULATE);
        off[i] = total;
        total += ((size_t)stacks[i]->channels() * views[i].width * views[i].height *
                      (views[i].out_dtype == DART_F64 ? 8 : 4) + 255) & ~(size_t)255;
    }
    void *buf = nullptr;
    HIP_TRY(hipMalloc(&buf, total), "hipMalloc(autotune images)");
    std::vector<void *> imgs(n);
    for (int32_t i = 0; i < n; i++) imgs[i] = (char *)buf + off[i];
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const dart_tuning saved = tuning_for(nullptr);
    std::vector<dart_tuning> cands;
    // Measured on MI355X: the L2 working set of the resident waves dominates,
    // so the sweep covers low occupancies, row-like tiles and both spatial orders.
    const int shapes[][2] = {{64, 1}, {32, 2}, {16, 4}, {8, 8}};
    const int waves[] = {12, 16, 8};  // (ties go to the earliest: 12 first)
    const int orders[] = {0, 3, 1, 2, 4};
    for (auto &sh : shapes)
        for (int w : waves)
            for (int order : orders)
                for (int orient = 0; orient < 2; orient++)
                    cands.push_back({sh[0], sh[1], w, order, orient, 0, 8});
    // Brick candidates: every power-of-two shape (sides up to 16) holding one
    // 128-B cache line of records, and, for stacks with an emissivity plane
    // (which renders read for the cells at rest), one line of the plane.
    // Which one wins depends on the view set: lines that extend along the
    // rays' directions are used whole by one ray, lines across the image plane
    // are only partly covered when rays are sparser than cells.
    std::vector<std::array<int, 3>> bricks;
    if (rebrick) {
        const uint32_t rb = record_bytes(stacks[0]->dev.store);
        std::vector<int> per_line = {(int)std::max(1u, 128u / rb)};
        if (jplane_eligible(stacks[0])) per_line.push_back((int)(128u / (rb / 4)));
        for (int pl : per_line)
            for (int bx = 1; bx <= std::min(pl, 16); bx *= 2)
                for (int by = 1; by <= 16 && bx * by <= pl; by *= 2) {
                    const int bz = pl / (bx * by);
                    if (bx * by * bz == pl && bz <= 16) bricks.push_back({bx, by, bz});
                }
    } else {
        bricks = {{0, 0, 0}};
    }
    // one warm-up call (plans and captures the graph), then the best of two replays
    auto measure = [&](const dart_tuning &c, float *ms_out) -> dart_status {
        for (int32_t i = 0; i < n; i++) {
            stacks[i]->tuning = c;
            stacks[i]->tuned = true;
        }
        dart_status r = dart_render_batch(stacks, vv.data(), n, imgs.data(), nullptr, nullptr, hip_stream);
        if (r != DART_OK) return r;
        // best of several replays: about 40 ms of timing per candidate, at
        // least 2 and at most 48 replays (short batches are noisier: a
        // sub-millisecond batch gets dozens)
        float ms_min = INFINITY;
        int reps = 2;
        for (int rep = 0; rep < reps; rep++) {
            (void)hipEventRecord(e0, stream);
            r = dart_render_batch(stacks, vv.data(), n, imgs.data(), nullptr, nullptr, hip_stream);
            (void)hipEventRecord(e1, stream);
            (void)hipEventSynchronize(e1);
            if (r != DART_OK) return r;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms_min = std::min(ms_min, ms);
            if (rep == 0) reps = std::max(2, std::min(48, (int)(40.0f / std::max(ms, 1e-3f))));
        }
        *ms_out = ms_min;
        return DART_OK;
    };
    auto rebrick_all = [&](const std::array<int, 3> &br) -> dart_status {
        for (int32_t i = 0; i < n; i++) {
            bool seen = false;
            for (int32_t k = 0; k < i; k++) seen |= stacks[k] == stacks[i];
            if (seen) continue;
            dart_status r = dart_stack_rebrick(stacks[i], br.data(), hip_stream);
            if (r != DART_OK) return r;
        }
        return DART_OK;
    };
    // Candidates within 2% of the fastest count as ties (timing noise); a tie
    // goes to the earliest candidate in the sweep order, so repeated tunings of
    // one workload settle on the same choice.
    auto pick = [](const std::vector<float> &ms) {
        const float lo = *std::min_element(ms.begin(), ms.end());
        for (size_t k = 0; k < ms.size(); k++)
            if (ms[k] <= 1.02f * lo) return k;
        return (size_t)0;
    };
    double best_ms = INFINITY;
    dart_tuning best = saved;
    dart_status result = DART_OK;
    // Stage 1: brick shapes under a few representative launch shapes.
    if (rebrick) {
        const dart_tuning probes[] = {{64, 1, 12, 0, 0, 0, 8}, {64, 1, 12, 0, 1, 0, 8},
                                      {8, 8, 12, 0, 0, 0, 8}};
        std::vector<float> brick_ms;
        for (auto &br : bricks) {
            result = rebrick_all(br);
            if (result != DART_OK) break;
            float b_ms = INFINITY;
            for (const dart_tuning &c : probes) {
                float ms = 0;
                result = measure(c, &ms);
                if (result != DART_OK) break;
                b_ms = std::min(b_ms, ms);
            }
            if (result != DART_OK) break;
            brick_ms.push_back(b_ms);
        }
        if (result == DART_OK) result = rebrick_all(bricks[pick(brick_ms)]);
    }
    // Stage 2: launch shapes on the chosen layout.  A candidate with orient = 1
    // that turns no view's tiles is the same launch as its orient = 0 twin and
    // is not timed again (timing noise would otherwise pick between the two).
    if (result == DART_OK) {
        std::vector<RayView> rvs(n);
        for (int32_t i = 0; i < n && result == DART_OK; i++)
            result = resolve_view(stacks[i], &vv[i], &rvs[i]);
        std::vector<dart_tuning> kept;
        for (const dart_tuning &c : cands) {
            bool turns = false;
            for (int32_t i = 0; i < n; i++) turns |= orient_flips(rvs[i], c);
            if (c.orient && !turns) continue;
            kept.push_back(c);
        }
        cands.swap(kept);
        std::vector<float> cand_ms;
        for (const dart_tuning &c : cands) {
            if (result != DART_OK) break;
            float ms = 0;
            result = measure(c, &ms);
            if (result != DART_OK) break;
            cand_ms.push_back(ms);
        }
        if (result == DART_OK) {
            const size_t k = pick(cand_ms);
            best = cands[k];
            best_ms = cand_ms[k];
        }
    }
    // Stage 3: cells per batch and depth-synchronous marching on the chosen
    // launch shape.  Stages 1 and 2 time 8 cells per batch (more loads in
    // flight per wave; the better default measured), and 8 is swept first
    // here, so that it wins ties: a stable choice keeps counter rows
    // applicable.
    if (result == DART_OK) {
        std::vector<dart_tuning> c3;
        std::vector<float> c3_ms;
        for (int k : {8, 4})
        for (int gap : {0, 1, 2, 3, 4, 6}) {
            if (k == 8 && gap == 0) {  // the launch shape as chosen, already timed
                c3.push_back(best);
                c3_ms.push_back((float)best_ms);
                continue;
            }
            dart_tuning c = best;
            c.cells_per_batch = k;
            c.depth_sync = gap;
            float ms = 0;
            result = measure(c, &ms);
            if (result != DART_OK) break;
            c3.push_back(c);
            c3_ms.push_back(ms);
        }
        if (result == DART_OK) {
            const size_t k = pick(c3_ms);
            best = c3[k];
            best_ms = c3_ms[k];
        }
    }
    for (int32_t i = 0; i < n; i++) {
        stacks[i]->tuning = best;
        stacks[i]->tuned = result == DART_OK;
    }
    (void)hipStreamSynchronize(stream);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (result != DART_OK) return result;
    if (best_out) *best_out = best;
    if (best_ms_out) *best_ms_out = best_ms;
    return DART_OK;
}

// ------------------------------------------------------------------ counting / probe

// Distinct marked bits over one view: records (line_log2 < 0) or 128-byte
// lines of the resident layout (2^line_log2 records each).
static dart_status count_marked(const dart_stack *s, const dart_view *v, int line_log2,
                                bool moving_only, uint64_t *out, void *hip_stream) {
    if (!out) return fail(DART_E_INVAL, "output pointer is NULL");
    if (s && s->labelled()) return fail(DART_E_INVAL, "count the sub-domains of a labelled stack");
    RayView rv;
    dart_status st = resolve_view(s, v, &rv);
    if (st != DART_OK) return st;
    hipStream_t stream = (hipStream_t)hip_stream;
    const uint64_t bits =
        line_log2 < 0 ? (uint64_t)s->dev.n[0] * s->dev.n[1] * s->dev.n[2] * s->dev.n_epochs
                      : ((s->dev.epoch_stride * s->dev.n_epochs) >> line_log2) + 1;
    const uint64_t words = (bits + 31) / 32;
    const uint64_t u64s = (words + 1) / 2 + 1;
    unsigned long long *bm = nullptr;
    HIP_TRY(hipMalloc(&bm, u64s * 8), "hipMalloc(bitmap)");
    unsigned long long *cnt = bm + (u64s - 1);
    hipError_t e = launch_fill_u64(bm, u64s, 0ull, stream);
    if (e == hipSuccess) e = launch_mark(rv, (uint32_t *)bm, line_log2, moving_only, stream);
    if (e == hipSuccess) e = launch_popcount((const uint32_t *)bm, words, cnt, stream);
    unsigned long long c = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&c, cnt, sizeof(c), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(bm);
    if (e != hipSuccess) return hip_fail(e, "count samples");
    *out = c;
    return DART_OK;
}

extern "C" dart_status dart_count_samples(const dart_stack *s, const dart_view *v,
                                          uint64_t *samples_out, void *hip_stream) {
    return count_marked(s, v, -1, false, samples_out, hip_stream);
}

extern "C" dart_status dart_count_lines(const dart_stack *s, const dart_view *v,
                                        uint64_t *lines_out, void *hip_stream) {
    if (!s) return fail(DART_E_INVAL, "NULL stack");
    const uint32_t rb = record_bytes(s->dev.store);
    int line_log2 = 0;
    while ((rb << (line_log2 + 1)) <= 128u) line_log2++;
    return count_marked(s, v, line_log2, false, lines_out, hip_stream);
}

extern "C" dart_status dart_count_bytes(const dart_stack *s, const dart_view *v,
                                        uint64_t *compulsory_out, uint64_t *line_bytes_out,
                                        void *hip_stream) {
    if (!s || !v) return fail(DART_E_INVAL, "NULL argument");
    if (s->labelled()) return fail(DART_E_INVAL, "count the sub-domains of a labelled stack");
    hipStream_t stream = (hipStream_t)hip_stream;
    dart_status st = refresh_jplane(s, stream, true);
    if (st != DART_OK) return st;
    const uint32_t rb = record_bytes(s->dev.store);
    auto lines_of = [](uint32_t elem) {
        int l = 0;
        while ((elem << (l + 1)) <= 128u) l++;
        return l;
    };
    const bool plane = !(v->flags & (DART_RECORDS_ONLY | DART_NO_KAHAN)) && jplane_ready(s);
    uint64_t samples = 0, lines = 0;
    st = count_marked(s, v, -1, false, &samples, hip_stream);
    if (st == DART_OK && line_bytes_out)
        st = count_marked(s, v, lines_of(plane ? rb / 4 : rb), false, &lines, hip_stream);
    if (st != DART_OK) return st;
    uint64_t comp = samples * (plane ? rb / 4 : rb), lb = lines * 128;
    if (plane) {
        // samples marked to be read whole cost their records as well
        uint64_t whole = 0, wlines = 0;
        st = count_marked(s, v, -1, true, &whole, hip_stream);
        if (st == DART_OK && line_bytes_out)
            st = count_marked(s, v, lines_of(rb), true, &wlines, hip_stream);
        if (st != DART_OK) return st;
        comp += whole * rb;
        lb += wlines * 128;
    }
    if (compulsory_out) *compulsory_out = comp;
    if (line_bytes_out) *line_bytes_out = lb;
    return DART_OK;
}

// Read-only bandwidth probe: every 16-byte word of src is loaded once and
// folded into a per-thread checksum, which is stored only if it equals one
// particular value.  The store keeps the loads from being removed; for the
// bench's buffer of ones it never happens (and if it did, the sink is valid
// device memory).
// Each thread keeps READ_PROBE_DEPTH independent 16-B loads in flight per
// iteration (coalesced across the grid), so the pass measures bandwidth rather
// than the latency of one load per thread.
constexpr int READ_PROBE_DEPTH = 8;

__global__ void __launch_bounds__(256) k_read_probe(const uint4 *__restrict__ src, uint64_t n,
                                                    uint32_t *__restrict__ sink) {
    uint32_t acc = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride * READ_PROBE_DEPTH) {
        uint4 w[READ_PROBE_DEPTH];
#pragma unroll
        for (int k = 0; k < READ_PROBE_DEPTH; k++) {
            const uint64_t ik = i + (uint64_t)k * stride;
            w[k] = ik < n ? src[ik] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int k = 0; k < READ_PROBE_DEPTH; k++) acc ^= w[k].x ^ w[k].y ^ w[k].z ^ w[k].w;
    }
    if (acc == 0x7fc00001u) sink[0] = acc;
}

// Gather probe: every 128-B line of the buffer read once, in an order that
// scatters neighbouring lines over the whole buffer (line k goes to line
// k * odd mod 2^b, a permutation).  Eight consecutive lanes read the eight
// 16-B words of one line, so a wave's load instruction touches eight unrelated
// lines: the access pattern of a gather over bricked records, without the
// reuse.
__global__ void __launch_bounds__(256) k_gather_probe(const uint4 *__restrict__ src,
                                                      uint64_t n_lines, uint32_t *__restrict__ sink) {
    uint32_t acc = 0;
    const uint64_t nw = n_lines * 8u, mask = n_lines - 1u;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
         i += stride * READ_PROBE_DEPTH) {
        uint4 w[READ_PROBE_DEPTH];
#pragma unroll
        for (int k = 0; k < READ_PROBE_DEPTH; k++) {
            const uint64_t ik = i + (uint64_t)k * stride;
            const uint64_t line = ((ik >> 3) * 0x9E3779B97F4A7C15ull) & mask;
            w[k] = ik < nw ? src[line * 8u + (ik & 7u)] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int k = 0; k < READ_PROBE_DEPTH; k++) acc ^= w[k].x ^ w[k].y ^ w[k].z ^ w[k].w;
    }
    if (acc == 0x7fc00001u) sink[0] = acc;
}

// Device word the probes write only if their XOR of the data hits one value;
// one per device (allocated on first use, on the current device).
static hipError_t probe_sink(uint32_t **out) {
    static std::map<int, uint32_t *> sinks;
    static std::mutex sink_mu;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(sink_mu);
    uint32_t *&sink = sinks[dev];
    if (!sink) {
        e = hipMalloc((void **)&sink, 256);
        if (e != hipSuccess) {
            sink = nullptr;
            return e;
        }
    }
    *out = sink;
    return hipSuccess;
}

extern "C" dart_status dart_gather_probe(const void *src, uint64_t bytes, int32_t reps,
                                         void *hip_stream) {
    const uint64_t n_lines = bytes / 128u;
    if (!src || bytes == 0 || bytes % 128u || (n_lines & (n_lines - 1u)) || reps < 1)
        return fail(DART_E_INVAL, "gather probe: bytes must be 128 times a power of two, reps > 0");
    hipStream_t stream = (hipStream_t)hip_stream;
    uint32_t *sink = nullptr;
    HIP_TRY(probe_sink(&sink), "hipMalloc(probe sink)");
    const uint64_t blocks = std::min<uint64_t>((n_lines * 8u + 255u) / 256u, 1u << 14);
    for (int32_t r = 0; r < reps; r++) {
        hipLaunchKernelGGL(k_gather_probe, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (const uint4 *)src, n_lines, sink);
        HIP_TRY(hipGetLastError(), "gather probe kernel");
    }
    return DART_OK;
}

extern "C" dart_status dart_bandwidth_probe(void *dst, const void *src, uint64_t bytes,
                                            int32_t reps, void *hip_stream) {
    if (!src || bytes == 0 || bytes % 16 || reps < 1)
        return fail(DART_E_INVAL, "bad probe arguments");
    hipStream_t stream = (hipStream_t)hip_stream;
    if (!dst) {
        // read-only: the loads feed an XOR that is stored only if it hits one
        // value (so the compiler keeps them); the sink must be valid memory
        uint32_t *sink = nullptr;
        HIP_TRY(probe_sink(&sink), "hipMalloc(probe sink)");
        const uint64_t n = bytes / 16;
        const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 1u << 14);
        for (int32_t r = 0; r < reps; r++) {
            hipLaunchKernelGGL(k_read_probe, dim3((unsigned)blocks), dim3(256), 0, stream,
                               (const uint4 *)src, n, sink);
            HIP_TRY(hipGetLastError(), "read probe kernel");
        }
        return DART_OK;
    }
    for (int32_t r = 0; r < reps; r++)
        HIP_TRY(launch_copy(dst, src, bytes, stream), "copy kernel");
    return DART_OK;
}
