// dart_stream.hip -- out-of-core rendering: the epochs stay in the caller's
// memory and stream through a ring of device epoch slots.
//
// The paper renders snapshot by snapshot and adds partial images into one
// buffer per camera (Sec. 4, Fig. 5); this is that chronology with the lookback
// sum split exactly: epoch interval [t_m, t_{m+1}) is rendered from the two
// epochs m and m+1 alone, over the cells whose retarded time falls in it
// (half-open, the last interval closed), and every interval adds into the
// images.  Intervals no view can see, and epochs no needed interval uses, are
// skipped without being read (the paper's proposed flexload, Sec. 5.2).  While
// interval m renders on the caller's stream, the next epoch is uploaded and
// converted on a copy stream into a free slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <set>
#include <vector>

#include "dart_runtime.h"

using namespace dart;

#define ST_TRY(call, what)                          \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

struct dart_streamer {
    int device = 0;
    int32_t M = 0;
    std::vector<double> times;
    dart_dtype storage = DART_F32;
    int32_t ring_n = 0;
    dart_stack *ring = nullptr;           // ring_n epoch slots, bricked like a stack
    double *d_times = nullptr;            // the whole series, and 1 / (t_{m+1} - t_m)
    double *d_invdt = nullptr;
    void *stage_j = nullptr, *stage_b = nullptr;  // one epoch of host source (b inside j's block)
    size_t stage_bytes = 0;
    unsigned long long *err = nullptr;    // [M] first bad element per loaded epoch
    unsigned long long *acc = nullptr;    // flux[n], steps[n], queue heads
    size_t acc_cap = 0;
    RayView *d_views = nullptr;
    size_t views_cap = 0;
    Tile *d_tiles = nullptr;
    size_t tiles_cap = 0;
    void *h_desc = nullptr;               // pinned descriptor staging
    size_t h_desc_cap = 0;
    hipEvent_t desc_done{};
    bool desc_pending = false;
    char *img_stage = nullptr;            // device images for host-destined views
    size_t img_cap = 0;
    hipStream_t copy = nullptr;
    std::vector<hipEvent_t> ready, freed;
    std::mutex mu;
    dart_stream_stats last{};
};

static hipError_t grow(void **p, size_t *cap, size_t need) {
    if (need <= *cap) return hipSuccess;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc(p, need);
    if (e == hipSuccess) *cap = need;
    return e;
}

extern "C" dart_status dart_streamer_create(const int32_t dims[3], const double cell[3],
                                            int32_t n_epochs, const double *epoch_times,
                                            dart_dtype storage, int32_t ring_epochs,
                                            const int32_t brick[3], dart_streamer **out) {
    if (out) *out = nullptr;
    if (!out || !epoch_times) return fail(DART_E_INVAL, "NULL argument");
    if (ring_epochs < 3 || ring_epochs > 64)
        return fail(DART_E_INVAL, "ring_epochs must be in [3, 64]");
    if (n_epochs < 1) return fail(DART_E_INVAL, "n_epochs must be >= 1");
    // the ring is a stack of ring_epochs slots; its own times are placeholders
    std::vector<double> slot_t(ring_epochs);
    for (int32_t k = 0; k < ring_epochs; k++) slot_t[k] = k;
    dart_stack *ring = nullptr;
    dart_status st = dart_stack_create(dims, cell, ring_epochs, slot_t.data(), storage, 0, &ring);
    if (st != DART_OK) return st;
    std::unique_ptr<dart_streamer> s(new dart_streamer);
    s->ring = ring;
    auto undo = [&](dart_status r) {
        (void)dart_free_epochs(s->ring);
        s->ring = nullptr;
        return r;
    };
    // series times: validated like a stack's
    for (int32_t m = 0; m < n_epochs; m++)
        if (!std::isfinite(epoch_times[m]) || (m > 0 && !(epoch_times[m] > epoch_times[m - 1])))
            return undo(fail(DART_E_INVAL, "epoch times must be finite and strictly increasing"));
    if (brick) {
        st = dart_stack_rebrick(ring, brick, nullptr);
        if (st != DART_OK) return undo(st);
    }
    s->device = ring->device;
    s->M = n_epochs;
    s->times.assign(epoch_times, epoch_times + n_epochs);
    s->storage = storage;
    s->ring_n = ring_epochs;
    std::vector<double> inv(n_epochs, 0.0);
    for (int32_t m = 0; m + 1 < n_epochs; m++) inv[m] = 1.0 / (s->times[m + 1] - s->times[m]);
    hipError_t e = hipMalloc(&s->d_times, n_epochs * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&s->d_invdt, n_epochs * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&s->err, n_epochs * sizeof(unsigned long long));
    if (e == hipSuccess)
        e = hipMemcpy(s->d_times, s->times.data(), n_epochs * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(s->d_invdt, inv.data(), n_epochs * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->desc_done, hipEventDisableTiming);
    s->ready.resize(ring_epochs);
    s->freed.resize(ring_epochs);
    for (int32_t k = 0; k < ring_epochs && e == hipSuccess; k++) {
        e = hipEventCreateWithFlags(&s->ready[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->freed[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        dart_streamer *raw = s.release();
        (void)dart_streamer_destroy(raw);
        return hip_fail(e, "streamer set-up");
    }
    *out = s.release();
    return DART_OK;
}

extern "C" dart_status dart_streamer_destroy(dart_streamer *s) {
    if (!s) return fail(DART_E_INVAL, "streamer is NULL");
    if (s->copy) (void)hipStreamSynchronize(s->copy);
    if (s->desc_pending) (void)hipEventSynchronize(s->desc_done);
    for (hipEvent_t ev : s->ready) if (ev) (void)hipEventSynchronize(ev), (void)hipEventDestroy(ev);
    for (hipEvent_t ev : s->freed) if (ev) (void)hipEventSynchronize(ev), (void)hipEventDestroy(ev);
    if (s->desc_done) (void)hipEventDestroy(s->desc_done);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    if (s->ring) {
        (void)hipDeviceSynchronize();
        (void)dart_free_epochs(s->ring);
    }
    // (stage_b points into stage_j's allocation)
    for (void *p : {(void *)s->d_times, (void *)s->d_invdt, s->stage_j, (void *)s->err,
                    (void *)s->acc, (void *)s->d_views, (void *)s->d_tiles, (void *)s->img_stage})
        if (p) (void)hipFree(p);
    if (s->h_desc) (void)hipHostFree(s->h_desc);
    delete s;
    return DART_OK;
}

extern "C" dart_status dart_streamer_get_stats(const dart_streamer *s, dart_stream_stats *out) {
    if (!s || !out) return fail(DART_E_INVAL, "NULL argument");
    *out = s->last;
    return DART_OK;
}

// The intervals [t_m, t_{m+1}] that view v can see: its retarded times over the
// grid's box are t_obs - s for s between the extreme projections of the box
// corners on s_hat (from the camera centre).  Single-epoch series: interval 0.
static void view_intervals(const dart_streamer *s, const RayView &rv, bool lookback,
                           std::vector<int32_t> &out) {
    const int32_t M = s->M;
    if (M == 1) {
        if (rv.fixed_m >= 0 || lookback) out.push_back(0);
        return;
    }
    if (!lookback) {
        if (rv.fixed_m >= 0) out.push_back(rv.fixed_m);
        return;
    }
    double smin = INFINITY, smax = -INFINITY;
    for (int c = 0; c < 8; c++) {
        double sv = 0.0;
        for (int a = 0; a < 3; a++) {
            const double x = (c >> a & 1) ? rv.st.n[a] * rv.st.cell[a] : 0.0;
            sv += (x - rv.centre[a]) * rv.shat[a];
        }
        smin = std::min(smin, sv);
        smax = std::max(smax, sv);
    }
    const double tlo = std::max(rv.t_obs - smax, s->times[0]);
    const double thi = std::min(rv.t_obs - smin, s->times[M - 1]);
    if (tlo > thi) return;
    for (int32_t m = 0; m + 1 < M; m++)
        if (s->times[m + 1] >= tlo && s->times[m] <= thi) out.push_back(m);
}

extern "C" dart_status dart_streamer_render(dart_streamer *s, dart_dtype src_dtype,
                                            const void *emissivity, const void *velocity,
                                            uint32_t src_flags, const dart_view *views, int32_t n,
                                            void *const *images, double *flux_out,
                                            uint64_t *steps_out, void *hip_stream) {
    if (!s || !emissivity || !velocity) return fail(DART_E_INVAL, "NULL argument");
    if (n < 1 || !views || !images) return fail(DART_E_INVAL, "bad view arguments");
    if (src_dtype != DART_F64 && src_dtype != DART_F32)
        return fail(DART_E_INVAL, "src_dtype must be DART_F64 or DART_F32");
    if (src_flags & ~(uint32_t)DART_DEVICE_PTRS) return fail(DART_E_INVAL, "unknown source flags");
    for (int32_t i = 0; i < n; i++)
        if (views[i].flags & DART_EXACT_TIME)
            return fail(DART_E_INVAL, "view %d: DART_EXACT_TIME is not streamed (a cell cut by an "
                        "interval boundary would count in both intervals)", i);
    std::lock_guard<std::mutex> lock(s->mu);
    hipStream_t stream = (hipStream_t)hip_stream;
    const int32_t M = s->M, R = s->ring_n;
    const StackDev &rd = s->ring->dev;
    const uint64_t ncell = (uint64_t)rd.n[0] * rd.n[1] * rd.n[2];
    const size_t rb = record_bytes(rd.store);
    const size_t esz = src_dtype == DART_F64 ? 8 : 4;
    const bool dev_src = (src_flags & DART_DEVICE_PTRS) != 0;
    for (int32_t i = 0; i < n; i++)
        if (!images[i]) return fail(DART_E_INVAL, "images[%d] is NULL", i);

    // a stack object describing the whole series, for view validation
    dart_stack whole;
    whole.dev = rd;
    whole.dev.n_epochs = M;
    whole.storage = s->storage;
    whole.times = s->times;
    whole.filled.assign(M, 1);
    whole.device = s->device;
    std::vector<RayView> rvs(n);
    std::vector<std::vector<int32_t>> need(n);
    for (int32_t i = 0; i < n; i++) {
        dart_status st = resolve_view(&whole, &views[i], &rvs[i]);
        if (st != DART_OK) return fail(st, "view %d: %s", i, dart_last_error());
        view_intervals(s, rvs[i], !(views[i].flags & DART_NO_LOOKBACK), need[i]);
    }
    std::set<int32_t> ivals;
    for (auto &v : need) ivals.insert(v.begin(), v.end());
    std::set<int32_t> eps;
    for (int32_t m : ivals) {
        eps.insert(m);
        if (M > 1) eps.insert(m + 1);
    }
    const std::vector<int32_t> order(eps.begin(), eps.end());  // load order
    std::vector<int32_t> slot(M, -1), rank(M, -1), last_use(M, -1);
    for (size_t r = 0; r < order.size(); r++) {
        slot[order[r]] = (int32_t)(r % R);
        rank[order[r]] = (int32_t)r;
    }
    const std::vector<int32_t> iv(ivals.begin(), ivals.end());
    for (size_t k = 0; k < iv.size(); k++) {
        last_use[iv[k]] = (int32_t)k;
        if (M > 1) last_use[iv[k] + 1] = (int32_t)k;
    }

    // device images: the caller's, or staging for host-destined views
    std::vector<void *> dimg(n);
    std::vector<size_t> img_bytes(n), img_off(n);
    size_t stage_total = 0;
    for (int32_t i = 0; i < n; i++) {
        img_bytes[i] = (size_t)views[i].width * views[i].height * (rvs[i].out_f64 ? 8 : 4);
        if (!(views[i].flags & DART_DEVICE_PTRS)) {
            img_off[i] = stage_total;
            stage_total += (img_bytes[i] + 255) & ~(size_t)255;
        }
    }
    ST_TRY(hipSetDevice(s->device), "hipSetDevice");
    ST_TRY(grow((void **)&s->img_stage, &s->img_cap, std::max<size_t>(stage_total, 256)), "image staging");
    for (int32_t i = 0; i < n; i++)
        dimg[i] = (views[i].flags & DART_DEVICE_PTRS) ? images[i] : (void *)(s->img_stage + img_off[i]);

    // one descriptor set for every interval: interval stacks over ring slots
    const dart_tuning tun = tuning_for(nullptr);
    std::vector<std::unique_ptr<dart_stack>> istacks;
    std::vector<Group> groups;
    std::vector<size_t> gbegin;  // first group of each interval
    for (int32_t m : iv) {
        std::unique_ptr<dart_stack> is(new dart_stack);
        is->dev = rd;
        const int32_t ne = M > 1 ? 2 : 1;
        is->dev.n_epochs = ne;
        is->dev.data = (const char *)rd.data + (size_t)slot[m] * rd.epoch_stride * rb;
        is->dev.epoch_stride = M > 1 ? (int64_t)(slot[m + 1] - slot[m]) * rd.epoch_stride : rd.epoch_stride;
        is->dev.times = s->d_times + m;
        is->dev.inv_dt = s->d_invdt + m;
        is->storage = s->storage;
        is->times.assign(s->times.begin() + m, s->times.begin() + m + ne);
        is->filled.assign(ne, 1);
        is->device = s->device;
        std::vector<const dart_stack *> sts;
        std::vector<dart_view> vv;
        std::vector<void *> im;
        std::vector<int32_t> gidx;
        for (int32_t i = 0; i < n; i++)
            if (std::find(need[i].begin(), need[i].end(), m) != need[i].end()) {
                dart_view v = views[i];
                // FP64 ray parameters for every storage type: a chord midpoint at
                // an interval boundary then compares the same in both intervals,
                // so each cell is summed (and counted) exactly once
                v.flags = (v.flags & ~(DART_KERNEL_PLAIN)) | DART_DEVICE_PTRS | DART_ACCUMULATE |
                          DART_FORCE_F64_DDA;
                vv.push_back(v);
                sts.push_back(is.get());
                im.push_back(dimg[i]);
                gidx.push_back(i);
            }
        std::vector<Group> g;
        dart_status st = plan_batch(sts.data(), vv.data(), (int32_t)vv.size(), im.data(), tun, g);
        if (st != DART_OK) return st;
        const bool lo_open = M > 1 && m + 1 < M - 1;
        for (Group &gr : g)
            for (RayView &rv : gr.views) {
                // [t_m, t_{m+1}) in t is (t_obs - t_{m+1}, t_obs - t_m] in s.  The
                // open end becomes the next double above s_lo: the kernel's
                // s >= s_lo test in FP64 ray parameters is then s > the end,
                // with no extra per-cell test
                if (!(rv.flags & F_NO_LOOKBACK) && lo_open) rv.s_lo = std::nextafter(rv.s_lo, INFINITY);
                rv.acc_index = gidx[rv.acc_index];
            }
        gbegin.push_back(groups.size());
        for (Group &gr : g) groups.push_back(std::move(gr));
        istacks.push_back(std::move(is));
    }
    gbegin.push_back(groups.size());
    size_t nv = 0, nt = 0;
    assign_offsets(groups, &nv, &nt);
    const size_t desc = nv * sizeof(RayView) + nt * sizeof(Tile);
    if (s->desc_pending) {
        ST_TRY(hipEventSynchronize(s->desc_done), "descriptor staging");
        s->desc_pending = false;
    }
    if (desc > s->h_desc_cap) {
        if (s->h_desc) (void)hipHostFree(s->h_desc);
        s->h_desc = nullptr;
        s->h_desc_cap = 0;
        ST_TRY(hipHostMalloc(&s->h_desc, std::max<size_t>(desc, 4096), hipHostMallocDefault), "pinned staging");
        s->h_desc_cap = std::max<size_t>(desc, 4096);
    }
    ST_TRY(grow((void **)&s->d_views, &s->views_cap, std::max<size_t>(nv, 1) * sizeof(RayView)), "views");
    ST_TRY(grow((void **)&s->d_tiles, &s->tiles_cap, std::max<size_t>(nt, 1) * sizeof(Tile)), "tiles");
    const size_t acc_n = 2 * (size_t)n + 4 * std::max<size_t>(groups.size(), 1);
    ST_TRY(grow((void **)&s->acc, &s->acc_cap, acc_n * 8), "accumulators");
    if (nv > 0) {
        pack_descriptors(groups, nv, s->h_desc);
        ST_TRY(hipMemcpyAsync(s->d_views, s->h_desc, nv * sizeof(RayView), hipMemcpyHostToDevice, stream), "H2D views");
        ST_TRY(hipMemcpyAsync(s->d_tiles, (char *)s->h_desc + nv * sizeof(RayView), nt * sizeof(Tile),
                              hipMemcpyHostToDevice, stream), "H2D tiles");
        ST_TRY(hipEventRecord(s->desc_done, stream), "event");
        s->desc_pending = true;
    }
    ST_TRY(launch_fill_u64(s->acc, acc_n, 0ull, stream), "clear accumulators");
    ST_TRY(launch_fill_u64(s->err, M, ~0ull, stream), "clear error flags");
    for (int32_t i = 0; i < n; i++)
        if (!(views[i].flags & DART_ACCUMULATE))
            ST_TRY(hipMemsetAsync(dimg[i], 0, img_bytes[i], stream), "clear image");
    // the copy stream starts after everything above (buffers of the last call)
    hipEvent_t start;
    ST_TRY(hipEventCreateWithFlags(&start, hipEventDisableTiming), "event");
    (void)hipEventRecord(start, stream);
    (void)hipStreamWaitEvent(s->copy, start, 0);
    (void)hipEventDestroy(start);

    if (!dev_src) {
        ST_TRY(grow(&s->stage_j, &s->stage_bytes, ncell * esz * 4), "source staging");
        s->stage_b = (char *)s->stage_j + ncell * esz;
    }
    std::vector<char> slot_used(R, 0);
    size_t next = 0;
    uint64_t uploaded = 0;
    const int cus = device_cus(s->device);
    const int blocks = std::max(1, cus * tun.waves_per_cu / 4);
    auto load = [&](int32_t e) -> dart_status {
        const int32_t k = slot[e];
        if (slot_used[k]) ST_TRY(hipStreamWaitEvent(s->copy, s->freed[k], 0), "wait slot");
        slot_used[k] = 1;
        const char *hj = (const char *)emissivity + (size_t)e * ncell * esz;
        const char *hb = (const char *)velocity + (size_t)e * ncell * esz * 3;
        const void *dj = hj, *db = hb;
        if (!dev_src) {
            ST_TRY(hipMemcpyAsync(s->stage_j, hj, ncell * esz, hipMemcpyHostToDevice, s->copy), "H2D j");
            ST_TRY(hipMemcpyAsync(s->stage_b, hb, ncell * esz * 3, hipMemcpyHostToDevice, s->copy), "H2D beta");
            uploaded += ncell * esz * 4;
            dj = s->stage_j;
            db = s->stage_b;
        }
        // convert into slot k; a bad element is reported in err[e]
        ST_TRY(launch_convert(esz == 8, rd.store, dj, db, k, 1, rd, (void *)rd.data, s->err + e,
                              s->copy), "convert kernel");
        ST_TRY(hipEventRecord(s->ready[k], s->copy), "event");
        return DART_OK;
    };
    for (size_t k = 0; k < iv.size(); k++) {
        const int32_t m = iv[k];
        const int32_t hi = M > 1 ? m + 1 : m;
        // load every epoch up to R - 2 ahead of this interval's later epoch
        while (next < order.size() && rank[order[next]] <= rank[hi] + (R - 2)) {
            dart_status st = load(order[next]);
            if (st != DART_OK) return st;
            next++;
        }
        ST_TRY(hipStreamWaitEvent(stream, s->ready[slot[m]], 0), "wait epoch");
        if (hi != m) ST_TRY(hipStreamWaitEvent(stream, s->ready[slot[hi]], 0), "wait epoch");
        for (size_t gi = gbegin[k]; gi < gbegin[k + 1]; gi++) {
            const Group &g = groups[gi];
            BatchLaunch bl;
            bl.views = s->d_views + g.view_off;
            bl.tiles = s->d_tiles + g.tile_off;
            bl.n_tiles = (uint32_t)g.tiles.size();
            bl.head = (uint32_t *)(s->acc + 2 * (size_t)n + 4 * gi);
            bl.n_queues = g.n_queues;
            for (uint32_t q = 0; q <= g.n_queues; q++) bl.q_begin[q] = g.q_begin[q];
            bl.flux_acc = (double *)s->acc;
            bl.step_acc = s->acc + n;
            const int variant = (tun.depth_sync > 0 ? KV_SYNC : 0) | (g.labelled ? KV_LABELLED : 0) |
                                (tun.cells_per_batch == 8 ? KV_K8 : 0);
            ST_TRY(launch_batch(g.store, g.f64, variant, bl, blocks, stream), "interval kernel");
        }
        for (int32_t e : {m, hi})
            if (last_use[e] == (int32_t)k) ST_TRY(hipEventRecord(s->freed[slot[e]], stream), "event");
    }
    // results
    for (int32_t i = 0; i < n; i++)
        if (!(views[i].flags & DART_DEVICE_PTRS))
            ST_TRY(hipMemcpyAsync(images[i], dimg[i], img_bytes[i], hipMemcpyDeviceToHost, stream), "D2H image");
    std::vector<unsigned long long> acc(2 * (size_t)n), bad(M);
    ST_TRY(hipMemcpyAsync(acc.data(), s->acc, acc.size() * 8, hipMemcpyDeviceToHost, stream), "D2H acc");
    ST_TRY(hipStreamSynchronize(s->copy), "sync copy stream");
    ST_TRY(hipMemcpyAsync(bad.data(), s->err, M * 8, hipMemcpyDeviceToHost, stream), "D2H err");
    ST_TRY(hipStreamSynchronize(stream), "sync");
    for (int32_t e = 0; e < M; e++)
        if (bad[e] != ~0ull) {
            const uint64_t c = bad[e] % ncell;
            return fail(DART_E_RANGE, "non-finite value or |beta| >= 1 at epoch %d, cell (x=%llu, "
                        "y=%llu, z=%llu)", e, (unsigned long long)(c % rd.n[0]),
                        (unsigned long long)((c / rd.n[0]) % rd.n[1]),
                        (unsigned long long)(c / ((uint64_t)rd.n[0] * rd.n[1])));
        }
    for (int32_t i = 0; i < n; i++) {
        if (flux_out) memcpy(&flux_out[i], &acc[i], sizeof(double));
        if (steps_out) steps_out[i] = acc[n + i];
    }
    s->last.epochs_loaded = (int32_t)order.size();
    s->last.epochs_skipped = M - (int32_t)order.size();
    s->last.intervals = (int32_t)iv.size();
    s->last.bytes_uploaded = uploaded;
    return DART_OK;
}
