// dart_server.hip -- render-request server with continuous batching.
//
// A scheduler thread owns the device side of every request.  Requests wait in
// a FIFO until admission: a request is admitted when its output image (and a
// share of the wave's descriptors) fits in the server's HBM arena and fewer
// than max_inflight requests are admitted.  Whenever one of the server's
// streams is idle, every admitted request that is not yet running forms the
// next wave: one batched plan (persistent tile-queue kernels), launched on that
// stream, so waves on different streams overlap on the device.  A host
// callback at the end of each wave stamps the completion time; the scheduler
// then delivers the images (device-to-device, or through pinned staging to
// host memory), frees the arena space and admits waiting requests.
#include <hip/hip_runtime.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dart.h"
#include "dart_internal.h"
#include "dart_runtime.h"

using namespace dart;
using Clock = std::chrono::steady_clock;

namespace {

// First-fit allocator over one contiguous region (offsets only).
class Arena {
  public:
    void init(size_t size) {
        size_ = size;
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

  private:
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Req {
    uint64_t ticket = 0;
    const dart_stack *stack = nullptr;
    dart_view view{};
    void *dest = nullptr;
    bool host_dest = false;
    size_t img_bytes = 0;
    size_t desc_bound = 0;  // upper bound of the request's share of a wave's descriptors
    size_t dev_off = 0, host_off = 0;
    bool admitted = false;
    bool waited = false;  // counted once in admission_waits
    Clock::time_point t_submit;
    double latency_ms = 0, flux = 0;
    uint64_t steps = 0;
    int state = 0;  // 0 queued, 1 admitted, 2 running, 3 done, 4 failed
    dart_status err = DART_OK;
    std::string err_msg;
};

struct Wave {
    std::vector<Req *> reqs;
    int stream_idx = 0;
    bool done = false;
    Clock::time_point t_plan;    // the scheduler starts planning the wave
    Clock::time_point t_launch;  // its device work is enqueued
    Clock::time_point t_done;    // the completion callback ran
    struct dart_server *srv = nullptr;
};

}  // namespace

struct dart_server {
    int device = 0;
    size_t budget = 0;
    int max_inflight = 0;
    std::vector<hipStream_t> streams;
    std::vector<bool> stream_busy;
    // per stream: descriptor buffer on the device and its pinned upload staging
    // (also the flux / step readback), fixed at creation and outside the budget
    std::vector<void *> desc_dev, desc_host;
    size_t desc_cap = 0;
    // per stream: events around a wave's device work (upload .. readback) and
    // around its render kernels, and when its previous wave completed
    std::vector<hipEvent_t> ev_begin, ev_kbegin, ev_kend, ev_end;
    std::vector<Clock::time_point> stream_free_at;
    std::vector<bool> stream_waited;  // requests were queued when the stream's last wave retired
    void *dev_base = nullptr;    // device arena: images and wave descriptors
    void *host_base = nullptr;   // pinned arena: descriptor uploads, flux readback, host images
    size_t host_size = 0;
    Arena dev_arena, host_arena;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req *> queue;                        // submitted, waiting for admission / a wave
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    std::vector<std::unique_ptr<Wave>> waves;       // in flight
    uint64_t next_ticket = 1;
    int admitted = 0;
    bool stop = false;
    std::thread thr;
    dart_server_stats stats{};
    dart_server_timeline tl{};
};

static double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

static void on_wave_done(void *p) {
    Wave *w = (Wave *)p;
    dart_server *srv = w->srv;
    std::lock_guard<std::mutex> g(srv->mu);
    w->done = true;
    w->t_done = Clock::now();
    srv->cv.notify_all();
}

// Frees a finished wave's resources and publishes its results.  Caller holds mu.
static void retire(dart_server *srv, Wave *w) {
    const size_t n = w->reqs.size();
    {
        // the completion callback ran after every event of the wave: all complete
        const int k = w->stream_idx;
        float dev_ms = 0, ker_ms = 0;
        if (hipEventElapsedTime(&dev_ms, srv->ev_begin[k], srv->ev_end[k]) == hipSuccess &&
            hipEventElapsedTime(&ker_ms, srv->ev_kbegin[k], srv->ev_kend[k]) == hipSuccess) {
            srv->tl.device_ms += dev_ms;
            srv->tl.kernel_ms += ker_ms;
        }
        srv->tl.callback_to_retire_ms += ms_between(w->t_done, Clock::now());
        srv->tl.waves_timed++;
        srv->stream_free_at[k] = w->t_done;
        srv->stream_waited[k] = !srv->queue.empty();
    }
    const unsigned long long *acc_h = (const unsigned long long *)srv->desc_host[w->stream_idx];
    for (size_t i = 0; i < n; i++) {
        Req *r = w->reqs[i];
        double f;
        memcpy(&f, &acc_h[i], sizeof(f));
        r->flux = f;
        r->steps = acc_h[n + i];
        if (r->host_dest)
            memcpy(r->dest, (char *)srv->host_base + r->host_off, r->img_bytes);
        r->latency_ms =
            std::chrono::duration<double, std::milli>(w->t_done - r->t_submit).count();
        r->state = 3;
        srv->dev_arena.release(r->dev_off, r->img_bytes);
        if (r->host_dest) srv->host_arena.release(r->host_off, r->img_bytes);
        const_cast<dart_stack *>(r->stack)->pinned--;
        srv->admitted--;
        srv->stats.completed++;
    }
    srv->stream_busy[w->stream_idx] = false;
    srv->stats.bytes_in_use = srv->dev_arena.used();
}

static void fail_wave(dart_server *srv, Wave *w, dart_status st, const std::string &msg) {
    for (Req *r : w->reqs) {
        r->state = 4;
        r->err = st;
        r->err_msg = msg;
        srv->dev_arena.release(r->dev_off, r->img_bytes);
        if (r->host_dest) srv->host_arena.release(r->host_off, r->img_bytes);
        const_cast<dart_stack *>(r->stack)->pinned--;
        srv->admitted--;
    }
    srv->stream_busy[w->stream_idx] = false;
}

// Admission: FIFO, stop at the first request that does not fit.  Caller holds mu.
static void admit(dart_server *srv) {
    auto wait = [srv](Req *r) {
        if (!r->waited) {
            r->waited = true;
            srv->stats.admission_waits++;
        }
    };
    for (Req *r : srv->queue) {
        if (r->admitted) continue;
        if (srv->admitted >= srv->max_inflight) {
            wait(r);
            return;
        }
        size_t doff = 0, hoff = 0;
        if (!srv->dev_arena.alloc(r->img_bytes, &doff)) {
            wait(r);
            return;
        }
        if (r->host_dest && !srv->host_arena.alloc(r->img_bytes, &hoff)) {
            srv->dev_arena.release(doff, r->img_bytes);
            wait(r);
            return;
        }
        r->dev_off = doff;
        r->host_off = hoff;
        r->admitted = true;
        r->state = 1;
        const_cast<dart_stack *>(r->stack)->pinned++;
        srv->admitted++;
        srv->stats.bytes_in_use = srv->dev_arena.used();
        if (srv->stats.bytes_in_use > srv->stats.bytes_peak)
            srv->stats.bytes_peak = srv->stats.bytes_in_use;
    }
}

// Builds and launches one wave from the admitted requests at the queue front.
// Called with mu held; releases it around the HIP calls.
static void launch_wave(dart_server *srv, std::unique_lock<std::mutex> &lk, int sidx) {
    std::unique_ptr<Wave> w(new Wave());
    w->srv = srv;
    w->stream_idx = sidx;
    w->t_plan = Clock::now();
    // 256-B alignment of the accumulators + 64 B per request (flux, steps and
    // queue heads) on top of each request's descriptor bound
    size_t bound = 320;
    while (!srv->queue.empty() && srv->queue.front()->admitted &&
           (w->reqs.empty() || bound + srv->queue.front()->desc_bound <= srv->desc_cap)) {
        bound += srv->queue.front()->desc_bound;
        w->reqs.push_back(srv->queue.front());
        srv->queue.pop_front();
    }
    if (w->reqs.empty()) return;
    const int32_t n = (int32_t)w->reqs.size();
    std::vector<const dart_stack *> stacks(n);
    std::vector<dart_view> views(n);
    std::vector<void *> imgs(n);
    for (int32_t i = 0; i < n; i++) {
        Req *r = w->reqs[i];
        r->state = 2;
        stacks[i] = r->stack;
        views[i] = r->view;
        views[i].flags |= DART_DEVICE_PTRS;
        imgs[i] = (char *)srv->dev_base + r->dev_off;
    }
    dart_tuning tun = tuning_for(stacks[0]);
    // Every wave is planned here, on the scheduler thread, while the other
    // streams render.  Orders 1 and 4 estimate every tile's ray length and
    // sort by it (at saturation, tens of ms of host time per wave of
    // hundreds of requests, more than the wave's device time); waves keep the
    // tuned shape with tiles in row order instead.
    if (tun.order == 1 || tun.order == 4) tun.order = 0;
    std::vector<Group> groups;
    dart_status st = plan_batch(stacks.data(), views.data(), n, imgs.data(), tun, groups);
    if (st != DART_OK) {
        fail_wave(srv, w.get(), st, dart_last_error());
        return;
    }
    size_t nv = 0, nt = 0;
    assign_offsets(groups, &nv, &nt);
    const size_t acc_u64 = 2 * (size_t)n + 4 * groups.size();
    const size_t desc_bytes = nv * sizeof(RayView) + nt * sizeof(Tile);
    const size_t acc_off = (desc_bytes + 255) & ~(size_t)255;
    if (acc_off + acc_u64 * 8 > srv->desc_cap) {
        // cannot happen: the per-request bounds cover the plan
        fail_wave(srv, w.get(), DART_E_INTERNAL, "wave descriptors exceed their buffer");
        return;
    }
    srv->stream_busy[sidx] = true;
    srv->stats.waves++;
    if ((uint64_t)n > srv->stats.max_wave_requests) srv->stats.max_wave_requests = n;
    Wave *wp = w.get();
    srv->waves.push_back(std::move(w));
    char *hstage = (char *)srv->desc_host[sidx];
    char *ddesc = (char *)srv->desc_dev[sidx];
    unsigned long long *dacc = (unsigned long long *)(ddesc + acc_off);
    pack_descriptors(groups, nv, hstage);
    hipStream_t stream = srv->streams[sidx];
    const Clock::time_point t_planned = Clock::now();
    // the stream's idle time before this wave while requests were waiting:
    // from its last wave's completion, if the queue held requests then
    const double idle_ms =
        srv->stream_waited[sidx] ? ms_between(srv->stream_free_at[sidx], wp->t_plan) : 0.0;
    srv->stream_waited[sidx] = false;
    lk.unlock();
    hipError_t e = hipEventRecord(srv->ev_begin[sidx], stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ddesc, hstage, desc_bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(srv->ev_kbegin[sidx], stream);
    if (e == hipSuccess)
        e = enqueue_plan(groups, n, dacc, (const RayView *)ddesc,
                         (const Tile *)(ddesc + nv * sizeof(RayView)), tun, srv->device, stream);
    if (e == hipSuccess) e = hipEventRecord(srv->ev_kend[sidx], stream);
    for (int32_t i = 0; i < n && e == hipSuccess; i++) {
        Req *r = wp->reqs[i];
        if (r->host_dest)
            e = hipMemcpyAsync((char *)srv->host_base + r->host_off, imgs[i], r->img_bytes,
                               hipMemcpyDeviceToHost, stream);
        else
            e = hipMemcpyAsync(r->dest, imgs[i], r->img_bytes, hipMemcpyDeviceToDevice, stream);
    }
    // the flux and step accumulators overwrite the (already consumed) descriptor staging
    if (e == hipSuccess)
        e = hipMemcpyAsync(hstage, dacc, (size_t)n * 16, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipEventRecord(srv->ev_end[sidx], stream);
    if (e == hipSuccess) {
        for (int32_t i = 0; i < n; i++) note_use(stacks[i], stream);
        e = hipLaunchHostFunc(stream, on_wave_done, wp);
    }
    const Clock::time_point t_enqueued = Clock::now();
    lk.lock();
    wp->t_launch = t_enqueued;
    srv->tl.plan_ms += ms_between(wp->t_plan, t_planned);
    srv->tl.enqueue_ms += ms_between(t_planned, t_enqueued);
    srv->tl.stream_idle_ms += idle_ms;
    if (e != hipSuccess) {
        // the device work may still be queued: wait for the stream before freeing
        lk.unlock();
        (void)hipStreamSynchronize(stream);
        lk.lock();
        fail_wave(srv, wp, DART_E_DEVICE, hipGetErrorString(e));
        for (auto it = srv->waves.begin(); it != srv->waves.end(); ++it)
            if (it->get() == wp) {
                srv->waves.erase(it);
                break;
            }
    }
}

static void scheduler(dart_server *srv) {
    (void)hipSetDevice(srv->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        // retire finished waves
        for (size_t i = 0; i < srv->waves.size();) {
            if (srv->waves[i]->done) {
                retire(srv, srv->waves[i].get());
                srv->waves.erase(srv->waves.begin() + i);
                srv->cv.notify_all();
            } else {
                i++;
            }
        }
        admit(srv);
        // launch on an idle stream when admitted work is waiting
        bool launched = false;
        if (!srv->queue.empty() && srv->queue.front()->admitted) {
            for (size_t k = 0; k < srv->streams.size(); k++)
                if (!srv->stream_busy[k]) {
                    const size_t before = srv->queue.size();
                    launch_wave(srv, lk, (int)k);
                    launched = srv->queue.size() != before;
                    break;
                }
        }
        if (launched) continue;
        if (srv->stop && srv->queue.empty() && srv->waves.empty()) break;
        srv->cv.wait(lk);
    }
}

extern "C" dart_status dart_server_create(size_t hbm_budget_bytes, int32_t max_inflight,
                                          int32_t n_streams, dart_server **out) {
    if (!out) return fail(DART_E_INVAL, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes < (1u << 20)) return fail(DART_E_INVAL, "budget below 1 MiB");
    if (max_inflight < 1) return fail(DART_E_INVAL, "max_inflight must be >= 1");
    if (n_streams < 1 || n_streams > 8) return fail(DART_E_INVAL, "n_streams must be in [1, 8]");
    std::unique_ptr<dart_server> srv(new dart_server());
    if (hipGetDevice(&srv->device) != hipSuccess) return fail(DART_E_DEVICE, "hipGetDevice");
    srv->budget = hbm_budget_bytes;
    srv->max_inflight = max_inflight;
    hipError_t e = hipMalloc(&srv->dev_base, hbm_budget_bytes);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(server arena)");
    srv->host_size = std::min(hbm_budget_bytes, (size_t)1 << 30);
    e = hipHostMalloc(&srv->host_base, srv->host_size, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipFree(srv->dev_base);
        return hip_fail(e, "hipHostMalloc(server staging)");
    }
    srv->dev_arena.init(hbm_budget_bytes);
    srv->host_arena.init(srv->host_size);
    for (int32_t k = 0; k < n_streams; k++) {
        hipStream_t s;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (hipStream_t q : srv->streams) (void)hipStreamDestroy(q);
            (void)hipFree(srv->dev_base);
            (void)hipHostFree(srv->host_base);
            return hip_fail(e, "hipStreamCreate");
        }
        srv->streams.push_back(s);
        srv->stream_busy.push_back(false);
    }
    // room for at least one 1024^2 request of 1x64 tiles, up to 64 MiB per stream
    srv->desc_cap = std::max((size_t)4 << 20, std::min((size_t)64 << 20, hbm_budget_bytes / 4));
    for (int32_t k = 0; k < n_streams; k++) {
        void *d = nullptr, *h = nullptr;
        e = hipMalloc(&d, srv->desc_cap);
        if (e == hipSuccess) e = hipHostMalloc(&h, srv->desc_cap, hipHostMallocDefault);
        if (e != hipSuccess) {
            if (d) (void)hipFree(d);
            for (void *q : srv->desc_dev) (void)hipFree(q);
            for (void *q : srv->desc_host) (void)hipHostFree(q);
            for (hipStream_t q : srv->streams) (void)hipStreamDestroy(q);
            (void)hipFree(srv->dev_base);
            (void)hipHostFree(srv->host_base);
            return hip_fail(e, "server descriptor buffers");
        }
        srv->desc_dev.push_back(d);
        srv->desc_host.push_back(h);
    }
    for (int32_t k = 0; k < n_streams && e == hipSuccess; k++) {
        hipEvent_t ev[4] = {};
        for (int q = 0; q < 4 && e == hipSuccess; q++) e = hipEventCreate(&ev[q]);
        srv->ev_begin.push_back(ev[0]);
        srv->ev_kbegin.push_back(ev[1]);
        srv->ev_kend.push_back(ev[2]);
        srv->ev_end.push_back(ev[3]);
    }
    if (e != hipSuccess) {
        for (auto *v : {&srv->ev_begin, &srv->ev_kbegin, &srv->ev_kend, &srv->ev_end})
            for (hipEvent_t q : *v)
                if (q) (void)hipEventDestroy(q);
        for (void *q : srv->desc_dev) (void)hipFree(q);
        for (void *q : srv->desc_host) (void)hipHostFree(q);
        for (hipStream_t q : srv->streams) (void)hipStreamDestroy(q);
        (void)hipFree(srv->dev_base);
        (void)hipHostFree(srv->host_base);
        return hip_fail(e, "server events");
    }
    srv->stream_free_at.assign(n_streams, Clock::now());
    srv->stream_waited.assign(n_streams, false);
    dart_server *p = srv.get();
    srv->thr = std::thread(scheduler, p);
    *out = srv.release();
    return DART_OK;
}

extern "C" dart_status dart_submit(dart_server *srv, const dart_stack *s, const dart_view *v,
                                   void *image, uint64_t *ticket) {
    if (!srv || !s || !v || !image || !ticket) return fail(DART_E_INVAL, "NULL argument");
    // (the stack's emissivity plane is packed here, in the caller's thread,
    // when the records changed since it was last packed)
    dart_status st = refresh_jplane(s, nullptr, true);
    if (st != DART_OK) return st;
    RayView rv;
    st = resolve_view(s, v, &rv);
    if (st != DART_OK) return st;
    if (v->out_dtype != DART_F32) return fail(DART_E_INVAL, "the server renders float32 images");
    if (s->vector()) return fail(DART_E_INVAL, "the server does not render vector stacks");
    if (v->flags & DART_ACCUMULATE)
        return fail(DART_E_INVAL, "the server does not accept DART_ACCUMULATE");
    std::unique_ptr<Req> r(new Req());
    r->stack = s;
    r->view = *v;
    r->dest = image;
    r->host_dest = !(v->flags & DART_DEVICE_PTRS);
    r->img_bytes = (size_t)v->width * v->height * 4;
    // any 64-pixel tile shape w x h cuts the image into at most
    // (W/w + 1)(H/h + 1) <= WH/64 + W + H + 1 tiles
    r->desc_bound = sizeof(RayView) + 64 +
                    ((size_t)v->width * v->height / 64 + v->width + v->height + 1) * sizeof(Tile);
    if (r->desc_bound + 256 > srv->desc_cap)
        return fail(DART_E_NOMEM, "a %dx%d image needs more wave descriptors than the server holds",
                    v->width, v->height);
    if (r->img_bytes + (1u << 20) > srv->budget ||
        (r->host_dest && r->img_bytes + (1u << 20) > srv->host_size))
        return fail(DART_E_NOMEM, "a %dx%d image cannot fit the server budget", v->width,
                    v->height);
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->stop) return fail(DART_E_BUSY, "server is shutting down");
    r->ticket = srv->next_ticket++;
    *ticket = r->ticket;
    srv->queue.push_back(r.get());
    srv->reqs.emplace(r->ticket, std::move(r));
    srv->stats.submitted++;
    srv->cv.notify_all();
    return DART_OK;
}

static dart_status collect(dart_server *srv, Req *r, double *flux, uint64_t *steps,
                           double *latency_ms, uint64_t ticket) {
    dart_status st = r->state == 4 ? r->err : DART_OK;
    std::string msg = r->err_msg;
    if (st == DART_OK) {
        if (flux) *flux = r->flux;
        if (steps) *steps = r->steps;
        if (latency_ms) *latency_ms = r->latency_ms;
    }
    srv->reqs.erase(ticket);
    if (st != DART_OK) return fail(st, "request failed: %s", msg.c_str());
    return DART_OK;
}

extern "C" dart_status dart_poll(dart_server *srv, uint64_t ticket, int32_t *done, double *flux,
                                 uint64_t *steps, double *latency_ms) {
    if (!srv || !done) return fail(DART_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> g(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(DART_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Req *r = it->second.get();
    if (r->state < 3) {
        *done = 0;
        return DART_OK;
    }
    *done = 1;
    return collect(srv, r, flux, steps, latency_ms, ticket);
}

extern "C" dart_status dart_wait(dart_server *srv, uint64_t ticket, double *flux, uint64_t *steps,
                                 double *latency_ms) {
    if (!srv) return fail(DART_E_INVAL, "NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(DART_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Req *r = it->second.get();
    srv->cv.wait(lk, [r] { return r->state >= 3; });
    return collect(srv, r, flux, steps, latency_ms, ticket);
}

extern "C" dart_status dart_server_get_stats(dart_server *srv, dart_server_stats *st) {
    if (!srv || !st) return fail(DART_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> g(srv->mu);
    *st = srv->stats;
    st->bytes_in_use = srv->dev_arena.used();
    return DART_OK;
}

extern "C" dart_status dart_server_destroy(dart_server *srv) {
    if (!srv) return fail(DART_E_INVAL, "NULL server");
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
        srv->cv.notify_all();
    }
    srv->thr.join();
    for (hipStream_t s : srv->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (auto *v : {&srv->ev_begin, &srv->ev_kbegin, &srv->ev_kend, &srv->ev_end})
        for (hipEvent_t q : *v) (void)hipEventDestroy(q);
    for (void *q : srv->desc_dev) (void)hipFree(q);
    for (void *q : srv->desc_host) (void)hipHostFree(q);
    (void)hipFree(srv->dev_base);
    (void)hipHostFree(srv->host_base);
    delete srv;
    return DART_OK;
}

extern "C" dart_status dart_server_get_timeline(dart_server *srv, dart_server_timeline *tl) {
    if (!srv || !tl) return fail(DART_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> g(srv->mu);
    *tl = srv->tl;
    return DART_OK;
}
