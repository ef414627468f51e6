// dart_noalloc.hip -- the batched render without any device allocation.
//
// dart_render_batch keeps its accumulators, queue heads and view / tile
// descriptors in a per-stream workspace that grows with hipMalloc.  Callers
// that cannot allocate (code under stream capture, tight serving loops,
// hosts that forbid it) use dart_render_batch_noalloc instead: the same plan
// and the same kernels, with that scratch in one fixed-size array of device
// memory that lives as long as the process.
//
// Host code never passes the array's name to a kernel or a copy: that name is
// a host-side stand-in.  Its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and kept in a table; every
// launch and copy uses the kept address.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/dart.h"
#include "dart_internal.h"
#include "dart_runtime.h"

using namespace dart;

#define HIP_TRY_STATUS(call, what)                     \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

namespace {

// Accumulators (flux and cell-steps per view, queue heads per launch group),
// then the view descriptors, then the tile descriptors.  Each GPU holds its
// own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[DART_NOALLOC_SCRATCH_BYTES];

struct DeviceScratch {
    unsigned char *ptr = nullptr;  // device address of `scratch` on this device
    std::mutex mu;                 // one host-side enqueue at a time per device
};

std::mutex g_table_mu;
std::map<int, std::unique_ptr<DeviceScratch>> g_table;

dart_status scratch_of(int device, DeviceScratch **out) {
    std::lock_guard<std::mutex> g(g_table_mu);
    std::unique_ptr<DeviceScratch> &slot = g_table[device];
    if (!slot) {
        void *p = nullptr;
        // (called with `device` current: the address of this device's copy)
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_table.erase(device);
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                            "hipGetSymbolAddress(scratch)");
        }
        slot.reset(new DeviceScratch());
        slot->ptr = (unsigned char *)p;
    }
    *out = slot.get();
    return DART_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" dart_status dart_render_batch_noalloc(const dart_stack *const *stacks,
                                                 const dart_view *views, int32_t n,
                                                 void *const *images, double *flux_out,
                                                 uint64_t *steps_out, void *hip_stream) {
    if (n < 0 || (n > 0 && (!stacks || !views || !images)))
        return fail(DART_E_INVAL, "bad batch arguments");
    if (n == 0) return DART_OK;
    for (int32_t i = 0; i < n; i++) {
        if (!stacks[i]) return fail(DART_E_INVAL, "stacks[%d] is NULL", i);
        if (!(views[i].flags & DART_DEVICE_PTRS))
            return fail(DART_E_INVAL, "view %d: images must be device memory (DART_DEVICE_PTRS)", i);
        if (views[i].flags & DART_KERNEL_PLAIN)
            return fail(DART_E_INVAL, "view %d: DART_KERNEL_PLAIN is not available here", i);
    }
    {
        std::vector<std::pair<const void *, int32_t>> dst;
        for (int32_t i = 0; i < n; i++) dst.emplace_back(images[i], i);
        std::sort(dst.begin(), dst.end());
        for (size_t k = 1; k < dst.size(); k++)
            if (dst[k].first == dst[k - 1].first)
                return fail(DART_E_INVAL, "views %d and %d write the same image", dst[k - 1].second,
                            dst[k].second);
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    dart_status st = DART_OK;
    for (int32_t i = 0; i < n; i++) {
        st = refresh_vector(stacks[i], stream);
        // (an emissivity plane is repacked in place, never allocated here)
        if (st == DART_OK) st = refresh_jplane(stacks[i], stream, false);
        if (st != DART_OK) return st;
    }
    const dart_tuning tun = tuning_for(stacks[0]);
    std::vector<Group> groups;
    st = plan_batch(stacks, views, n, images, tun, groups);
    if (st != DART_OK) return st;
    size_t nv = 0, nt = 0;
    assign_offsets(groups, &nv, &nt);
    const size_t acc_words = 2 * (size_t)n + 4 * groups.size();
    const size_t desc_off = align256(acc_words * sizeof(unsigned long long));
    const size_t desc_bytes = nv * sizeof(RayView) + nt * sizeof(Tile);
    if (desc_off + desc_bytes > (size_t)DART_NOALLOC_SCRATCH_BYTES)
        return fail(DART_E_INVAL,
                    "%d views in %zu tiles need %zu bytes of scratch; the fixed scratch holds %zu "
                    "(use dart_render_batch, or fewer or smaller views per call)",
                    n, nt, desc_off + desc_bytes, (size_t)DART_NOALLOC_SCRATCH_BYTES);
    int device = 0;
    HIP_TRY_STATUS(hipGetDevice(&device), "hipGetDevice");
    DeviceScratch *sc = nullptr;
    st = scratch_of(device, &sc);
    if (st != DART_OK) return st;
    std::lock_guard<std::mutex> g(sc->mu);
    std::vector<unsigned char> host(desc_bytes);
    pack_descriptors(groups, nv, host.data());
    unsigned long long *acc = (unsigned long long *)sc->ptr;
    const RayView *dviews = (const RayView *)(sc->ptr + desc_off);
    const Tile *dtiles = (const Tile *)(sc->ptr + desc_off + nv * sizeof(RayView));
    // Stream-ordered after earlier work that reads the scratch; the wait makes
    // sure the pageable host copy has been consumed before it goes out of scope.
    HIP_TRY_STATUS(hipMemcpyAsync(sc->ptr + desc_off, host.data(), desc_bytes,
                                  hipMemcpyHostToDevice, stream),
                   "H2D descriptors");
    HIP_TRY_STATUS(hipStreamSynchronize(stream), "sync");
    HIP_TRY_STATUS(enqueue_plan(groups, n, acc, dviews, dtiles, tun, device, stream),
                   "batch kernels");
    for (int32_t i = 0; i < n; i++) note_use(stacks[i], stream);
    if (flux_out || steps_out) {
        std::vector<unsigned long long> h(2 * (size_t)n);
        HIP_TRY_STATUS(hipMemcpyAsync(h.data(), acc, h.size() * sizeof(unsigned long long),
                                      hipMemcpyDeviceToHost, stream),
                       "D2H accumulators");
        HIP_TRY_STATUS(hipStreamSynchronize(stream), "sync");
        for (int32_t i = 0; i < n; i++) {
            if (flux_out) memcpy(&flux_out[i], &h[i], sizeof(double));
            if (steps_out) steps_out[i] = h[n + i];
        }
    }
    return DART_OK;
}
