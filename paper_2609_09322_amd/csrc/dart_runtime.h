// dart_runtime.h -- host-side objects shared by the runtime and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/dart.h"
#include "dart_internal.h"

namespace dart {
// Process-wide, never repeated: a stack created where a freed one lived, or
// re-laid, never matches a cached plan of another.
uint64_t next_generation();
}  // namespace dart

struct dart_stack {
    dart::StackDev dev{};
    dart_dtype storage = DART_F32;
    std::vector<double> times;
    std::vector<char> filled;
    uint64_t bytes = 0;
    uint64_t generation = dart::next_generation();  // renewed whenever the resident layout
                                                    // or data change
    int device = 0;
    dart_tuning tuning{32, 2, 8, 0, 1, 0, 4};
    bool placed = false;               // set by dart_stack_set_placement
    double origin[3] = {0, 0, 0}, centre[3] = {0, 0, 0};
    bool tuned = false;
    std::mutex mu;
    std::vector<std::pair<hipStream_t, hipEvent_t>> uses;  // last render per stream
    std::atomic<int> pinned{0};                            // server requests holding the stack
    // labelled stack: its sub-domains (owned by the caller) and their device
    // descriptors; a stack that is a sub-domain counts the labelled stacks
    // holding it in `refs`
    std::vector<dart_stack *> parts;
    dart::Block *dev_blocks = nullptr;
    std::atomic<int> refs{0};
    bool labelled() const { return !parts.empty(); }
    // vector stack: its components (owned by the caller, counted in refs);
    // dev is component 0's
    std::vector<dart_stack *> comps;
    void *packed = nullptr;             // emissivity of components 1.., packed (device)
    std::vector<uint64_t> packed_gen;   // the components' generations when packed
    // emissivity plane (StackDev::jplane) of a plain FP32 / 16-bit stack: built
    // at the first render after the records change, when memory allows
    void *jplane = nullptr;
    uint64_t jplane_bytes = 0;
    // the generation it was packed from (0: never); read without the lock by
    // planners on other threads, so published after the pack has completed
    std::atomic<uint64_t> jplane_gen{0};
    uint64_t jplane_no_room = 0;        // a generation for which hipMalloc failed
    bool vector() const { return !comps.empty(); }
    int channels() const { return comps.empty() ? 1 : (int)comps.size(); }
};

namespace dart {

dart_status fail(dart_status st, const char *fmt, ...);
dart_status hip_fail(hipError_t e, const char *what);
int device_cus(int dev);
uint32_t record_bytes(int store);
dart_status resolve_view(const dart_stack *s, const dart_view *v, RayView *rv);
// Packs the stack's emissivity plane when it is missing or stale (allocating it
// only if may_alloc); a stack without one is rendered from whole records.
dart_status refresh_jplane(const dart_stack *s, hipStream_t stream, bool may_alloc);
bool jplane_ready(const dart_stack *s);
void note_use(const dart_stack *s, hipStream_t stream);
bool stack_busy(const dart_stack *s);
dart_tuning tuning_for(const dart_stack *s);
// Vector stacks: repacks the components' emissivity on `stream` if any
// component was refilled since it was packed (after renders that read the
// packed copy have finished).  No-op for other stacks.
dart_status refresh_vector(const dart_stack *s, hipStream_t stream);

// One launch group of a batch: views of one storage type and ray precision.
struct Group {
    int store = 0;
    bool f64 = false;
    bool labelled = false;  // views of labelled stacks (kernels with the block loop)
    bool vec = false;       // views of vector stacks
    bool exact = false;     // views with exact temporal integration
    bool jp = false;        // views that read their stacks' emissivity planes
    bool jp32 = false;      // ... through 32-bit offsets (planes of at most 4 GiB)
    std::vector<RayView> views;
    // queued tiles [0, q_begin[n_queues]), then n_clear tiles whose rays all
    // miss the grid (their pixels are set to 0 by a fill kernel)
    std::vector<Tile> tiles;
    std::vector<Tile> clear;  // (planner scratch)
    uint32_t n_clear = 0;
    size_t view_off = 0, tile_off = 0;  // offsets in the uploaded descriptor arrays
    uint32_t n_queues = 8;
    uint32_t q_begin[MAX_QUEUES + 1] = {};  // chunk bounds in `tiles`
};

dart_status plan_batch(const dart_stack *const *stacks, const dart_view *views, int32_t n,
                       void *const *images, const dart_tuning &tun, std::vector<Group> &groups);

// Per-(device, stream) scratch: accumulators, descriptor arrays, image staging,
// pinned upload staging and the last captured batch graph.
struct Workspace {
    hipStream_t stream = nullptr;
    int device = 0;
    std::mutex mu;
    unsigned long long *acc = nullptr;  // flux[n] (as double bits), steps[n], queue heads
    size_t acc_cap = 0;
    RayView *views = nullptr;
    size_t views_cap = 0;
    Tile *tiles = nullptr;
    size_t tiles_cap = 0;
    unsigned long long *img = nullptr;  // staging for host-destined images
    size_t img_cap = 0;
    void *stage = nullptr;              // pinned host staging for descriptor uploads
    size_t stage_cap = 0;
    hipEvent_t stage_done{};
    bool stage_ready = false;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uint8_t> graph_key;
    // the last batch plan (descriptors already on the device), replayed when
    // the next call has the same key
    std::vector<Group> plan_groups;
    std::vector<uint8_t> plan_key;
    bool plan_ready = false;
};

Workspace *get_workspace(hipStream_t stream);
hipError_t ws_reserve(Workspace *ws, size_t n_views, size_t n_tiles, size_t img_u64,
                      size_t n_queue_slots);
hipError_t enqueue_plan(const std::vector<Group> &groups, int32_t n, unsigned long long *acc,
                        const RayView *dviews, const Tile *dtiles, const dart_tuning &tun,
                        int device, hipStream_t stream);
void assign_offsets(std::vector<Group> &groups, size_t *n_views, size_t *n_tiles);
void pack_descriptors(const std::vector<Group> &groups, size_t n_views, void *dst);

}  // namespace dart
