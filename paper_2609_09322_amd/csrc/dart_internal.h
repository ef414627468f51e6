// dart_internal.h -- descriptors shared by the HIP kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dart {

enum Store : int { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };

enum : uint32_t {
    F_NO_LOOKBACK = 0x1u,
    F_NO_BEAMING = 0x2u,
    F_NEAREST = 0x4u,
    F_NO_KAHAN = 0x8u,
    F_F64_DDA = 0x10u,
    F_DEVICE_PTRS = 0x20u,
    F_ACCUMULATE = 0x80u,
    F_EXACT = 0x100u,
    F_PLANE32 = 0x1000u,  // the view's emissivity plane is read through 32-bit offsets
};

// Resident stack as the kernels see it.  Records (j, bx, by, bz) are stored
// epoch-major; inside an epoch the cells are grouped in bricks of
// 2^lb[0] x 2^lb[1] x 2^lb[2] cells (x fastest inside a brick, bricks x-fastest).
struct StackDev {
    const void *data;       // resident records
    // Emissivity plane: the j field of every record packed alone, at the
    // record's own index, in the storage type (FP32, or the 16-bit bits); its
    // sign bit is set when the record must be read whole (velocity bits not
    // all zero, or j itself negative or -0).  Null: read whole records.
    const void *jplane;
    const double *times;    // [M] epoch times (device)
    const double *inv_dt;   // [M] 1 / (t_{m+1} - t_m), 0 for the last epoch (device)
    int64_t epoch_stride;   // records from one epoch to the next (padded to whole bricks;
                            // negative for a streamed interval whose later epoch sits
                            // in an earlier ring slot)
    int32_t n[3];           // cells per axis
    int32_t nb[3];          // bricks per axis
    int32_t lb[3];          // log2 of the brick shape
    int32_t n_epochs;
    int32_t store;          // Store
    double cell[3];
};

// One sub-domain of a labelled stack: its grid and the camera centre in the
// grid's own coordinates (the domain centre minus the grid's origin).
struct Block {
    StackDev st;
    double centre[3];
};

// One view, resolved on the host in FP64.
struct RayView {
    double shat[3], eu[3], ev[3], centre[3];
    double inv_shat[3];     // 1 / s_hat per axis (0 where s_hat has a zero component)
    float shat_hi[3];       // s_hat rounded to FP32, and the rest: s_hat = hi + lo to
    float shat_lo[3];       // ~2^-48, for the FP32 Doppler of 16-bit stacks
    double ps;              // pixel scale
    double t_obs;
    double s_lo, s_hi;      // temporal window expressed in s: [t_obs - t_{M-1}, t_obs - t_0]
                            // (a half-open end is the next representable value inside)
    double p;               // 2 + alpha
    uint32_t flags;
    int32_t width, height;
    int32_t fixed_m;        // NO_LOOKBACK: epoch bracket at t_obs (-1: t_obs outside coverage)
    double fixed_w;         // NO_LOOKBACK: weight of epoch fixed_m + 1
    float fixed_wf;         // the same rounded to FP32 (read as such by FP32 walks)
    double sync_gap;        // batched kernel: depth-synchronous horizon (length), 0 = off
    void *image;            // [height][width] float or double (device)
    int32_t out_f64;
    int32_t acc_index;      // slot in the flux / step accumulators
    int32_t tile_w_log2;    // batched kernel: tile width 1 << tile_w_log2, height 64 >> it
    StackDev st;            // the stack (a labelled stack: its first sub-domain)
    const Block *blocks;    // labelled stack: its sub-domains (device), else null
    int32_t n_blocks;       // 0 for a plain stack
    // vector stack: n_chan components (2..4) with the same grid and layout;
    // st is component 0 (its velocity sets D for all), chan_data[c - 1] the
    // emissivity of component c packed one value per record index.  Images
    // are [n_chan][height][width].  n_chan = 1 otherwise.
    int32_t n_chan;
    const void *chan_data[3];
};

struct Tile {
    uint32_t view;
    uint16_t tx, ty;
};

constexpr int MAX_QUEUES = 8;

// Launch parameters of the persistent batched kernel.
struct BatchLaunch {
    const RayView *views;
    const Tile *tiles;
    uint32_t n_tiles;
    uint32_t *head;         // tile queue heads, one per XCD queue
    uint32_t n_queues;      // at most MAX_QUEUES
    uint32_t q_begin[9];    // queue q holds tiles [q_begin[q], q_begin[q + 1])
    double *flux_acc;
    unsigned long long *step_acc;
};

// Host-side launchers (dart_kernels.hip).
hipError_t launch_plain(const RayView &v, double *flux_acc, unsigned long long *step_acc,
                        hipStream_t s);
// Kernel variant bits: 1 depth-synchronous wavefronts, 2 the launch's views are
// labelled stacks (block loop), 4 exact temporal integration, 8 eight cells per
// batch (else four), 16 vector stacks (only alone: no other bit but 8), 32 the
// views' stacks have an emissivity plane (not with 2 or 16).
enum : int {
    KV_SYNC = 1, KV_LABELLED = 2, KV_EXACT = 4, KV_K8 = 8, KV_VEC = 16, KV_JP = 32,
    KV_JP32 = 64,  // with KV_JP: the plane through 32-bit byte offsets (F_PLANE32)
};
hipError_t launch_batch(int store, bool f64_dda, int variant, const BatchLaunch &bl,
                        int grid_blocks, hipStream_t s);
// Marks the samples of positive weight of a render of v (moving_only: only
// those whose record must be read whole, see StackDev::jplane) in a bitmap of
// records (line_log2 < 0) or of lines of 2^line_log2 elements of the record
// index space.
hipError_t launch_mark(const RayView &v, uint32_t *bitmap, int line_log2, bool moving_only,
                       hipStream_t s);
hipError_t launch_popcount(const uint32_t *bitmap, uint64_t words, unsigned long long *out,
                           hipStream_t s);
hipError_t launch_convert(int src_f64, int store, const void *j, const void *beta, int32_t m0,
                          int32_t count, const StackDev &st, void *data,
                          unsigned long long *err, hipStream_t s);
hipError_t launch_rebrick(int store, const StackDev &from, const StackDev &to, void *dst,
                          hipStream_t s);
// One epoch of a stack back in the caller's layout, widened to FP64 (FP64
// stacks) or FP32 (the others): j [ncell], beta [ncell][3] (device).
hipError_t launch_read_epoch(const StackDev &st, int32_t m, void *j, void *beta, hipStream_t s);
// Emissivity fields of n resident records into a packed array (vector stacks).
hipError_t launch_pack_j(int store, const void *records, void *out, uint64_t n, hipStream_t s);
// The emissivity plane of n records (StackDev::jplane); FP32 and 16-bit storage.
hipError_t launch_pack_jplane(int store, const void *records, void *out, uint64_t n,
                              hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long value,
                           hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t s);
// Writes 0 to every pixel (and channel) of n tiles of the given views.
hipError_t launch_clear_tiles(const RayView *views, const Tile *tiles, uint32_t n, hipStream_t s);

}  // namespace dart
