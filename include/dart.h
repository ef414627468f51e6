/*
 * dart.h -- C ABI of the MI355X lookback ray-marching library (libdart.so).
 *
 * The library evaluates, for every pixel of an orthographic image, the
 * optically thin intensity sum of the paper's Eq. 19 (Sec. 2.5):
 *
 *     I = sum_n sum_m W_{n,m} D_{n,m}^p j_{n,m} ds_n ,      p = 2 + alpha
 *
 * over the cells n a pixel ray crosses (3D DDA, Sec. 2.4, Eq. 11), with the
 * epoch pair m chosen at the cell's retarded time tbar_n = t_obs - s_n / c
 * (Eq. 2, c = 1) and weighted linearly in time (Eqs. 6-7), and with the
 * Doppler factor D = sqrt(1 - beta^2) / (1 + beta . s_hat) of Eq. 14.  Only
 * cells whose retarded time lies inside the epoch coverage [t_0, t_{M-1}]
 * are visited (the fast-forward of Sec. 5.1).  The output is at the reference
 * frequency, so the prefactor (nu / nu0')^alpha of Eq. 19 is 1.
 *
 * Conventions shared by every call:
 *  - alpha is the positive index of S ~ nu^-alpha; the per-cell exponent is
 *    p = 2 + alpha (the paper writes 2 - alpha with alpha = -0.6 by default).
 *  - Lengths are in the caller's unit; times are in that unit / c.
 *  - The grid spans [0, nx dx) x [0, ny dy) x [0, nz dz); cells are half-open.
 *  - theta is the polar angle (degrees) of the direction toward the observer
 *    n_hat = (sin th cos ph, sin th sin ph, cos th) from +z, phi its azimuth
 *    from +x; rays travel along s_hat = -n_hat.  Image axes:
 *    e_u = (-sin ph, cos ph, 0) (columns), e_v = (-cos th cos ph,
 *    -cos th sin ph, sin th) (rows).  Pixel (i, j) has its ray through
 *    C + (i + 1/2 - W/2) ps e_u + (j + 1/2 - H/2) ps e_v, C the grid centre;
 *    row 0 is the bottom row.  Images are row-major [height][width].
 *  - s is measured along the ray from the plane through C normal to s_hat;
 *    the retarded time of a cell is t_obs - s_mid with s_mid its chord
 *    midpoint.  Cells with s_mid outside the epoch coverage contribute 0.
 *  - Flux = sum of pixel intensities x ps^2 (Eq. 22 up to 1/L^2).
 *  - One cell-step = one (ray, cell) pair with a positive chord inside the
 *    temporal window.
 *
 * Errors: every call returns a dart_status; no exception crosses the ABI.  On
 * error the outputs are left untouched (and *out = NULL for constructors) and
 * dart_last_error() returns a thread-local message.
 *
 * Threading: stacks are read-only after loading and may be rendered from
 * several host threads and streams at once.  The server object is
 * thread-safe.  Every call uses the HIP device that is current on the calling
 * thread; a stack must be rendered on the device it was loaded on.
 */
#ifndef DART_H
#define DART_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DART_OK = 0,
    DART_E_INVAL = -1,    /* malformed argument */
    DART_E_RANGE = -2,    /* |beta| >= 1 or a non-finite value in the fields */
    DART_E_NOMEM = -3,    /* device or host allocation failed / over budget */
    DART_E_DEVICE = -4,   /* a HIP runtime call failed */
    DART_E_BUSY = -5,     /* object still in use (renders in flight, full queue) */
    DART_E_INTERNAL = -6
} dart_status;

typedef enum { DART_F64 = 0, DART_F32 = 1, DART_F16 = 2, DART_BF16 = 3 } dart_dtype;

/* flags (dart_view.flags, and the load flags where noted) */
#define DART_NO_LOOKBACK 0x1u   /* routine B: tbar = t_obs for every cell (Eq. 3, Eq. 10) */
#define DART_NO_BEAMING 0x2u    /* routine A: D = 1 */
#define DART_NEAREST_EPOCH 0x4u /* weight 1 on the epoch closest to tbar (ties: earlier) */
#define DART_NO_KAHAN 0x8u      /* plain (uncompensated) FP32 accumulation (such views read
                                   whole records, not the emissivity plane) */
#define DART_FORCE_F64_DDA 0x10u /* FP64 ray parameters (DDA crossings, retarded times) for
                                    16-bit stacks too; FP64 and FP32 stacks always use them,
                                    16-bit stacks when a ray may cross more than 4096 cells */
#define DART_DEVICE_PTRS 0x20u  /* load: field pointers are device pointers;
                                   view: the image pointer is a device pointer */
#define DART_KERNEL_PLAIN 0x40u /* dart_render_batch: force the one-launch-per-image kernel */
#define DART_EXACT_TIME 0x100u  /* view: cut every chord where the retarded time passes an
                                   epoch time (and at the window ends) and weight each piece
                                   at its own midpoint: the exact integral of the field that is
                                   constant in each cell and linear in time between epochs,
                                   instead of Eq. 19's one sample per cell (Eqs. 6-7, Sec. 6.1).
                                   A cell still counts as one cell-step.  Lookback with linear
                                   interpolation only (not with DART_NEAREST_EPOCH); not
                                   accepted by dart_streamer_render */
#define DART_RECORDS_ONLY 0x200u /* view: read the whole record of every cell instead of the
                                   stack's emissivity plane (see dart_stack_get_info); the
                                   image is the same bit for bit: for comparisons */
#define DART_PLANE_ADDR64 0x400u /* view: address the emissivity plane through 64-bit
                                   pointers, as planes over 4 GiB always are, instead of the
                                   32-bit offsets used for smaller ones; the image is the same
                                   bit for bit: for comparisons */
#define DART_ACCUMULATE 0x80u   /* view: add the render to the values already in the image
                                   instead of overwriting them, so partial renders of
                                   sub-domains sum into one buffer (Sec. 4, Fig. 5; Sec. 6.2).
                                   Device images only (DART_DEVICE_PTRS); calls that add into
                                   one image run in stream order; not accepted by dart_submit */

typedef struct dart_stack dart_stack;
typedef struct dart_server dart_server;

/* ---------------------------------------------------------------- stacks --
 * dart_load_epochs: copy M epochs of emissivity j'_{nu0'} and velocity beta
 * (the method's inputs, Sec. 2.5) into a resident device stack.
 *   dims[3]      nx, ny, nz > 0 (cells)
 *   cell[3]      dx, dy, dz > 0 and finite
 *   n_epochs     M >= 1;  epoch_times[M] finite and strictly increasing
 *   src_dtype    DART_F64 or DART_F32: element type of the two arrays
 *   storage      resident element type; DART_F16 / DART_BF16 round to nearest even
 *   emissivity   [M][nz][ny][nx], C order (x fastest)
 *   velocity     [M][nz][ny][nx][3] (beta_x, beta_y, beta_z)
 *   flags        DART_DEVICE_PTRS: arrays are device memory, converted in
 *                place on hip_stream.  Either way the call returns after the
 *                conversion and its validation have finished, so the caller may
 *                release the arrays on return.
 *   hip_stream   hipStream_t or NULL (default stream)
 * Every value must be finite and |beta| < 1 before and after rounding to the
 * storage type, else DART_E_RANGE names the first bad element.
 * The stack owns its device memory until dart_free_epochs.
 */
dart_status dart_load_epochs(const int32_t dims[3], const double cell[3], int32_t n_epochs,
                             const double *epoch_times, dart_dtype src_dtype, dart_dtype storage,
                             const void *emissivity, const void *velocity, uint32_t flags,
                             void *hip_stream, dart_stack **out);

/* Two-phase loading for stacks that cannot be staged whole: create an empty
 * stack, then fill epochs [m0, m0 + count) from arrays laid out as
 * [count][nz][ny][nx] and [count][nz][ny][nx][3].  A stack can be rendered once
 * every epoch has been filled (DART_E_INVAL otherwise). */
dart_status dart_stack_create(const int32_t dims[3], const double cell[3], int32_t n_epochs,
                              const double *epoch_times, dart_dtype storage, uint32_t flags,
                              dart_stack **out);
dart_status dart_stack_set_epochs(dart_stack *s, int32_t m0, int32_t count, dart_dtype src_dtype,
                                  const void *emissivity, const void *velocity, uint32_t flags,
                                  void *hip_stream);

/* Releases the stack; DART_E_BUSY (and nothing freed) while a render that
 * reads it is still running on the device. */
dart_status dart_free_epochs(dart_stack *s);

/* Emissivity plane.  A plain stack with FP32, FP16 or BF16 records also keeps
 * its emissivity alone, one value per record at the record's own index (a
 * quarter of the record bytes), packed on the device by the first render
 * after its records change (not inside a stream capture, and by
 * dart_render_batch_noalloc only into a plane already allocated).  The value's
 * sign bit marks records that must be read whole: any velocity bit set, or a
 * negative (or -0) emissivity.  A render reads the plane, and whole records
 * only of the marked elements; a jet's volume at rest is then read at a
 * quarter of the bytes.  Images, flux
 * and cell-steps are bit for bit those of whole-record reads
 * (DART_RECORDS_ONLY).  Without room for the plane (hipMalloc fails) renders
 * read whole records, as do views with DART_NO_KAHAN.  Planes of at most 4 GiB
 * are read through 32-bit offsets, larger ones through 64-bit addresses
 * (DART_PLANE_ADDR64 asks for those on any plane).  FP64, labelled, vector and
 * streamed stacks have none. */
typedef struct {
    int32_t dims[3];
    int32_t n_epochs;
    dart_dtype storage;
    int32_t brick[3];      /* resident brick shape (cells) */
    uint64_t device_bytes; /* resident bytes: records, and the emissivity plane once packed */
} dart_stack_info;
dart_status dart_stack_get_info(const dart_stack *s, dart_stack_info *info);

/* Copies epoch m of a plain stack back in the caller's layout of
 * dart_load_epochs (emissivity [nz][ny][nx], velocity [nz][ny][nx][3]): the
 * values the renders read (the inputs j' and beta of Sec. 2.5 after rounding
 * to the storage type), each widened exactly, to FP64 for FP64 stacks and to
 * FP32 for the others.  Inspection only: the storage error of a 16-bit stack
 * is a render of these values against a render of the source fields.
 *   flags   DART_DEVICE_PTRS: the two arrays are device memory (stream-ordered,
 *           the call returns once the copy is enqueued); otherwise host memory
 *           (staged through a temporary device buffer, the call returns after
 *           the copy)
 * DART_E_INVAL for labelled or vector stacks, m outside [0, M) or an epoch
 * never filled; the arrays are untouched on error. */
dart_status dart_stack_read_epoch(const dart_stack *s, int32_t m, void *emissivity,
                                  void *velocity, uint32_t flags, void *hip_stream);

/* Places the stack inside a larger domain, for renders of sub-domains whose
 * partial images add up to the render of the whole (optically thin emission
 * is additive along a ray; the paper's partial renders of sub-regions,
 * Sec. 6.2).  origin[3]: position of the grid's lower corner; centre[3]: the
 * point every camera is centred on and through which the s = 0 plane of the
 * retarded time passes (for a slab: the centre of the whole domain).
 * Defaults: origin 0, centre = the grid's own centre.  Finite values only. */
dart_status dart_stack_set_placement(dart_stack *s, const double origin[3], const double centre[3]);

/* Labelled mode (Sec. 4; partial renders of sub-regions, Sec. 6.2): one stack
 * made of non-overlapping sub-domains, each a stack with its own dims and cell
 * size, placed in the domain with dart_stack_set_placement (all with the same
 * domain centre), and all with the same storage type, device and epoch times.
 * A render of it (dart_render, dart_render_batch, dart_submit) marches every
 * ray through each sub-domain in order and sums them in one pass.  The
 * sub-domains stay owned by the caller; while a labelled stack holds them they
 * cannot be freed, re-laid or re-placed (DART_E_BUSY), but their epochs may be
 * refilled with dart_stack_set_epochs.  Overlapping sub-domains would be
 * counted twice: the caller keeps them disjoint (the leaf blocks of a
 * refinement hierarchy).  Free it with dart_free_epochs.  dart_stack_get_info
 * reports the first sub-domain's dims and brick and the bytes of all of them;
 * dart_stack_rebrick, dart_stack_set_epochs, dart_stack_set_placement,
 * dart_count_samples, dart_count_lines and dart_autotune with rebrick != 0
 * return DART_E_INVAL for it.  n_blocks in [1, 65536]; on error *out = NULL. */
dart_status dart_labelled_create(dart_stack *const *blocks, int32_t n_blocks, dart_stack **out);

/* Vector sums (the line integral of Eq. 1 for a vector-valued emissivity, e.g.
 * the Stokes components a polarised emitter would carry; the paper names
 * polarisation as future work, Sec. 7): one stack made of n in [2, 4]
 * component stacks with the same dims, cell size, brick shape, layout,
 * placement, storage type, device and epoch times.  The emissivity of
 * components 1.. is also kept packed (one value per cell and epoch, a quarter
 * of the record bytes each), refreshed by the next render after a component's
 * epochs are refilled; dart_stack_get_info counts it.  A render marches each ray
 * once: the chords, epoch weights (Eqs. 6-7) and the Doppler factor D^p of
 * component 0's velocity (Eq. 14) are applied to the emissivity of every
 * component, each summed on its own as in Eq. 19.  The other components'
 * velocities are not read (the caller gives them the same field; a rotation
 * of the polarisation plane by aberration is not modelled).  Component c of
 * pixel (i, j) equals the scalar render of (j_c, component 0's velocity).
 * Images are [n][height][width] at the view's image pointer (host or device,
 * as for one scalar image); flux and cell steps refer to component 0.
 * dart_render, dart_render_batch (vector and scalar views mix freely) accept
 * it; dart_submit, DART_EXACT_TIME, dart_labelled_create, dart_stack_rebrick,
 * dart_stack_set_epochs, dart_stack_set_placement and dart_autotune with
 * rebrick != 0 return DART_E_INVAL for it; batched renders of it march without
 * depth sync.  The components stay owned by the caller and cannot be freed,
 * re-laid or re-placed while the vector stack holds them (DART_E_BUSY); their
 * epochs may be refilled.  Free it with dart_free_epochs.  On error *out = NULL. */
dart_status dart_vector_create(dart_stack *const *components, int32_t n, dart_stack **out);

/* Re-lays the resident stack with a new brick shape (powers of two, each
 * 1..16, at most 4096 cells per brick); the current shape returns at once.
 * Uses a second copy of the stack when device memory allows, else (when the
 * epoch size does not change) re-lays one epoch at a time in place through a
 * one-epoch buffer.  If that in-place pass fails part-way the stack reports
 * its epochs as unfilled and renders on it return DART_E_INVAL until they are
 * loaded again.  Synchronises the stream. */
dart_status dart_stack_rebrick(dart_stack *s, const int32_t brick[3], void *hip_stream);

/* ---------------------------------------------------------------- render --
 * One observation (N cameras per call in the batch form).
 *   theta_deg, phi_deg  orientation (finite)
 *   width, height       image size in pixels (> 0)
 *   pixel_scale         length per pixel (> 0, finite)
 *   t_obs               observer time
 *   alpha               spectral index, p = 2 + alpha (finite)
 *   flags               DART_NO_LOOKBACK | DART_NO_BEAMING | DART_NEAREST_EPOCH |
 *                       DART_NO_KAHAN | DART_FORCE_F64_DDA | DART_DEVICE_PTRS
 *   out_dtype           DART_F32, or DART_F64 (FP64 stacks only)
 */
typedef struct {
    double theta_deg, phi_deg;
    int32_t width, height;
    double pixel_scale;
    double t_obs;
    double alpha;
    uint32_t flags;
    dart_dtype out_dtype;
} dart_view;

/* Plain kernel: one launch, one thread per pixel.
 *   image      [height][width] of out_dtype; host memory unless the view has
 *              DART_DEVICE_PTRS (then stream-ordered)
 *   flux_out   nullable host pointer: sum I ps^2
 *   steps_out  nullable host pointer: cell-steps of the image
 * With a host image or a non-NULL flux_out/steps_out the call waits for the
 * stream; otherwise it returns once the work is enqueued. */
dart_status dart_render(const dart_stack *s, const dart_view *v, void *image, double *flux_out,
                        uint64_t *steps_out, void *hip_stream);

/* Batched form: n (stack, view, image) triples rendered by one persistent,
 * tile-queue launch per (storage type, precision) group.  Stacks may differ.
 * images[i] follows views[i].flags like dart_render; flux_out[n] and
 * steps_out[n] are nullable host arrays.  A call whose arguments equal those of
 * the previous call on the same stream replays a captured hipGraph. */
dart_status dart_render_batch(const dart_stack *const *stacks, const dart_view *views, int32_t n,
                              void *const *images, double *flux_out, uint64_t *steps_out,
                              void *hip_stream);

/* The batched render for callers that cannot allocate device memory: code
 * under stream capture, tight serving loops, hosts that forbid hipMalloc.
 * Same arguments, plan, kernels and results as dart_render_batch (pixels and
 * cell-steps identical; flux equal up to the order of the FP64 atomic
 * additions that sum it), but its accumulators and view / tile
 * descriptors live in a fixed array of DART_NOALLOC_SCRATCH_BYTES of device
 * memory that the library holds on each GPU it runs on until the process
 * ends.  The call makes no hipMalloc, hipFree or pinned-host allocation.
 *   images     device memory only: every view needs DART_DEVICE_PTRS
 *              (DART_KERNEL_PLAIN is refused)
 *   flux_out, steps_out  nullable host arrays [n]; when given, the call waits
 *              for the stream
 * The call uploads the descriptors with a pageable copy and waits for the
 * stream once before launching, so it returns after earlier work on the
 * stream has finished; without flux_out / steps_out it returns once the
 * render is enqueued.  A batch whose accumulators and descriptors (2n + 4
 * words per launch group, then 384 bytes per view and 8 per 64-pixel
 * tile) exceed the scratch returns DART_E_INVAL before anything is enqueued.
 * Every call on one GPU shares that GPU's scratch and overwrites what the last
 * call left there: calls on one stream are ordered, but calls that overlap on
 * one GPU from different streams or host threads race. */
#define DART_NOALLOC_SCRATCH_BYTES (16u << 20)
dart_status dart_render_batch_noalloc(const dart_stack *const *stacks, const dart_view *views,
                                      int32_t n, void *const *images, double *flux_out,
                                      uint64_t *steps_out, void *hip_stream);

/* ------------------------------------------------------------- streaming --
 * Out-of-core rendering (Sec. 4, Fig. 5: snapshot by snapshot into one image
 * buffer per camera; Sec. 5.2 and 6.2: data larger than device memory, and
 * skipping snapshots no camera needs).  The epochs stay in the caller's memory
 * and pass through a ring of `ring_epochs` device slots: epoch interval
 * [t_m, t_{m+1}) is rendered from epochs m and m + 1 alone over the cells whose
 * retarded time lies in it (the last interval closed) and added into the
 * images, so the result is the same lookback sum as a resident render (cell
 * steps identical; pixels differ only by the rounding of the per-interval
 * partial sums).  Streamed renders use FP64 ray parameters for every storage
 * type (DART_FORCE_F64_DDA), so a chord midpoint on an interval boundary falls
 * on the same side in both intervals.  Intervals no view can see are skipped and their epochs never
 * read.  The next epoch is uploaded and converted on an internal copy stream
 * while the current interval renders; host sources overlap with rendering only
 * when they are in pinned memory.
 *   dims, cell, n_epochs, epoch_times, storage: as for dart_load_epochs.
 *   ring_epochs: device epoch slots, in [3, 64] (3 is enough for overlap).
 *   brick: brick shape of the slots (nullable: the default one).
 * Device memory held: ring_epochs epochs in the storage type, one epoch of
 * source data (host sources), descriptors and staging for host images. */
typedef struct dart_streamer dart_streamer;
typedef struct {
    int32_t epochs_loaded;   /* epochs the last render call converted into the ring */
    int32_t epochs_skipped;  /* epochs no needed interval used (never read) */
    int32_t intervals;       /* epoch intervals the last call rendered */
    int32_t reserved;
    uint64_t bytes_uploaded; /* host-to-device source bytes of the last call */
} dart_stream_stats;
dart_status dart_streamer_create(const int32_t dims[3], const double cell[3], int32_t n_epochs,
                                 const double *epoch_times, dart_dtype storage,
                                 int32_t ring_epochs, const int32_t brick[3], dart_streamer **out);
/* Renders n views of the epoch series (emissivity [M][nz][ny][nx], velocity
 * [M][nz][ny][nx][3], src_dtype DART_F32 or DART_F64; src_flags
 * DART_DEVICE_PTRS when they are device arrays).  Views, images, flux_out and
 * steps_out as for dart_render_batch (the batched kernel with the current
 * dart_set_tuning shape); DART_ACCUMULATE adds into a device image, otherwise
 * it is cleared first.  Synchronises the stream before returning.  A bad value
 * in an epoch the call reads returns DART_E_RANGE naming it (the images are
 * then undefined).  Calls on one streamer are serialised. */
dart_status dart_streamer_render(dart_streamer *s, dart_dtype src_dtype, const void *emissivity,
                                 const void *velocity, uint32_t src_flags,
                                 const dart_view *views, int32_t n, void *const *images,
                                 double *flux_out, uint64_t *steps_out, void *hip_stream);
dart_status dart_streamer_get_stats(const dart_streamer *s, dart_stream_stats *out);
dart_status dart_streamer_destroy(dart_streamer *s);

/* Launch-shape parameters of the batched kernel (see dart_autotune). */
typedef struct {
    int32_t tile_w, tile_h;  /* pixels per wavefront tile, tile_w * tile_h == 64 */
    int32_t waves_per_cu;    /* resident waves per compute unit for the persistent grid */
    int32_t order;           /* tile queue order: 0 row-major, 1 longest estimated tile
                                first, 2 Z-order (Morton), 3 rows from the image's middle
                                outward (the upper half upward, then the lower half
                                downward), 4 whole rows, longest first, dealt round
                                robin to the per-XCD queues */
    int32_t orient;          /* 1: per view, turn the tile so that its long side follows
                                the image-plane projection of the bricks' long axis
                                (lanes of a wavefront then share cache lines) */
    int32_t depth_sync;      /* 0: each ray walks its own cells; n > 0: the rays of a
                                wavefront march together, no ray more than n cell
                                lengths (largest cell side) ahead of the rearmost, so
                                neighbouring rays read shared lines at the same time */
    int32_t cells_per_batch; /* cells a lane walks before it requests their records in one
                                go: 4 or 8 (0 means 4).  More cells keep more loads in
                                flight per wavefront and cost registers; the pixels do
                                not depend on it */
} dart_tuning;

/* Times the batched kernel on the given views over candidate tile shapes,
 * occupancies, tile orders, orientations and (if rebrick != 0) brick shapes,
 * then over cells per batch and depth sync for the chosen shape, and keeps the
 * fastest for later dart_render_batch calls on these stacks (candidates within
 * 2% of the fastest count as ties; the first in the sweep wins).  Errors:
 * DART_E_INVAL for bad arguments, or for labelled or vector stacks with
 * rebrick != 0; a HIP failure is returned as such, and the stacks are then
 * marked untuned (their renders use the process-wide dart_set_tuning shape).
 * best_out and best_ms_out are nullable. */
dart_status dart_autotune(dart_stack *const *stacks, const dart_view *views, int32_t n,
                          int32_t rebrick, dart_tuning *best_out, double *best_ms_out,
                          void *hip_stream);
dart_status dart_set_tuning(const dart_tuning *t);
dart_status dart_get_tuning(dart_tuning *t);

/* Number of distinct (cell, epoch) samples that receive a positive weight on
 * any ray of the image: the compulsory stack bytes of a render are this count
 * times the record size.  Untimed instrumentation (bitmap + counting pass). */
dart_status dart_count_samples(const dart_stack *s, const dart_view *v, uint64_t *samples_out,
                               void *hip_stream);

/* Number of distinct 128-byte lines of the stack's current layout that hold
 * those samples: times 128 it is the fewest bytes a render of the view can
 * fetch at cache-line granularity with this brick shape.  Untimed
 * instrumentation, as above. */
dart_status dart_count_lines(const dart_stack *s, const dart_view *v, uint64_t *lines_out,
                             void *hip_stream);

/* The same counts as renders read the stack: with the emissivity plane (packed
 * first if it is missing or stale), each sample of positive weight costs one
 * plane value (a quarter of a record) and, when its record carries the
 * read-whole mark, the record as well; without it (DART_RECORDS_ONLY,
 * DART_NO_KAHAN, or no plane) a record.  compulsory_out: those bytes; line_bytes_out: the distinct
 * 128-byte lines of the plane and of the records that hold them, times 128.
 * The image bytes are not included.  Either output may be NULL.  Untimed
 * instrumentation, as above. */
dart_status dart_count_bytes(const dart_stack *s, const dart_view *v, uint64_t *compulsory_out,
                             uint64_t *line_bytes_out, void *hip_stream);

/* Bytes of one resident record (j, beta_x, beta_y, beta_z) of a stack. */
dart_status dart_record_bytes(const dart_stack *s, uint32_t *bytes_out);

/* Streaming copy of `bytes` (multiple of 16) from src to dst, both device
 * memory: the measured HBM bandwidth reference. reps > 0 copies are enqueued.
 * dst = NULL: a read-only pass over src instead (each 16-byte word loaded
 * once, several independent loads in flight per thread, nothing written): the
 * reference for kernels that mostly read. */
dart_status dart_bandwidth_probe(void *dst, const void *src, uint64_t bytes, int32_t reps,
                                 void *hip_stream);

/* Gather probe: reads every 128-byte line of src (device memory) once, in a
 * scattered order (line k is read as line k * odd mod the line count), eight
 * consecutive threads reading the eight 16-byte words of one line, several
 * loads in flight per thread.  The bandwidth reference for kernels that gather
 * whole lines from scattered addresses.  bytes must be 128 times a power of
 * two (else DART_E_INVAL, nothing enqueued); reps > 0 passes are enqueued on
 * hip_stream.  Nothing is written. */
dart_status dart_gather_probe(const void *src, uint64_t bytes, int32_t reps, void *hip_stream);

/* ---------------------------------------------------------------- serving --
 * A render server keeps stacks resident (the caller's) and runs a host
 * scheduler thread that batches requests as they arrive (continuous batching):
 * every admitted, unfinished request is rendered by the next wave, waves run
 * on several streams and overlap on the device.  Output images are staged in
 * server-owned device memory; admission waits until the staged images of the
 * requests in flight fit in hbm_budget_bytes and fewer than max_inflight are
 * admitted.  Wave descriptors live in per-stream buffers fixed at creation
 * (budget / 4, clamped to [4, 64] MiB per stream, outside the budget); a wave
 * takes admitted requests in arrival order while their descriptors fit.
 *   image      destination [height][width] float32 (host memory, or device
 *              memory with DART_DEVICE_PTRS in the view flags); must stay valid
 *              until the ticket completes.
 *   ticket     out: identifies the request.
 * dart_poll: done = 1 once the image is written; flux, cell-steps and latency
 * (ms from submission to completion) are then valid, and the ticket is
 * retired.  dart_wait blocks until done.  flux, steps, latency_ms are nullable.
 * dart_server_destroy waits for every request.
 */
dart_status dart_server_create(size_t hbm_budget_bytes, int32_t max_inflight, int32_t n_streams,
                               dart_server **out);
dart_status dart_submit(dart_server *srv, const dart_stack *s, const dart_view *v, void *image,
                        uint64_t *ticket);
dart_status dart_poll(dart_server *srv, uint64_t ticket, int32_t *done, double *flux,
                      uint64_t *steps, double *latency_ms);
dart_status dart_wait(dart_server *srv, uint64_t ticket, double *flux, uint64_t *steps,
                      double *latency_ms);
dart_status dart_server_destroy(dart_server *srv);

typedef struct {
    uint64_t submitted, completed, waves;
    uint64_t max_wave_requests;
    uint64_t bytes_in_use, bytes_peak;
    uint64_t admission_waits;  /* requests that had to wait for memory or a slot */
} dart_server_stats;
dart_status dart_server_get_stats(dart_server *srv, dart_server_stats *st);

/* Where a server's waves spend their time, summed over the waves retired so
 * far (waves_timed of them).  Host side, per wave: planning (tile lists and
 * descriptors), enqueueing (the descriptor upload, the render launches, the
 * image copies and the completion callback), and the time from the
 * completion callback to the scheduler publishing the results.  Device side,
 * from events on the wave's stream: its whole device work (descriptor upload
 * to accumulator readback) and its render kernels alone (kernels of waves on
 * other streams run meanwhile, so these overlap).  stream_idle_ms sums, over
 * the waves, how long their stream sat idle with requests waiting: from its
 * previous wave's completion, when requests were queued at that moment, to
 * the start of planning this one.  All times in ms. */
typedef struct {
    uint64_t waves_timed;
    double plan_ms, enqueue_ms, callback_to_retire_ms;
    double device_ms, kernel_ms;
    double stream_idle_ms;
} dart_server_timeline;
dart_status dart_server_get_timeline(dart_server *srv, dart_server_timeline *tl);

/* Thread-local text describing the last non-OK status on this thread. */
const char *dart_last_error(void);

/* Library version string. */
const char *dart_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DART_H */
