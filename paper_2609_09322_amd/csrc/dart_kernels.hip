// dart_kernels.hip -- gfx950 kernels of the lookback ray-marching hot path.
//
// Per pixel ray (paper Sec. 2.3-2.5, Eqs. 2, 4-11, 14, 18-19):
//   * ray setup in FP64: pixel-centre origin, slab test against the grid box,
//     clip to the temporal window [t_obs - t_{M-1}, t_obs - t_0] in s
//     (the fast-forward of Sec. 5.1);
//   * 3D DDA (Eq. 11): per axis the crossings of cell planes are equally spaced
//     by ds_a = dx_a / |s_hat . x_a|; the k-th crossing is base_a + k ds_a,
//     evaluated from the integer crossing count (no drift);
//   * per cell: chord ds_n = exit - entry, retarded time at the chord midpoint,
//     epoch pair by a monotone pointer (tbar only decreases along the ray),
//     linear weight (Eqs. 6-7), two record gathers, D^p per epoch (Eq. 14 with
//     p = 2 + alpha) and Kahan-compensated accumulation of Eq. 19.
// The same device routine serves the one-launch-per-image kernel and the
// persistent tile-queue kernel; a MARK instantiation records the (cell, epoch)
// samples a render touches instead of summing them.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "dart_internal.h"

namespace dart {

// ------------------------------------------------------------------ records

__device__ __forceinline__ uint32_t cell_offset(const StackDev &st, int x, int y, int z) {
    const uint32_t bx = (uint32_t)x >> st.lb[0], by = (uint32_t)y >> st.lb[1],
                   bz = (uint32_t)z >> st.lb[2];
    const uint32_t lx = (uint32_t)x & ((1u << st.lb[0]) - 1u);
    const uint32_t ly = (uint32_t)y & ((1u << st.lb[1]) - 1u);
    const uint32_t lz = (uint32_t)z & ((1u << st.lb[2]) - 1u);
    const uint32_t brick = (bz * (uint32_t)st.nb[1] + by) * (uint32_t)st.nb[0] + bx;
    const uint32_t inner = (lz << (st.lb[0] + st.lb[1])) | (ly << st.lb[0]) | lx;
    return (brick << (st.lb[0] + st.lb[1] + st.lb[2])) | inner;
}

// Raw records as clang vector types: (j, beta_x, beta_y, beta_z) in the
// storage type; 16-bit records are two 32-bit words (j | bx << 16, by | bz << 16).
typedef double rec_f64 __attribute__((ext_vector_type(4)));
typedef float rec_f32 __attribute__((ext_vector_type(4)));
typedef unsigned int rec_h16 __attribute__((ext_vector_type(2)));

template <int S> struct RecT;
template <> struct RecT<ST_F64> { using raw = rec_f64; using val = double; };
template <> struct RecT<ST_F32> { using raw = rec_f32; using val = float; };
template <> struct RecT<ST_F16> { using raw = rec_h16; using val = float; };
template <> struct RecT<ST_BF16> { using raw = rec_h16; using val = float; };

// Records are read through global-address-space pointers (plain global loads).
template <int S>
__device__ __forceinline__ typename RecT<S>::raw load_grec(
    const typename RecT<S>::raw __attribute__((address_space(1))) *p) {
    return *p;
}

__device__ __forceinline__ float h2f(uint32_t bits16) {
    return __half2float(__ushort_as_half((unsigned short)bits16));
}

template <int S, typename V>
__device__ __forceinline__ void decode(const typename RecT<S>::raw &r, V &j, V &bx, V &by, V &bz) {
    if constexpr (S == ST_F64 || S == ST_F32) {
        j = r.x; bx = r.y; by = r.z; bz = r.w;
    } else if constexpr (S == ST_F16) {
        j = h2f(r.x & 0xffffu); bx = h2f(r.x >> 16); by = h2f(r.y & 0xffffu); bz = h2f(r.y >> 16);
    } else {
        j = __uint_as_float(r.x << 16); bx = __uint_as_float(r.x & 0xffff0000u);
        by = __uint_as_float(r.y << 16); bz = __uint_as_float(r.y & 0xffff0000u);
    }
}

// The velocity bits of a record, OR-ed into one word: zero exactly when the
// three components are +0.  (A -0 component makes it non-zero; such records
// take the general path, where they also give D = 1.)
template <int S>
__device__ __forceinline__ uint32_t beta_bits(const typename RecT<S>::raw &r) {
    if constexpr (S == ST_F16 || S == ST_BF16) {
        return (r.x & 0xffff0000u) | r.y;
    } else if constexpr (S == ST_F32) {
        return __float_as_uint(r.y) | __float_as_uint(r.z) | __float_as_uint(r.w);
    } else {
        const uint64_t b = (uint64_t)__double_as_longlong(r.y) |
                           (uint64_t)__double_as_longlong(r.z) |
                           (uint64_t)__double_as_longlong(r.w);
        return (uint32_t)b | (uint32_t)(b >> 32);
    }
}

// The rest-frame emissivity j of a record.
template <int S>
__device__ __forceinline__ typename RecT<S>::val record_j(const typename RecT<S>::raw &r) {
    if constexpr (S == ST_F64 || S == ST_F32) return r.x;
    else if constexpr (S == ST_F16) return h2f(r.x & 0xffffu);
    else return __uint_as_float(r.x << 16);
}

// D^p of one record (Eq. 14 raised to p), and its rest-frame emissivity in j.
template <int S>
__device__ __forceinline__ typename RecT<S>::val boost_factor(const typename RecT<S>::raw &r,
                                                             const RayView &v, bool beaming,
                                                             typename RecT<S>::val &j) {
    using V = typename RecT<S>::val;
    V bx, by, bz;
    decode<S, V>(r, j, bx, by, bz);
    if (!beaming || (bx == V(0) && by == V(0) && bz == V(0))) return V(1);
    if constexpr (S == ST_F64) {
        double q = fma(-bx, bx, fma(-by, by, fma(-bz, bz, 1.0)));
        double rr = fma(bx, v.shat[0], fma(by, v.shat[1], fma(bz, v.shat[2], 1.0)));
        return exp2(v.p * (0.5 * log2(q) - log2(rr)));
    } else if constexpr (S == ST_F32) {
        double dx = bx, dy = by, dz = bz;
        double q = fma(-dx, dx, fma(-dy, dy, fma(-dz, dz, 1.0)));
        double rr = fma(dx, v.shat[0], fma(dy, v.shat[1], fma(dz, v.shat[2], 1.0)));
        float p = (float)v.p;
        float e = fmaf(0.5f * p, __builtin_amdgcn_logf((float)q), -p * __builtin_amdgcn_logf((float)rr));
        return __builtin_amdgcn_exp2f(e);
    } else {
        float q = fmaf(-bx, bx, fmaf(-by, by, fmaf(-bz, bz, 1.0f)));
        float rr = fmaf(bx, v.shat_hi[0], fmaf(by, v.shat_hi[1], fmaf(bz, v.shat_hi[2], 1.0f)));
        rr += fmaf(bx, v.shat_lo[0], fmaf(by, v.shat_lo[1], bz * v.shat_lo[2]));
        float p = (float)v.p;
        float e = fmaf(0.5f * p, __builtin_amdgcn_logf(q), -p * __builtin_amdgcn_logf(rr));
        return __builtin_amdgcn_exp2f(e);
    }
}

// Rest-frame emissivity times D^p of one record (Eq. 14 raised to p, times j).
// FP64 stacks: all in FP64.  FP32 stacks: 1 - beta^2 and 1 + beta.s in FP64
// (the two quantities that cancel at high Lorentz factor), logs in FP32.
// 16-bit stacks: FP32 FMA chains starting from 1, with s_hat split in two
// floats: rounding s_hat to FP32 alone moves 1 + beta.s by ~6e-8 absolute,
// which near the beaming peak (1 + beta.s ~ 0.05 at Lorentz factor 4) is a
// systematic ~1e-6 relative error of D^p over the whole image.  (The factor is
// exactly 1 without beaming or at rest, and j * 1 is j.)
// (The product is rounded on its own, never fused into the interpolation that
// uses it, so every path that meets a sample, from the emissivity plane or
// from whole records, gives it the same bits.)
template <int S>
__device__ __forceinline__ typename RecT<S>::val boosted(const typename RecT<S>::raw &r,
                                                        const RayView &v, bool beaming) {
#pragma clang fp contract(off)
    typename RecT<S>::val j;
    const typename RecT<S>::val f = boost_factor<S>(r, v, beaming, j);
    return j * f;
}

// Emissivity of another component of a vector stack, packed one value per
// (epoch, cell) in the stack's storage type at the record's index.
template <int S> struct JFieldT;
template <> struct JFieldT<ST_F64> { using raw = double; };
template <> struct JFieldT<ST_F32> { using raw = float; };
template <> struct JFieldT<ST_F16> { using raw = unsigned short; };
template <> struct JFieldT<ST_BF16> { using raw = unsigned short; };

template <int S>
__device__ __forceinline__ typename RecT<S>::val decode_j(typename JFieldT<S>::raw w) {
    if constexpr (S == ST_F64 || S == ST_F32) return w;
    else if constexpr (S == ST_F16) return h2f((uint32_t)w);
    else return __uint_as_float((uint32_t)w << 16);
}

// decode_j(b) - decode_j(a) in FP32, of two loaded plane elements (16-bit
// elements as their bits zero-extended to 32, as the load leaves them).  FP16:
// one mixed-precision fma, b * 1 - a with both operands converted exactly and
// one rounding: the same value as the difference of the converted elements,
// without the two conversions.
template <int S, typename Q>
__device__ __forceinline__ float plane_diff(Q a, Q b) {
    using JF = typename JFieldT<S>::raw;
    if constexpr (S == ST_F16) {
        float d;
        asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel_hi:[1,0,1]" : "=v"(d) : "v"(b), "v"(a));
        return d;
    } else {
        return (float)decode_j<S>((JF)b) - (float)decode_j<S>((JF)a);
    }
}

// Emissivity plane (StackDev::jplane): one element per record, j alone in the
// storage type, with its sign bit standing for "read the whole record": set
// when the velocity bits are not all zero or j itself has its sign bit set
// (negative, or -0).  An element without the mark is the record's j, exactly.
template <int S>
__device__ __forceinline__ uint32_t jplane_bits(typename JFieldT<S>::raw w) {
    if constexpr (S == ST_F32) return __float_as_uint(w);
    else return (uint32_t)w;
}
// the mark of an element, or of the OR of several elements' bits
template <int S>
__device__ __forceinline__ uint32_t jplane_mark(uint32_t bits) {
    if constexpr (S == ST_F32) return bits >> 31;
    else return (bits >> 15) & 1u;
}
template <int S>
__device__ __forceinline__ typename JFieldT<S>::raw jplane_element(const typename RecT<S>::raw &r) {
    if constexpr (S == ST_F32) {
        const uint32_t jb = __float_as_uint(r.x);
        const uint32_t mark = (beta_bits<S>(r) != 0u || (jb >> 31)) ? 1u : 0u;
        return __uint_as_float((jb & 0x7fffffffu) | (mark << 31));
    } else {
        const uint32_t jb = r.x & 0xffffu;
        const uint32_t mark = (beta_bits<S>(r) != 0u || (jb >> 15)) ? 1u : 0u;
        return (typename JFieldT<S>::raw)((jb & 0x7fffu) | (mark << 15));
    }
}

// ------------------------------------------------------------------ one ray

// DDA state of one ray.  Per axis the plane crossings ahead of the ray form the
// sequence base + c * ds_axis (c = crossings made so far along that axis): the
// cell's chord is [max of the planes behind, min of the planes ahead].  The
// planes behind are not kept: the largest of them is the previous cell's exit
// (or, for the first cell, the largest of the planes behind the start).
// Crossing counts are kept in the ray precision (exact integers there).
// The cell indices are not kept either: the walk needs only the record offset
// (updated per step, below) and the end of the ray, which includes the first
// crossing of a grid face, evaluated with the same expression as the walk's.
template <typename R>
struct Ray {
    R c0, c1, c2;        // crossings made per axis
    R b0, b1, b2;        // s of the first plane ahead per axis
    R d0, d1, d2;        // plane spacing per axis (Eq. 11)
    R sa0, sa1, sa2;     // s of the plane ahead
    R entry;             // s where the ray enters the current cell
    R stop;              // min(first crossing of a grid face, end of the window)
    uint32_t off;        // record offset of the current cell inside its epoch
};

// The record offset of cell (x, y, z) inside its epoch is a sum of one term per
// axis: with bricks of 2^a x 2^b x 2^c cells (L = a + b + c bits per brick),
//   offset = ((bz nb1 + by) nb0 + bx) 2^L + lz 2^(a+b) + ly 2^a + lx
//          = X(x) + Y(y) + Z(z),
//   X(x) = x + (x >> a)(2^L - 2^a)
//   Y(y) = y 2^a + (y >> b)(nb0 2^L - 2^(a+b))
//   Z(z) = z 2^(a+b) + (z >> c)(nb1 nb0 2^L - 2^(a+b+c))
// (the same value cell_offset returns), so a step along one axis changes one
// term.  The products wrap modulo 2^32 like the offsets themselves.
//
// A step of +-1 along x changes X by +-1, or by +-(1 + 2^L - 2^a) when it
// crosses into the next brick, which is when the current cell is the last of
// its brick in the direction of the step: x mod 2^a is 2^a - 1 (stepping up)
// or 0 (stepping down); y and z alike.  The position of a cell inside its brick
// is the low L bits of its offset, (lz << (a+b)) | (ly << a) | lx, so the test
// reads the offset itself.  All rays of a view step the same way along each
// axis, so these increments and tests are uniform over a wavefront: the walk
// updates the offset with an and, a compare and a select per axis, two selects
// of the stepping axis and an add, without multiplies.
struct OffsetSteps {
    uint32_t field[3];   // bits of lx, ly, lz in the offset
    uint32_t last[3];    // their value in the last cell of a brick along the step
    uint32_t inner[3];   // offset change of a step inside a brick
    uint32_t cross[3];   // offset change of a step across a brick face
};

__device__ __forceinline__ OffsetSteps offset_steps(const StackDev &st, const RayView &v) {
    OffsetSteps o;
    const uint32_t a = st.lb[0], b = st.lb[1], c = st.lb[2], L = a + b + c;
    const uint32_t nb0 = st.nb[0], nb1 = st.nb[1];
    const uint32_t in_[3] = {1u, 1u << a, 1u << (a + b)};
    const uint32_t k[3] = {(1u << L) - (1u << a), (nb0 << L) - (1u << (a + b)),
                           ((nb1 * nb0) << L) - (1u << L)};
    const uint32_t lb[3] = {a, b, c};
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const bool down = v.shat[q] < 0.0;
        o.field[q] = ((1u << lb[q]) - 1u) * in_[q];
        o.last[q] = down ? 0u : o.field[q];
        // (unsigned negation: a step down subtracts modulo 2^32)
        const uint32_t inner = down ? 0u - in_[q] : in_[q];
        const uint32_t cross = inner + (down ? 0u - k[q] : k[q]);
        // Both held in vector registers for the whole walk: the per-step
        // select between them reads its condition from a scalar register
        // pair, and an instruction takes at most one scalar operand.
        asm("v_mov_b32 %0, %1" : "=v"(o.inner[q]) : "s"(inner));
        asm("v_mov_b32 %0, %1" : "=v"(o.cross[q]) : "s"(cross));
    }
    return o;
}
__device__ __forceinline__ uint32_t off_x(const StackDev &st, int x) {
    const uint32_t a = st.lb[0], L = st.lb[0] + st.lb[1] + st.lb[2];
    return (uint32_t)x + ((uint32_t)x >> a) * ((1u << L) - (1u << a));
}
__device__ __forceinline__ uint32_t off_y(const StackDev &st, int y) {
    const uint32_t a = st.lb[0], b = st.lb[1], L = st.lb[0] + st.lb[1] + st.lb[2];
    return ((uint32_t)y << a) + ((uint32_t)y >> b) * (((uint32_t)st.nb[0] << L) - (1u << (a + b)));
}
__device__ __forceinline__ uint32_t off_z(const StackDev &st, int z) {
    const uint32_t ab = st.lb[0] + st.lb[1], c = st.lb[2], L = ab + c;
    return ((uint32_t)z << ab) +
           ((uint32_t)z >> c) * ((((uint32_t)st.nb[1] * (uint32_t)st.nb[0]) << L) - (1u << L));
}

// FP64 set-up of pixel (pi, pj): slab test, clip to the window, starting cell
// and crossing sequences.  False when no cell of the ray can contribute.
// cell (if given) receives the starting cell's indices.
template <typename R>
__device__ __forceinline__ bool ray_setup(const RayView &v, const StackDev &st,
                                          const double *centre, int pi, int pj, Ray<R> &r,
                                          int *cell = nullptr) {
    const double u = (pi + 0.5 - 0.5 * v.width) * v.ps;
    const double w = (pj + 0.5 - 0.5 * v.height) * v.ps;
    double o[3];
#pragma unroll
    for (int a = 0; a < 3; a++) o[a] = centre[a] + u * v.eu[a] + w * v.ev[a];
    double s_in = -INFINITY, s_out = INFINITY;
    bool hit = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double d = v.shat[a];
        const double hi = st.n[a] * st.cell[a];
        if (d == 0.0) {
            if (o[a] < 0.0 || o[a] >= hi) hit = false;
        } else {
            const double t0 = (0.0 - o[a]) * v.inv_shat[a], t1 = (hi - o[a]) * v.inv_shat[a];
            s_in = fmax(s_in, fmin(t0, t1));
            s_out = fmin(s_out, fmax(t0, t1));
        }
    }
    const double s_start = fmax(s_in, v.s_lo);
    const double s_stop = fmin(s_out, v.s_hi);
    if (!hit || !(s_start < s_stop) || !(s_in < s_out)) return false;
    if ((v.flags & F_NO_LOOKBACK) && v.fixed_m < 0) return false;
    int idx[3];
    R base[3], sp[3];
    R stop = (R)s_stop;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double d = v.shat[a];
        const double x = o[a] + s_start * d;
        int k = (int)floor(x / st.cell[a]);
        k = k < 0 ? 0 : (k >= st.n[a] ? st.n[a] - 1 : k);
        idx[a] = k;
        if (d == 0.0) {
            base[a] = (R)INFINITY;
            sp[a] = (R)0;
        } else {
            const double plane = (d > 0.0 ? (k + 1) : k) * st.cell[a];
            base[a] = (R)((plane - o[a]) * v.inv_shat[a]);
            sp[a] = (R)(st.cell[a] * fabs(v.inv_shat[a]));
            // the grid face ahead is the plane after c_face crossings; the walk
            // reaches it as fma(c_face, ds, base), the value taken here
            const int c_face = d > 0.0 ? st.n[a] - 1 - k : k;
            stop = fmin(stop, fma((R)c_face, sp[a], base[a]));
        }
    }
    r.c0 = r.c1 = r.c2 = (R)0;
    r.b0 = base[0]; r.b1 = base[1]; r.b2 = base[2];
    r.d0 = sp[0]; r.d1 = sp[1]; r.d2 = sp[2];
    r.sa0 = base[0]; r.sa1 = base[1]; r.sa2 = base[2];
    const R sb0 = v.shat[0] != 0.0 ? base[0] - sp[0] : (R)-INFINITY;
    const R sb1 = v.shat[1] != 0.0 ? base[1] - sp[1] : (R)-INFINITY;
    const R sb2 = v.shat[2] != 0.0 ? base[2] - sp[2] : (R)-INFINITY;
    r.entry = fmax(sb0, fmax(sb1, sb2));
    r.stop = stop;
    r.off = off_x(st, idx[0]) + off_y(st, idx[1]) + off_z(st, idx[2]);
    if (cell) {
        cell[0] = idx[0]; cell[1] = idx[1]; cell[2] = idx[2];
    }
    return r.entry < r.stop;
}

// max(a, b) of two walk positions (never NaN).  FP32: one v_max_f32 (fmaxf
// would first quiet both operands); FP64: a compare and select.  (Equal
// operands give the same value either way, up to the sign of a zero, which no
// use of the entry distinguishes.)
__device__ __forceinline__ float later_of(float a, float b) {
    float m;
    asm("v_max_f32 %0, %1, %2" : "=v"(m) : "v"(a), "v"(b));
    return m;
}
__device__ __forceinline__ double later_of(double a, double b) { return a > b ? a : b; }

// The axis of the next crossing (ties: x before y before z); exit is
// min(sa0, sa1, sa2), the current cell's exit.
template <typename R>
__device__ __forceinline__ void step_axis(const Ray<R> &r, const R exit, bool &ax, bool &ay,
                                          bool &az) {
    ax = r.sa0 == exit;
    ay = !ax && r.sa1 == exit;
    az = !ax && !ay;
}

// Step to the neighbour across the nearest face; false when the ray has ended
// (it crossed a grid face or the end of the window).  exit becomes the next
// cell's entry.  Written without branches: the lanes of a wavefront step along
// different axes, and every axis takes the same few selects instead of three
// divergent paths.  An axis that does not step keeps its count, so its
// recomputed plane is the same value.  Since the crossings are taken in order
// of s, every cell entered before the crossing that ends the ray has entry
// below stop; a cell entered on a tie with it has no chord.
template <typename R>
__device__ __forceinline__ bool ray_advance(const OffsetSteps &os, Ray<R> &r, const R exit) {
    // (bitwise, not short-circuit, logic: every select below is evaluated on
    // every lane, with no branch)
    const bool ax = r.sa0 == exit;
    const bool ey = r.sa1 == exit;
    const bool ay = ey & !ax, az = !(ax | ey);
    // brick face ahead along each axis, from the current cell's offset
    const uint32_t dx = (r.off & os.field[0]) == os.last[0] ? os.cross[0] : os.inner[0];
    const uint32_t dy = (r.off & os.field[1]) == os.last[1] ? os.cross[1] : os.inner[1];
    const uint32_t dz = (r.off & os.field[2]) == os.last[2] ? os.cross[2] : os.inner[2];
    const uint32_t dyz = ey ? dy : dz;
    r.off += ax ? dx : dyz;
    r.c0 += ax ? (R)1 : (R)0;
    r.c1 += ay ? (R)1 : (R)0;
    r.c2 += az ? (R)1 : (R)0;
    r.sa0 = fma(r.c0, r.d0, r.b0);
    r.sa1 = fma(r.c1, r.d1, r.b1);
    r.sa2 = fma(r.c2, r.d2, r.b2);
    r.entry = later_of(exit, r.entry);
    return r.entry < r.stop;
}

// Epoch bracket in s: a_m = t_obs - t_m decreases with m; the bracket m holds
// a_{m+1} <= s_mid <= a_m.  s_mid only grows along a ray, so m only moves down.
template <typename R>
struct Bracket {
    int m;
    R am, am1, inv_dt;
};

typedef const double __attribute__((address_space(1))) gdouble;
typedef double __attribute__((address_space(3))) ldsdouble;

// Epoch table of a view in LDS, one per wavefront: (t_obs - t_m, 1 / (t_{m+1} -
// t_m)) for m < n_epochs, so that a lane whose bracket moves reads it from LDS
// instead of waiting on a global load in the middle of a batch.  Views with
// more epochs read global memory (the same values).
constexpr int EPOCH_TAB_MAX = 64;

// Fills the calling wavefront's table for stack st seen at t_obs (all lanes).
__device__ __forceinline__ void epoch_tab_fill(ldsdouble *tab, const StackDev &st, double t_obs) {
    gdouble *t = (gdouble *)st.times, *idt = (gdouble *)st.inv_dt;
    const int lane = threadIdx.x & 63;
    for (int m = lane; m < st.n_epochs; m += 64) {
        tab[2 * m] = t_obs - t[m];
        tab[2 * m + 1] = idt[m];
    }
    // the wavefront's own writes, before any lane reads another lane's entry
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R>
__device__ __forceinline__ R epoch_a(const RayView &v, const StackDev &st, const ldsdouble *tab,
                                     int m) {
    return tab ? (R)tab[2 * m] : (R)(v.t_obs - ((gdouble *)st.times)[m]);
}
template <typename R>
__device__ __forceinline__ R epoch_inv_dt(const StackDev &st, const ldsdouble *tab, int m) {
    return tab ? (R)tab[2 * m + 1] : (R)((gdouble *)st.inv_dt)[m];
}

template <typename R>
__device__ __forceinline__ void bracket_init(const RayView &v, const StackDev &st, bool lookback,
                                             Bracket<R> &b, const ldsdouble *tab = nullptr) {
    const int M = st.n_epochs;
    b.m = lookback ? (M >= 2 ? M - 2 : 0) : v.fixed_m;
    b.am = epoch_a<R>(v, st, tab, b.m);
    b.am1 = M >= 2 ? epoch_a<R>(v, st, tab, b.m + 1) : b.am;
    b.inv_dt = M >= 2 ? epoch_inv_dt<R>(st, tab, b.m) : (R)0;
}

template <typename R>
__device__ __forceinline__ void bracket_seek(const RayView &v, const StackDev &st, R mid,
                                             Bracket<R> &b, const ldsdouble *tab = nullptr) {
    while (b.m > 0 && mid > b.am) {
        b.m--;
        b.am1 = b.am;
        b.am = epoch_a<R>(v, st, tab, b.m);
        b.inv_dt = epoch_inv_dt<R>(st, tab, b.m);
    }
}

// The same, keeping `base` (the elements of epoch b.m) in step with the
// bracket.
template <typename R, typename P>
__device__ __forceinline__ void bracket_seek(const RayView &v, const StackDev &st, R mid,
                                             Bracket<R> &b, const ldsdouble *tab, P &base,
                                             P data, int64_t estride) {
    while (b.m > 0 && mid > b.am) {
        b.m--;
        b.am1 = b.am;
        b.am = epoch_a<R>(v, st, tab, b.m);
        b.inv_dt = epoch_inv_dt<R>(st, tab, b.m);
        base = data + (int64_t)b.m * estride;
    }
}

// The walk's bracket in doubled units, for mid2 = entry + exit (twice the
// chord midpoint): thr2 = 2 a_m, or +inf at m = 0 where the bracket cannot
// move (one compare per cell instead of two); am2 = 2 a_m, am1_2 = 2 a_{m+1},
// hdt = inv_dt / 2.  Doubling and halving are exact, so every test on mid2 and
// the weight (am2 - mid2) hdt equal those on the midpoint itself, and the walk
// saves the halving of every midpoint.
template <typename R>
struct Doubled {
    R thr2, am2, am1_2, hdt;
};
template <typename R>
__device__ __forceinline__ void doubled_of(const Bracket<R> &b, Doubled<R> &d) {
    d.am2 = (R)2 * b.am;
    d.am1_2 = (R)2 * b.am1;
    d.hdt = (R)0.5 * b.inv_dt;
    d.thr2 = b.m > 0 ? d.am2 : (R)INFINITY;
}

// bracket_seek for mid = mid2 / 2, keeping d and `base` (the elements of epoch
// b.m) in step with the bracket.
template <typename R, typename P>
__device__ __forceinline__ void bracket_seek2(const RayView &v, const StackDev &st, R mid2,
                                              Bracket<R> &b, Doubled<R> &d, const ldsdouble *tab,
                                              P &base, P data, int64_t estride) {
    if (mid2 > d.thr2) {
        do {
            b.m--;
            b.am1 = b.am;
            b.am = epoch_a<R>(v, st, tab, b.m);
            b.inv_dt = epoch_inv_dt<R>(st, tab, b.m);
        } while (b.m > 0 && mid2 > (R)2 * b.am);
        base = data + (int64_t)b.m * estride;
        doubled_of(b, d);
    }
}

// Exact-time pieces start at s: the bracket of the retarded times just below
// t_obs - s, so a piece that starts on an epoch time takes the earlier interval.
template <typename R>
__device__ __forceinline__ void bracket_seek_from(const RayView &v, const StackDev &st, R s,
                                                  Bracket<R> &b, const ldsdouble *tab = nullptr) {
    while (b.m > 0 && s >= b.am) {
        b.m--;
        b.am1 = b.am;
        b.am = epoch_a<R>(v, st, tab, b.m);
        b.inv_dt = epoch_inv_dt<R>(st, tab, b.m);
    }
}

// Sample marking for the compulsory-bytes count: sets the (epoch, cell) bits
// of positive weight in `bitmap` ([M][nz][ny][nx] bits).
// line_log2 >= 0 marks instead the lines of 2^line_log2 elements of the record
// index space that hold those samples (128-byte lines of the records, or of the
// emissivity plane): bit (record index in the stack) >> line_log2.
// moving_only: only the samples whose record carries the emissivity plane's
// read-whole mark.
template <int S, typename R>
__device__ __forceinline__ void mark_ray(const RayView &v, int pi, int pj, uint32_t *bitmap,
                                         int line_log2, bool moving_only) {
    using Raw = typename RecT<S>::raw;
    Ray<R> r;
    const StackDev &st = v.st;
    int cell[3];
    if (!ray_setup(v, st, v.centre, pi, pj, r, cell)) return;
    const int step[3] = {v.shat[0] > 0.0 ? 1 : -1, v.shat[1] > 0.0 ? 1 : -1,
                         v.shat[2] > 0.0 ? 1 : -1};
    const bool lookback = !(v.flags & F_NO_LOOKBACK);
    const bool single = (v.flags & F_NEAREST) || st.n_epochs == 1;
    const R r_lo = (R)v.s_lo, r_hi = (R)v.s_hi;
    Bracket<R> br;
    bracket_init(v, st, lookback, br);
    const OffsetSteps os = offset_steps(st, v);
    const uint64_t ncell = (uint64_t)st.n[0] * st.n[1] * st.n[2];
    for (int guard = st.n[0] + st.n[1] + st.n[2] + 3; guard > 0; guard--) {
        const R entry = r.entry;
        const R exit = fmin(r.sa0, fmin(r.sa1, r.sa2));
        if (entry >= r.stop) break;
        const R ds = exit - entry, mid = (R)0.5 * (entry + exit);
        if (ds > (R)0 && mid >= r_lo && mid <= r_hi) {
            R wt = (R)v.fixed_w;
            if (lookback) {
                bracket_seek(v, st, mid, br);
                wt = (br.am - mid) * br.inv_dt;
            }
            int m0 = br.m;
            if (single && st.n_epochs >= 2) {
                const bool later = lookback ? (mid - br.am1) < (br.am - mid) : wt > (R)0.5;
                m0 = later ? br.m + 1 : br.m;
            }
            uint64_t lin, stride;
            if (line_log2 < 0) {
                lin = ((uint64_t)cell[2] * st.n[1] + cell[1]) * st.n[0] + cell[0];
                stride = ncell;
            } else {
                lin = r.off;
                stride = st.epoch_stride;
            }
            const int sh = line_log2 < 0 ? 0 : line_log2;
            // (the whole-record mark of the sample of epoch m)
            auto whole = [&](int m) {
                const Raw *rec = (const Raw *)st.data + ((int64_t)m * st.epoch_stride + r.off);
                if constexpr (S == ST_F64) {
                    return beta_bits<S>(*rec) != 0u || signbit(rec->x);
                } else {
                    return jplane_mark<S>(jplane_bits<S>(jplane_element<S>(*rec))) != 0u;
                }
            };
            if ((single || wt < (R)1) && (!moving_only || whole(m0))) {
                const uint64_t b = ((uint64_t)m0 * stride + lin) >> sh;
                atomicOr(&bitmap[b >> 5], 1u << (b & 31));
            }
            if (!single && wt > (R)0 && (!moving_only || whole(m0 + 1))) {
                const uint64_t b = ((uint64_t)(m0 + 1) * stride + lin) >> sh;
                atomicOr(&bitmap[b >> 5], 1u << (b & 31));
            }
        }
        bool ax, ay, az;
        step_axis(r, exit, ax, ay, az);
        cell[0] += ax ? step[0] : 0;
        cell[1] += ay ? step[1] : 0;
        cell[2] += az ? step[2] : 0;
        if (!ray_advance(os, r, exit)) break;
    }
}

// Adds term to the compensated sum (sum, comp) (Kahan); a zero term leaves
// both as they are, so cells not taken in a batch do not perturb the sum.
// Without compensation (kahan false) comp stays 0, and the same steps are a
// plain add.  (The sum starts at +0 and never becomes -0, so skipping a zero
// term is the same as adding it.)
// The steps are never fused with the product that made the term, and the
// test stays a branch (an empty volatile asm keeps the compiler from turning
// it into selects, which would cost two more vector instructions per term).
template <typename A>
__device__ __forceinline__ void kahan_add(A &sum, A &comp, A term, bool kahan) {
#pragma clang fp contract(off)
    if (term != (A)0) {
        asm volatile("");
        const A yk = term - comp;
        const A tk = sum + yk;
        comp = kahan ? (tk - sum) - yk : (A)0;
        sum = tk;
    }
}

// The epoch interpolation a + w (b - a) of a sample's two values, as one fma
// after the difference, in every path alike.
__device__ __forceinline__ float lerp_w(float a, float b, float w) {
#pragma clang fp contract(off)
    return fmaf(w, b - a, a);
}
__device__ __forceinline__ double lerp_w(double a, double b, double w) {
#pragma clang fp contract(off)
    return fma(w, b - a, a);
}
// The same with the difference given (the emissivity plane's FP16 difference
// is one mixed-precision fma).
__device__ __forceinline__ float lerp_d(float a, float d, float w) { return fmaf(w, d, a); }

// Cells walked per batch (K): a lane walks K cells of its ray, then issues all
// their record loads back to back, then consumes them.  The batched kernel
// comes with K = 4 and K = 8 (a tuning choice); the plain kernel uses 4.
constexpr int CELLS_PER_BATCH = 4;

// Minimum over the 64 lanes of a wavefront (every lane active), in six
// instructions that each take the minimum of a lane's value and a DPP-moved
// one: within each row of 16 lanes (swap neighbours, swap pairs, mirror the
// half row, mirror the row: every lane then holds its row's minimum), then the
// last lane of row 0 into row 1 and of row 2 into row 3 (row_bcast:15), then
// the last lane of row 1 into rows 2 and 3 (row_bcast:31): lane 63 holds the
// wavefront's minimum.  No LDS round trips.  The operands are entries of the
// walk (never NaN), so v_min_f32 needs no quieting of its operands; every
// source lane of these moves is active.  Each move reads a register the
// previous instruction wrote, which takes two wait states (s_nop 1).
__device__ __forceinline__ float wave_min(float x) {
    asm("s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "s_nop 1\n\t"
        "v_min_f32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
        "s_nop 1"
        : "+v"(x));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}
__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fmin(x, __shfl_xor(x, off, 64));
    return x;
}

// lo <= s <= hi (lo <= hi, no NaN): in FP32 one median-of-three and a compare.
__device__ __forceinline__ bool in_window(float s, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(s, lo, hi) == s;
}
__device__ __forceinline__ bool in_window(double s, double lo, double hi) {
    return s >= lo && s <= hi;
}

// Marching modes (SYNC):
//   0  each lane walks its own ray, K cells per batch;
//   1  depth-synchronous wavefront: a batch only takes cells whose entry lies
//      within v.sync_gap of the wavefront's rearmost ray, so neighbouring
//      rays reach the cells (and cache lines) they share at the same time
//      instead of some batches apart.  Every lane then stays in the loop
//      until all rays of the wavefront have ended, including lanes whose ray
//      misses the grid.
// EX (exact temporal integration): a cell's chord is cut where the ray's
// retarded time passes an epoch time and at the window ends; each piece lies
// in one epoch interval, where the interpolated field is linear along the ray,
// so the midpoint value times the piece is its exact integral.  A batch slot
// then takes one piece instead of one cell; a cell counts as one cell-step.
// (Linear interpolation with lookback only: the host clears EX otherwise.)
// VEC (vector stacks): the same walk, weights and D^p also integrate the
// emissivity of components 1..n_chan-1, each with its own compensated sum,
// returned in ext[0..2].
// SINGLE: one epoch per cell (nearest-epoch mode, or a one-epoch stack), a
// property of the view and stack, so each lane's walk has no per-cell test.
//
// Marches pixel (pi, pj) of view v and returns its intensity (FP64 for the
// caller's reductions); adds the counted cell-steps to nsteps.
//
// The walk does not depend on the data it reads, so each lane first walks a
// batch of K cells (chord, epoch weight, record addresses), then requests the
// 2K records at once and consumes them after a single wait: many gathers per
// lane in flight instead of one dependent load per step.  (K is 4 or 8 in the
// batched kernel, CELLS_PER_BATCH in the plain one.)
//
// JP: 0 whole records; 1 the emissivity plane through 64-bit addresses; 2 the
// plane through 32-bit byte offsets from its start (planes of at most 4 GiB):
// a cell's offset is one add and a shift, and the elements of its two epochs
// are loaded at that offset from two wavefront-uniform bases.
template <int S, typename R, int SYNC, bool EX, int K, bool VEC, bool SINGLE, int JP>
__device__ __forceinline__ double march_walk(const RayView &v, const StackDev &st,
                                             const double *centre, int pi, int pj, bool in_image,
                                             const ldsdouble *tab, uint32_t &nsteps,
                                             double *ext) {
    using A = typename std::conditional<S == ST_F64, double, float>::type;
    using V = typename RecT<S>::val;
    using Raw = typename RecT<S>::raw;
    using GRaw = const Raw __attribute__((address_space(1)));
    using JF = typename JFieldT<S>::raw;
    using GJ = const JF __attribute__((address_space(1)));
    static_assert(!(JP && (VEC || S == ST_F64)), "no emissivity plane for these stacks");
    // The walk addresses elements of the emissivity plane (JP) or records:
    // both have the record index space, so one offset serves either.
    using E = typename std::conditional<JP != 0, JF, Raw>::type;
    using GE = const E __attribute__((address_space(1)));
    constexpr bool O32 = JP == 2;
    constexpr uint32_t ESH = sizeof(JF) == 2 ? 1u : 2u;  // log2 of the element size
    using GB = const uint8_t __attribute__((address_space(1)));
    // a cell's element: its address, or (O32) its byte offset in the plane
    using Addr = typename std::conditional<O32, uint32_t, GE *>::type;
    constexpr int NX = VEC ? 3 : 1;  // extra component slots
    if constexpr (VEC) {
#pragma unroll
        for (int c = 0; c < NX; c++) ext[c] = 0.0;
    }
    Ray<R> r;
    bool alive = in_image && ray_setup(v, st, centre, pi, pj, r);
    if (SYNC == 0 && !alive) return 0.0;
    const bool lookback = !(v.flags & F_NO_LOOKBACK);
    const bool beaming = !(v.flags & F_NO_BEAMING);
    const int M = st.n_epochs;
    constexpr bool single = SINGLE;
    // (views without compensation are never given the emissivity plane)
    const bool kahan = JP != 0 || !(v.flags & F_NO_KAHAN);
    const R r_lo = (R)v.s_lo, r_hi = (R)v.s_hi;
    constexpr bool DOUBLED = std::is_same<R, float>::value || JP != 0;
    const R lo2 = (R)2 * r_lo, hi2 = (R)2 * r_hi;  // the window for mid2 (exact)
    const R gap = (R)v.sync_gap;
    GRaw *gdata = (GRaw *)st.data;
    GE *wdata = JP ? (GE *)st.jplane : (GE *)st.data;
    const int64_t estride = st.epoch_stride;
    // offset of the second record: the next epoch, or the same record when
    // only one epoch is used
    const int64_t second = single ? 0 : estride;
    Bracket<R> br;
    bracket_init(v, st, lookback, br, tab);
    Doubled<R> dbl;
    doubled_of(br, dbl);
    const OffsetSteps os = offset_steps(st, v);
    // elements of epoch br.m: their address, or (O32) the index of the first
    Addr abase;
    if constexpr (O32) abase = 0u;
    else abase = wdata;
    Addr ebase = abase + (int64_t)br.m * estride;
    int ebase_m = br.m;
    // (O32) the two epochs' loads: one byte offset from two bases
    GB *pb0 = (GB *)wdata, *pb1 = pb0 + second * (int64_t)sizeof(E);
    auto cell_addr = [&](Addr e) -> Addr {
        if constexpr (O32) return (e + r.off) << ESH;
        else return e + r.off;
    };
    A sum = 0, comp = 0;
    A xsum[NX], xcomp[NX];
#pragma unroll
    for (int c = 0; c < NX; c++) xsum[c] = xcomp[c] = 0;
    const int nx = VEC ? v.n_chan - 1 : 0;
    uint32_t count = 0;
    // A ray crosses at most n0 + n1 + n2 - 2 cells (in EX, each cell is cut at
    // most once more per epoch time and window end).  Every batch takes a cell
    // or piece of each live ray (SYNC == 0), or at least of the wavefront's
    // rearmost ray, so the batches are bounded; the bound only guards against
    // a walk that does not advance.
    int guard = (st.n[0] + st.n[1] + st.n[2] + (EX ? M + 3 : 1)) * (SYNC != 0 ? 64 : 1);
    R piece = -(R)INFINITY;  // EX: start of the part of the current cell not yet taken
    bool cell_counted = false;
    // Weights of the batch's cells.  A cell not taken keeps the weight of an
    // earlier batch (finite, and multiplied by a zero chord), so no default
    // is written per cell.
    A cw[K];
#pragma unroll
    for (int k = 0; k < K; k++) cw[k] = (A)0;

    for (;;) {
        if (--guard < 0) break;
        R lim = (R)0;  // depth-synchronous horizon: cells entered before it are taken
        if (SYNC != 0) {
            const R front = wave_min(alive ? r.entry : (R)INFINITY);
            if (front == (R)INFINITY) break;  // uniform: every ray has ended
            lim = front + gap;
            // (at least just past the rearmost entry, whatever the rounding)
            if (!(lim > front)) lim = nextafter(front, (R)INFINITY);
        } else if (!alive) {
            break;
        }
        Addr addr[K];
        A cds[K];  // chord, already in the accumulation type
#pragma unroll
        for (int k = 0; k < K; k++) {
            addr[k] = abase;  // a valid element for cells not taken in this batch
            cds[k] = (A)0;
            if (alive) {
                const R entry = r.entry;
                const R exit = fmin(r.sa0, fmin(r.sa1, r.sa2));
                // (a live ray's cell has entry < stop: checked at set-up and
                // by every step)
                if (EX && (SYNC == 0 || entry < lim)) {
                    // one piece [a, b] of the cell: from where the last piece
                    // ended (or the cell's entry, or the window's start) to the
                    // next epoch time or the end of cell or window
                    const R a = fmax(fmax(entry, piece), r_lo);
                    const R end = fmin(exit, r_hi);
                    bool more = false;
                    R b = a;
                    if (a < end) {
                        // bracket of the retarded times just below t_obs - a
                        bracket_seek_from(v, st, a, br, tab);
                        b = fmin(end, br.am);
                        more = b < end;
                    }
                    const R ds = b - a, mid = (R)0.5 * (a + b);
                    const bool contrib = ds > (R)0;
                    const R wt = (br.am - mid) * br.inv_dt;
                    if (br.m != ebase_m) {
                        ebase = abase + (int64_t)br.m * estride;
                        ebase_m = br.m;
                    }
                    addr[k] = cell_addr(ebase);
                    cds[k] = contrib ? (A)ds : (A)0;
                    cw[k] = (A)wt;
                    count += (contrib && !cell_counted) ? 1u : 0u;
                    cell_counted |= contrib;
                    if (more) {
                        piece = b;
                    } else {
                        piece = -(R)INFINITY;
                        cell_counted = false;
                        alive = ray_advance(os, r, exit);
                    }
                } else if (!EX && (SYNC == 0 || entry < lim)) {
                    // (the rearmost ray has entry == front < lim, so each batch
                    // takes at least one cell or ends a ray)
                    // The midpoint is kept doubled (one compare for the
                    // bracket, no halving), except by FP64 rays over whole
                    // records: there the doubled form made the compiler's
                    // schedule hold twice the registers (290 against 146)
                    const R ds = exit - entry;
                    const R mid2 = entry + exit, mid = (R)0.5 * mid2;
                    const bool contrib = ds > (R)0 && (DOUBLED ? in_window(mid2, lo2, hi2)
                                                                 : in_window(mid, r_lo, r_hi));
                    // (FP32 walks read the weight stored in FP32: no conversion
                    // per cell)
                    R wt = std::is_same<R, float>::value ? (R)v.fixed_wf : (R)v.fixed_w;
                    if (lookback) {
                        if constexpr (DOUBLED) {
                            bracket_seek2(v, st, mid2, br, dbl, tab, ebase, abase, estride);
                            wt = (dbl.am2 - mid2) * dbl.hdt;
                        } else {
                            bracket_seek(v, st, mid, br, tab, ebase, abase, estride);
                            wt = (br.am - mid) * br.inv_dt;
                        }
                    }
                    Addr e0 = ebase;
                    if constexpr (single) {
                        if (M >= 2) {
                            bool later;
                            if constexpr (DOUBLED)
                                later = lookback ? (mid2 - dbl.am1_2) < (dbl.am2 - mid2)
                                                 : wt > (R)0.5;
                            else
                                later = lookback ? (mid - br.am1) < (br.am - mid) : wt > (R)0.5;
                            if (later) e0 = ebase + estride;
                        }
                        wt = (R)0;
                    }
                    addr[k] = cell_addr(e0);
                    cds[k] = contrib ? (A)ds : (A)0;
                    cw[k] = (A)wt;
                    count += contrib ? 1u : 0u;
                    alive = ray_advance(os, r, exit);
                }
            }
        }
        Raw r0[K], r1[K];
        JF j0[K][NX], j1[K][NX];
        if constexpr (JP) {
            // Emissivity elements first.  When no element of the batch, on
            // any lane, carries the read-whole mark, every record it reads is
            // at rest with j >= 0 and the element is its j: the batch is
            // consumed from the elements with the arithmetic of the record
            // path, and its sums are bit for bit those of the records.
            // (Marks on cells that contribute nothing send the batch to the
            // marked path below too, which is never wrong, and saves a test
            // per cell.)
            // (16-bit elements held zero-extended, as loaded)
            using QJ = typename std::conditional<sizeof(JF) == 2, uint32_t, JF>::type;
            QJ q0[K], q1[K];
#pragma unroll
            for (int k = 0; k < K; k++) {
                if constexpr (O32) {
                    q0[k] = (QJ) * (GJ *)(pb0 + addr[k]);
                    q1[k] = (QJ) * (GJ *)(pb1 + addr[k]);
                } else {
                    q0[k] = (QJ)addr[k][0];
                    q1[k] = (QJ)addr[k][second];
                }
            }
            uint32_t any_bits = 0u;
#pragma unroll
            for (int k = 0; k < K; k++)
                any_bits |= jplane_bits<S>((JF)q0[k]) | jplane_bits<S>((JF)q1[k]);
            if (!__any(jplane_mark<S>(any_bits) != 0u)) {
#pragma unroll
                for (int k = 0; k < K; k++) {
                    const A val = lerp_d((A)decode_j<S>((JF)q0[k]), plane_diff<S>(q0[k], q1[k]), cw[k]);
                    const A term = cds[k] * val;
                    kahan_add(sum, comp, term, kahan);
                }
                continue;
            }
            // Whole records only of the marked elements.  An element without
            // the mark is its record's j (>= 0, at rest), whose Doppler factor
            // is exactly 1, so every sample below has the value the record
            // path gives it, bit for bit, and only the lanes and cells that
            // need a record load it.
            bool mk0[K], mk1[K];
#pragma unroll
            for (int k = 0; k < K; k++) {
                mk0[k] = jplane_mark<S>(jplane_bits<S>((JF)q0[k])) != 0u;
                mk1[k] = jplane_mark<S>(jplane_bits<S>((JF)q1[k])) != 0u;
                GRaw *ra;
                if constexpr (O32) ra = gdata + (addr[k] >> ESH);
                else ra = gdata + (addr[k] - wdata);
                r0[k] = Raw{};
                r1[k] = Raw{};
                if (mk0[k]) r0[k] = load_grec<S>(ra);
                if (mk1[k]) r1[k] = load_grec<S>(ra + second);
            }
#pragma unroll
            for (int k = 0; k < K; k++) {
                const A b0 = mk0[k] ? (A)boosted<S>(r0[k], v, beaming) : (A)decode_j<S>((JF)q0[k]);
                const A b1 = mk1[k] ? (A)boosted<S>(r1[k], v, beaming) : (A)decode_j<S>((JF)q1[k]);
                const A val = lerp_w(b0, b1, cw[k]);
                const A term = cds[k] * val;
                kahan_add(sum, comp, term, kahan);
            }
            continue;
        } else {
#pragma unroll
            for (int k = 0; k < K; k++) {
                r0[k] = load_grec<S>(addr[k]);
                r1[k] = load_grec<S>(addr[k] + second);
                if constexpr (VEC) {
                    // the same record index in the other components
                    const int64_t ri = addr[k] - wdata;
#pragma unroll
                    for (int c = 0; c < NX; c++) {
                        j0[k][c] = j1[k][c] = (JF)0;
                        if (c < nx) {
                            GJ *cd = (GJ *)v.chan_data[c];
                            j0[k][c] = cd[ri];
                            j1[k][c] = cd[ri + second];
                        }
                    }
                }
            }
        }
        // Every lane consumes all K cells: a cell not taken, past the end of
        // the ray or outside the window has ds = 0 (its records, validated at
        // load, are finite), and an unconditional use keeps the compiler from
        // sinking the loads back into a branch.
        //
        // When no record that contributes to the batch, on any lane of the
        // wavefront, has a velocity (the bulk of a jet's volume is at rest),
        // every Doppler factor is exactly 1: the batch is consumed without
        // decoding velocities, with the same arithmetic on j as the general
        // path (j * 1 = j), so the sums are bit for bit the same.
        bool at_rest = !beaming;
        if constexpr (!VEC) {
            if (beaming) {
                uint32_t moving = 0u;
#pragma unroll
                for (int k = 0; k < K; k++)
                    moving |= cds[k] != (A)0 ? (beta_bits<S>(r0[k]) | beta_bits<S>(r1[k])) : 0u;
                at_rest = !__any(moving != 0u);
            }
        }
        if (!VEC && at_rest) {
#pragma unroll
            for (int k = 0; k < K; k++) {
                const A val = lerp_w((A)record_j<S>(r0[k]), (A)record_j<S>(r1[k]), cw[k]);
                const A term = cds[k] * val;
                kahan_add(sum, comp, term, kahan);
            }
            continue;
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
            V f0 = V(1), f1 = V(1);
            A val, b1;
            if constexpr (VEC) {
                V jj0, jj1;
                f0 = boost_factor<S>(r0[k], v, beaming, jj0);
                f1 = boost_factor<S>(r1[k], v, beaming, jj1);
                val = (A)(jj0 * f0);
                b1 = (A)(jj1 * f1);
            } else {
                val = (A)boosted<S>(r0[k], v, beaming);
                b1 = (A)boosted<S>(r1[k], v, beaming);
            }
            val = lerp_w(val, b1, cw[k]);
            if constexpr (VEC) {
#pragma unroll
                for (int c = 0; c < NX; c++) {
                    if (c < nx) {
                        A xv = (A)(decode_j<S>(j0[k][c]) * f0);
                        const A xb = (A)(decode_j<S>(j1[k][c]) * f1);
                        xv = lerp_w(xv, xb, cw[k]);
                        const A xt = cds[k] * xv;
                        kahan_add(xsum[c], xcomp[c], xt, kahan);
                    }
                }
            }
            const A term = cds[k] * val;
            // a zero term leaves the compensated sum as it is, so cells not
            // taken in a batch do not perturb it (rounding of sum - comp)
            kahan_add(sum, comp, term, kahan);
        }
    }
    nsteps += count;
    if constexpr (VEC) {
#pragma unroll
        for (int c = 0; c < NX; c++) ext[c] = (double)xsum[c] - (double)xcomp[c];
    }
    return (double)sum - (double)comp;
}

template <int S, typename R, int SYNC, bool EX, int K, bool VEC = false, int JP = 0>
__device__ __forceinline__ double march(const RayView &v, const StackDev &st,
                                        const double *centre, int pi, int pj, bool in_image,
                                        const ldsdouble *tab, uint32_t &nsteps,
                                        double *ext = nullptr) {
    // uniform over the launch's view (flags, epoch count): a scalar branch
    if ((v.flags & F_NEAREST) || st.n_epochs == 1)
        return march_walk<S, R, SYNC, EX, K, VEC, true, JP>(v, st, centre, pi, pj, in_image, tab,
                                                             nsteps, ext);
    return march_walk<S, R, SYNC, EX, K, VEC, false, JP>(v, st, centre, pi, pj, in_image, tab,
                                                          nsteps, ext);
}

// Intensity of pixel (pi, pj): one march through the stack, or, for a labelled
// stack (LAB), one march through each of its sub-domains in order, summed
// (emission adds along the ray; sub-domains do not overlap).  The block loop
// is uniform over the wavefront, as the depth-synchronous mode needs.
// Vector stacks (VEC, never with LAB) also return components 1.. in ext.
template <int S, typename R, int SYNC, bool LAB, bool EX, int K, bool VEC = false,
          int JP = 0>
__device__ __forceinline__ double pixel_value(const RayView &v, int pi, int pj, bool in_image,
                                              const ldsdouble *tab, uint32_t &nsteps,
                                              double *ext = nullptr) {
    // (labelled stacks get kernels of their own: the block loop would
    // otherwise raise the register count, and lower the occupancy, of every
    // plain render)
    static_assert(!(LAB && VEC), "vector stacks are not labelled");
    static_assert(!(LAB && JP), "labelled stacks read whole records");
    if constexpr (!LAB) {
        return march<S, R, SYNC, EX, K, VEC, JP>(v, v.st, v.centre, pi, pj, in_image, tab, nsteps,
                                                 ext);
    } else {
        double acc = 0.0;
        for (int b = 0; b < v.n_blocks; b++)
            acc += march<S, R, SYNC, EX, K>(v, v.blocks[b].st, v.blocks[b].centre, pi, pj,
                                         in_image, tab, nsteps);
        return acc;
    }
}

// ------------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Pixel (pi, pj) of image plane c ([n_chan][height][width]; c = 0 for a
// scalar stack).
__device__ __forceinline__ void store_pixel(const RayView &v, int pi, int pj, double val,
                                            int c = 0) {
    const size_t o = ((size_t)c * v.height + pj) * v.width + pi;
    const bool add = (v.flags & F_ACCUMULATE) != 0;
    if (v.out_f64) {
        double *p = (double *)v.image + o;
        *p = add ? *p + val : val;
    } else {
        float *p = (float *)v.image + o;
        *p = add ? (float)((double)*p + val) : (float)val;
    }
}

// ------------------------------------------------------------------ kernels

// Plain kernel: one thread per pixel in row order, one launch per image.
template <int S, typename R, bool LAB, bool EX, bool VEC = false, int JP = 0>
__global__ void __launch_bounds__(256) k_plain(RayView v, double *flux_acc,
                                               unsigned long long *step_acc) {
    __shared__ double s_tab[4][2 * EPOCH_TAB_MAX];
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long npix = (long long)v.width * v.height;
    ldsdouble *tab = nullptr;
    if (v.st.n_epochs <= EPOCH_TAB_MAX) {
        tab = (ldsdouble *)&s_tab[threadIdx.x >> 6][0];
        epoch_tab_fill(tab, v.st, v.t_obs);
    }
    double val = 0.0;
    uint32_t ns = 0;
    if (idx < npix) {
        const int pi = (int)(idx % v.width), pj = (int)(idx / v.width);
        double ext[3];
        val = pixel_value<S, R, 0, LAB, EX, CELLS_PER_BATCH, VEC, JP>(v, pi, pj, true, tab, ns,
                                                                      ext);
        store_pixel(v, pi, pj, val);
        if constexpr (VEC)
            for (int c = 1; c < v.n_chan; c++) store_pixel(v, pi, pj, ext[c - 1], c);
    }
    const double fs = wave_sum(val);
    const uint32_t cs = wave_sum_u32(ns);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&flux_acc[v.acc_index], fs * v.ps * v.ps);
        atomicAdd(&step_acc[v.acc_index], (unsigned long long)cs);
    }
}

// Persistent kernel: every wavefront pulls 64-pixel tiles (tile_w x tile_h)
// from a queue until all are done.  Tiles are split into n_queues contiguous
// chunks (bounds from the planner); a wave starts on chunk (block index mod
// n_queues), which under
// round-robin workgroup dispatch is the chunk of its own XCD, and moves on to
// the other chunks when its own runs dry.
template <int S, typename R, int SYNC, bool LAB, bool EX, int K, bool VEC = false,
          int JP = 0>
__global__ void __launch_bounds__(256) k_batch(BatchLaunch bl,
                                               const RayView *__restrict__ views,
                                               const Tile *__restrict__ tiles) {
    // (descriptors through read-only, non-aliased pointers: uniform reads of
    // them become scalar loads instead of round trips through the vector
    // memory path that the gathers keep busy)
    __shared__ double s_tab[4][2 * EPOCH_TAB_MAX];
    ldsdouble *const wave_tab = (ldsdouble *)&s_tab[threadIdx.x >> 6][0];
    uint32_t tab_view = 0xffffffffu;  // view whose epochs the table holds
    const int lane = threadIdx.x & 63;
    const uint32_t nq = bl.n_queues;
    const uint32_t q0 = blockIdx.x % nq;
    for (uint32_t qi = 0; qi < nq;) {
        const uint32_t q = (q0 + qi) % nq;
        const uint32_t begin = bl.q_begin[q], end = bl.q_begin[q + 1];
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(&bl.head[q], 1u);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= end - begin) {
            qi++;
            continue;
        }
        const Tile tile = tiles[begin + t];
        const uint32_t vi = __builtin_amdgcn_readfirstlane(tile.view);
        const RayView &v = views[vi];
        const bool use_tab = v.st.n_epochs <= EPOCH_TAB_MAX;
        if (use_tab && vi != tab_view) {
            epoch_tab_fill(wave_tab, v.st, v.t_obs);
            tab_view = vi;
        }
        const uint32_t tw_log2 = (uint32_t)__builtin_amdgcn_readfirstlane(v.tile_w_log2);
        const int pi = (int)(__builtin_amdgcn_readfirstlane(tile.tx) << tw_log2) +
                       (lane & ((1 << tw_log2) - 1));
        const int pj = (int)(__builtin_amdgcn_readfirstlane(tile.ty) << (6 - tw_log2)) +
                       (lane >> tw_log2);
        uint32_t ns = 0;
        const bool in_image = pi < v.width && pj < v.height;
        double ext[3];
        const double val = pixel_value<S, R, SYNC, LAB, EX, K, VEC, JP>(
            v, pi, pj, in_image, use_tab ? wave_tab : nullptr, ns, ext);
        if (in_image) {
            store_pixel(v, pi, pj, val);
            if constexpr (VEC)
                for (int c = 1; c < v.n_chan; c++) store_pixel(v, pi, pj, ext[c - 1], c);
        }
        const double fs = wave_sum(val);
        const uint32_t cs = wave_sum_u32(ns);
        if (lane == 0) {
            atomicAdd(&bl.flux_acc[v.acc_index], fs * v.ps * v.ps);
            atomicAdd(&bl.step_acc[v.acc_index], (unsigned long long)cs);
        }
    }
}

// Zero fill of the tiles a batch does not march (every ray of them misses the
// grid): four 64-pixel tiles per 256-thread block, each lane one pixel in the
// tile layout of k_batch, every channel.
__global__ void __launch_bounds__(256) k_clear_tiles(const RayView *__restrict__ views,
                                                     const Tile *__restrict__ tiles, uint32_t n) {
    const uint32_t k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= n) return;
    const Tile tile = tiles[k];
    const RayView &v = views[tile.view];
    const int lane = threadIdx.x & 63;
    const uint32_t tw_log2 = (uint32_t)v.tile_w_log2;
    const int pi = (int)((uint32_t)tile.tx << tw_log2) + (lane & ((1 << tw_log2) - 1));
    const int pj = (int)((uint32_t)tile.ty << (6 - tw_log2)) + (lane >> tw_log2);
    if (pi < v.width && pj < v.height)
        for (int c = 0; c < v.n_chan; c++) store_pixel(v, pi, pj, 0.0, c);
}

// Sample marking for the compulsory-bytes count (untimed instrumentation).
template <int S, typename R>
__global__ void __launch_bounds__(256) k_mark(RayView v, uint32_t *bitmap, int line_log2,
                                              bool moving_only) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long npix = (long long)v.width * v.height;
    if (idx >= npix) return;
    mark_ray<S, R>(v, (int)(idx % v.width), (int)(idx / v.width), bitmap, line_log2, moving_only);
}

__global__ void __launch_bounds__(256) k_popcount(const uint32_t *bm, uint64_t words,
                                                  unsigned long long *out) {
    unsigned long long c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * blockDim.x)
        c += __popc(bm[i]);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, c);
}

// Emissivity fields of n records (the first field of each) into a packed
// array of the same indexing.
template <int S>
__global__ void __launch_bounds__(256) k_pack_j(const typename RecT<S>::raw *__restrict__ rec,
                                                typename JFieldT<S>::raw *__restrict__ out,
                                                uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if constexpr (S == ST_F64 || S == ST_F32) out[i] = rec[i].x;
        else out[i] = (unsigned short)(rec[i].x & 0xffffu);
    }
}

template <int S>
__global__ void __launch_bounds__(256) k_pack_jplane(const typename RecT<S>::raw *__restrict__ rec,
                                                     typename JFieldT<S>::raw *__restrict__ out,
                                                     uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = jplane_element<S>(rec[i]);
}

__global__ void __launch_bounds__(256) k_fill_u64(unsigned long long *p, uint64_t n,
                                                  unsigned long long value) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void __launch_bounds__(256) k_copy(float4 *__restrict__ dst,
                                              const float4 *__restrict__ src, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ------------------------------------------------------------------ load / convert

__device__ __forceinline__ uint32_t f2bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ uint32_t f2h_rne(float f) {
    return (uint32_t)__half_as_ushort(__float2half_rn(f));
}

// A value of the source type as an FP32 value that rounds to nearest even in
// one step to FP16 or BF16.  FP32 sources pass unchanged.  FP64 sources are
// rounded to FP32 by round-to-odd (truncate, then set the last bit if the
// truncation was inexact): with at least two more significant bits than the
// 16-bit format at every magnitude, the second rounding of a round-to-odd
// result equals a direct rounding of the FP64 value (Boldo and Melquiond,
// "Emulation of FMA and correctly rounded sums: proved algorithms using
// rounding to odd", IEEE Trans. Computers 57, 2008).
__device__ __forceinline__ float narrow_for16(float v) { return v; }
__device__ __forceinline__ float narrow_for16(double v) {
    float f = __double2float_rz(v);
    if ((double)f != v) f = __uint_as_float(__float_as_uint(f) | 1u);
    return f;
}

// caller layout (one epoch: j [nz][ny][nx], beta [nz][ny][nx][3]) -> resident
// records, with validation: every value finite, |beta| < 1 in the source type
// and again after rounding to the storage type.  The first bad element (as
// epoch * ncell + cell) is kept by atomicMin in *err.
template <typename Src, int S>
__global__ void __launch_bounds__(256) k_convert(const Src *__restrict__ j,
                                                 const Src *__restrict__ beta, int32_t m,
                                                 StackDev st, void *data,
                                                 unsigned long long *err) {
    const uint32_t n0 = st.n[0], n1 = st.n[1];
    const uint64_t ncell = (uint64_t)n0 * n1 * st.n[2];
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
         c += (uint64_t)gridDim.x * blockDim.x) {
        const double jv = (double)j[c];
        const double bx = (double)beta[3 * c], by = (double)beta[3 * c + 1],
                     bz = (double)beta[3 * c + 2];
        bool ok = isfinite(jv) && isfinite(bx) && isfinite(by) && isfinite(bz) &&
                  (bx * bx + by * by + bz * bz) < 1.0;
        const uint32_t x = (uint32_t)(c % n0), y = (uint32_t)((c / n0) % n1),
                       z = (uint32_t)(c / ((uint64_t)n0 * n1));
        const uint64_t rec = (uint64_t)m * st.epoch_stride + cell_offset(st, x, y, z);
        double qj, qx, qy, qz;
        if constexpr (S == ST_F64) {
            double2 *p = (double2 *)data;
            p[2 * rec] = double2{jv, bx};
            p[2 * rec + 1] = double2{by, bz};
            qj = jv; qx = bx; qy = by; qz = bz;
        } else if constexpr (S == ST_F32) {
            float4 r{(float)jv, (float)bx, (float)by, (float)bz};
            ((float4 *)data)[rec] = r;
            qj = r.x; qx = r.y; qy = r.z; qz = r.w;
        } else if constexpr (S == ST_F16) {
            const Src *bc = beta + 3 * c;
            uint32_t hj = f2h_rne(narrow_for16(j[c])), hx = f2h_rne(narrow_for16(bc[0])),
                     hy = f2h_rne(narrow_for16(bc[1])), hz = f2h_rne(narrow_for16(bc[2]));
            ((uint2 *)data)[rec] = uint2{hj | (hx << 16), hy | (hz << 16)};
            qj = h2f(hj); qx = h2f(hx); qy = h2f(hy); qz = h2f(hz);
        } else {
            const Src *bc = beta + 3 * c;
            uint32_t hj = f2bf16_rne(narrow_for16(j[c])), hx = f2bf16_rne(narrow_for16(bc[0])),
                     hy = f2bf16_rne(narrow_for16(bc[1])), hz = f2bf16_rne(narrow_for16(bc[2]));
            ((uint2 *)data)[rec] = uint2{hj | (hx << 16), hy | (hz << 16)};
            qj = __uint_as_float(hj << 16); qx = __uint_as_float(hx << 16);
            qy = __uint_as_float(hy << 16); qz = __uint_as_float(hz << 16);
        }
        // the stored velocity must stay strictly sub-luminal in the arithmetic
        // the render uses (FP64, and the FP32 FMA chain of 16-bit stacks)
        ok = ok && isfinite(qj) && (1.0 - (qx * qx + qy * qy + qz * qz)) > 0.0;
        if constexpr (S == ST_F16 || S == ST_BF16) {
            const float fx = (float)qx, fy = (float)qy, fz = (float)qz;
            ok = ok && fmaf(-fx, fx, fmaf(-fy, fy, fmaf(-fz, fz, 1.0f))) > 0.0f;
        }
        if (!ok) atomicMin(err, (unsigned long long)((uint64_t)m * ncell + c));
    }
}

template <int RB>
struct RawRec { uint32_t w[RB / 4]; };

template <int RB>
__global__ void __launch_bounds__(256) k_rebrick(StackDev from, StackDev to, int32_t m,
                                                 RawRec<RB> *__restrict__ dst) {
    const uint32_t n0 = from.n[0], n1 = from.n[1];
    const uint64_t ncell = (uint64_t)n0 * n1 * from.n[2];
    const RawRec<RB> *src = (const RawRec<RB> *)from.data;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
         c += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t x = (uint32_t)(c % n0), y = (uint32_t)((c / n0) % n1),
                       z = (uint32_t)(c / ((uint64_t)n0 * n1));
        dst[(uint64_t)m * to.epoch_stride + cell_offset(to, x, y, z)] =
            src[(uint64_t)m * from.epoch_stride + cell_offset(from, x, y, z)];
    }
}

// One epoch of resident records back in the caller's layout (j [nz][ny][nx],
// beta [nz][ny][nx][3]), each value widened exactly to Out (FP64 for FP64
// stacks, FP32 otherwise).
template <int S, typename Out>
__global__ void __launch_bounds__(256) k_read_epoch(StackDev st, int32_t m, Out *__restrict__ j,
                                                    Out *__restrict__ beta) {
    using Raw = typename RecT<S>::raw;
    using V = typename RecT<S>::val;
    const uint32_t n0 = st.n[0], n1 = st.n[1];
    const uint64_t ncell = (uint64_t)n0 * n1 * st.n[2];
    const Raw *src = (const Raw *)st.data;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
         c += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t x = (uint32_t)(c % n0), y = (uint32_t)((c / n0) % n1),
                       z = (uint32_t)(c / ((uint64_t)n0 * n1));
        const Raw r = src[(uint64_t)m * st.epoch_stride + cell_offset(st, x, y, z)];
        V vj, vx, vy, vz;
        decode<S, V>(r, vj, vx, vy, vz);
        j[c] = (Out)vj;
        beta[3 * c] = (Out)vx;
        beta[3 * c + 1] = (Out)vy;
        beta[3 * c + 2] = (Out)vz;
    }
}

// ------------------------------------------------------------------ launchers

static inline unsigned grid_for(uint64_t n, unsigned cap = 1u << 16) {
    uint64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

template <int S, typename R>
static hipError_t plain_impl(const RayView &v, double *flux_acc, unsigned long long *step_acc,
                             hipStream_t s) {
    const dim3 g((unsigned)(((uint64_t)v.width * v.height + 255) / 256)), b(256);
    const bool lab = v.n_blocks > 0, ex = (v.flags & F_EXACT) != 0;
    if constexpr (S != ST_F64) {
        // (the planner gives an emissivity plane only to plain stacks)
        if (v.st.jplane && !lab && v.n_chan == 1) {
            if (v.flags & F_PLANE32) {
                if (ex) hipLaunchKernelGGL((k_plain<S, R, false, true, false, 2>), g, b, 0, s, v, flux_acc, step_acc);
                else hipLaunchKernelGGL((k_plain<S, R, false, false, false, 2>), g, b, 0, s, v, flux_acc, step_acc);
            } else {
                if (ex) hipLaunchKernelGGL((k_plain<S, R, false, true, false, 1>), g, b, 0, s, v, flux_acc, step_acc);
                else hipLaunchKernelGGL((k_plain<S, R, false, false, false, 1>), g, b, 0, s, v, flux_acc, step_acc);
            }
            return hipGetLastError();
        }
    }
    if (v.n_chan > 1) hipLaunchKernelGGL((k_plain<S, R, false, false, true>), g, b, 0, s, v, flux_acc, step_acc);
    else if (lab && ex) hipLaunchKernelGGL((k_plain<S, R, true, true>), g, b, 0, s, v, flux_acc, step_acc);
    else if (lab) hipLaunchKernelGGL((k_plain<S, R, true, false>), g, b, 0, s, v, flux_acc, step_acc);
    else if (ex) hipLaunchKernelGGL((k_plain<S, R, false, true>), g, b, 0, s, v, flux_acc, step_acc);
    else hipLaunchKernelGGL((k_plain<S, R, false, false>), g, b, 0, s, v, flux_acc, step_acc);
    return hipGetLastError();
}

hipError_t launch_plain(const RayView &v, double *flux_acc, unsigned long long *step_acc,
                        hipStream_t s) {
    const bool f64 = (v.flags & F_F64_DDA) != 0;
    switch (v.st.store) {
        case ST_F64: return plain_impl<ST_F64, double>(v, flux_acc, step_acc, s);
        case ST_F32: return f64 ? plain_impl<ST_F32, double>(v, flux_acc, step_acc, s)
                                : plain_impl<ST_F32, float>(v, flux_acc, step_acc, s);
        case ST_F16: return f64 ? plain_impl<ST_F16, double>(v, flux_acc, step_acc, s)
                                : plain_impl<ST_F16, float>(v, flux_acc, step_acc, s);
        case ST_BF16: return f64 ? plain_impl<ST_BF16, double>(v, flux_acc, step_acc, s)
                                 : plain_impl<ST_BF16, float>(v, flux_acc, step_acc, s);
    }
    return hipErrorInvalidValue;
}

template <int S, typename R, int SYNC, bool LAB, bool EX, int JP = 0>
static void batch_launch_k(const BatchLaunch &bl, bool k8, int grid_blocks, hipStream_t s) {
    const dim3 g((unsigned)grid_blocks), b(256);
    if (k8)
        hipLaunchKernelGGL((k_batch<S, R, SYNC, LAB, EX, 8, false, JP>), g, b, 0, s, bl, bl.views,
                           bl.tiles);
    else
        hipLaunchKernelGGL((k_batch<S, R, SYNC, LAB, EX, 4, false, JP>), g, b, 0, s, bl, bl.views,
                           bl.tiles);
}

template <int S, typename R>
static hipError_t batch_impl(const BatchLaunch &bl, int variant, int grid_blocks, hipStream_t s) {
    const bool k8 = (variant & KV_K8) != 0;
    if (variant & KV_VEC) {
        // vector stacks: own marching mode only (no depth sync, labels or
        // exact time)
        const dim3 g((unsigned)grid_blocks), b(256);
        if (k8)
            hipLaunchKernelGGL((k_batch<S, R, 0, false, false, 8, true>), g, b, 0, s, bl, bl.views,
                               bl.tiles);
        else
            hipLaunchKernelGGL((k_batch<S, R, 0, false, false, 4, true>), g, b, 0, s, bl, bl.views,
                               bl.tiles);
        return hipGetLastError();
    }
    if constexpr (S != ST_F64) {
        if ((variant & KV_JP) && (variant & KV_JP32)) {
            switch (variant & 7) {
                case 0: batch_launch_k<S, R, 0, false, false, 2>(bl, k8, grid_blocks, s); break;
                case 1: batch_launch_k<S, R, 1, false, false, 2>(bl, k8, grid_blocks, s); break;
                case 4: batch_launch_k<S, R, 0, false, true, 2>(bl, k8, grid_blocks, s); break;
                case 5: batch_launch_k<S, R, 1, false, true, 2>(bl, k8, grid_blocks, s); break;
                default: return hipErrorInvalidValue;  // (labelled stacks read whole records)
            }
            return hipGetLastError();
        }
        if (variant & KV_JP) {
            switch (variant & 7) {
                case 0: batch_launch_k<S, R, 0, false, false, 1>(bl, k8, grid_blocks, s); break;
                case 1: batch_launch_k<S, R, 1, false, false, 1>(bl, k8, grid_blocks, s); break;
                case 4: batch_launch_k<S, R, 0, false, true, 1>(bl, k8, grid_blocks, s); break;
                case 5: batch_launch_k<S, R, 1, false, true, 1>(bl, k8, grid_blocks, s); break;
                default: return hipErrorInvalidValue;  // (labelled stacks read whole records)
            }
            return hipGetLastError();
        }
    }
    switch (variant & 7) {
        case 0: batch_launch_k<S, R, 0, false, false>(bl, k8, grid_blocks, s); break;
        case 1: batch_launch_k<S, R, 1, false, false>(bl, k8, grid_blocks, s); break;
        case 2: batch_launch_k<S, R, 0, true, false>(bl, k8, grid_blocks, s); break;
        case 3: batch_launch_k<S, R, 1, true, false>(bl, k8, grid_blocks, s); break;
        case 4: batch_launch_k<S, R, 0, false, true>(bl, k8, grid_blocks, s); break;
        case 5: batch_launch_k<S, R, 1, false, true>(bl, k8, grid_blocks, s); break;
        case 6: batch_launch_k<S, R, 0, true, true>(bl, k8, grid_blocks, s); break;
        default: batch_launch_k<S, R, 1, true, true>(bl, k8, grid_blocks, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_batch(int store, bool f64, int variant, const BatchLaunch &bl, int grid_blocks,
                        hipStream_t s) {
    switch (store) {
        case ST_F64: return batch_impl<ST_F64, double>(bl, variant, grid_blocks, s);
        case ST_F32: return f64 ? batch_impl<ST_F32, double>(bl, variant, grid_blocks, s)
                                : batch_impl<ST_F32, float>(bl, variant, grid_blocks, s);
        case ST_F16: return f64 ? batch_impl<ST_F16, double>(bl, variant, grid_blocks, s)
                                : batch_impl<ST_F16, float>(bl, variant, grid_blocks, s);
        case ST_BF16: return f64 ? batch_impl<ST_BF16, double>(bl, variant, grid_blocks, s)
                                 : batch_impl<ST_BF16, float>(bl, variant, grid_blocks, s);
    }
    return hipErrorInvalidValue;
}

template <int S, typename R>
static hipError_t mark_impl(const RayView &v, uint32_t *bitmap, int line_log2, bool moving_only,
                            hipStream_t s) {
    const uint64_t npix = (uint64_t)v.width * v.height;
    hipLaunchKernelGGL((k_mark<S, R>), dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, s, v,
                       bitmap, line_log2, moving_only);
    return hipGetLastError();
}

hipError_t launch_mark(const RayView &v, uint32_t *bitmap, int line_log2, bool moving_only,
                       hipStream_t s) {
    const bool f64 = (v.flags & F_F64_DDA) != 0;
    const bool mo = moving_only;
    switch (v.st.store) {
        case ST_F64: return mark_impl<ST_F64, double>(v, bitmap, line_log2, mo, s);
        case ST_F32: return f64 ? mark_impl<ST_F32, double>(v, bitmap, line_log2, mo, s)
                                : mark_impl<ST_F32, float>(v, bitmap, line_log2, mo, s);
        case ST_F16: return f64 ? mark_impl<ST_F16, double>(v, bitmap, line_log2, mo, s)
                                : mark_impl<ST_F16, float>(v, bitmap, line_log2, mo, s);
        case ST_BF16: return f64 ? mark_impl<ST_BF16, double>(v, bitmap, line_log2, mo, s)
                                 : mark_impl<ST_BF16, float>(v, bitmap, line_log2, mo, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_popcount(const uint32_t *bitmap, uint64_t words, unsigned long long *out,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_popcount, dim3(grid_for(words, 8192)), dim3(256), 0, s, bitmap, words,
                       out);
    return hipGetLastError();
}

template <typename Src, int S>
static hipError_t convert_impl(const void *j, const void *beta, int32_t m0, int32_t count,
                               const StackDev &st, void *data, unsigned long long *err,
                               hipStream_t s) {
    const uint64_t ncell = (uint64_t)st.n[0] * st.n[1] * st.n[2];
    const unsigned g = grid_for(ncell, 1u << 15);
    for (int32_t q = 0; q < count; q++) {
        hipLaunchKernelGGL((k_convert<Src, S>), dim3(g), dim3(256), 0, s,
                           (const Src *)j + (size_t)q * ncell,
                           (const Src *)beta + (size_t)q * ncell * 3, m0 + q, st, data, err);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_convert(int src_f64, int store, const void *j, const void *beta, int32_t m0,
                          int32_t count, const StackDev &st, void *data,
                          unsigned long long *err, hipStream_t s) {
    if (src_f64) {
        switch (store) {
            case ST_F64: return convert_impl<double, ST_F64>(j, beta, m0, count, st, data, err, s);
            case ST_F32: return convert_impl<double, ST_F32>(j, beta, m0, count, st, data, err, s);
            case ST_F16: return convert_impl<double, ST_F16>(j, beta, m0, count, st, data, err, s);
            case ST_BF16: return convert_impl<double, ST_BF16>(j, beta, m0, count, st, data, err, s);
        }
    } else {
        switch (store) {
            case ST_F64: return convert_impl<float, ST_F64>(j, beta, m0, count, st, data, err, s);
            case ST_F32: return convert_impl<float, ST_F32>(j, beta, m0, count, st, data, err, s);
            case ST_F16: return convert_impl<float, ST_F16>(j, beta, m0, count, st, data, err, s);
            case ST_BF16: return convert_impl<float, ST_BF16>(j, beta, m0, count, st, data, err, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int RB>
static hipError_t rebrick_impl(const StackDev &from, const StackDev &to, void *dst,
                               hipStream_t s) {
    const uint64_t ncell = (uint64_t)from.n[0] * from.n[1] * from.n[2];
    for (int32_t m = 0; m < from.n_epochs; m++) {
        hipLaunchKernelGGL((k_rebrick<RB>), dim3(grid_for(ncell, 1u << 15)), dim3(256), 0, s,
                           from, to, m, (RawRec<RB> *)dst);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_rebrick(int store, const StackDev &from, const StackDev &to, void *dst,
                          hipStream_t s) {
    switch (store) {
        case ST_F64: return rebrick_impl<32>(from, to, dst, s);
        case ST_F32: return rebrick_impl<16>(from, to, dst, s);
        case ST_F16:
        case ST_BF16: return rebrick_impl<8>(from, to, dst, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_read_epoch(const StackDev &st, int32_t m, void *j, void *beta, hipStream_t s) {
    const uint64_t ncell = (uint64_t)st.n[0] * st.n[1] * st.n[2];
    const dim3 g(grid_for(ncell, 1u << 15)), b(256);
    switch (st.store) {
        case ST_F64:
            hipLaunchKernelGGL((k_read_epoch<ST_F64, double>), g, b, 0, s, st, m, (double *)j,
                               (double *)beta);
            break;
        case ST_F32:
            hipLaunchKernelGGL((k_read_epoch<ST_F32, float>), g, b, 0, s, st, m, (float *)j,
                               (float *)beta);
            break;
        case ST_F16:
            hipLaunchKernelGGL((k_read_epoch<ST_F16, float>), g, b, 0, s, st, m, (float *)j,
                               (float *)beta);
            break;
        case ST_BF16:
            hipLaunchKernelGGL((k_read_epoch<ST_BF16, float>), g, b, 0, s, st, m, (float *)j,
                               (float *)beta);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack_j(int store, const void *records, void *out, uint64_t n, hipStream_t s) {
    const dim3 g(grid_for(n, 1u << 15)), b(256);
    switch (store) {
        case ST_F64:
            hipLaunchKernelGGL(k_pack_j<ST_F64>, g, b, 0, s, (const rec_f64 *)records, (double *)out, n);
            break;
        case ST_F32:
            hipLaunchKernelGGL(k_pack_j<ST_F32>, g, b, 0, s, (const rec_f32 *)records, (float *)out, n);
            break;
        case ST_F16:
            hipLaunchKernelGGL(k_pack_j<ST_F16>, g, b, 0, s, (const rec_h16 *)records,
                               (unsigned short *)out, n);
            break;
        case ST_BF16:
            hipLaunchKernelGGL(k_pack_j<ST_BF16>, g, b, 0, s, (const rec_h16 *)records,
                               (unsigned short *)out, n);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pack_jplane(int store, const void *records, void *out, uint64_t n,
                              hipStream_t s) {
    const dim3 g(grid_for(n, 1u << 15)), b(256);
    switch (store) {
        case ST_F32:
            hipLaunchKernelGGL(k_pack_jplane<ST_F32>, g, b, 0, s, (const rec_f32 *)records,
                               (float *)out, n);
            break;
        case ST_F16:
            hipLaunchKernelGGL(k_pack_jplane<ST_F16>, g, b, 0, s, (const rec_h16 *)records,
                               (unsigned short *)out, n);
            break;
        case ST_BF16:
            hipLaunchKernelGGL(k_pack_jplane<ST_BF16>, g, b, 0, s, (const rec_h16 *)records,
                               (unsigned short *)out, n);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_clear_tiles(const RayView *views, const Tile *tiles, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_tiles, dim3((n + 3) / 4), dim3(256), 0, s, views, tiles, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n, unsigned long long value,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 4096)), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, uint64_t bytes, hipStream_t s) {
    const uint64_t n = bytes / 16;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n, 1u << 14)), dim3(256), 0, s, (float4 *)dst,
                       (const float4 *)src, n);
    return hipGetLastError();
}

}  // namespace dart
