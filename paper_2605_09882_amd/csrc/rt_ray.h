// Device-side walk of one ray through the leaf-only linear octree, shared
// by the kernels of this library (compiled into each HIP source that
// includes it).
//
// Walk of one ray (sec. 2.3.1 DDA + Morton lookup, sec. 2.3.2 slab chord),
// the step definition of the CPU reference, in FP64 and bit-identical to it:
//   probe p = floor(Q 2^D) (integer finest cell);
//   loop: k = Morton(p); i = leaf holding k (largest key <= k);
//         edge = 2^(D - level_i);
//         anchor = p rounded down to the edge;
//         far-plane times tf_a = (plane_a h - Q_a) / m_a for bounding axes
//         (1/m_a finite), +inf for the others;
//         t_out = min(tf_x, tf_y, tf_z) in that order;
//         l = t_out - t_in (clamped at 0, t_in kept), accumulate rho_i l;
//         axes with tf_a == t_out step to the neighbour cell, the others
//         take floor(fma(m_a, t_out, Q_a) 2^D) clamped to the leaf;
//         stop when p leaves [0, 2^D)^3.
// The kernel evaluates the same roundings with fewer operations: with
// Qs = Q 2^D, ms = m 2^D and ih = (1/m) 2^-D (exact power-of-two scalings),
//   (plane h - Q) (1/m) == (plane - Qs) ih   and
//   fma(m, t, Q) 2^D   == fma(ms, t, Qs)
// hold bit for bit, because scaling by a power of two commutes with
// rounding (no operand here is subnormal or overflows for directions with
// |m_a| <= 2^1000).  Non-bounding axes get ih = +inf and the upper face as
// plane (which lies strictly above Qs), so their far time is +inf without a
// select.  Sources that include this header are compiled with
// -ffp-contract=off: every FP operation rounds as written.
#pragma once

#include "rt_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace rt {
namespace ray {

constexpr int kBlock = 256;         // threads per block of every walk kernel
constexpr int kLutBits = 10;        // Morton spread table covers depths <= 10

// ---------------------------------------------------------------------
// Morton keys: spread the bits of each coordinate three apart.
// ---------------------------------------------------------------------

__device__ __forceinline__ uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ uint64_t spread21(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// (a << s) | b in one instruction (the compiler splits it when the operands
// arrive from separate loads).
__device__ __forceinline__ uint32_t shl_or(uint32_t a, int s, uint32_t b) {
    uint32_t r;
    asm("v_lshl_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "i"(s), "v"(b));
    return r;
}

// 32-bit keys (depth <= 10) read the spread bits from a table in LDS.
__device__ __forceinline__ uint32_t morton(const uint32_t *lut, int x, int y, int z, uint32_t) {
    return shl_or(lut[z], 2, shl_or(lut[y], 1, lut[x]));
}

__device__ __forceinline__ uint64_t morton(const uint32_t *, int x, int y, int z, uint64_t) {
    return spread21((uint64_t)x) | (spread21((uint64_t)y) << 1) | (spread21((uint64_t)z) << 2);
}

template <typename KeyT>
struct Tree {
    const KeyT *__restrict__ keys;      // n + 1 keys (sentinel 8^D last)
    const uint8_t *__restrict__ levels;  // n leaf levels
    const uint32_t *__restrict__ top;   // 8^top_level + 1 leaf indices
    KeyT cell_mask;  // 8^(depth - top_level) - 1: keys per table cell, minus one
    int depth;
    int top_shift;  // 3 * (depth - top_level)
};

// Fills the block's Morton spread table (32-bit keys only); all threads of
// the block must call it.
template <typename KeyT>
__device__ __forceinline__ void init_lut(uint32_t *lut, int depth) {
    if (sizeof(KeyT) == 4) {
        for (int j = threadIdx.x; j < (1 << depth); j += blockDim.x) lut[j] = spread10((uint32_t)j);
    }
    __syncthreads();
}

// The leaf holding key k: the largest index i with keys[i] <= k, and its
// level.  top[c] locates the level-top_level cell c of k: its flags say
// whether the cell is refined to depth D everywhere (the leaf follows from
// the key's offset in the cell, at level D) or covered by one leaf.
// Otherwise the cell's leaves are top[c] .. top[c+1]-1 (a leaf starting
// before the next cell's first key and reaching into it would be coarser
// than the cell and cover all of it), found by binary search.
template <typename KeyT>
__device__ __forceinline__ uint32_t find_leaf(const Tree<KeyT> &t, KeyT k, int &level) {
    const uint32_t c = (uint32_t)(k >> t.top_shift);
    const uint32_t e = t.top[c];
    if (e & kTopFull) {
        level = t.depth;
        // e = index | kTopFull (the only flag a full cell carries)
        return e + (uint32_t)(k & t.cell_mask) - kTopFull;
    }
    uint32_t lo = e & kTopIndex;
    if (!(e & kTopOne)) {
        uint32_t hi = t.top[c + 1] & kTopIndex;
        while (hi - lo > 1u) {
            const uint32_t mid = (lo + hi) >> 1;
            if (t.keys[mid] <= k)
                lo = mid;
            else
                hi = mid;
        }
    }
    level = t.levels[lo];
    return lo;
}

// ---------------------------------------------------------------------
// State of one ray and one step of its walk
// ---------------------------------------------------------------------

struct Ray {
    double qx, qy, qz;  // Q 2^D
    double mx, my, mz;  // m 2^D
    double ix, iy, iz;  // (1/m) 2^-D, +inf for non-bounding axes
    int ux, uy, uz;     // 1: far plane is the upper face (m > 0, or non-bounding); 0: lower
    int cx, cy, cz;     // probe cell
    double t_in;
    int steps;
};

// Sets up the ray; false for an invalid ray (source outside [0,1)^3,
// non-finite direction, or no bounding axis).
__device__ __forceinline__ bool ray_init(Ray &r, int depth, const double *q, const double *m) {
    const double scale = (double)(1 << depth);  // 2^D
    const double h = 1.0 / scale;               // 2^-D
    const double Qx = q[0], Qy = q[1], Qz = q[2];
    const double Mx = m[0], My = m[1], Mz = m[2];
    if (!(Qx >= 0.0 && Qx < 1.0 && Qy >= 0.0 && Qy < 1.0 && Qz >= 0.0 && Qz < 1.0)) return false;
    if (!(isfinite(Mx) && isfinite(My) && isfinite(Mz))) return false;
    const double inx = 1.0 / Mx, iny = 1.0 / My, inz = 1.0 / Mz;
    const bool bx = isfinite(inx), by = isfinite(iny), bz = isfinite(inz);
    if (!(bx || by || bz)) return false;
    r.qx = Qx * scale;
    r.qy = Qy * scale;
    r.qz = Qz * scale;
    r.mx = Mx * scale;
    r.my = My * scale;
    r.mz = Mz * scale;
    r.ix = bx ? inx * h : (double)INFINITY;
    r.iy = by ? iny * h : (double)INFINITY;
    r.iz = bz ? inz * h : (double)INFINITY;
    r.ux = (!bx || Mx > 0.0) ? 1 : 0;
    r.uy = (!by || My > 0.0) ? 1 : 0;
    r.uz = (!bz || Mz > 0.0) ? 1 : 0;
    r.cx = (int)floor(r.qx);
    r.cy = (int)floor(r.qy);
    r.cz = (int)floor(r.qz);
    r.t_in = 0.0;
    r.steps = 0;
    return true;
}

// Integer helpers of the step, each one VALU instruction on gfx950.
// (x << s) + a
__device__ __forceinline__ int shl_add(int x, int s, int a) {
    return (int)((uint32_t)x << s) + a;
}
// a + b - 1.  (Written out, the compiler keeps b - 1 of the per-ray b in
// registers of its own for the whole walk; volatile keeps the instruction
// where it stands rather than inside a branch.)
__device__ __forceinline__ int add_m1(int a, int b) {
    int r;
    asm volatile("v_add3_u32 %0, %1, %2, -1" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
// x clamped to [lo, hi] (lo <= hi): the median of the three.  (The compiler
// forms v_med3_i32 only for constant bounds; min(max()) would be two.)
__device__ __forceinline__ int med3(int x, int lo, int hi) {
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}
// max(a, b) of two doubles that are never NaN: the plain v_max_f64.  (fmax
// first quiets its operands, two more instructions, because the compiler
// cannot tell that a loop-carried value is never a signalling NaN.)
__device__ __forceinline__ double max_nonnan(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// First half of a step: the leaf that holds the probe, and its level.
template <typename KeyT>
__device__ __forceinline__ uint32_t ray_locate(const Ray &r, const Tree<KeyT> &t,
                                               const uint32_t *lut, int &level) {
    return find_leaf(t, morton(lut, r.cx, r.cy, r.cz, KeyT(0)), level);
}

// Second half: the chord l of the ray in leaf i, and the probe moved into
// the next cell; done is set when it has left the box.  The leaf value is
// not needed here, so its load (issued by the caller between the halves)
// overlaps with this arithmetic.
//
// The integer forms below give the cells of the step definition exactly.  With the leaf
// edge 2^sh and anchor a = c & -2^sh, the far plane is a + 2^sh on an upper
// face and a on a lower one, i.e. a + (u << sh).  An exit axis moves to
// a + 2^sh (up) or a - 1 (down), i.e. plane + u - 1.  Another axis takes the
// floor of its position clamped to [a, a + 2^sh - 1]; truncation gives the
// same clamped cell, since the two differ only below 0 <= a.  In a finest
// leaf (sh = 0) that clamp leaves the probe's own cell, so only the exit
// axes move (a plain DDA step).
template <typename KeyT>
__device__ __forceinline__ void ray_advance(Ray &r, const Tree<KeyT> &t, int level, double &l,
                                            bool &done) {
    const int sh = t.depth - level;
    const int msk = (int)(0xffffffffu << sh);  // -2^sh
    const int ax = r.cx & msk, ay = r.cy & msk, az = r.cz & msk;
    const int px = shl_add(r.ux, sh, ax), py = shl_add(r.uy, sh, ay), pz = shl_add(r.uz, sh, az);
    // the cell an exit axis moves to
    const int ex_x = add_m1(px, r.ux), ex_y = add_m1(py, r.uy), ex_z = add_m1(pz, r.uz);

    // slab method: far planes of the leaf's box along the ray
    const double tfx = ((double)px - r.qx) * r.ix;
    const double tfy = ((double)py - r.qy) * r.iy;
    const double tfz = ((double)pz - r.qz) * r.iz;
    // min in the order x, y, z; the far times are never +0 (a zero far time
    // is (0) * (negative 1/m) = -0) nor NaN, so fmin returns the same bits
    // as the compare chain
    const double t_out = fmin(fmin(tfx, tfy), tfz);

    // chord, clamped at 0: t_in moves to t_out unless rounding put t_out
    // behind it (max(t_in, t_out) - t_in is t_out - t_in or a zero; a zero
    // chord's sign never changes a sum)
    const double t_next = max_nonnan(r.t_in, t_out);
    l = t_next - r.t_in;
    r.t_in = t_next;
    ++r.steps;

    int nx = r.cx, ny = r.cy, nz = r.cz;
    if (sh != 0) {
        // the anchors again, from a copy of the mask the compiler cannot
        // see through: it would otherwise keep the three anchors live across
        // the slab arithmetic, in registers that bound the occupancy
        int m = msk;
        asm("" : "+v"(m));
        const int bx = r.cx & m, by = r.cy & m, bz = r.cz & m;
        const int hi = ~m;  // 2^sh - 1
        nx = med3((int)fma(r.mx, t_out, r.qx), bx, bx + hi);
        ny = med3((int)fma(r.my, t_out, r.qy), by, by + hi);
        nz = med3((int)fma(r.mz, t_out, r.qz), bz, bz + hi);
    }
    r.cx = tfx == t_out ? ex_x : nx;
    r.cy = tfy == t_out ? ex_y : ny;
    r.cz = tfz == t_out ? ex_z : nz;
    const unsigned side = 1u << t.depth;
    done = ((unsigned)r.cx >= side) | ((unsigned)r.cy >= side) | ((unsigned)r.cz >= side);
}

// Walks a whole ray; the visitor fetches what it needs of leaf i
// (Visitor::fetch) as soon as i is known and sees every visited leaf in
// order (Visitor::step).  Returns the number of leaves, or -1 for an
// invalid ray or one longer than the 3 * 2^D + 3 steps a valid walk takes.
template <bool kCount = false, typename KeyT, typename Visitor>
__device__ __forceinline__ int walk_ray(const Tree<KeyT> &t, const uint32_t *lut,
                                        const double *q, const double *m, Visitor &v) {
    Ray r;
    if (!ray_init(r, t.depth, q, m)) return -1;
    const int max_steps = 3 * (1 << t.depth) + 3;
    // one step; true when the ray has left the box
    auto step = [&]() {
        int level;
        const uint32_t i = ray_locate(r, t, lut, level);
        const auto value = v.fetch(i);
        double l;
        bool done;
        ray_advance(r, t, level, l, done);
        v.step(value, i, l);
        return done;
    };
    // two steps per iteration: the loop-carried values then alternate
    // between two registers instead of being copied back every step
    for (;;) {
        if (r.steps >= max_steps) return -1;
        if (step()) break;
        if (r.steps >= max_steps) return -1;
        if (step()) break;
    }
    return kCount ? r.steps : 0;
}

// ---------------------------------------------------------------------
// Visitors
// ---------------------------------------------------------------------

struct SumF64 {
    const double *__restrict__ rho;
    double N;
    __device__ __forceinline__ double fetch(uint32_t i) const { return rho[i]; }
    __device__ __forceinline__ void step(double r, uint32_t, double l) { N = N + r * l; }
};

struct SumF32Kahan {
    const float *__restrict__ rho;
    float S, c;
    // 32-bit byte offset (fewer than 2^30 leaves): one shift, no 64-bit
    // address arithmetic
    __device__ __forceinline__ float fetch(uint32_t i) const {
        return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(rho) + (i << 2));
    }
    __device__ __forceinline__ void step(float r, uint32_t, double l) {
        const float y = r * (float)l - c;
        const float t = S + y;
        c = (t - S) - y;
        S = t;
    }
};

struct HashSteps {
    uint64_t h;
    __device__ __forceinline__ int fetch(uint32_t) const { return 0; }
    __device__ __forceinline__ void step(int, uint32_t i, double) {
        h = (h ^ (uint64_t)i) * 0x100000001b3ull;
    }
};

struct RecordVisits {
    int32_t *__restrict__ out;
    int64_t cap;
    int64_t n;
    __device__ __forceinline__ int fetch(uint32_t) const { return 0; }
    __device__ __forceinline__ void step(int, uint32_t i, double) {
        if (n < cap) out[n] = (int32_t)i;
        ++n;
    }
};

struct RayIndex {
    int64_t s, d, off;
};

__device__ __forceinline__ RayIndex ray_index(const RayBatch &r, int64_t ray) {
    RayIndex x;
    x.d = ray / r.n_src;
    x.s = ray - x.d * r.n_src;
    x.off = x.s * r.stride_src + x.d * r.stride_dir;
    return x;
}

template <typename KeyT>
inline Tree<KeyT> tree_of(const TreeView &v) {
    Tree<KeyT> t;
    t.keys = static_cast<const KeyT *>(v.keys);
    t.levels = v.levels;
    t.top = v.top;
    t.depth = v.depth;
    t.top_shift = 3 * (v.depth - v.top_level);
    // keys per table cell; beyond 2^32 no cell can hold that many leaves
    const int bits = 3 * (v.depth - v.top_level);
    t.cell_mask = bits >= 8 * (int)sizeof(KeyT) ? (KeyT)~KeyT(0) : (KeyT)((KeyT(1) << bits) - 1);
    return t;
}

// Blocks for total work items, one per thread: a dispatch counts its work
// items in 32 bits, so larger launches are capped there and the kernels'
// grid-stride loops take the rest.
inline unsigned grid_for(int64_t total) {
    int64_t blocks = (total + kBlock - 1) / kBlock;
    const int64_t cap = (((int64_t)1 << 32) - 1) / kBlock;
    return (unsigned)(blocks < cap ? blocks : cap);
}

}  // namespace ray
}  // namespace rt
