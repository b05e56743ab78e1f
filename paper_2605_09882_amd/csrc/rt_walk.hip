// HIP kernels of the reverse ray walk for gfx950 (MI355X).
//
// One ray per lane.  Rays are numbered r = d * n_src + s (direction-major),
// so the 64 lanes of a wavefront carry consecutive sources in one direction:
// with Morton-ordered sources their rays run parallel through a compact
// neighbourhood, share leaves and key-search probes in cache, and store
// their results to consecutive addresses when stride_src = 1.
//
// Walk of one ray (sec. 2.3.1 DDA + Morton lookup, sec. 2.3.2 slab chord),
// the same step definition as the CPU reference, in FP64 with no
// floating-point contraction (this file is compiled with -ffp-contract=off;
// the one fused multiply-add of the position update is written as fma):
//   probe p = floor(Q 2^D) (integer finest cell);
//   loop: k = Morton(p); i = leaf holding k (largest key <= k);
//         edge = 2^(D - level), with 8^(D-level) = key[i+1] - key[i];
//         anchor = p rounded down to the edge;
//         far-plane times tf_a = (plane_a h - Q_a) / m_a for bounding axes
//         (1/m_a finite), taken from a per-ray reciprocal;
//         t_out = min(tf_x, tf_y, tf_z) in that order;
//         l = t_out - t_in (clamped at 0), accumulate rho_i l;
//         axes with tf_a == t_out step to the neighbour cell, the others
//         take floor(fma(m_a, t_out, Q_a) 2^D) clamped to the leaf;
//         stop when p leaves [0, 2^D)^3.
#include "rt_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace rt {
namespace {

constexpr int kBlock = 256;
constexpr int kTopLevelMax = 7;  // 8^7 + 1 entries = 8 MB of table at most

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

template <typename KeyT>
__device__ __forceinline__ KeyT morton(int x, int y, int z);

template <>
__device__ __forceinline__ uint32_t morton<uint32_t>(int x, int y, int z) {
    return spread10((uint32_t)x) | (spread10((uint32_t)y) << 1) | (spread10((uint32_t)z) << 2);
}

template <>
__device__ __forceinline__ uint64_t morton<uint64_t>(int x, int y, int z) {
    return spread21((uint64_t)x) | (spread21((uint64_t)y) << 1) | (spread21((uint64_t)z) << 2);
}

__device__ __forceinline__ int ctz_key(uint32_t v) { return __builtin_ctz(v); }
__device__ __forceinline__ int ctz_key(uint64_t v) { return __builtin_ctzll(v); }

template <typename KeyT>
struct Tree {
    const KeyT *__restrict__ keys;     // n + 1 keys (sentinel 8^D last)
    const uint32_t *__restrict__ top;  // 8^top_level + 1 leaf indices
    int depth;
    int top_shift;  // 3 * (depth - top_level)
};

// Largest leaf index i with keys[i] <= k.  The top table narrows the range
// to the leaves that meet the level-top_level cell of k; the rest is a
// binary search in the sorted keys.
template <typename KeyT>
__device__ __forceinline__ uint32_t find_leaf(const Tree<KeyT> &t, KeyT k) {
    const uint32_t c = (uint32_t)(k >> t.top_shift);
    uint32_t lo = t.top[c];
    uint32_t hi = t.top[c + 1] + 1u;
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (t.keys[mid] <= k)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------
// The walk.  Visitor::step(leaf, l) is called once per visited leaf, in
// order.  Returns the number of leaves visited, or -1 for an invalid ray
// (source outside [0,1)^3, non-finite or all-zero direction, or a walk
// longer than the 3 * 2^D + 3 steps a valid ray can take).
// ---------------------------------------------------------------------

template <typename KeyT, typename Visitor>
__device__ __forceinline__ int walk_ray(const Tree<KeyT> &t, double qx, double qy, double qz,
                                        double mx, double my, double mz, Visitor &v) {
    const int D = t.depth;
    const int side = 1 << D;
    const double scale = (double)side;  // 2^D, exact
    const double h = 1.0 / scale;       // 2^-D, exact

    if (!(qx >= 0.0 && qx < 1.0 && qy >= 0.0 && qy < 1.0 && qz >= 0.0 && qz < 1.0)) return -1;
    if (!(isfinite(mx) && isfinite(my) && isfinite(mz))) return -1;
    const double ix = 1.0 / mx, iy = 1.0 / my, iz = 1.0 / mz;
    const bool bx = isfinite(ix), by = isfinite(iy), bz = isfinite(iz);
    if (!(bx || by || bz)) return -1;
    const bool px = mx > 0.0, py = my > 0.0, pz = mz > 0.0;

    int cx = (int)floor(qx * scale);
    int cy = (int)floor(qy * scale);
    int cz = (int)floor(qz * scale);

    double t_in = 0.0;
    const int max_steps = 3 * side + 3;
    int steps = 0;
    for (;;) {
        if (steps >= max_steps) return -1;
        const KeyT k = morton<KeyT>(cx, cy, cz);
        const uint32_t i = find_leaf(t, k);
        const KeyT span = t.keys[i + 1] - t.keys[i];  // 8^(D - level)
        const int lg = ctz_key(span) / 3;
        const int size = 1 << lg;
        const int ax = cx & ~(size - 1);
        const int ay = cy & ~(size - 1);
        const int az = cz & ~(size - 1);

        // slab method: far planes of the leaf's box along the ray
        const double tfx = bx ? ((double)(px ? ax + size : ax) * h - qx) * ix : INFINITY;
        const double tfy = by ? ((double)(py ? ay + size : ay) * h - qy) * iy : INFINITY;
        const double tfz = bz ? ((double)(pz ? az + size : az) * h - qz) * iz : INFINITY;
        double t_out = tfx;
        if (tfy < t_out) t_out = tfy;
        if (tfz < t_out) t_out = tfz;

        double l = t_out - t_in;
        if (l < 0.0)
            l = 0.0;
        else
            t_in = t_out;
        v.step(i, l);
        ++steps;

        // advance the probe into the next cell
        if (bx && tfx == t_out) {
            cx = px ? ax + size : ax - 1;
        } else {
            int c = (int)floor(fma(mx, t_out, qx) * scale);
            cx = c < ax ? ax : (c > ax + size - 1 ? ax + size - 1 : c);
        }
        if (by && tfy == t_out) {
            cy = py ? ay + size : ay - 1;
        } else {
            int c = (int)floor(fma(my, t_out, qy) * scale);
            cy = c < ay ? ay : (c > ay + size - 1 ? ay + size - 1 : c);
        }
        if (bz && tfz == t_out) {
            cz = pz ? az + size : az - 1;
        } else {
            int c = (int)floor(fma(mz, t_out, qz) * scale);
            cz = c < az ? az : (c > az + size - 1 ? az + size - 1 : c);
        }
        if ((unsigned)cx >= (unsigned)side || (unsigned)cy >= (unsigned)side ||
            (unsigned)cz >= (unsigned)side)
            break;
    }
    return steps;
}

// ---------------------------------------------------------------------
// Visitors
// ---------------------------------------------------------------------

struct SumF64 {
    const double *__restrict__ rho;
    double N;
    __device__ __forceinline__ void step(uint32_t i, double l) { N = N + rho[i] * l; }
};

struct SumF32Kahan {
    const float *__restrict__ rho;
    float S, c;
    __device__ __forceinline__ void step(uint32_t i, double l) {
        const float y = rho[i] * (float)l - c;
        const float t = S + y;
        c = (t - S) - y;
        S = t;
    }
};

struct ScatterGrad {
    float *__restrict__ grad;
    float g;
    __device__ __forceinline__ void step(uint32_t i, double l) {
        unsafeAtomicAdd(grad + i, g * (float)l);
    }
};

struct HashSteps {
    uint64_t h;
    __device__ __forceinline__ void step(uint32_t i, double) {
        h = (h ^ (uint64_t)i) * 0x100000001b3ull;
    }
};

struct RecordVisits {
    int32_t *__restrict__ out;
    int64_t cap;
    int64_t n;
    __device__ __forceinline__ void step(uint32_t i, double) {
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

// ---------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_forward_f64(Tree<KeyT> t, RayBatch r,
                                                        const double *__restrict__ rho,
                                                        double kappa, double *__restrict__ N,
                                                        double *__restrict__ A, int64_t total) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ray < total;
         ray += stride) {
        const RayIndex x = ray_index(r, ray);
        const double *q = r.src + 3 * x.s;
        const double *m = r.dirs + 3 * x.d;
        SumF64 v{rho, 0.0};
        const int steps = walk_ray(t, q[0], q[1], q[2], m[0], m[1], m[2], v);
        const double n = steps < 0 ? (double)NAN : v.N;
        N[x.off] = n;
        if (A) A[x.off] = exp(-kappa * n);
    }
}

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_forward_f32k(Tree<KeyT> t, RayBatch r,
                                                         const float *__restrict__ rho,
                                                         float kappa, float *__restrict__ N,
                                                         float *__restrict__ A, int64_t total) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ray < total;
         ray += stride) {
        const RayIndex x = ray_index(r, ray);
        const double *q = r.src + 3 * x.s;
        const double *m = r.dirs + 3 * x.d;
        SumF32Kahan v{rho, 0.0f, 0.0f};
        const int steps = walk_ray(t, q[0], q[1], q[2], m[0], m[1], m[2], v);
        const float n = steps < 0 ? (float)NAN : v.S;
        N[x.off] = n;
        if (A) A[x.off] = expf(-kappa * n);
    }
}

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_backward(Tree<KeyT> t, RayBatch r, float kappa,
                                                     const float *__restrict__ gN,
                                                     const float *__restrict__ gA,
                                                     const float *__restrict__ A,
                                                     float *__restrict__ grad, int64_t total) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ray < total;
         ray += stride) {
        const RayIndex x = ray_index(r, ray);
        float g = gN ? gN[x.off] : 0.0f;
        if (gA) g = g - kappa * A[x.off] * gA[x.off];
        if (g == 0.0f) continue;  // the ray adds nothing
        const double *q = r.src + 3 * x.s;
        const double *m = r.dirs + 3 * x.d;
        ScatterGrad v{grad, g};
        walk_ray(t, q[0], q[1], q[2], m[0], m[1], m[2], v);
    }
}

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_trace(Tree<KeyT> t, RayBatch r,
                                                  int32_t *__restrict__ steps_out,
                                                  uint64_t *__restrict__ hash_out,
                                                  int64_t total) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ray < total;
         ray += stride) {
        const RayIndex x = ray_index(r, ray);
        const double *q = r.src + 3 * x.s;
        const double *m = r.dirs + 3 * x.d;
        HashSteps v{0xcbf29ce484222325ull};
        const int steps = walk_ray(t, q[0], q[1], q[2], m[0], m[1], m[2], v);
        if (steps_out) steps_out[x.off] = steps;
        if (hash_out) hash_out[x.off] = v.h;
    }
}

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_trace_sample(Tree<KeyT> t, RayBatch r,
                                                         const int64_t *__restrict__ sample,
                                                         int64_t n_sample,
                                                         int32_t *__restrict__ visited,
                                                         int64_t cap, int64_t total) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_sample) return;
    int32_t *out = visited + j * cap;
    const int64_t ray = sample[j];
    int64_t n = 0;
    if (ray >= 0 && ray < total) {
        const RayIndex x = ray_index(r, ray);
        const double *q = r.src + 3 * x.s;
        const double *m = r.dirs + 3 * x.d;
        RecordVisits v{out, cap, 0};
        walk_ray(t, q[0], q[1], q[2], m[0], m[1], m[2], v);
        n = v.n;
    }
    for (int64_t e = n; e < cap; ++e) out[e] = -1;
}

template <typename KeyT>
Tree<KeyT> tree_of(const TreeView &v) {
    Tree<KeyT> t;
    t.keys = static_cast<const KeyT *>(v.keys);
    t.top = v.top;
    t.depth = v.depth;
    t.top_shift = 3 * (v.depth - v.top_level);
    return t;
}

unsigned grid_for(int64_t total) {
    int64_t blocks = (total + kBlock - 1) / kBlock;
    const int64_t cap = (int64_t)1 << 30;
    return (unsigned)(blocks < cap ? blocks : cap);
}

}  // namespace

int top_table_level(int depth) { return depth < kTopLevelMax ? depth : kTopLevelMax; }

hipError_t launch_forward(const TreeView &tree, const RayBatch &rays, const void *rho,
                          int precision, double kappa, void *N, void *A, hipStream_t stream) {
    const int64_t total = rays.n_src * rays.n_dirs;
    const unsigned grid = grid_for(total);
    if (precision == 0) {
        if (tree.wide_keys)
            hipLaunchKernelGGL(k_forward_f64<uint64_t>, dim3(grid), dim3(kBlock), 0, stream,
                               tree_of<uint64_t>(tree), rays, (const double *)rho, kappa,
                               (double *)N, (double *)A, total);
        else
            hipLaunchKernelGGL(k_forward_f64<uint32_t>, dim3(grid), dim3(kBlock), 0, stream,
                               tree_of<uint32_t>(tree), rays, (const double *)rho, kappa,
                               (double *)N, (double *)A, total);
    } else {
        if (tree.wide_keys)
            hipLaunchKernelGGL(k_forward_f32k<uint64_t>, dim3(grid), dim3(kBlock), 0, stream,
                               tree_of<uint64_t>(tree), rays, (const float *)rho, (float)kappa,
                               (float *)N, (float *)A, total);
        else
            hipLaunchKernelGGL(k_forward_f32k<uint32_t>, dim3(grid), dim3(kBlock), 0, stream,
                               tree_of<uint32_t>(tree), rays, (const float *)rho, (float)kappa,
                               (float *)N, (float *)A, total);
    }
    return hipGetLastError();
}

hipError_t launch_backward(const TreeView &tree, const RayBatch &rays, double kappa,
                           const float *gN, const float *gA, const float *A, float *grad,
                           hipStream_t stream) {
    const int64_t total = rays.n_src * rays.n_dirs;
    const unsigned grid = grid_for(total);
    if (tree.wide_keys)
        hipLaunchKernelGGL(k_backward<uint64_t>, dim3(grid), dim3(kBlock), 0, stream,
                           tree_of<uint64_t>(tree), rays, (float)kappa, gN, gA, A, grad, total);
    else
        hipLaunchKernelGGL(k_backward<uint32_t>, dim3(grid), dim3(kBlock), 0, stream,
                           tree_of<uint32_t>(tree), rays, (float)kappa, gN, gA, A, grad, total);
    return hipGetLastError();
}

hipError_t launch_trace(const TreeView &tree, const RayBatch &rays, int32_t *steps,
                        uint64_t *hash, const int64_t *sample, int64_t n_sample,
                        int32_t *visited, int64_t cap, hipStream_t stream) {
    const int64_t total = rays.n_src * rays.n_dirs;
    if (steps || hash) {
        const unsigned grid = grid_for(total);
        if (tree.wide_keys)
            hipLaunchKernelGGL(k_trace<uint64_t>, dim3(grid), dim3(kBlock), 0, stream,
                               tree_of<uint64_t>(tree), rays, steps, hash, total);
        else
            hipLaunchKernelGGL(k_trace<uint32_t>, dim3(grid), dim3(kBlock), 0, stream,
                               tree_of<uint32_t>(tree), rays, steps, hash, total);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_sample > 0) {
        const unsigned grid = (unsigned)((n_sample + kBlock - 1) / kBlock);
        if (tree.wide_keys)
            hipLaunchKernelGGL(k_trace_sample<uint64_t>, dim3(grid), dim3(kBlock), 0, stream,
                               tree_of<uint64_t>(tree), rays, sample, n_sample, visited, cap,
                               total);
        else
            hipLaunchKernelGGL(k_trace_sample<uint32_t>, dim3(grid), dim3(kBlock), 0, stream,
                               tree_of<uint32_t>(tree), rays, sample, n_sample, visited, cap,
                               total);
    }
    return hipGetLastError();
}

}  // namespace rt
