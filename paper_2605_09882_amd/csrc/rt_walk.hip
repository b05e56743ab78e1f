// HIP kernels of the reverse ray walk for gfx950 (MI355X): column densities
// (FP64 and FP32-Kahan), their adjoint, and traversal records.
//
// One ray per lane.  Rays are numbered r = d * n_src + s (direction-major),
// so the 64 lanes of a wavefront carry consecutive sources in one direction:
// with Morton-ordered sources their rays run parallel through a compact
// neighbourhood, share leaves and key-search probes in cache, and store
// their results to consecutive addresses when stride_src = 1.  The walk of
// one ray (sec. 2.3.1 DDA + Morton lookup, sec. 2.3.2 slab chord) is in
// rt_ray.h.
#include "rt_ray.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace rt {
namespace {

using namespace ray;

constexpr int kWaves = kBlock / 64;

// Adjoint scatter aggregation: per wavefront, a kAggWays-way set-associative
// table in LDS of (leaf, partial dL/drho) pairs, moved to global memory
// every kFlushEvery steps of the wavefront and when it ends.
constexpr int kAggSlots = 512;
constexpr int kAggWays = 4;
constexpr int kAggSets = kAggSlots / kAggWays;
static_assert(kAggWays == 4, "a set's tags are read as one uint4");
constexpr int kFlushEvery = 16;
constexpr uint32_t kEmpty = 0xffffffffu;
// Before the table, lanes that share a leaf in the same step are summed
// across the wavefront: the groups of the first kMaxPeel pending lanes are
// examined, and those of at least kPeelMin lanes are summed.
constexpr int kPeelMin = 4;
constexpr int kMaxPeel = 1;
// Owner election cells per wavefront (slot mod kOwnerSlots; an alias only
// turns an owner into an atomic adder).
constexpr int kOwnerSlots = 128;

// ---------------------------------------------------------------------
// Forward kernels
// ---------------------------------------------------------------------

// The FP64 exp of the epilogue stays out of line: inlined, its constants and
// temporaries are live across the walk loop (72 VGPRs and 7 waves per SIMD;
// out of line the kernel fits 8).
__device__ __noinline__ double exp_f64(double x) { return exp(x); }

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_forward_f64(Tree<KeyT> t, RayBatch r,
                                                        const double *__restrict__ rho,
                                                        double kappa, double *__restrict__ N,
                                                        double *__restrict__ A, int64_t total) {
    __shared__ uint32_t lut[1 << kLutBits];
    init_lut<KeyT>(lut, t.depth);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ray < total;
         ray += stride) {
        const RayIndex x = ray_index(r, ray);
        SumF64 v{rho, 0.0};
        const int steps = walk_ray(t, lut, r.src + 3 * x.s, r.dirs + 3 * x.d, v);
        const double n = steps < 0 ? (double)NAN : v.N;
        N[x.off] = n;
        if (A) A[x.off] = exp_f64(-kappa * n);
    }
}

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_forward_f32k(Tree<KeyT> t, RayBatch r,
                                                         const float *__restrict__ rho,
                                                         float kappa, float *__restrict__ N,
                                                         float *__restrict__ A, int64_t total) {
    __shared__ uint32_t lut[1 << kLutBits];
    init_lut<KeyT>(lut, t.depth);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ray < total;
         ray += stride) {
        const RayIndex x = ray_index(r, ray);
        SumF32Kahan v{rho, 0.0f, 0.0f};
        const int steps = walk_ray(t, lut, r.src + 3 * x.s, r.dirs + 3 * x.d, v);
        const float n = steps < 0 ? (float)NAN : v.S;
        N[x.off] = n;
        if (A) A[x.off] = expf(-kappa * n);
    }
}

// ---------------------------------------------------------------------
// Adjoint kernel
//
// Every step adds g * l (formed in FP32) to dL/drho of the leaf, which is
// accumulated in FP64: a coarse leaf collects the contributions of millions
// of rays, and in an FP32 running sum the late, small ones would be rounded
// away.  Neighbouring rays of a
// wavefront cross the same leaves within a few steps of each other (all of
// them share a coarse leaf at once), so the additions are first combined
// in a per-wavefront table in LDS (after lanes of the same step that share
// a leaf have been summed across the wavefront).  The leaf selects a set of
// kAggWays slots (set = leaf mod kAggSets); a lane reads the set's tags at
// once and adds into the slot holding its leaf, or claims the first empty
// slot, or, when the set is full or the claim is lost to another leaf,
// adds straight to global memory (see table_add).  Every kFlushEvery steps, and
// when the wavefront finishes, its lanes move the table to global memory
// with one atomic per occupied slot.  The wavefront steps in lockstep (loop
// condition uniform over the wavefront) so that all of its lanes take part
// in every flush.
// ---------------------------------------------------------------------

// Sum of v over the 64 lanes of the wavefront (all lanes must be active),
// with DPP lane shifts only: an inclusive scan inside each row of 16 lanes
// (shifts by 1, 2, 4, 8 lanes), then the row totals carried across rows
// (row broadcasts of lanes 15 and 31); lane 63 ends with the total.
template <int kCtrl, int kRowMask, bool kBoundZero>
__device__ __forceinline__ float dpp(float src) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, src),
                                                                 kCtrl, kRowMask, 0xf, kBoundZero));
}

__device__ __forceinline__ float wave_total(float v) {
    v += dpp<0x111, 0xf, true>(v);   // row_shr:1
    v += dpp<0x112, 0xf, true>(v);   // row_shr:2
    v += dpp<0x114, 0xf, true>(v);   // row_shr:4
    v += dpp<0x118, 0xf, true>(v);   // row_shr:8
    v += dpp<0x142, 0xa, false>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp<0x143, 0xc, false>(v);  // row_bcast:31 into rows 2 and 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Adds v to the table entry of leaf (or to global memory when its set is
// full).  Called by every lane of the wavefront in the same instruction
// (lanes without a pending value take no part).  LDS atomics are slow when
// many lanes issue them, so the table is updated with plain loads and
// stores, made safe by the order in which one wavefront's LDS accesses
// complete: a lane claims an empty way by storing its leaf and reading it
// back (the value that sticks wins; lanes of the same leaf share the way),
// then the lanes elect one owner per slot (each stores its lane number in
// the slot's owner cell, the value that sticks names the owner).  The owner
// adds with a plain load and store, and only the other lanes of that slot --
// lanes of the same step on the same leaf -- add atomically, after the
// owner's store.
__device__ __forceinline__ void table_add(uint32_t *tag, float *sum, uint32_t *owner,
                                          double *__restrict__ grad, uint32_t leaf, float v,
                                          bool pending, int lane) {
    int slot = -1;
    int claim = -1;
    if (pending) {
        const int set = (int)(leaf & (kAggSets - 1)) * kAggWays;
        // the set's 4 tags in one 16-byte LDS read (sets are 16-byte aligned)
        const uint4 ways = *reinterpret_cast<const uint4 *>(tag + set);
        const uint32_t tgs[kAggWays] = {ways.x, ways.y, ways.z, ways.w};
        int empty = -1;
#pragma unroll
        for (int way = 0; way < kAggWays; ++way) {
            if (tgs[way] == leaf) slot = set + way;
            if (tgs[way] == kEmpty && empty < 0) empty = set + way;
        }
        claim = slot < 0 && empty >= 0 ? empty : -1;
    }
    // claim an empty way: every claiming lane stores its leaf, the value that
    // sticks wins; lanes of the same leaf share the claim
    if (claim >= 0) __hip_atomic_store(tag + claim, leaf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (claim >= 0 && __hip_atomic_load(tag + claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == leaf)
        slot = claim;
    if (pending && slot < 0) unsafeAtomicAdd(grad + leaf, (double)v);
    uint32_t *cell = owner + (slot & (kOwnerSlots - 1));
    if (slot >= 0)
        __hip_atomic_store(cell, (uint32_t)lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const bool own = slot >= 0 && __hip_atomic_load(cell, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP) == (uint32_t)lane;
    if (own) sum[slot] = sum[slot] + v;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the owners' stores come first
    if (slot >= 0 && !own) atomicAdd(sum + slot, v);
}

__device__ __forceinline__ void flush_table(uint32_t *tag, float *sum, double *__restrict__ grad,
                                            int lane) {
    for (int j = lane; j < kAggSlots; j += 64) {
        const uint32_t k = tag[j];
        if (k != kEmpty) {
            unsafeAtomicAdd(grad + k, (double)sum[j]);
            tag[j] = kEmpty;
            sum[j] = 0.0f;
        }
    }
}

// Per-wavefront aggregation state of the adjoint: the table, its owner
// cells, and the steps since the last flush.
struct AggTable {
    uint32_t *tag;
    float *sum;
    uint32_t *owner;
    int since_flush;
};

// The adjoint walk of the wavefront's rays, in lockstep (loop condition
// uniform over the wavefront, so that all 64 lanes take part in the
// wavefront-wide sums and in every flush): each step of an active lane adds
// g * l to its leaf.  st holds the lane's ray, set up by the caller.  Peel:
// sum the largest group of lanes on one leaf across the wavefront first (it
// pays in the adjoint alone; in the fused pass, where the walks of other
// wavefronts keep the VALU busy, it costs more than it saves).
template <bool Peel, typename KeyT>
__device__ __forceinline__ void scatter_rays(const Tree<KeyT> &t, const uint32_t *lut, Ray &st,
                                             bool active, float g, int max_steps, AggTable &agg,
                                             double *__restrict__ grad, int lane) {
    // one step of the wavefront (all 64 lanes call it)
    auto step = [&]() {
        uint32_t leaf = kEmpty;
        float v = 0.0f;
        if (active) {
            double l;
            bool done;
            int level;
            leaf = ray_locate(st, t, lut, level);
            ray_advance(st, t, level, l, done);
            v = g * (float)l;
            if (done || st.steps >= max_steps) active = false;
        }
        // all 64 lanes are active here: sum the groups of lanes that share a
        // leaf (coarse leaves hold many rays at once)
        bool pending = leaf != kEmpty;
        bool cand = pending;  // not yet examined for a shared leaf
        for (int peel = 0; Peel && peel < kMaxPeel; ++peel) {
            const uint64_t cm = __ballot(cand);
            if (cm == 0) break;
            const int leader = __ffsll((unsigned long long)cm) - 1;
            const uint32_t L = (uint32_t)__builtin_amdgcn_readlane((int)leaf, leader);
            const bool mine = cand && leaf == L;
            if (__popcll(__ballot(mine)) >= kPeelMin) {
                const float total = wave_total(mine ? v : 0.0f);
                if (mine) {
                    // the group's total travels in the leader's lane
                    v = lane == leader ? total : 0.0f;
                    pending = lane == leader;
                }
            }
            if (mine) cand = false;
        }
        table_add(agg.tag, agg.sum, agg.owner, grad, leaf, v, pending, lane);
        if (++agg.since_flush == kFlushEvery) {
            flush_table(agg.tag, agg.sum, grad, lane);
            agg.since_flush = 0;
        }
    };
    // two steps per iteration, as in walk_ray: the ray state then alternates
    // between two sets of registers instead of being copied back every step
    for (;;) {
        if (!__any(active)) break;
        step();
        if (!__any(active)) break;
        step();
    }
}

// The LDS of the adjoint kernels: the Morton spread table and one
// aggregation table per wavefront.
struct alignas(16) AdjointShared {
    uint32_t tag[kWaves][kAggSlots];
    float sum[kWaves][kAggSlots];
    uint32_t lut[1 << kLutBits];
    uint32_t owner[kWaves][kOwnerSlots];
};

template <typename KeyT>
__device__ __forceinline__ AggTable init_adjoint(AdjointShared &sh, int depth, int wave, int lane) {
    AggTable agg{sh.tag[wave], sh.sum[wave], sh.owner[wave], 0};
    for (int j = lane; j < kAggSlots; j += 64) {
        agg.tag[j] = kEmpty;
        agg.sum[j] = 0.0f;
    }
    init_lut<KeyT>(sh.lut, depth);  // ends with a block barrier
    return agg;
}

template <typename KeyT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_backward(
    Tree<KeyT> t, RayBatch r, float kappa,
                                                     const float *__restrict__ gN,
                                                     const float *__restrict__ gA,
                                                     const float *__restrict__ A,
                                                     double *__restrict__ grad, int64_t total) {
    __shared__ AdjointShared sh;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    AggTable agg = init_adjoint<KeyT>(sh, t.depth, wave, lane);
    const int max_steps = 3 * (1 << t.depth) + 3;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // base is uniform over the wavefront: all its lanes run every iteration
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (wave << 6); base < total;
         base += stride) {
        const int64_t ray = base + lane;
        Ray st;
        float g = 0.0f;
        bool active = false;
        if (ray < total) {
            const RayIndex x = ray_index(r, ray);
            g = gN ? gN[x.off] : 0.0f;
            if (gA) g = g - kappa * A[x.off] * gA[x.off];
            if (g != 0.0f) active = ray_init(st, t.depth, r.src + 3 * x.s, r.dirs + 3 * x.d);
        }
        scatter_rays<true>(t, sh.lut, st, active, g, max_steps, agg, grad, lane);
    }
    flush_table(agg.tag, agg.sum, grad, lane);
}

// ---------------------------------------------------------------------
// Forward and adjoint in one pass, for a loss linear in N and A:
// L = sum_r (wN_r N_r + wA_r A_r), so g_r = wN_r - kappa A_r wA_r is known as
// soon as the ray's forward walk ends.  A wavefront walks its rays for the
// FP32-Kahan column (the bits of k_forward_f32k), stores N and A, and walks
// them again to scatter g * l; both walks step in lockstep and share the ray
// state.  The second walk finds the leaves of the first still in cache, and
// the scatter of some wavefronts overlaps the walks of others.  Asked for 7
// waves per SIMD (the adjoint's LDS allows 7 blocks per CU), the compiler
// fits it in 72 VGPRs; the only values it spills belong to the per-ray
// set-up, none to the walks.
// ---------------------------------------------------------------------

// Out of line, as exp_f64: inlined, its constants would stay live across
// both walks.
__device__ __noinline__ float exp_f32(float x) { return expf(x); }

template <typename KeyT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7, 8))) void k_forward_adjoint(
    Tree<KeyT> t, RayBatch r, const float *__restrict__ rho, float kappa,
    const float *__restrict__ wN, const float *__restrict__ wA, float *__restrict__ N,
    float *__restrict__ A, double *__restrict__ grad, int64_t total) {
    __shared__ AdjointShared sh;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    AggTable agg = init_adjoint<KeyT>(sh, t.depth, wave, lane);
    const int max_steps = 3 * (1 << t.depth) + 3;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (wave << 6); base < total;
         base += stride) {
        const int64_t ray = base + lane;
        Ray st;
        RayIndex x{0, 0, 0};
        bool valid = false;
        if (ray < total) {
            x = ray_index(r, ray);
            valid = ray_init(st, t.depth, r.src + 3 * x.s, r.dirs + 3 * x.d);
        }
        // forward: the FP32-Kahan column, as SumF32Kahan in walk_ray
        SumF32Kahan v{rho, 0.0f, 0.0f};
        bool active = valid;
        bool too_long = false;
        auto step = [&]() {
            if (active) {
                double l;
                bool done;
                int level;
                const uint32_t leaf = ray_locate(st, t, sh.lut, level);
                const float value = v.fetch(leaf);
                ray_advance(st, t, level, l, done);
                v.step(value, leaf, l);
                if (done) {
                    active = false;
                } else if (st.steps >= max_steps) {
                    active = false;
                    too_long = true;
                }
            }
        };
        // lockstep, two steps per iteration (see scatter_rays)
        for (;;) {
            if (!__any(active)) break;
            step();
            if (!__any(active)) break;
            step();
        }
        float g = 0.0f;
        if (ray < total) {
            const float n = valid && !too_long ? v.S : (float)NAN;
            const float a = exp_f32(-kappa * n);
            N[x.off] = n;
            if (A) A[x.off] = a;
            if (wN) g = wN[x.off];
            if (wA) g = g - kappa * a * wA[x.off];
            active = valid && !too_long && g != 0.0f &&
                     ray_init(st, t.depth, r.src + 3 * x.s, r.dirs + 3 * x.d);
        }
        scatter_rays<false>(t, sh.lut, st, active, g, max_steps, agg, grad, lane);
    }
    flush_table(agg.tag, agg.sum, grad, lane);
}

// ---------------------------------------------------------------------
// Trace kernels
// ---------------------------------------------------------------------

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_trace(Tree<KeyT> t, RayBatch r,
                                                  int32_t *__restrict__ steps_out,
                                                  uint64_t *__restrict__ hash_out,
                                                  int64_t total) {
    __shared__ uint32_t lut[1 << kLutBits];
    init_lut<KeyT>(lut, t.depth);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t ray = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ray < total;
         ray += stride) {
        const RayIndex x = ray_index(r, ray);
        HashSteps v{0xcbf29ce484222325ull};
        const int steps = walk_ray<true>(t, lut, r.src + 3 * x.s, r.dirs + 3 * x.d, v);
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
    __shared__ uint32_t lut[1 << kLutBits];
    init_lut<KeyT>(lut, t.depth);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_sample; j += stride) {
        int32_t *out = visited + j * cap;
        const int64_t ray = sample[j];
        int64_t n = 0;
        if (ray >= 0 && ray < total) {
            const RayIndex x = ray_index(r, ray);
            RecordVisits v{out, cap, 0};
            walk_ray(t, lut, r.src + 3 * x.s, r.dirs + 3 * x.d, v);
            n = v.n;
        }
        for (int64_t e = n; e < cap; ++e) out[e] = -1;
    }
}

}  // namespace

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
                           const float *gN, const float *gA, const float *A, double *grad,
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

hipError_t launch_forward_adjoint(const TreeView &tree, const RayBatch &rays, const float *rho,
                                  double kappa, const float *wN, const float *wA, float *N, float *A,
                                  double *grad, hipStream_t stream) {
    const int64_t total = rays.n_src * rays.n_dirs;
    const unsigned grid = grid_for(total);
    if (tree.wide_keys)
        hipLaunchKernelGGL(k_forward_adjoint<uint64_t>, dim3(grid), dim3(kBlock), 0, stream,
                           tree_of<uint64_t>(tree), rays, rho, (float)kappa, wN, wA, N, A, grad,
                           total);
    else
        hipLaunchKernelGGL(k_forward_adjoint<uint32_t>, dim3(grid), dim3(kBlock), 0, stream,
                           tree_of<uint32_t>(tree), rays, rho, (float)kappa, wN, wA, N, A, grad,
                           total);
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
        const unsigned grid = grid_for(n_sample);
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
