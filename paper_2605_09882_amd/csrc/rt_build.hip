// HIP kernels that build the contribution grid on the GPU (gfx950): the
// leaf-only linear octree of the density + uniformity rule (sec. 2.4) from
// a uniform grid of 8^D values in Morton order.
//
// A cell of level L < D is split iff max >= floor and (max - min) >= rel max
// over the fine cells it covers; the leaves are the unsplit cells whose
// ancestors are all split, plus the fine cells under split level-(D-1)
// cells.  A leaf's value is the mean of its fine cells, formed level by
// level as the mean of the 8 children's values (summed in child order).
//
// 1. Pyramid (k_pyramid): one block reduces a level-(Lin - k) cell from
//    its 8^k descendants at level Lin (k <= 3, 512 threads), writing max,
//    min, mean and the split flag of the k levels above Lin; the fine grid
//    is read once, then each pass reads the previous pass's top level.
// 2. Count (k_count): each thread owns the 8 fine cells of one level-(D-1)
//    cell, finds the first unsplit ancestor top-down, and counts the leaves
//    that start in its cells (8 if the level-(D-1) cell is split, else 1
//    when its first fine cell starts the leaf, else 0); blocks of 256
//    threads (2048 fine cells) sum their counts.
// 3. Offsets (k_scan_blocks): one block turns the block counts into
//    exclusive offsets and the leaf total.
// 4. Emit (k_emit): the count of step 2 again, a block-wide exclusive scan
//    of the thread counts (wavefront shuffles, then the 4 wavefront totals),
//    and each thread writes its leaves at their offsets: leaves come out in
//    Morton order without a sort.
#include "rt_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

namespace rt {
namespace {

constexpr int kEmitBlock = 256;                // threads per count / emit block
constexpr int kCellsPerBlock = 8 * kEmitBlock;  // fine cells per count / emit block
constexpr int kScanBlock = 1024;

__host__ __device__ constexpr int64_t cells_before(int level) {
    return (((int64_t)1 << (3 * level)) - 1) / 7;
}

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace layout at depth D: max, min and mean (f64) and the split flag
// (u8) of every cell of levels 0 .. D-1, then one i64 offset per count /
// emit block, each array 256-byte aligned.
constexpr size_t workspace_bytes_at(int depth) {
    return 3 * align256(8 * (size_t)cells_before(depth)) + align256((size_t)cells_before(depth)) +
           align256(8 * (size_t)((((int64_t)1 << (3 * (depth - 1))) + kEmitBlock - 1) / kEmitBlock));
}

struct Pyramid {
    double *mx, *mn, *mean;  // cells of levels 0 .. D-1, level L at cells_before(L)
    uint8_t *split;
};

// Reduces k levels above Lin.  Block size 8^k; block b covers level-Lin
// cells b 8^k .. (b+1) 8^k - 1.  from_grid: level Lin is the fine grid.
__global__ __launch_bounds__(512) void k_pyramid(const double *__restrict__ grid, Pyramid p,
                                                 int Lin, int k, int from_grid, double floor_,
                                                 double rel) {
    __shared__ double s_mx[512], s_mn[512], s_mean[512];
    const int t = threadIdx.x;
    const int64_t width = (int64_t)1 << (3 * k);  // level-Lin cells of this block
    const int64_t cell = (int64_t)blockIdx.x * width + t;
    if (from_grid) {
        const double v = grid[cell];
        s_mx[t] = v;
        s_mn[t] = v;
        s_mean[t] = v;
    } else {
        const int64_t at = cells_before(Lin) + cell;
        s_mx[t] = p.mx[at];
        s_mn[t] = p.mn[at];
        s_mean[t] = p.mean[at];
    }
    __syncthreads();
    int64_t count = width;
    for (int j = 1; j <= k; ++j) {
        count >>= 3;
        const int L = Lin - j;
        double hi = 0.0, lo = 0.0, sum = 0.0;
        if (t < count) {
            hi = s_mx[8 * t];
            lo = s_mn[8 * t];
            sum = s_mean[8 * t];
            for (int c = 1; c < 8; ++c) {
                hi = fmax(hi, s_mx[8 * t + c]);
                lo = fmin(lo, s_mn[8 * t + c]);
                sum = sum + s_mean[8 * t + c];
            }
        }
        __syncthreads();
        if (t < count) {
            const double mean = sum / 8.0;
            s_mx[t] = hi;
            s_mn[t] = lo;
            s_mean[t] = mean;
            const int64_t at = cells_before(L) + (int64_t)blockIdx.x * count + t;
            p.mx[at] = hi;
            p.mn[at] = lo;
            p.mean[at] = mean;
            p.split[at] = (uint8_t)(hi >= floor_ && (hi - lo) >= rel * hi);
        }
        __syncthreads();
    }
}

// Leaves that start in the 8 fine cells of level-(D-1) cell q, and the
// level and value index of the leaf holding them: 8 fine leaves when q is
// split, else one leaf of level L < D starting at fine cell 8q when 8q is
// aligned to it, else none.
struct Owned {
    int count;
    int level;
};

__device__ __forceinline__ Owned owned_leaves(const uint8_t *__restrict__ split, int D, int64_t q) {
    Owned o;
    int L = 0;
    // the first unsplit ancestor of q (q itself at level D-1)
    while (L < D && split[cells_before(L) + (q >> (3 * (D - 1 - L)))]) ++L;
    o.level = L;
    if (L == D) {
        o.count = 8;
    } else {
        const int64_t first = 8 * q;
        const int64_t span = (int64_t)1 << (3 * (D - L));
        o.count = (first & (span - 1)) == 0 ? 1 : 0;
    }
    return o;
}

__global__ __launch_bounds__(kEmitBlock) void k_count(const uint8_t *__restrict__ split, int D,
                                                      int64_t n_parents,
                                                      int64_t *__restrict__ block_counts) {
    __shared__ int s_sum[kEmitBlock / 64];
    const int64_t q = (int64_t)blockIdx.x * kEmitBlock + threadIdx.x;
    int c = 0;
    if (q < n_parents) c = owned_leaves(split, D, q).count;
    // block sum: wavefront sums, then the 4 wavefront totals
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t total = 0;
        for (int w = 0; w < kEmitBlock / 64; ++w) total += s_sum[w];
        block_counts[blockIdx.x] = total;
    }
}

// Exclusive offsets of n block counts, in place, and the total in *n_out.
__global__ __launch_bounds__(kScanBlock) void k_scan_blocks(int64_t *__restrict__ counts, int64_t n,
                                                            int64_t *__restrict__ n_out) {
    __shared__ int64_t s_wave[kScanBlock / 64];
    __shared__ int64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t base = 0; base < n; base += kScanBlock) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < n ? counts[i] : 0;
        int64_t incl = v;  // inclusive scan inside the wavefront
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        int64_t before = s_carry;
        for (int w = 0; w < wave; ++w) before += s_wave[w];
        if (i < n) counts[i] = before + incl - v;
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) s_carry = before + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_out = s_carry;
}

__global__ __launch_bounds__(kEmitBlock) void k_emit(const double *__restrict__ grid, Pyramid p, int D,
                                                     int64_t n_parents,
                                                     const int64_t *__restrict__ block_offsets,
                                                     uint64_t *__restrict__ keys,
                                                     uint8_t *__restrict__ levels,
                                                     double *__restrict__ values) {
    __shared__ int s_wave[kEmitBlock / 64];
    const int64_t q = (int64_t)blockIdx.x * kEmitBlock + threadIdx.x;
    Owned o{0, 0};
    if (q < n_parents) o = owned_leaves(p.split, D, q);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = o.count;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += s_wave[w];
    int64_t pos = block_offsets[blockIdx.x] + before + incl - o.count;
    const int64_t first = 8 * q;
    if (o.count == 8) {
        for (int c = 0; c < 8; ++c) {
            keys[pos + c] = (uint64_t)(first + c);
            levels[pos + c] = (uint8_t)D;
            values[pos + c] = grid[first + c];
        }
    } else if (o.count == 1) {
        keys[pos] = (uint64_t)first;
        levels[pos] = (uint8_t)o.level;
        values[pos] = p.mean[cells_before(o.level) + (first >> (3 * (D - o.level)))];
    }
}

// Scratch of rt_grid_tree_static, for callers that cannot allocate: the
// workspace of the deepest grid it takes, held by every GPU the library runs
// on until the process ends.  Host code never uses the array's name as an
// address (on the host it is a stand-in, not device memory): it takes the
// device address from hipGetSymbolAddress, once per device.
constexpr size_t kStaticScratchBytes = workspace_bytes_at(kStaticGridMaxDepth);
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

}  // namespace

size_t grid_tree_workspace_bytes(int depth) { return workspace_bytes_at(depth); }

size_t grid_tree_static_scratch_bytes() { return kStaticScratchBytes; }

hipError_t grid_tree_static_scratch(void **ptr) {
    constexpr int kMaxDevices = 256;
    static std::mutex lock;
    static void *addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(lock);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_grid_tree(const double *grid, int depth, double floor_, double rel,
                            void *workspace, uint64_t *keys, uint8_t *levels, double *values,
                            int64_t *n_out, hipStream_t stream) {
    const int D = depth;
    const int64_t cells = cells_before(D);
    unsigned char *w = static_cast<unsigned char *>(workspace);
    Pyramid p;
    p.mx = reinterpret_cast<double *>(w);
    w += align256(8 * (size_t)cells);
    p.mn = reinterpret_cast<double *>(w);
    w += align256(8 * (size_t)cells);
    p.mean = reinterpret_cast<double *>(w);
    w += align256(8 * (size_t)cells);
    p.split = w;
    w += align256((size_t)cells);
    int64_t *block_counts = reinterpret_cast<int64_t *>(w);

    for (int Lin = D; Lin > 0;) {
        const int k = Lin < 3 ? Lin : 3;
        const unsigned blocks = (unsigned)((int64_t)1 << (3 * (Lin - k)));
        hipLaunchKernelGGL(k_pyramid, dim3(blocks), dim3(1u << (3 * k)), 0, stream, grid, p, Lin, k,
                           Lin == D ? 1 : 0, floor_, rel);
        Lin -= k;
    }
    const int64_t parents = (int64_t)1 << (3 * (D - 1));
    const unsigned blocks = (unsigned)((parents + kEmitBlock - 1) / kEmitBlock);
    hipLaunchKernelGGL(k_count, dim3(blocks), dim3(kEmitBlock), 0, stream, p.split, D, parents,
                       block_counts);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanBlock), 0, stream, block_counts,
                       (int64_t)blocks, n_out);
    hipLaunchKernelGGL(k_emit, dim3(blocks), dim3(kEmitBlock), 0, stream, grid, p, D, parents,
                       block_counts, keys, levels, values);
    return hipGetLastError();
}

}  // namespace rt
