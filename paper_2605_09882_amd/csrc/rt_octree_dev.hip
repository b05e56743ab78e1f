// The octree's search structures staged on the device from leaf arrays
// that are already in device memory (rt_build_octree_device): the same
// checks and the same bytes as the host path of rt_octree.cpp, computed by
// kernels so that a tree built on the GPU never travels to the host.
//
//   k_check   one thread per leaf: level <= D, key aligned to its span,
//             keys strictly increasing, each leaf ending where the next
//             begins (the last at 8^D), the first at key 0; the smallest
//             failing index of each kind is kept with an atomic minimum;
//   k_stage   the key copy (narrowed to 32 bits for D <= 10) with the
//             sentinel 8^D;
//   k_top     one thread per top-table cell: binary searches for the leaf
//             holding the cell's first finest cell and for the next cell's,
//             and the FULL / ONE flags of the entry (the rule of the host
//             path).
#include "rt_internal.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rt {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_init_status(int64_t *status) {
    if (threadIdx.x < 2) status[threadIdx.x] = INT64_MAX;
}

// status[0]: first index i >= 1 with keys[i] <= keys[i-1]; status[1]: first
// index with a tiling error.
__global__ __launch_bounds__(kBlock) void k_check(const uint64_t *__restrict__ keys,
                                                  const uint8_t *__restrict__ levels, int64_t n,
                                                  int D, int64_t *status) {
    const uint64_t end = (uint64_t)1 << (3 * D);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t k = keys[i];
        const int L = levels[i];
        if (i > 0 && k <= keys[i - 1]) atomicMin((long long *)&status[0], (long long)i);
        bool bad = L > D || (i == 0 && k != 0);
        if (!bad) {
            const uint64_t span = (uint64_t)1 << (3 * (D - L));
            const uint64_t next = i + 1 < n ? keys[i + 1] : end;
            bad = (k & (span - 1)) != 0 || k + span != next;
        }
        if (bad) atomicMin((long long *)&status[1], (long long)i);
    }
}

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_stage(const uint64_t *__restrict__ keys, int64_t n,
                                                  int D, KeyT *__restrict__ out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride)
        out[i] = i < n ? (KeyT)keys[i] : (KeyT)((uint64_t)1 << (3 * D));
}

// Index of the leaf holding the finest cell with key base: the largest i
// with keys[i] <= base (keys[0] = 0 <= base; keys[n] read as +inf).
__device__ __forceinline__ int64_t leaf_holding(const uint64_t *__restrict__ keys, int64_t n,
                                                uint64_t base) {
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] <= base)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// One thread per top-table cell c: the leaf holding the cell's first finest
// cell, and its flags (the rule of the host path).  The thread finds the
// next cell's first leaf itself, so no thread reads another's output.
__global__ __launch_bounds__(kBlock) void k_top(const uint64_t *__restrict__ keys,
                                                const uint8_t *__restrict__ levels, int64_t n, int D,
                                                int lt, int shift, int64_t ncell,
                                                uint32_t *__restrict__ top) {
    const int64_t per_cell = shift < 31 ? (int64_t)1 << shift : INT64_MAX;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= ncell; c += stride) {
        if (c == ncell) {
            top[c] = (uint32_t)n;
            continue;
        }
        const int64_t lo = leaf_holding(keys, n, (uint64_t)c << shift);
        const int64_t nx = c + 1 == ncell ? n : leaf_holding(keys, n, (uint64_t)(c + 1) << shift);
        uint32_t flag = 0;
        if (nx - lo == per_cell && levels[lo] == D)
            flag = kTopFull;
        else if (levels[lo] <= lt)
            flag = kTopOne;
        top[c] = (uint32_t)lo | flag;
    }
}

unsigned blocks_for(int64_t work) {
    int64_t b = (work + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return (unsigned)(b < 65536 ? b : 65536);
}

}  // namespace

hipError_t launch_octree_check(const uint64_t *keys, const uint8_t *levels, int64_t n, int depth,
                               int64_t *status, hipStream_t stream) {
    hipLaunchKernelGGL(k_init_status, dim3(1), dim3(64), 0, stream, status);
    hipLaunchKernelGGL(k_check, dim3(blocks_for(n)), dim3(kBlock), 0, stream, keys, levels, n, depth,
                       status);
    return hipGetLastError();
}

hipError_t launch_octree_stage(const uint64_t *keys, const uint8_t *levels, int64_t n, int depth,
                               int top_level, void *key_out, uint8_t *level_out, uint32_t *top,
                               hipStream_t stream) {
    if (depth > 10)
        hipLaunchKernelGGL(k_stage<uint64_t>, dim3(blocks_for(n + 1)), dim3(kBlock), 0, stream, keys, n,
                           depth, static_cast<uint64_t *>(key_out));
    else
        hipLaunchKernelGGL(k_stage<uint32_t>, dim3(blocks_for(n + 1)), dim3(kBlock), 0, stream, keys, n,
                           depth, static_cast<uint32_t *>(key_out));
    hipError_t e = hipMemcpyAsync(level_out, levels, (size_t)n, hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return e;
    const int shift = 3 * (depth - top_level);
    const int64_t ncell = (int64_t)1 << (3 * top_level);
    hipLaunchKernelGGL(k_top, dim3(blocks_for(ncell + 1)), dim3(kBlock), 0, stream, keys, levels, n,
                       depth, top_level, shift, ncell, top);
    return hipGetLastError();
}

}  // namespace rt
