// Leaf-only linear octree (sec. 2.3.1): validation of the leaves on the host
// and staging of the search structures (keys, levels, top table) in the
// caller's device workspace.
#include "raytheia.h"
#include "rt_internal.h"

#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

namespace {

constexpr int kTopLevelMax = 9;  // at most 8^9 + 1 table entries (512 MiB)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace layout: key copy (with sentinel), level copy, top table.
struct Layout {
    size_t keys, levels, top;
    size_t total() const { return keys + levels + top; }
};

Layout workspace_layout(int64_t n, int depth) {
    const size_t ksize = depth <= 10 ? 4 : 8;
    const int lt = rt::top_table_level(depth, n);
    Layout l;
    l.keys = align256(ksize * (size_t)(n + 1));
    l.levels = align256((size_t)n);
    l.top = align256(4 * (((size_t)1 << (3 * lt)) + 1));
    return l;
}

// Leaf indices travel in the low 30 bits of a top-table entry.
constexpr int64_t kMaxLeaves = ((int64_t)1 << 30) - 2;

// The host handle of a tree staged at base with layout lay.
rt_octree *new_handle(unsigned char *base, const Layout &lay, int64_t n, int depth, int device) {
    rt_octree *t = new (std::nothrow) rt_octree;
    if (!t) return nullptr;
    t->view.keys = base;
    t->view.levels = base + lay.keys;
    t->view.top = reinterpret_cast<const uint32_t *>(base + lay.keys + lay.levels);
    t->view.n = n;
    t->view.depth = depth;
    t->view.top_level = rt::top_table_level(depth, n);
    t->view.wide_keys = depth > 10 ? 1 : 0;
    t->device = device;
    return t;
}

// Argument checks shared by both build calls (everything but the leaves).
int check_build_args(int64_t n_leaves, int max_depth, void *d_workspace, size_t workspace_bytes,
                     rt_octree **out) {
    if (!out) return rt::fail(RT_ERR_ARG, "null output handle pointer");
    *out = nullptr;
    if (max_depth < 1 || max_depth > 21)
        return rt::fail(RT_ERR_ARG, "max_depth %d not in 1..21", max_depth);
    if (n_leaves < 1 || n_leaves > kMaxLeaves)
        return rt::fail(RT_ERR_ARG, "n_leaves %lld not in 1..2^30-2", (long long)n_leaves);
    if (!d_workspace) return rt::fail(RT_ERR_WORKSPACE, "null workspace");
    if (((uintptr_t)d_workspace & 255) != 0)
        return rt::fail(RT_ERR_WORKSPACE, "workspace not 256-byte aligned");
    const size_t need = workspace_layout(n_leaves, max_depth).total();
    if (workspace_bytes < need)
        return rt::fail(RT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    return RT_OK;
}

}  // namespace

namespace rt {

// The top table has at most two entries per leaf (8 bytes per leaf), at the
// deepest level that allows, capped at the tree depth and at kTopLevelMax.
int top_table_level(int depth, int64_t n_leaves) {
    int lt = 0;
    while (lt < depth && lt < kTopLevelMax && ((int64_t)1 << (3 * (lt + 1))) <= 2 * n_leaves) ++lt;
    return lt;
}

}  // namespace rt

using rt::device_status;
using rt::fail;
using rt::ok;

extern "C" {

size_t rt_octree_workspace_bytes(int64_t n_leaves, int max_depth) {
    if (n_leaves < 1 || n_leaves > kMaxLeaves || max_depth < 1 || max_depth > 21) return 0;
    return workspace_layout(n_leaves, max_depth).total();
}

int rt_build_octree(const uint64_t *keys, const uint8_t *levels, int64_t n_leaves, int max_depth,
                    void *d_workspace, size_t workspace_bytes, void *stream, rt_octree **out) {
    if (!out) return fail(RT_ERR_ARG, "null output handle pointer");
    *out = nullptr;
    if (!keys || !levels) return fail(RT_ERR_ARG, "null keys or levels");
    if (max_depth < 1 || max_depth > 21) return fail(RT_ERR_ARG, "max_depth %d not in 1..21", max_depth);
    if (n_leaves < 1 || n_leaves > kMaxLeaves)
        return fail(RT_ERR_ARG, "n_leaves %lld not in 1..2^30-2", (long long)n_leaves);
    const int D = max_depth;
    for (int64_t i = 1; i < n_leaves; ++i)
        if (keys[i] <= keys[i - 1])
            return fail(RT_ERR_UNSORTED, "keys[%lld] <= keys[%lld]", (long long)i, (long long)(i - 1));
    const uint64_t end = (uint64_t)1 << (3 * D);
    uint64_t next = 0;
    for (int64_t i = 0; i < n_leaves; ++i) {
        if (levels[i] > D)
            return fail(RT_ERR_TILING, "levels[%lld] = %d exceeds depth %d", (long long)i, levels[i], D);
        const uint64_t span = (uint64_t)1 << (3 * (D - levels[i]));
        if (keys[i] & (span - 1))
            return fail(RT_ERR_TILING, "keys[%lld] not aligned to its level", (long long)i);
        if (keys[i] != next)
            return fail(RT_ERR_TILING, "gap or overlap before leaf %lld", (long long)i);
        next = keys[i] + span;
    }
    if (next != end) return fail(RT_ERR_TILING, "leaves end at key %llu, not 8^D", (unsigned long long)next);
    int st = check_build_args(n_leaves, D, d_workspace, workspace_bytes, out);
    if (st != RT_OK) return st;
    const Layout lay = workspace_layout(n_leaves, D);
    const size_t kb = lay.keys, lb = lay.levels;

    // stage keys (+ sentinel), levels and the top table in one host buffer
    std::vector<unsigned char> host(lay.total(), 0);
    const bool wide = D > 10;
    if (wide) {
        uint64_t *k = reinterpret_cast<uint64_t *>(host.data());
        std::memcpy(k, keys, sizeof(uint64_t) * n_leaves);
        k[n_leaves] = end;
    } else {
        uint32_t *k = reinterpret_cast<uint32_t *>(host.data());
        for (int64_t i = 0; i < n_leaves; ++i) k[i] = (uint32_t)keys[i];
        k[n_leaves] = (uint32_t)end;
    }
    std::memcpy(host.data() + kb, levels, (size_t)n_leaves);
    const int lt = rt::top_table_level(D, n_leaves);
    const int64_t ncell = (int64_t)1 << (3 * lt);
    const int shift = 3 * (D - lt);
    uint32_t *top = reinterpret_cast<uint32_t *>(host.data() + kb + lb);
    int64_t i = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        const uint64_t base = (uint64_t)c << shift;
        while (i + 1 < n_leaves && keys[i + 1] <= base) ++i;
        top[c] = (uint32_t)i;
    }
    top[ncell] = (uint32_t)n_leaves;
    // flags: the cell is refined to depth D everywhere (its leaves follow its
    // keys one to one), or a single leaf covers it.  As many leaves as
    // finest cells means depth D throughout, except for a one-cell table
    // cell, which also meets that count when it is the last finest cell of
    // a coarser leaf: hence the level test.
    const int64_t per_cell = shift < 31 ? (int64_t)1 << shift : INT64_MAX;
    for (int64_t c = 0; c < ncell; ++c) {
        const int64_t lo = top[c], nx = top[c + 1] & rt::kTopIndex;
        if (nx - lo == per_cell && levels[lo] == D)
            top[c] |= rt::kTopFull;
        else if (levels[lo] <= lt)
            top[c] |= rt::kTopOne;
    }

    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return device_status(e, "hipGetDevice");
    hipStream_t s = static_cast<hipStream_t>(stream);
    e = hipMemcpyAsync(d_workspace, host.data(), lay.total(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return device_status(e, "hipMemcpyAsync(octree)");
    e = hipStreamSynchronize(s);  // the staging buffer dies with this call
    if (e != hipSuccess) return device_status(e, "hipStreamSynchronize");

    rt_octree *t = new_handle(static_cast<unsigned char *>(d_workspace), lay, n_leaves, D, device);
    if (!t) return fail(RT_ERR_ARG, "out of host memory");
    *out = t;
    return ok();
}

int rt_build_octree_device(const uint64_t *d_keys, const uint8_t *d_levels, int64_t n_leaves,
                           int max_depth, void *d_workspace, size_t workspace_bytes, void *stream,
                           rt_octree **out) {
    int st = check_build_args(n_leaves, max_depth, d_workspace, workspace_bytes, out);
    if (st != RT_OK) return st;
    if (!d_keys || !d_levels) return fail(RT_ERR_ARG, "null keys or levels");
    const int D = max_depth;
    const Layout lay = workspace_layout(n_leaves, D);
    unsigned char *base = static_cast<unsigned char *>(d_workspace);
    uint32_t *top = reinterpret_cast<uint32_t *>(base + lay.keys + lay.levels);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return device_status(e, "hipGetDevice");
    // the first 16 bytes of the top table's region hold the check results
    int64_t *status = reinterpret_cast<int64_t *>(top);
    e = rt::launch_octree_check(d_keys, d_levels, n_leaves, D, status, s);
    if (e != hipSuccess) return device_status(e, "octree check launch");
    int64_t found[2];
    e = hipMemcpyAsync(found, status, sizeof found, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return device_status(e, "hipMemcpyAsync(check)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_status(e, "hipStreamSynchronize");
    if (found[0] != INT64_MAX)
        return fail(RT_ERR_UNSORTED, "keys[%lld] <= keys[%lld]", (long long)found[0],
                    (long long)(found[0] - 1));
    if (found[1] != INT64_MAX)
        return fail(RT_ERR_TILING, "leaf %lld: level above the depth, key not aligned to its level, "
                    "a gap or an overlap after it, or a first key other than 0", (long long)found[1]);
    e = rt::launch_octree_stage(d_keys, d_levels, n_leaves, D, rt::top_table_level(D, n_leaves), base,
                                base + lay.keys, top, s);
    if (e != hipSuccess) return device_status(e, "octree staging launch");
    rt_octree *t = new_handle(base, lay, n_leaves, D, device);
    if (!t) return fail(RT_ERR_ARG, "out of host memory");
    *out = t;
    return ok();
}

void rt_octree_free(rt_octree *tree) { delete tree; }

int64_t rt_octree_leaves(const rt_octree *tree) { return tree ? tree->view.n : -1; }

int rt_octree_depth(const rt_octree *tree) { return tree ? tree->view.depth : -1; }

}  // extern "C"
