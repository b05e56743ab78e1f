// C ABI of the reverse ray-walk library: argument and octree validation on
// the host, HEALPix directions, staging of the octree's search structures in
// the caller's workspace, and dispatch to the HIP kernels.
#include "raytheia.h"
#include "rt_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

struct rt_octree {
    rt::TreeView view;
    int device;
};

namespace {

thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int ok() {
    g_last_error.clear();
    return RT_OK;
}

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

bool valid_precision(int p) { return p == RT_FP64 || p == RT_FP32_KAHAN; }

// Common checks of a batch of rays; fills the kernel-side description.
int check_rays(const rt_octree *tree, const double *d_src, int64_t n_src, const double *d_dirs,
               int64_t n_dirs, int64_t stride_src, int64_t stride_dir, rt::RayBatch *rays) {
    if (!tree) return fail(RT_ERR_ARG, "null octree handle");
    if (!d_src || !d_dirs) return fail(RT_ERR_ARG, "null source or direction pointer");
    if (n_src < 1 || n_dirs < 1) return fail(RT_ERR_ARG, "n_src and n_dirs must be >= 1");
    if (n_src > INT64_MAX / 3 || n_dirs > INT64_MAX / n_src)
        return fail(RT_ERR_ARG, "n_src * n_dirs overflows");
    if (stride_src < 0 || stride_dir < 0) return fail(RT_ERR_ARG, "negative output stride");
    // largest output offset must be representable
    if ((stride_src > 0 && n_src - 1 > INT64_MAX / stride_src) ||
        (stride_dir > 0 && n_dirs - 1 > INT64_MAX / stride_dir) ||
        (n_src - 1) * stride_src > INT64_MAX - (n_dirs - 1) * stride_dir)
        return fail(RT_ERR_ARG, "output offsets overflow");
    rays->src = d_src;
    rays->n_src = n_src;
    rays->dirs = d_dirs;
    rays->n_dirs = n_dirs;
    rays->stride_src = stride_src;
    rays->stride_dir = stride_dir;
    return RT_OK;
}

int device_status(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(RT_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

}  // namespace

extern "C" {

int rt_abi_version(void) { return RT_ABI_VERSION; }

const char *rt_status_string(int status) {
    switch (status) {
        case RT_OK: return "ok";
        case RT_ERR_ARG: return "invalid argument";
        case RT_ERR_UNSORTED: return "leaf keys not strictly increasing";
        case RT_ERR_TILING: return "leaves do not tile the box";
        case RT_ERR_RANGE: return "value out of range";
        case RT_ERR_DEVICE: return "HIP runtime error";
        case RT_ERR_WORKSPACE: return "workspace too small or misaligned";
        default: return "unknown status";
    }
}

const char *rt_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------
// HEALPix RING pixel centres, computed pixel by pixel: the pixel index is
// mapped to its ring i (north cap, equatorial belt or south cap) and its
// position j inside the ring; the ring gives z = cos(theta), the position
// the azimuth (Gorski et al. 2005, the direction set of sec. 2.1).
// ---------------------------------------------------------------------

int64_t rt_healpix_npix(int nside) {
    if (nside < 1 || nside > (1 << 20)) return -1;
    return 12 * (int64_t)nside * (int64_t)nside;
}

namespace {

// Largest r with 2 r (r - 1) <= p (ring of a north-cap pixel p, 1-based).
int64_t cap_ring(int64_t p) {
    int64_t r = (int64_t)std::floor(0.5 * (1.0 + std::sqrt(1.0 + 2.0 * (double)p)));
    while (2 * r * (r - 1) > p) --r;
    while (2 * (r + 1) * r <= p) ++r;
    return r;
}

}  // namespace

int rt_healpix_dirs(int nside, double *dirs_out) {
    const int64_t npix = rt_healpix_npix(nside);
    if (npix < 0) return fail(RT_ERR_ARG, "nside %d out of range [1, 2^20]", nside);
    if (!dirs_out) return fail(RT_ERR_ARG, "null output pointer");
    const double pi = 3.14159265358979323846;
    const int64_t ns = nside;
    const int64_t ncap = 2 * ns * (ns - 1);  // pixels in the north polar cap
    const double fns = (double)ns;
    for (int64_t p = 0; p < npix; ++p) {
        double z, phi;
        if (p < ncap) {  // north cap: ring i has 4i pixels
            const int64_t i = cap_ring(p);
            const int64_t j = p - 2 * i * (i - 1);  // 0-based position
            z = 1.0 - (double)(i * i) / (3.0 * fns * fns);
            phi = ((double)j + 0.5) * (pi / (2.0 * (double)i));
        } else if (p < npix - ncap) {  // belt: 4 nside pixels per ring
            const int64_t q = p - ncap;
            const int64_t i = q / (4 * ns) + ns;
            const int64_t j = q % (4 * ns);
            z = 4.0 / 3.0 - 2.0 * (double)i / (3.0 * fns);
            const double shift = ((i + ns) & 1) ? 0.0 : 0.5;  // half-pixel offset
            phi = ((double)j + shift) * (pi / (2.0 * fns));
        } else {  // south cap, mirror of the north cap
            const int64_t q = npix - 1 - p;
            const int64_t i = cap_ring(q);
            const int64_t jm = q - 2 * i * (i - 1);      // position from the end
            const int64_t j = 4 * i - 1 - jm;
            z = -(1.0 - (double)(i * i) / (3.0 * fns * fns));
            phi = ((double)j + 0.5) * (pi / (2.0 * (double)i));
        }
        const double st = std::sqrt((1.0 - z) * (1.0 + z));
        dirs_out[3 * p + 0] = st * std::cos(phi);
        dirs_out[3 * p + 1] = st * std::sin(phi);
        dirs_out[3 * p + 2] = z;
    }
    return ok();
}

// ---------------------------------------------------------------------
// Octree
// ---------------------------------------------------------------------

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

    if (!d_workspace) return fail(RT_ERR_WORKSPACE, "null workspace");
    if (((uintptr_t)d_workspace & 255) != 0) return fail(RT_ERR_WORKSPACE, "workspace not 256-byte aligned");
    const Layout lay = workspace_layout(n_leaves, D);
    const size_t kb = lay.keys, lb = lay.levels;
    if (workspace_bytes < lay.total())
        return fail(RT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes,
                    lay.total());

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

    rt_octree *t = new (std::nothrow) rt_octree;
    if (!t) return fail(RT_ERR_ARG, "out of host memory");
    unsigned char *base = static_cast<unsigned char *>(d_workspace);
    t->view.keys = base;
    t->view.levels = base + kb;
    t->view.top = reinterpret_cast<const uint32_t *>(base + kb + lb);
    t->view.n = n_leaves;
    t->view.depth = D;
    t->view.top_level = lt;
    t->view.wide_keys = wide ? 1 : 0;
    t->device = device;
    *out = t;
    return ok();
}

void rt_octree_free(rt_octree *tree) { delete tree; }

int64_t rt_octree_leaves(const rt_octree *tree) { return tree ? tree->view.n : -1; }

int rt_octree_depth(const rt_octree *tree) { return tree ? tree->view.depth : -1; }

// ---------------------------------------------------------------------
// Walks
// ---------------------------------------------------------------------

int rt_columns(const rt_octree *tree, const void *d_rho, int precision, const double *d_src,
               int64_t n_src, const double *d_dirs, int64_t n_dirs, double kappa, void *d_N,
               void *d_A, int64_t stride_src, int64_t stride_dir, void *stream) {
    rt::RayBatch rays;
    int st = check_rays(tree, d_src, n_src, d_dirs, n_dirs, stride_src, stride_dir, &rays);
    if (st != RT_OK) return st;
    if (!valid_precision(precision)) return fail(RT_ERR_ARG, "unknown precision %d", precision);
    if (!d_rho || !d_N) return fail(RT_ERR_ARG, "null rho or N");
    if (!std::isfinite(kappa)) return fail(RT_ERR_ARG, "kappa not finite");
    hipError_t e = rt::launch_forward(tree->view, rays, d_rho, precision, kappa, d_N, d_A,
                                      static_cast<hipStream_t>(stream));
    return device_status(e, "forward walk launch");
}

int rt_columns_backward(const rt_octree *tree, const double *d_src, int64_t n_src,
                        const double *d_dirs, int64_t n_dirs, double kappa, const float *d_gN,
                        const float *d_gA, const float *d_A, int64_t stride_src,
                        int64_t stride_dir, double *d_grad_rho, void *stream) {
    rt::RayBatch rays;
    int st = check_rays(tree, d_src, n_src, d_dirs, n_dirs, stride_src, stride_dir, &rays);
    if (st != RT_OK) return st;
    if (!d_grad_rho) return fail(RT_ERR_ARG, "null gradient output");
    if (d_gA && !d_A) return fail(RT_ERR_ARG, "dL/dA given without A");
    if (!std::isfinite(kappa)) return fail(RT_ERR_ARG, "kappa not finite");
    if (!d_gN && !d_gA) return ok();  // zero upstream gradient: nothing to add
    hipError_t e = rt::launch_backward(tree->view, rays, kappa, d_gN, d_gA, d_A, d_grad_rho,
                                       static_cast<hipStream_t>(stream));
    return device_status(e, "adjoint walk launch");
}

int rt_columns_trace(const rt_octree *tree, const double *d_src, int64_t n_src,
                     const double *d_dirs, int64_t n_dirs, int32_t *d_steps, uint64_t *d_hash,
                     int64_t stride_src, int64_t stride_dir, const int64_t *d_sample,
                     int64_t n_sample, int32_t *d_visited, int64_t cap, void *stream) {
    rt::RayBatch rays;
    int st = check_rays(tree, d_src, n_src, d_dirs, n_dirs, stride_src, stride_dir, &rays);
    if (st != RT_OK) return st;
    if (n_sample < 0) return fail(RT_ERR_ARG, "negative n_sample");
    if (n_sample > 0 && (!d_sample || !d_visited || cap < 1))
        return fail(RT_ERR_ARG, "sample rays need d_sample, d_visited and cap >= 1");
    if (n_sample > 0 && n_sample > INT64_MAX / cap) return fail(RT_ERR_ARG, "n_sample * cap overflows");
    hipError_t e = rt::launch_trace(tree->view, rays, d_steps, d_hash, d_sample, n_sample,
                                    d_visited, cap, static_cast<hipStream_t>(stream));
    return device_status(e, "trace walk launch");
}

}  // extern "C"
