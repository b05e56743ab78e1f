// C ABI of the reverse ray-walk library: error reporting, HEALPix
// directions, argument validation and dispatch to the HIP kernels.  The
// octree calls are in rt_octree.cpp.
#include "raytheia.h"
#include "rt_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

namespace {

thread_local std::string g_last_error;

}  // namespace

namespace rt {

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

int device_status(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(RT_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

int check_rays(const rt_octree *tree, const double *d_src, int64_t n_src, const double *d_dirs,
               int64_t n_dirs, int64_t stride_src, int64_t stride_dir, RayBatch *rays) {
    if (!tree) return fail(RT_ERR_ARG, "null octree handle");
    if (!d_src || !d_dirs) return fail(RT_ERR_ARG, "null source or direction pointer");
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail(RT_ERR_DEVICE, "hipGetDevice failed");
    if (device != tree->device)
        return fail(RT_ERR_ARG, "the octree lives on device %d, the current device is %d", tree->device,
                    device);
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

}  // namespace rt

namespace {

using rt::check_rays;
using rt::device_status;
using rt::fail;
using rt::ok;

bool valid_precision(int p) { return p == RT_FP64 || p == RT_FP32_KAHAN; }

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

namespace {

// Centre of pixel j (0-based, azimuth ascending) of ring i (1-based from the
// north pole, 1 .. 4 nside - 1), as a unit vector: caps have 4 i' pixels
// (i' the ring counted from the nearer pole) centred at z = +-(1 - i'^2 / (3
// nside^2)), phi = (j + 1/2) pi / (2 i'); belt rings have 4 nside pixels at
// z = 4/3 - 2 i / (3 nside), phi = (j + s) pi / (2 nside), s = 1/2 when
// i + nside is even and 0 otherwise.
void ring_pixel_centre(int64_t ns, int64_t i, int64_t j, double *out) {
    const double pi = 3.14159265358979323846;
    const double fns = (double)ns;
    double z, phi;
    if (i < ns) {  // north cap
        z = 1.0 - (double)(i * i) / (3.0 * fns * fns);
        phi = ((double)j + 0.5) * (pi / (2.0 * (double)i));
    } else if (i <= 3 * ns) {  // belt
        z = 4.0 / 3.0 - 2.0 * (double)i / (3.0 * fns);
        const double shift = ((i + ns) & 1) ? 0.0 : 0.5;  // half-pixel offset
        phi = ((double)j + shift) * (pi / (2.0 * fns));
    } else {  // south cap, mirror of the north cap
        const int64_t r = 4 * ns - i;
        z = -(1.0 - (double)(r * r) / (3.0 * fns * fns));
        phi = ((double)j + 0.5) * (pi / (2.0 * (double)r));
    }
    const double st = std::sqrt((1.0 - z) * (1.0 + z));
    out[0] = st * std::cos(phi);
    out[1] = st * std::sin(phi);
    out[2] = z;
}

// Even (odd) bits of x packed together: the x (y) coordinate of a NESTED
// in-face index.
int64_t compact_bits(uint64_t x) {
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0f0f0f0f0f0f0f0full;
    x = (x | (x >> 4)) & 0x00ff00ff00ff00ffull;
    x = (x | (x >> 8)) & 0x0000ffff0000ffffull;
    x = (x | (x >> 16)) & 0x00000000ffffffffull;
    return (int64_t)x;
}

}  // namespace

int rt_healpix_dirs(int nside, double *dirs_out) {
    const int64_t npix = rt_healpix_npix(nside);
    if (npix < 0) return fail(RT_ERR_ARG, "nside %d out of range [1, 2^20]", nside);
    if (!dirs_out) return fail(RT_ERR_ARG, "null output pointer");
    const int64_t ns = nside;
    const int64_t ncap = 2 * ns * (ns - 1);  // pixels in the north polar cap
    for (int64_t p = 0; p < npix; ++p) {
        int64_t i, j;
        if (p < ncap) {  // north cap: ring i has 4i pixels
            i = cap_ring(p);
            j = p - 2 * i * (i - 1);
        } else if (p < npix - ncap) {  // belt: 4 nside pixels per ring
            const int64_t q = p - ncap;
            i = q / (4 * ns) + ns;
            j = q % (4 * ns);
        } else {  // south cap, counted from the last pixel
            const int64_t q = npix - 1 - p;
            const int64_t r = cap_ring(q);
            i = 4 * ns - r;
            j = 4 * r - 1 - (q - 2 * r * (r - 1));
        }
        ring_pixel_centre(ns, i, j, dirs_out + 3 * p);
    }
    return ok();
}

int rt_healpix_dirs_nested(int nside, double *dirs_out) {
    const int64_t npix = rt_healpix_npix(nside);
    if (npix < 0) return fail(RT_ERR_ARG, "nside %d out of range [1, 2^20]", nside);
    if (nside & (nside - 1)) return fail(RT_ERR_ARG, "NESTED needs nside a power of two, got %d", nside);
    if (!dirs_out) return fail(RT_ERR_ARG, "null output pointer");
    // Base pixel f (Gorski et al. 2005, the 12 faces): its southmost corner
    // lies on ring face_row[f] * nside (the equator 2 nside for the north
    // faces, 3 nside for the equatorial ones, the south pole 4 nside for the
    // south ones) at azimuth face_col[f] * pi / 4 (the azimuth of the face's
    // nside = 1 centre: pi/4 + k pi/2 for polar faces, k pi/2 on the equator).
    static const int face_row[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
    static const int face_col[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};
    const int64_t ns = nside;
    const int64_t per_face = ns * ns;
    for (int64_t p = 0; p < npix; ++p) {
        const int f = (int)(p / per_face);
        const uint64_t in_face = (uint64_t)(p % per_face);
        const int64_t ix = compact_bits(in_face), iy = compact_bits(in_face >> 1);
        // each step in x or y moves one ring north of the south corner
        const int64_t i = face_row[f] * ns - ix - iy - 1;  // ring, 1-based from the north
        // quarter: pixels of the ring per quarter turn; on_axis: 1 for the
        // belt rings with a centre at azimuth 0 (the others sit half a
        // pixel off it)
        int64_t quarter, on_axis;
        if (i < ns) {
            quarter = i;
            on_axis = 0;
        } else if (i > 3 * ns) {
            quarter = 4 * ns - i;
            on_axis = 0;
        } else {
            quarter = ns;
            on_axis = (i - ns) & 1;
        }
        // azimuth in half pixel steps from the face's corner, east positive
        int64_t pos = (face_col[f] * quarter + ix - iy + 1 + on_axis) / 2;  // 1-based in the ring
        if (pos > 4 * quarter) pos -= 4 * quarter;
        if (pos < 1) pos += 4 * quarter;
        ring_pixel_centre(ns, i, pos - 1, dirs_out + 3 * p);
    }
    return ok();
}

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

int rt_columns_with_adjoint(const rt_octree *tree, const float *d_rho, const double *d_src,
                            int64_t n_src, const double *d_dirs, int64_t n_dirs, double kappa,
                            const float *d_wN, const float *d_wA, float *d_N, float *d_A,
                            int64_t stride_src, int64_t stride_dir, double *d_grad_rho,
                            void *stream) {
    rt::RayBatch rays;
    int st = check_rays(tree, d_src, n_src, d_dirs, n_dirs, stride_src, stride_dir, &rays);
    if (st != RT_OK) return st;
    if (!d_rho || !d_N) return fail(RT_ERR_ARG, "null rho or N");
    if (!d_grad_rho) return fail(RT_ERR_ARG, "null gradient output");
    if (!std::isfinite(kappa)) return fail(RT_ERR_ARG, "kappa not finite");
    hipError_t e;
    if (!d_wN && !d_wA)  // zero loss weights: the forward alone
        e = rt::launch_forward(tree->view, rays, d_rho, RT_FP32_KAHAN, kappa, d_N, d_A,
                               static_cast<hipStream_t>(stream));
    else
        e = rt::launch_forward_adjoint(tree->view, rays, d_rho, kappa, d_wN, d_wA, d_N, d_A,
                                       d_grad_rho, static_cast<hipStream_t>(stream));
    return device_status(e, "forward and adjoint walk launch");
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

// ---------------------------------------------------------------------
// Contribution grid on the device
// ---------------------------------------------------------------------

size_t rt_grid_tree_workspace_bytes(int depth) {
    if (depth < 1 || depth > 10) return 0;
    return rt::grid_tree_workspace_bytes(depth);
}

int rt_grid_tree(const double *d_grid, int depth, double density_floor, double rel_uniformity,
                 void *d_workspace, size_t workspace_bytes, uint64_t *d_keys, uint8_t *d_levels,
                 double *d_values, int64_t *d_n_leaves, void *stream) {
    if (depth < 1 || depth > 10) return fail(RT_ERR_ARG, "depth %d not in 1..10", depth);
    if (!d_grid || !d_keys || !d_levels || !d_values || !d_n_leaves)
        return fail(RT_ERR_ARG, "null grid or output pointer");
    if (!std::isfinite(density_floor) || !std::isfinite(rel_uniformity))
        return fail(RT_ERR_ARG, "density_floor and rel_uniformity must be finite");
    if (!d_workspace) return fail(RT_ERR_WORKSPACE, "null workspace");
    if (((uintptr_t)d_workspace & 255) != 0) return fail(RT_ERR_WORKSPACE, "workspace not 256-byte aligned");
    const size_t need = rt::grid_tree_workspace_bytes(depth);
    if (workspace_bytes < need)
        return fail(RT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    hipError_t e = rt::launch_grid_tree(d_grid, depth, density_floor, rel_uniformity, d_workspace,
                                        d_keys, d_levels, d_values, d_n_leaves,
                                        static_cast<hipStream_t>(stream));
    return device_status(e, "grid tree launch");
}

int rt_grid_tree_static(const double *d_grid, int depth, double density_floor,
                        double rel_uniformity, uint64_t *d_keys, uint8_t *d_levels,
                        double *d_values, int64_t *d_n_leaves, void *stream) {
    if (depth < 1 || depth > rt::kStaticGridMaxDepth)
        return fail(RT_ERR_ARG, "depth %d not in 1..%d (the static scratch holds %zu bytes)", depth,
                    rt::kStaticGridMaxDepth, rt::grid_tree_static_scratch_bytes());
    if (!d_grid || !d_keys || !d_levels || !d_values || !d_n_leaves)
        return fail(RT_ERR_ARG, "null grid or output pointer");
    if (!std::isfinite(density_floor) || !std::isfinite(rel_uniformity))
        return fail(RT_ERR_ARG, "density_floor and rel_uniformity must be finite");
    void *scratch = nullptr;
    hipError_t e = rt::grid_tree_static_scratch(&scratch);
    if (e != hipSuccess) return device_status(e, "static scratch address");
    e = rt::launch_grid_tree(d_grid, depth, density_floor, rel_uniformity, scratch, d_keys,
                             d_levels, d_values, d_n_leaves, static_cast<hipStream_t>(stream));
    return device_status(e, "grid tree launch");
}

// ---------------------------------------------------------------------
// Angular-resolution comparison
// ---------------------------------------------------------------------

int rt_nested_reference(const double *d_fine, int64_t n_fine_dirs, const double *d_coarse,
                        int64_t n_coarse_dirs, int64_t n_src, double *d_ref, double *d_err,
                        void *stream) {
    if (!d_fine) return fail(RT_ERR_ARG, "null fine columns");
    if (n_coarse_dirs < 1 || n_src < 1 || n_fine_dirs < n_coarse_dirs)
        return fail(RT_ERR_ARG, "need n_src >= 1 and n_fine_dirs >= n_coarse_dirs >= 1");
    if (n_fine_dirs > INT64_MAX / n_src) return fail(RT_ERR_ARG, "n_fine_dirs * n_src overflows");
    if (n_fine_dirs % n_coarse_dirs != 0) return fail(RT_ERR_ARG, "n_fine_dirs not a multiple of n_coarse_dirs");
    const int64_t ratio = n_fine_dirs / n_coarse_dirs;
    if (ratio & (ratio - 1) || (__builtin_ctzll((unsigned long long)ratio) & 1))
        return fail(RT_ERR_ARG, "n_fine_dirs / n_coarse_dirs = %lld is not a power of 4", (long long)ratio);
    if (d_err && !d_coarse) return fail(RT_ERR_ARG, "relative errors need the coarse columns");
    if (!d_ref && !d_err) return ok();
    hipError_t e = rt::launch_nested_reference(d_fine, d_coarse, n_coarse_dirs, n_src, ratio, d_ref,
                                               d_err, static_cast<hipStream_t>(stream));
    return device_status(e, "nested reference launch");
}

// ---------------------------------------------------------------------
// Several fields per leaf
// ---------------------------------------------------------------------

namespace {

// rt_shielding and rt_shielding_f32: the same checks and parameters, fields
// in f64 (field_precision 0) or f32 (1).
int shielding_call(const rt_octree *tree, const void *d_fields, int field_precision, int n_fields,
                   const double *d_src, int64_t n_src, const double *d_dirs, int64_t n_dirs,
                   double length, const double *d_temp, double vturb, const double *line_A,
                   const double *line_nu, double gamma, double av0, double *d_rays,
                   double *d_av_eff, double *d_beta, void *stream) {
    rt::RayBatch rays;
    // the per-ray output is [n_fields][n_dirs][n_src]: strides 1 and n_src
    int st = check_rays(tree, d_src, n_src, d_dirs, n_dirs, 1, n_src, &rays);
    if (st != RT_OK) return st;
    if (n_fields < 1 || n_fields > RT_MAX_FIELDS)
        return fail(RT_ERR_ARG, "n_fields %d not in 1..%d", n_fields, RT_MAX_FIELDS);
    if (!d_fields) return fail(RT_ERR_ARG, "null fields");
    if (n_src * n_dirs > INT64_MAX / n_fields) return fail(RT_ERR_ARG, "per-ray output size overflows");
    if (!std::isfinite(length) || !std::isfinite(gamma) || gamma == 0.0 || !std::isfinite(av0))
        return fail(RT_ERR_ARG, "length, gamma and av0 must be finite and gamma non-zero");
    rt::ShieldingParams p;
    p.length = length;
    p.temp = d_temp;
    p.vturb = vturb;
    p.gamma = gamma;
    p.gamma_av0 = gamma * av0;
    for (int f = 0; f < rt::kMaxFields; ++f) p.coef[f] = 0.0;
    if (n_fields > 1) {
        if (!d_temp || !line_A || !line_nu)
            return fail(RT_ERR_ARG, "lines need source temperatures, line_A and line_nu");
        if (!std::isfinite(vturb)) return fail(RT_ERR_ARG, "vturb not finite");
        const double c = 2.99792458e10;  // speed of light, cm/s
        const double pi = 3.14159265358979323846;
        for (int f = 1; f < n_fields; ++f) {
            const double A = line_A[f - 1], nu = line_nu[f - 1];
            if (!std::isfinite(A) || !std::isfinite(nu) || !(nu > 0.0))
                return fail(RT_ERR_ARG, "line %d: A must be finite and nu finite and > 0", f);
            // the prefactor of the discretised line optical depth (sec. 2.4)
            p.coef[f] = A * (c * c * c) / (8.0 * pi * (nu * nu * nu));
            if (!std::isfinite(p.coef[f])) return fail(RT_ERR_ARG, "line %d: prefactor overflows", f);
        }
    }
    if (!d_rays && !d_av_eff && !d_beta) return ok();  // nothing requested
    hipError_t e = rt::launch_shielding(tree->view, rays, d_fields, field_precision, n_fields, p,
                                        d_rays, d_av_eff, n_fields > 1 ? d_beta : nullptr,
                                        static_cast<hipStream_t>(stream));
    return device_status(e, "shielding walk launch");
}

}  // namespace

int rt_shielding(const rt_octree *tree, const double *d_fields, int n_fields, const double *d_src,
                 int64_t n_src, const double *d_dirs, int64_t n_dirs, double length,
                 const double *d_temp, double vturb, const double *line_A, const double *line_nu,
                 double gamma, double av0, double *d_rays, double *d_av_eff, double *d_beta,
                 void *stream) {
    return shielding_call(tree, d_fields, 0, n_fields, d_src, n_src, d_dirs, n_dirs, length, d_temp,
                          vturb, line_A, line_nu, gamma, av0, d_rays, d_av_eff, d_beta, stream);
}

int rt_shielding_f32(const rt_octree *tree, const float *d_fields, int n_fields, const double *d_src,
                     int64_t n_src, const double *d_dirs, int64_t n_dirs, double length,
                     const double *d_temp, double vturb, const double *line_A,
                     const double *line_nu, double gamma, double av0, double *d_rays,
                     double *d_av_eff, double *d_beta, void *stream) {
    return shielding_call(tree, d_fields, 1, n_fields, d_src, n_src, d_dirs, n_dirs, length, d_temp,
                          vturb, line_A, line_nu, gamma, av0, d_rays, d_av_eff, d_beta, stream);
}

}  // extern "C"
