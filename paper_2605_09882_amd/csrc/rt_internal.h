// Internal interface between the C ABI sources (rt_abi.cpp, rt_octree.cpp)
// and the HIP kernels.  Not installed; the public interface is
// include/raytheia.h.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

struct rt_octree;

namespace rt {

// Top-table entry: the leaf index in the low 30 bits, plus
//   kTopFull: the cell is refined to the maximum depth everywhere, so leaf
//             index = entry + (key mod keys per cell) and level = D;
//   kTopOne:  a single leaf (the entry's) covers the whole cell.
// Without either flag the cell's leaves are entry .. next entry - 1.
constexpr uint32_t kTopFull = 0x80000000u;
constexpr uint32_t kTopOne = 0x40000000u;
constexpr uint32_t kTopIndex = 0x3fffffffu;

// Device view of a built octree.  keys holds n+1 entries: the n leaf keys
// and a sentinel 8^D, narrowed to 32 bits when D <= 10; levels the n leaf
// levels.  top[c] for the
// 8^top_level cells c of level top_level is the index of the leaf holding the
// cell's first finest cell; top[8^top_level] = n.  The leaf holding key k is
// then found in [top[c], top[c+1]] with c = k >> 3 (D - top_level).
struct TreeView {
    const void *keys;
    const uint8_t *levels;  // n refinement levels
    const uint32_t *top;
    int64_t n;
    int depth;
    int top_level;
    int wide_keys;  // 0: uint32_t keys, 1: uint64_t keys
};

// Rays (s, d) for s < n_src, d < n_dirs; outputs at s*stride_src + d*stride_dir.
struct RayBatch {
    const double *src;
    int64_t n_src;
    const double *dirs;
    int64_t n_dirs;
    int64_t stride_src;
    int64_t stride_dir;
};

// Level of the top table for a tree of the given depth and leaf count.
int top_table_level(int depth, int64_t n_leaves);

// Error reporting of the C ABI: fail() records the message for
// rt_last_error and returns status; ok() clears it and returns RT_OK;
// device_status() maps a HIP error to RT_ERR_DEVICE (or ok()).
int fail(int status, const char *fmt, ...);
int ok();
int device_status(hipError_t e, const char *what);

// Checks a batch of rays (handle, pointers, counts, output strides and
// their offset range) and fills its kernel-side description.
int check_rays(const rt_octree *tree, const double *d_src, int64_t n_src, const double *d_dirs,
               int64_t n_dirs, int64_t stride_src, int64_t stride_dir, RayBatch *rays);

hipError_t launch_forward(const TreeView &tree, const RayBatch &rays, const void *rho,
                          int precision, double kappa, void *N, void *A, hipStream_t stream);

hipError_t launch_backward(const TreeView &tree, const RayBatch &rays, double kappa,
                           const float *gN, const float *gA, const float *A, double *grad,
                           hipStream_t stream);

hipError_t launch_forward_adjoint(const TreeView &tree, const RayBatch &rays, const float *rho,
                                  double kappa, const float *wN, const float *wA, float *N, float *A,
                                  double *grad, hipStream_t stream);

// Several fields per leaf (rt_shielding): at most kMaxFields fields, field 0
// the hydrogen density, fields 1.. the population terms of the lines.
constexpr int kMaxFields = 8;

struct ShieldingParams {
    double length;            // box edge in cm
    const double *temp;       // device, [n_src] source temperatures (K), used when K > 1
    double vturb;             // turbulent speed, cm/s
    double gamma;             // dust attenuation factor
    double gamma_av0;         // gamma * av0
    double coef[kMaxFields];  // coef[f] = A_f c^3 / (8 pi nu_f^3) for f = 1 .. K-1
};

// fields: f64 [n][K] (field_precision 0) or f32 [n][K] (1).
hipError_t launch_shielding(const TreeView &tree, const RayBatch &rays, const void *fields,
                            int field_precision, int n_fields, const ShieldingParams &p,
                            double *ray_out, double *av_eff, double *beta, hipStream_t stream);

hipError_t launch_nested_reference(const double *fine, const double *coarse, int64_t n_coarse,
                                   int64_t n_src, int64_t ratio, double *ref, double *err,
                                   hipStream_t stream);

// Octree staging from device leaf arrays (rt_build_octree_device).
hipError_t launch_octree_check(const uint64_t *keys, const uint8_t *levels, int64_t n, int depth,
                               int64_t *status, hipStream_t stream);
hipError_t launch_octree_stage(const uint64_t *keys, const uint8_t *levels, int64_t n, int depth,
                               int top_level, void *key_out, uint8_t *level_out, uint32_t *top,
                               hipStream_t stream);

// Contribution grid from a uniform grid (rt_grid_tree).
size_t grid_tree_workspace_bytes(int depth);
// rt_grid_tree_static: grids up to this depth use the library's static
// scratch, whose device address on the current device the second call
// returns (looked up once per device).
constexpr int kStaticGridMaxDepth = 7;
size_t grid_tree_static_scratch_bytes();
hipError_t grid_tree_static_scratch(void **ptr);
hipError_t launch_grid_tree(const double *grid, int depth, double floor_, double rel,
                            void *workspace, uint64_t *keys, uint8_t *levels, double *values,
                            int64_t *n_out, hipStream_t stream);

// Measurement probes (rt_calib_*): bytes per stream block, and launches.
size_t calib_stream_granule();
hipError_t launch_calib_copy(const void *src, void *dst, size_t bytes, hipStream_t stream);
hipError_t launch_calib_read(const void *src, size_t bytes, uint32_t *sink, hipStream_t stream);
hipError_t launch_calib_valu(int kind, int64_t n_threads, int iters, uint32_t *out,
                             hipStream_t stream);

hipError_t launch_trace(const TreeView &tree, const RayBatch &rays, int32_t *steps,
                        uint64_t *hash, const int64_t *sample, int64_t n_sample,
                        int32_t *visited, int64_t cap, hipStream_t stream);

}  // namespace rt

// Host handle of a built octree (opaque in the public header).
struct rt_octree {
    rt::TreeView view;
    int device;
};
