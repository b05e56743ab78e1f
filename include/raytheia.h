/*
 * raytheia.h -- C ABI of the MI355X reverse ray-walk library.
 *
 * The library computes direction-dependent column integrals by reverse ray
 * tracing (Zhu et al., "RAYTHEIA", sec. 2): for every source point p and
 * every direction q, a ray starts at p and walks outward through a leaf-only
 * linear octree (the AMR contribution grid, sec. 2.2), leaf by leaf (DDA
 * stepping with a Morton-key lookup, sec. 2.3.1), takes the exact chord of
 * each leaf by the slab method (sec. 2.3.2), and accumulates
 *     N(p, q) = sum_k rho_k r_k        (the discrete integral of sec. 2.3)
 * and the attenuation A = exp(-kappa N) (solution of the absorption-only
 * transfer equation, sec. 2.1) up to the boundary of the unit box.  Around
 * that walk: its adjoint, several fields per walk (line optical depths,
 * escape probabilities and the effective visual extinction, sec. 2.4 and
 * 3), the angular-resolution comparison of sec. 3, and the construction of
 * the contribution grid from a uniform grid (sec. 2.4).
 *
 * Conventions (all calls):
 *   - The domain is the unit box [0,1)^3; cells are half-open.  A tree of
 *     maximum depth D (1..21) has finest cells of edge h = 2^-D.  A leaf's key
 *     is the Morton code at depth D of its minimum corner (bit b of the
 *     integer x coordinate -> key bit 3b, y -> 3b+1, z -> 3b+2); a leaf of
 *     level L spans 8^(D-L) consecutive keys.
 *   - "host" pointers are read during the call only.  "device" pointers are
 *     HIP device memory owned by the caller; the library only borrows them.
 *     The library never allocates device memory: the octree lives in a
 *     caller-provided workspace.
 *   - Every call returns an rt_status (0 = RT_OK, < 0 = error); nothing
 *     throws or aborts.  On error, rt_last_error() gives a message (thread-
 *     local).  Argument checks run synchronously on the host before any
 *     device work is queued (rt_build_octree_device checks its device leaf
 *     arrays with a kernel and waits for the result); device work is queued
 *     on the given stream (a hipStream_t passed as void*, NULL = the default
 *     stream) and runs asynchronously.
 *   - Calls that launch kernels may run concurrently on different streams,
 *     also on the same octree: the octree is read-only after building.
 *   - An octree belongs to the device that was current when it was built;
 *     walk calls with another device current fail with RT_ERR_ARG.  Their
 *     device pointers must address memory of that device: the kernels
 *     dereference them as they are, and the library cannot tell a host or
 *     foreign pointer from its own (a wrong one faults the GPU).
 */
#ifndef RAYTHEIA_H
#define RAYTHEIA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RT_OK = 0,
    RT_ERR_ARG = -1,       /* null pointer, bad size, bad nside/depth, overflow */
    RT_ERR_UNSORTED = -2,  /* leaf keys not strictly increasing */
    RT_ERR_TILING = -3,    /* leaves misaligned, overlapping, gapped, level > D */
    RT_ERR_RANGE = -4,     /* value outside its domain */
    RT_ERR_DEVICE = -5,    /* a HIP runtime call failed */
    RT_ERR_WORKSPACE = -6  /* workspace too small or misaligned */
} rt_status;

typedef enum {
    RT_FP64 = 0,       /* rho f64, N/A f64: FP64 slab tests and FP64 accumulation */
    RT_FP32_KAHAN = 1  /* rho f32, N/A f32: FP64 slab tests (same traversal as
                          RT_FP64), rho*l summed in FP32 with Kahan compensation */
} rt_precision;

typedef struct rt_octree rt_octree; /* opaque host handle */

/* ABI version of this header (incremented on incompatible changes). */
#define RT_ABI_VERSION 1
int rt_abi_version(void);

/* Static description of a status code; never NULL. */
const char *rt_status_string(int status);

/* Message of the last failing call on this thread ("" if none). */
const char *rt_last_error(void);

/* ---------------------------------------------------------------------
 * Directions (sec. 2.1: HEALPix pixel centres, N_rays = 12 * 4^l with
 * nside = 2^l; any nside >= 1 is accepted).
 * ------------------------------------------------------------------- */

/* Number of directions 12 * nside^2, or -1 if nside < 1 or nside > 2^20. */
int64_t rt_healpix_npix(int nside);

/* Writes the HEALPix RING-order pixel centres as unit vectors to host
 * memory dirs_out[npix][3] (rings from the north pole, azimuth ascending).
 * Errors: RT_ERR_ARG (bad nside, null pointer). */
int rt_healpix_dirs(int nside, double *dirs_out);

/* The same centres in NESTED order (Gorski et al. 2005): pixel
 * p = f nside^2 + i of base pixel f = 0..11, whose in-face index i
 * interleaves the face coordinates (bit b of x -> bit 2b, of y -> bit 2b+1).
 * The 4 pixels 4p .. 4p+3 at 2 nside subdivide pixel p at nside, which is
 * what comparisons across resolutions need (sec. 3: a ray's reference
 * column is the mean over the finer rays inside its pixel).  Each centre is
 * bit-identical to the RING table's centre of the same pixel.  Errors:
 * RT_ERR_ARG (bad nside, nside not a power of two, null pointer). */
int rt_healpix_dirs_nested(int nside, double *dirs_out);

/* ---------------------------------------------------------------------
 * Contribution grid: the leaf-only linear octree (sec. 2.3.1).
 * ------------------------------------------------------------------- */

/* Device bytes that rt_build_octree needs for n_leaves leaves at depth
 * max_depth; 0 if the arguments are invalid. */
size_t rt_octree_workspace_bytes(int64_t n_leaves, int max_depth);

/* Validates a leaf-only linear octree and stages its search structures in
 * the caller's device workspace.
 *   keys[n_leaves]   host, Morton keys of the leaves' minimum corners,
 *                    strictly increasing;
 *   levels[n_leaves] host, refinement level of each leaf (0..max_depth);
 *   max_depth        D, 1..21;
 *   d_workspace      device, >= rt_octree_workspace_bytes(n, D) bytes,
 *                    256-byte aligned; must stay allocated and unmodified
 *                    while the handle is used;
 *   stream           the upload is queued on it (the host arrays may be
 *                    reused as soon as the call returns).
 * The leaf values are not part of the octree: they are passed to every
 * rt_columns call (so values can change without rebuilding).
 * Errors: RT_ERR_ARG, RT_ERR_UNSORTED, RT_ERR_TILING (key[0] != 0, a key not
 * aligned to its leaf's span, a gap or overlap key[i] + 8^(D-level[i]) !=
 * key[i+1], or a last leaf not ending at 8^D), RT_ERR_WORKSPACE,
 * RT_ERR_DEVICE.  On success *out receives a handle to free with
 * rt_octree_free. */
int rt_build_octree(const uint64_t *keys, const uint8_t *levels, int64_t n_leaves,
                    int max_depth, void *d_workspace, size_t workspace_bytes, void *stream,
                    rt_octree **out);

/* rt_build_octree for leaf arrays already in device memory (for example the
 * output of rt_grid_tree): the same checks, made by kernels, and the same
 * workspace contents.  d_keys [n_leaves] u64 and d_levels [n_leaves] u8 are
 * device pointers; n_leaves is a host value.  The call waits for the checks
 * (it synchronises the stream once); the staging is then queued on stream,
 * and the leaf arrays must stay unchanged until it has run.  Errors as for
 * rt_build_octree (RT_ERR_UNSORTED names the first unsorted index,
 * RT_ERR_TILING the first leaf with a tiling error). */
int rt_build_octree_device(const uint64_t *d_keys, const uint8_t *d_levels, int64_t n_leaves,
                           int max_depth, void *d_workspace, size_t workspace_bytes, void *stream,
                           rt_octree **out);

/* Releases the host handle (the workspace stays the caller's). NULL is ok. */
void rt_octree_free(rt_octree *tree);

/* Leaf count and depth of a built octree (-1 for NULL). */
int64_t rt_octree_leaves(const rt_octree *tree);
int rt_octree_depth(const rt_octree *tree);

/* Device bytes of the workspace of rt_grid_tree at depth 1..10; 0 otherwise. */
size_t rt_grid_tree_workspace_bytes(int depth);

/* Builds the contribution grid on the device from a uniform grid by the
 * density + uniformity rule (sec. 2.4): starting from the root, a cell of
 * level L < depth is split into its 8 children iff, over the fine cells it
 * covers, max >= density_floor and (max - min) >= rel_uniformity * max; an
 * unsplit cell whose ancestors are all split, or a fine cell under a split
 * level-(depth-1) cell, is a leaf.  A leaf's value is the mean of its fine
 * cells, formed level by level as the mean of its 8 children's values
 * (summed in child order, divided by 8).
 *   d_grid      device f64 [8^depth], finite values in Morton order (fine cell
 *               i has Morton key i at this depth);
 *   depth       1..10;
 *   d_workspace device, >= rt_grid_tree_workspace_bytes(depth) bytes,
 *               256-byte aligned (the max/min/mean/split pyramid and the
 *               block offsets);
 *   d_keys, d_levels, d_values  device outputs with room for 8^depth
 *               entries: the leaves' Morton keys at this depth, levels and
 *               values, in key order (the input of rt_build_octree and of
 *               the walks);
 *   d_n_leaves  device int64 output, the leaf count.
 * Device work is queued on stream; nothing is read back.  Errors:
 * RT_ERR_ARG (depth, null pointers, non-finite parameters),
 * RT_ERR_WORKSPACE, RT_ERR_DEVICE. */
int rt_grid_tree(const double *d_grid, int depth, double density_floor, double rel_uniformity,
                 void *d_workspace, size_t workspace_bytes, uint64_t *d_keys, uint8_t *d_levels,
                 double *d_values, int64_t *d_n_leaves, void *stream);

/* rt_grid_tree for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same kernels, the same outputs, bit for bit, but the pyramid and the block
 * offsets live in a static scratch array of the library
 * (rt_grid_tree_workspace_bytes(7) = 7,498,752 bytes) instead of a caller
 * workspace.  Each GPU the
 * library runs on holds its own copy until the process ends; its device
 * address is looked up on the first call on that device.  The call
 * allocates nothing and needs no zeroed memory (every scratch byte is
 * written before it is read).  All calls on one GPU share that GPU's
 * scratch: calls that may overlap on one GPU (on different streams, or from
 * several host threads) race and must be serialised by the caller.
 *   depth   1..7 (grids of at most 128^3 cells); deeper grids are refused;
 *   other arguments as for rt_grid_tree.
 * Errors: RT_ERR_ARG (depth beyond 7, null pointers, non-finite
 * parameters), RT_ERR_DEVICE. */
int rt_grid_tree_static(const double *d_grid, int depth, double density_floor,
                        double rel_uniformity, uint64_t *d_keys, uint8_t *d_levels,
                        double *d_values, int64_t *d_n_leaves, void *stream);

/* ---------------------------------------------------------------------
 * Column densities (sec. 2.3: I(p,q) = sum_k f_k r_k with f = rho).
 * ------------------------------------------------------------------- */

/* Forward walk of every ray (s, d), s < n_src, d < n_dirs.
 *   d_rho    device, [n_leaves] leaf values, f64 for RT_FP64 and f32 for
 *            RT_FP32_KAHAN; finite and >= 0 (not checked);
 *   d_src    device, f64 [n_src][3] source points, each in [0,1)^3;
 *   d_dirs   device, f64 [n_dirs][3] ray directions (finite, not all zero;
 *            HEALPix unit vectors in the usual case);
 *   kappa    attenuation coefficient for A = exp(-kappa N);
 *   d_N      device output, N of ray (s, d) at d_N[s*stride_src + d*stride_dir]
 *            (f64 or f32 per precision);
 *   d_A      device output or NULL, A at the same offsets;
 * The layout stride_src = 1, stride_dir = n_src (direction-major) gives
 * coalesced stores.  A ray whose source lies outside [0,1)^3 or whose
 * direction is invalid yields N = A = NaN (no other effect).
 * Errors: RT_ERR_ARG (null pointers, n_src < 1, n_dirs < 1, n_src*n_dirs
 * overflow, bad precision, negative strides), RT_ERR_DEVICE. */
int rt_columns(const rt_octree *tree, const void *d_rho, int precision, const double *d_src,
               int64_t n_src, const double *d_dirs, int64_t n_dirs, double kappa, void *d_N,
               void *d_A, int64_t stride_src, int64_t stride_dir, void *stream);

/* Adjoint of rt_columns for a loss L(N, A): re-walks the same rays and
 * scatters g * l into the leaf gradient, where for each ray
 *     g = dL/dN - kappa * A * dL/dA      (A = exp(-kappa N)),
 * i.e. d_grad_rho[k] += sum over rays of g * r_k (N is linear in rho).
 *   d_gN     device f32, dL/dN at the rt_columns offsets, or NULL (= 0);
 *   d_gA     device f32, dL/dA, or NULL (= 0);
 *   d_A      device f32, the A of the forward call; required iff d_gA;
 *   d_grad_rho device f64 [n_leaves], accumulated with atomic adds (the
 *            caller zeroes it); the summation order is not deterministic.
 *            It must be coarse-grained device memory (hipMalloc, or a
 *            device tensor of a framework that allocates with it): the adds
 *            are the hardware FP64 atomics, which fine-grained, managed or
 *            host memory does not support and would lose without an error.
 * The traversal is the FP64 one of rt_columns; g * r is formed in FP32,
 * summed in FP32 over a few steps of neighbouring rays, then added to the
 * FP64 accumulator.  Errors: RT_ERR_ARG, RT_ERR_DEVICE. */
int rt_columns_backward(const rt_octree *tree, const double *d_src, int64_t n_src,
                        const double *d_dirs, int64_t n_dirs, double kappa, const float *d_gN,
                        const float *d_gA, const float *d_A, int64_t stride_src,
                        int64_t stride_dir, double *d_grad_rho, void *stream);

/* rt_columns (RT_FP32_KAHAN) and rt_columns_backward in one pass, for a loss
 * linear in N and A whose weights are known before the walk:
 *     L = sum over rays of (wN * N + wA * A),  so  g = wN - kappa * A * wA.
 * Each ray is walked for its column, N and A are stored, and the ray is
 * walked again to scatter g * r_k (the same two walks as the separate
 * calls, fused so that the second finds the leaves of the first in cache).
 *   d_rho    device f32 [n_leaves] leaf values;
 *   d_wN, d_wA  device f32 weights at the rt_columns offsets, or NULL (= 0);
 *   d_N      device f32 output; d_A device f32 output or NULL;
 *   d_grad_rho device f64 [n_leaves], accumulated (the caller zeroes it);
 *            coarse-grained device memory, as for rt_columns_backward.
 * N and A have the bits of rt_columns with RT_FP32_KAHAN; the gradient is
 * that of rt_columns_backward with d_gN = d_wN, d_gA = d_wA and the same A,
 * up to the order of its additions.  Invalid rays give N = A = NaN and add
 * nothing.  With both weights NULL only the forward runs.
 * Errors: RT_ERR_ARG, RT_ERR_DEVICE. */
int rt_columns_with_adjoint(const rt_octree *tree, const float *d_rho, const double *d_src,
                            int64_t n_src, const double *d_dirs, int64_t n_dirs, double kappa,
                            const float *d_wN, const float *d_wA, float *d_N, float *d_A,
                            int64_t stride_src, int64_t stride_dir, double *d_grad_rho,
                            void *stream);

/* Traversal record of every ray, for verification: the number of leaves
 * visited and a 64-bit FNV-1a-style hash of the visited leaf indices
 * (h = 0xcbf29ce484222325; per leaf index i: h = (h ^ i) * 0x100000001b3 mod
 * 2^64), written at the rt_columns offsets to d_steps (int32) and d_hash
 * (uint64).  In addition, for the n_sample rays listed in d_sample (device
 * int64 ray ids r = d * n_src + s), the first cap visited leaf indices go to
 * d_visited[j * cap ...] (int32, -1 after the end).  d_sample / d_visited may
 * be NULL when n_sample is 0.  Errors: RT_ERR_ARG, RT_ERR_DEVICE. */
int rt_columns_trace(const rt_octree *tree, const double *d_src, int64_t n_src,
                     const double *d_dirs, int64_t n_dirs, int32_t *d_steps, uint64_t *d_hash,
                     int64_t stride_src, int64_t stride_dir, const int64_t *d_sample,
                     int64_t n_sample, int32_t *d_visited, int64_t cap, void *stream);

/* ---------------------------------------------------------------------
 * Angular-resolution comparison (sec. 3).
 * ------------------------------------------------------------------- */

/* Reference values and relative errors of a coarse direction set against a
 * finer one, both in HEALPix NESTED order (rt_healpix_dirs_nested) with
 * n_fine_dirs = 4^k n_coarse_dirs: the reference of coarse ray (q, s) is the
 * mean of the fine rays q 4^k .. (q+1) 4^k - 1 of source s (the finer
 * pixels inside pixel q), summed in that order and divided by 4^k, and its
 * error is |coarse - reference| / reference (the relative column error of
 * sec. 3; inf or NaN where the reference is 0).
 *   d_fine    device f64 [n_fine_dirs][n_src] (rt_columns with stride_src = 1,
 *             stride_dir = n_src);
 *   d_coarse  device f64 [n_coarse_dirs][n_src], or NULL when d_err is NULL;
 *   d_ref, d_err  device outputs or NULL, f64 [n_coarse_dirs][n_src].
 * Errors: RT_ERR_ARG (null pointers, counts < 1, a ratio that is not a power
 * of 4, overflow), RT_ERR_DEVICE. */
int rt_nested_reference(const double *d_fine, int64_t n_fine_dirs, const double *d_coarse,
                        int64_t n_coarse_dirs, int64_t n_src, double *d_ref, double *d_err,
                        void *stream);

/* ---------------------------------------------------------------------
 * Several fields per leaf: line optical depths, escape probabilities and
 * the effective visual extinction (sec. 2.4 and sec. 3).
 * ------------------------------------------------------------------- */

/* Largest number of leaf fields of one rt_shielding call. */
#define RT_MAX_FIELDS 8

/* One walk per ray (s, d) integrates K = n_fields leaf fields at once,
 * I_f = sum_k F[k][f] r_k (FP64, visiting order, the traversal of
 * rt_columns), and the results are reduced over the n_dirs directions of
 * each source.  Field 0 is the hydrogen number density n_H (cm^-3); field
 * f = 1 .. K-1 is the level-population term [n_j g_i / g_j - n_i] (cm^-3)
 * of line f (sec. 2.4).  With N_f = length * I_f (cm^-2):
 *   du(s)    = sqrt(8 kB T_s / (pi m_p) + vturb^2), kB = 1.380649e-16 erg/K,
 *              m_p = 1.67262192369e-24 g (the line width of sec. 2.4: the mean
 *              thermal speed and the turbulent speed in quadrature);
 *   tau_f    = A_f c^3 / (8 pi nu_f^3) * N_f / du, c = 2.99792458e10 cm/s
 *              (the discretised line optical depth of sec. 2.4);
 *   beta_f(s) = (1/n_dirs) sum_d (1 - exp(-tau_f)) / tau_f, with the term 1
 *              at tau = 0, for either sign of tau (escape probability,
 *              sec. 2.4);
 *   av_eff(s) = -(1/gamma) ln((1/n_dirs) sum_d exp(-gamma av0 N_0))
 *              (effective visual extinction, sec. 3; evaluated without
 *              underflow for large columns).
 *   d_fields  device f64 [n_leaves][n_fields] (a leaf's fields contiguous);
 *   n_fields  K, 1..RT_MAX_FIELDS;
 *   d_src, d_dirs as for rt_columns;
 *   length    edge of the unit box in cm;
 *   d_temp    device f64 [n_src], source gas temperatures in K; required
 *             when n_fields > 1, else ignored (may be NULL);
 *   vturb     turbulent speed in cm/s;
 *   line_A, line_nu  host f64 [n_fields - 1], Einstein A (s^-1) and line
 *             frequency (Hz) of each line; required when n_fields > 1;
 *   gamma, av0  dust attenuation factor and A_V per unit column (the paper
 *             uses 3.02 and 6.29e-22 mag cm^2);
 *   d_rays    device output or NULL, f64 [n_fields][n_dirs][n_src]: N_0 in
 *             plane 0 and tau_f in plane f;
 *   d_av_eff  device output or NULL, f64 [n_src];
 *   d_beta    device output or NULL, f64 [n_fields - 1][n_src] (ignored
 *             when n_fields = 1).
 * One lane walks all directions of one source, so n_src should be large
 * (>= 10^5) to fill the GPU.  A source outside [0,1)^3, an invalid
 * direction, or du not finite and > 0 gives NaN in all outputs of that
 * source.  Errors: RT_ERR_ARG (null pointers, counts out of range, output
 * size overflow, non-finite length/gamma/av0/vturb/A, nu <= 0, gamma = 0),
 * RT_ERR_DEVICE. */
int rt_shielding(const rt_octree *tree, const double *d_fields, int n_fields, const double *d_src,
                 int64_t n_src, const double *d_dirs, int64_t n_dirs, double length,
                 const double *d_temp, double vturb, const double *line_A, const double *line_nu,
                 double gamma, double av0, double *d_rays, double *d_av_eff, double *d_beta,
                 void *stream);

/* rt_shielding with the leaf fields stored in FP32: d_fields is device f32
 * [n_leaves][n_fields], half the bytes per step of the walk.  Each field is
 * widened to FP64 (exactly) before the same FP64 products and sums, so the
 * outputs equal those of rt_shielding on the fields widened to f64.  Other
 * arguments, outputs and errors as for rt_shielding. */
int rt_shielding_f32(const rt_octree *tree, const float *d_fields, int n_fields, const double *d_src,
                     int64_t n_src, const double *d_dirs, int64_t n_dirs, double length,
                     const double *d_temp, double vturb, const double *line_A,
                     const double *line_nu, double gamma, double av0, double *d_rays,
                     double *d_av_eff, double *d_beta, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RAYTHEIA_H */
