// HIP kernel for several fields per leaf (gfx950): the walk of rt_ray.h
// integrates K leaf fields at once, and the per-ray columns are turned into
// line optical depths (sec. 2.4) and reduced over the directions of each
// source into escape probabilities (sec. 2.4) and the effective visual
// extinction (sec. 3).
//
// One source per lane, its directions walked one after another: the 64
// lanes of a wavefront hold 64 consecutive sources and walk the same
// direction at the same time, so their rays run parallel through one tube
// of the octree, as in the column kernels.  The reductions over directions
// stay in registers (no atomics, no per-ray buffer), and the K field values
// of a leaf are read together, K * 8 contiguous bytes per step.
//
// Per source s and direction d (I_f = sum_k F[k][f] r_k, visiting order):
//   N_f  = length * I_f;  du = sqrt(8 kB T_s / (pi m_p) + vturb^2);
//   tau_f = coef_f * N_f / du  (coef_f = A c^3 / (8 pi nu^3), from the host);
//   beta_f  = (1/Dn) sum_d (1 - exp(-tau_f)) / tau_f, the term being 1 at
//             tau = 0 and -expm1(-tau) / tau otherwise;
//   AV_eff = -(1/gamma) ln((1/Dn) sum_d exp(-gamma av0 N_0)), kept as a
//            running minimum x_min of x_d = gamma av0 N_0,d and the sum of
//            exp(-(x_d - x_min)), rescaled when the minimum moves, so that no
//            term underflows for large columns.
#include "rt_ray.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace rt {
namespace {

using namespace ray;

// CGS constants (CODATA 2018): Boltzmann constant and proton mass.
constexpr double kBoltzmann = 1.380649e-16;
constexpr double kProtonMass = 1.67262192369e-24;
constexpr double kPi = 3.14159265358979323846;

// The FP64 exp, expm1 and log run once per ray, not per step, and stay out
// of line: inlined, their constants are hoisted out of the direction loop
// and with their temporaries stay live across the walk, which costs 30-50
// VGPRs and half of the waves per SIMD.  Out of line, the kernel needs no
// more registers than the walk with its K sums.
__device__ __noinline__ double exp_term(double x) { return exp(x); }

// (1 - exp(-tau)) / tau, with its limit 1 at tau = 0.
__device__ __noinline__ double escape_term(double tau) {
    return tau == 0.0 ? 1.0 : -expm1(-tau) / tau;
}

__device__ __noinline__ double log_term(double x) { return log(x); }

template <int K, typename FieldT>
struct FieldValues {
    FieldT v[K];
};

// Visitor of walk_ray: reads the K fields of each leaf and accumulates
// I_f = I_f + F_f l in visiting order (two roundings, as in the FP64 column).
// Fields stored in FP32 are widened to FP64 (exactly) before the product.
template <int K, typename FieldT>
struct SumFields {
    const FieldT *__restrict__ F;  // [n][K]
    double I[K];
    __device__ __forceinline__ FieldValues<K, FieldT> fetch(uint32_t i) const {
        FieldValues<K, FieldT> x;
        const FieldT *p = F + (size_t)i * K;
#pragma unroll
        for (int f = 0; f < K; ++f) x.v[f] = p[f];
        return x;
    }
    __device__ __forceinline__ void step(const FieldValues<K, FieldT> &x, uint32_t, double l) {
#pragma unroll
        for (int f = 0; f < K; ++f) I[f] = I[f] + (double)x.v[f] * l;
    }
};

// Waves per SIMD the compiler is asked to fit, by field count and storage.
// The walk is latency-bound, so on coherent rays (sources on a lattice)
// waves hide more than the registers they cost; the registers spilled to
// reach them are all in the per-ray code, none in the step loop.  With the
// fields in FP32: 8 waves at K = 2, 7 at K = 3..4, 5 at K = 5..8, which
// take the lattice workloads 5-14% below 6 waves.  Sources drawn in
// proportion to the density scatter the rays, and there the extra waves
// cost 4-10% (more leaves in flight than the caches hold).  FP64 fields
// need more registers: 5 waves at K <= 4, 4 beyond.  K = 1 fits 8 waves
// with two spilled registers.
template <int K, typename FieldT>
constexpr int kMinWaves = K == 1   ? 8
                          : sizeof(FieldT) == 4 ? (K == 2 ? 8 : K <= 4 ? 7 : 5)
                                                : (K <= 4 ? 5 : 4);

template <typename KeyT, int K, typename FieldT>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(kMinWaves<K, FieldT>))) void k_shielding(Tree<KeyT> t,
                                                      const double *__restrict__ src,
                                                      int64_t n_src, const double *__restrict__ dirs,
                                                      int64_t n_dirs, const FieldT *__restrict__ F,
                                                      ShieldingParams p, double *__restrict__ rays,
                                                      double *__restrict__ av_eff,
                                                      double *__restrict__ beta) {
    __shared__ uint32_t lut[1 << kLutBits];
    init_lut<KeyT>(lut, t.depth);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t plane = n_dirs * n_src;  // one field of the per-ray output
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_src; s += stride) {
        double du = 1.0;
        bool bad = false;
        if (K > 1) {
            du = sqrt(8.0 * kBoltzmann * p.temp[s] / (kPi * kProtonMass) + p.vturb * p.vturb);
            bad = !(du > 0.0 && isfinite(du));
        }
        double xmin = (double)INFINITY, esum = 0.0;
        double bsum[K];
#pragma unroll
        for (int f = 0; f < K; ++f) bsum[f] = 0.0;
        for (int64_t d = 0; d < n_dirs && !bad; ++d) {
            SumFields<K, FieldT> v;
            v.F = F;
#pragma unroll
            for (int f = 0; f < K; ++f) v.I[f] = 0.0;
            if (walk_ray(t, lut, src + 3 * s, dirs + 3 * d, v) < 0) {
                bad = true;
                break;
            }
            const double nh = p.length * v.I[0];
            const double x = p.gamma_av0 * nh;
            if (x < xmin) {
                esum = esum * exp_term(-(xmin - x)) + 1.0;  // 0 * exp(-inf) = 0 on the first ray
                xmin = x;
            } else {
                esum = esum + exp_term(-(x - xmin));
            }
            if (rays) rays[d * n_src + s] = nh;
#pragma unroll
            for (int f = 1; f < K; ++f) {
                const double tau = p.coef[f] * (p.length * v.I[f]) / du;
                bsum[f] = bsum[f] + escape_term(tau);
                if (rays) rays[f * plane + d * n_src + s] = tau;
            }
        }
        if (bad) {
            if (rays)
                for (int f = 0; f < K; ++f)
                    for (int64_t d = 0; d < n_dirs; ++d) rays[f * plane + d * n_src + s] = (double)NAN;
            if (av_eff) av_eff[s] = (double)NAN;
            if (beta)
                for (int f = 1; f < K; ++f) beta[(f - 1) * n_src + s] = (double)NAN;
            continue;
        }
        if (av_eff) av_eff[s] = (xmin - log_term(esum / (double)n_dirs)) / p.gamma;
        if (beta) {
#pragma unroll
            for (int f = 1; f < K; ++f) beta[(f - 1) * n_src + s] = bsum[f] / (double)n_dirs;
        }
    }
}

template <typename KeyT, int K, typename FieldT>
void launch_k(const TreeView &tree, const RayBatch &rays, const FieldT *F, const ShieldingParams &p,
              double *ray_out, double *av_eff, double *beta, hipStream_t stream) {
    hipLaunchKernelGGL((k_shielding<KeyT, K, FieldT>), dim3(grid_for(rays.n_src)), dim3(kBlock), 0,
                       stream, tree_of<KeyT>(tree), rays.src, rays.n_src, rays.dirs, rays.n_dirs, F,
                       p, ray_out, av_eff, beta);
}

template <typename KeyT, typename FieldT>
void launch_key(const TreeView &tree, const RayBatch &rays, const FieldT *F, int K,
                const ShieldingParams &p, double *ray_out, double *av_eff, double *beta,
                hipStream_t stream) {
    switch (K) {
        case 1: launch_k<KeyT, 1>(tree, rays, F, p, ray_out, av_eff, beta, stream); break;
        case 2: launch_k<KeyT, 2>(tree, rays, F, p, ray_out, av_eff, beta, stream); break;
        case 3: launch_k<KeyT, 3>(tree, rays, F, p, ray_out, av_eff, beta, stream); break;
        case 4: launch_k<KeyT, 4>(tree, rays, F, p, ray_out, av_eff, beta, stream); break;
        case 5: launch_k<KeyT, 5>(tree, rays, F, p, ray_out, av_eff, beta, stream); break;
        case 6: launch_k<KeyT, 6>(tree, rays, F, p, ray_out, av_eff, beta, stream); break;
        case 7: launch_k<KeyT, 7>(tree, rays, F, p, ray_out, av_eff, beta, stream); break;
        case 8: launch_k<KeyT, 8>(tree, rays, F, p, ray_out, av_eff, beta, stream); break;
        default: break;
    }
}

template <typename FieldT>
hipError_t launch_fields(const TreeView &tree, const RayBatch &rays, const FieldT *fields,
                         int n_fields, const ShieldingParams &p, double *ray_out, double *av_eff,
                         double *beta, hipStream_t stream) {
    if (n_fields < 1 || n_fields > kMaxFields) return hipErrorInvalidValue;
    if (tree.wide_keys)
        launch_key<uint64_t>(tree, rays, fields, n_fields, p, ray_out, av_eff, beta, stream);
    else
        launch_key<uint32_t>(tree, rays, fields, n_fields, p, ray_out, av_eff, beta, stream);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_shielding(const TreeView &tree, const RayBatch &rays, const void *fields,
                            int field_precision, int n_fields, const ShieldingParams &p,
                            double *ray_out, double *av_eff, double *beta, hipStream_t stream) {
    if (field_precision == 0)
        return launch_fields(tree, rays, static_cast<const double *>(fields), n_fields, p, ray_out,
                             av_eff, beta, stream);
    return launch_fields(tree, rays, static_cast<const float *>(fields), n_fields, p, ray_out, av_eff,
                         beta, stream);
}

}  // namespace rt
