// HIP kernel of the angular-resolution comparison (sec. 3): the reference
// value of a coarse ray is the mean of the finer rays inside its HEALPix
// pixel -- in NESTED order the 4^k consecutive rays q 4^k .. (q+1) 4^k - 1 of
// the direction set k levels finer -- and its relative error is
// |coarse - reference| / reference.
//
// Both sets are direction-major, [dirs][n_src].  One thread per (coarse
// direction, source): adjacent lanes read adjacent sources of one fine
// direction, so every load is coalesced; the 4^k values are summed in
// order, then divided by 4^k.
#include "rt_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace rt {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_nested_reference(
    const double *__restrict__ fine, const double *__restrict__ coarse, int64_t n_coarse,
    int64_t n_src, int64_t ratio, double *__restrict__ ref, double *__restrict__ err) {
    const int64_t total = n_coarse * n_src;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int64_t q = i / n_src;
        const int64_t s = i - q * n_src;
        const double *f = fine + q * ratio * n_src + s;
        double sum = 0.0;
        for (int64_t k = 0; k < ratio; ++k) sum = sum + f[k * n_src];
        const double r = sum / (double)ratio;
        if (ref) ref[i] = r;
        if (err) err[i] = fabs(coarse[i] - r) / r;
    }
}

}  // namespace

hipError_t launch_nested_reference(const double *fine, const double *coarse, int64_t n_coarse,
                                   int64_t n_src, int64_t ratio, double *ref, double *err,
                                   hipStream_t stream) {
    const int64_t total = n_coarse * n_src;
    int64_t blocks = (total + kBlock - 1) / kBlock;
    const int64_t cap = (((int64_t)1 << 32) - 1) / kBlock;  // work items count in 32 bits
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_nested_reference, dim3((unsigned)blocks), dim3(kBlock), 0, stream, fine,
                       coarse, n_coarse, n_src, ratio, ref, err);
    return hipGetLastError();
}

}  // namespace rt
