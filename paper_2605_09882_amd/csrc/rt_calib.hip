// Measurement probes for the roofline of the walk kernels (gfx950): the
// achievable HBM bandwidth of a plain stream, and the VALU issue rate of
// instruction chains of known length.  They compute nothing of the method.
//
// Streams: 16-byte loads (and stores), four per lane issued back to back,
// 256 threads per block and one block per 16 KB, so that the dispatcher keeps
// every CU full of wavefronts with several 1 KB requests in flight each, and
// consecutive lanes touch consecutive 16-byte words.
//
// VALU probes: every lane runs kChains independent dependency chains of one
// instruction type for `iters` iterations; the loop counter is uniform
// (scalar), so a wavefront issues kChains vector instructions per iteration
// plus a constant prologue and epilogue.  With enough waves per SIMD to hide
// each chain's latency, the issue rate over the launch is the VALU ceiling
// for that instruction type.
#include "rt_internal.h"
#include "raytheia.h"
#include "raytheia_calib.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rt {
namespace {

constexpr int kStreamBlock = 256;
constexpr int kPerThread = 4;
constexpr int kChains = 8;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Each block moves kPerThread * 256 16-byte words (the caller passes whole
// blocks): every lane issues its kPerThread loads (words kStreamBlock apart)
// before it stores or combines any, so each wavefront keeps kPerThread 1 KB
// requests in flight.
__global__ __launch_bounds__(kStreamBlock) void k_copy16(const u32x4 *__restrict__ src,
                                                          u32x4 *__restrict__ dst) {
    const int64_t base = (int64_t)blockIdx.x * (kPerThread * kStreamBlock) + threadIdx.x;
    u32x4 v[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) v[u] = __builtin_nontemporal_load(src + base + u * kStreamBlock);
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) __builtin_nontemporal_store(v[u], dst + base + u * kStreamBlock);
}

// Read-only stream: XOR of every 32-bit word, one value per block (so the
// loads cannot be dropped), written to sink[blockIdx.x].
__global__ __launch_bounds__(kStreamBlock) void k_read16(const u32x4 *__restrict__ src,
                                                          uint32_t *__restrict__ sink) {
    __shared__ uint32_t s_part[kStreamBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * (kPerThread * kStreamBlock) + threadIdx.x;
    u32x4 v[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) v[u] = __builtin_nontemporal_load(src + base + u * kStreamBlock);
    uint32_t acc = 0;
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = s_part[0] ^ s_part[1] ^ s_part[2] ^ s_part[3];
}

// kind 0: v_fma_f64 chains; kind 1: v_xad_u32 chains ((a ^ k) + b, one
// instruction); kind 2: v_fma_f32 chains (packed FP32 is disabled for this
// library, so one lane op each).
__global__ __launch_bounds__(256) void k_valu_f64(int iters, uint32_t *__restrict__ out) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    double a[kChains];
    const double m = 1.0 - 1e-9 * (double)(threadIdx.x & 7);
    const double c = 1e-3 * (double)(tid & 15);
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = (double)(tid + j);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = fma(a[j], m, c);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[tid] = (uint32_t)(int64_t)s;
}

__global__ __launch_bounds__(256) void k_valu_i32(int iters, uint32_t *__restrict__ out) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a[kChains], k[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
        a[j] = (uint32_t)(tid * 7 + j);
        k[j] = 0x9e3779b9u * (uint32_t)(j + 1) ^ (uint32_t)tid;
    }
    for (int it = 0; it < iters; ++it) {
        uint32_t b[kChains];
#pragma unroll
        for (int j = 0; j < kChains; ++j) b[j] = (a[j] ^ k[j]) + a[(j + 1) % kChains];
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = b[j];
    }
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s ^= a[j];
    out[tid] = s;
}

__global__ __launch_bounds__(256) void k_valu_f32(int iters, uint32_t *__restrict__ out) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    float a[kChains];
    const float m = 1.0f - 1e-7f * (float)(threadIdx.x & 7);
    const float c = 1e-3f * (float)(tid & 15);
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = (float)(tid + j);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = fmaf(a[j], m, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[tid] = (uint32_t)(int32_t)s;
}

}  // namespace

size_t calib_stream_granule() { return (size_t)16 * kPerThread * kStreamBlock; }

hipError_t launch_calib_copy(const void *src, void *dst, size_t bytes, hipStream_t stream) {
    const unsigned blocks = (unsigned)(bytes / calib_stream_granule());
    hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(kStreamBlock), 0, stream,
                       static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst));
    return hipGetLastError();
}

hipError_t launch_calib_read(const void *src, size_t bytes, uint32_t *sink, hipStream_t stream) {
    const unsigned blocks = (unsigned)(bytes / calib_stream_granule());
    hipLaunchKernelGGL(k_read16, dim3(blocks), dim3(kStreamBlock), 0, stream,
                       static_cast<const u32x4 *>(src), sink);
    return hipGetLastError();
}

hipError_t launch_calib_valu(int kind, int64_t n_threads, int iters, uint32_t *out,
                             hipStream_t stream) {
    const unsigned blocks = (unsigned)(n_threads / 256);
    if (kind == 0)
        hipLaunchKernelGGL(k_valu_f64, dim3(blocks), dim3(256), 0, stream, iters, out);
    else if (kind == 1)
        hipLaunchKernelGGL(k_valu_i32, dim3(blocks), dim3(256), 0, stream, iters, out);
    else
        hipLaunchKernelGGL(k_valu_f32, dim3(blocks), dim3(256), 0, stream, iters, out);
    return hipGetLastError();
}

}  // namespace rt

using rt::fail;

extern "C" {

size_t rt_calib_stream_granule(void) { return rt::calib_stream_granule(); }

static int check_stream(const void *p, size_t bytes) {
    const size_t g = rt::calib_stream_granule();
    if (!p) return fail(RT_ERR_ARG, "null stream buffer");
    if (((uintptr_t)p & 15) != 0) return fail(RT_ERR_ARG, "stream buffer not 16-byte aligned");
    if (bytes == 0 || bytes % g != 0 || bytes / g > 0x7fffffffu)
        return fail(RT_ERR_ARG, "stream bytes %zu not a positive multiple of %zu (at most 2^31 - 1 of them)",
                    bytes, g);
    return RT_OK;
}

int rt_calib_copy(const void *d_src, void *d_dst, size_t bytes, void *stream) {
    int st = check_stream(d_src, bytes);
    if (st != RT_OK) return st;
    st = check_stream(d_dst, bytes);
    if (st != RT_OK) return st;
    const uintptr_t a = (uintptr_t)d_src, b = (uintptr_t)d_dst;
    if (a < b + bytes && b < a + bytes) return fail(RT_ERR_ARG, "copy buffers overlap");
    return rt::device_status(rt::launch_calib_copy(d_src, d_dst, bytes, static_cast<hipStream_t>(stream)),
                             "stream copy launch");
}

int rt_calib_read(const void *d_src, size_t bytes, uint32_t *d_sink, void *stream) {
    int st = check_stream(d_src, bytes);
    if (st != RT_OK) return st;
    if (!d_sink) return fail(RT_ERR_ARG, "null sink");
    return rt::device_status(rt::launch_calib_read(d_src, bytes, d_sink, static_cast<hipStream_t>(stream)),
                             "stream read launch");
}

int rt_calib_valu(int kind, int64_t n_threads, int iters, uint32_t *d_out, void *stream) {
    if (kind < 0 || kind > 2) return fail(RT_ERR_ARG, "unknown probe kind %d", kind);
    if (n_threads < 256 || n_threads % 256 != 0 || n_threads > 0x7fffff00LL)
        return fail(RT_ERR_ARG, "n_threads %lld not a positive multiple of 256 below 2^31", (long long)n_threads);
    if (iters < 1) return fail(RT_ERR_ARG, "iters must be >= 1");
    if (!d_out) return fail(RT_ERR_ARG, "null output");
    return rt::device_status(
        rt::launch_calib_valu(kind, n_threads, iters, d_out, static_cast<hipStream_t>(stream)),
        "VALU probe launch");
}

}  // extern "C"
