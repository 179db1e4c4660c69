// Peak-rate probes of the two arithmetic units the blind rotation runs on,
// measured at the occupancy of the throughput kernels (one workgroup of
// eight waves per compute unit, two waves per SIMD): independent FP64 fused
// multiply-add chains on the vector ALUs, and independent
// v_mfma_i32_16x16x64_i8 accumulations on the matrix cores. The kernels'
// fractions of peak are quoted against these beside the published figures.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/cemu_measure.h"
#include "cemu_internal.h"

namespace cemu {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 512;
constexpr int kFmaChains = 16;
constexpr int kMfmaChains = 8;

// Sixteen independent chains per lane: a <- a * m + c, which stays finite.
__global__ void fp64_fma_probe(double *__restrict__ sink, int iters)
{
    const int t = blockIdx.x * kProbeThreads + threadIdx.x;
    double a[kFmaChains];
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) a[k] = 1.0 + 1e-9 * t + 0.125 * k;
    const double m = 0.9999999, c = 1e-7;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kFmaChains; ++k) a[k] = fma(a[k], m, c);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) s += a[k];
    sink[t] = s;
}

// Eight independent accumulators per wave, one MFMA each per iteration.
__global__ void int8_mfma_probe(int *__restrict__ sink, int iters)
{
    const int t = blockIdx.x * kProbeThreads + threadIdx.x;
    const v4i a = v4i{t, t + 1, t + 2, t + 3};
    const v4i b = v4i{3 * t, t ^ 5, t + 7, 11};
    v4i acc[kMfmaChains];
#pragma unroll
    for (int k = 0; k < kMfmaChains; ++k) acc[k] = v4i{k, 0, 0, 0};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kMfmaChains; ++k) acc[k] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc[k], 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int k = 0; k < kMfmaChains; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    sink[t] = s;
}

// LDS bandwidth at the same occupancy: each wave writes (or reads) its own
// 8 KiB region as eight rows of 64 consecutive 16-byte slots per iteration
// (no bank conflicts), at a per-lane base plus immediate offsets, so that no
// address arithmetic sits between the accesses (with an address computed
// per access the reads measured about 40 % slower; the writes did not
// change).
typedef unsigned u4v __attribute__((ext_vector_type(4)));
constexpr int kLdsSlots = 4096;   // 16-byte slots, 64 KiB: wave w owns [512 w, 512 w + 512)

__global__ void lds_write_probe(unsigned *__restrict__ sink, int iters)
{
    __shared__ u4v buf[kLdsSlots];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    u4v *base = buf + 512 * w + lane;
    u4v v = u4v{(unsigned)tid, 1u, 2u, 3u};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r) base[64 * r] = v;
        v.x += 1u;
        __asm__ volatile("" ::: "memory");   // keep every store
    }
    __syncthreads();
    sink[blockIdx.x * kProbeThreads + tid] = buf[(tid * 7) & (kLdsSlots - 1)].x;
}

__global__ void lds_read_probe(unsigned *__restrict__ sink, int iters)
{
    __shared__ u4v buf[kLdsSlots];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int e = tid; e < kLdsSlots; e += kProbeThreads) buf[e] = u4v{(unsigned)e, 1u, 2u, 3u};
    __syncthreads();
    const u4v *base = buf + 512 * w + lane;
    u4v acc = u4v{0u, 0u, 0u, 0u};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r) acc ^= base[64 * r];
        __asm__ volatile("" ::: "memory");   // keep every load
    }
    sink[blockIdx.x * kProbeThreads + tid] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

std::string msg(const char *what, hipError_t e) { return std::string(what) + ": " + hipGetErrorString(e); }

// Milliseconds of one launch of f, bracketed by events on stream s.
template <class F>
int time_launch(hipStream_t s, F &&f, float *ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) {
        f();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e == hipSuccess ? CEMU_OK : fail(CEMU_ERR_HIP, msg("peak probe", e));
}

}  // namespace
}  // namespace cemu

using namespace cemu;

extern "C" int cemu_measure_peaks(double *fp64_flops_per_s, double *int8_ops_per_s, void *hip_stream)
{
    clear_error();
    if (!fp64_flops_per_s || !int8_ops_per_s) return fail(CEMU_ERR_NULL, "NULL result pointer");
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cus <= 0) return fail(CEMU_ERR_HIP, msg("device query", e));
    const size_t threads = (size_t)cus * kProbeThreads;
    void *sink = nullptr;
    if (hipMalloc(&sink, threads * sizeof(double)) != hipSuccess) return fail(CEMU_ERR_OOM, "probe buffer");
    hipStream_t s = (hipStream_t)hip_stream;
    const int fma_iters = 1 << 16, mfma_iters = 1 << 14;
    // Eight timed launches of each, alternating, and the fastest of each
    // counts: the first ones run while the clocks ramp up from idle (and the
    // code objects load).
    float ms_fma = 0.f, ms_mfma = 0.f;
    int rc = CEMU_OK;
    for (int rep = 0; rep < 8 && rc == CEMU_OK; ++rep) {
        float t = 0.f;
        rc = time_launch(s, [&] {
            hipLaunchKernelGGL(fp64_fma_probe, dim3(cus), dim3(kProbeThreads), 0, s, (double *)sink, fma_iters);
        }, &t);
        if (rc == CEMU_OK && t > 0.f && (ms_fma == 0.f || t < ms_fma)) ms_fma = t;
        if (rc == CEMU_OK)
            rc = time_launch(s, [&] {
                hipLaunchKernelGGL(int8_mfma_probe, dim3(cus), dim3(kProbeThreads), 0, s, (int *)sink, mfma_iters);
            }, &t);
        if (rc == CEMU_OK && t > 0.f && (ms_mfma == 0.f || t < ms_mfma)) ms_mfma = t;
    }
    (void)hipFree(sink);
    if (rc != CEMU_OK) return rc;
    if (!(ms_fma > 0.f) || !(ms_mfma > 0.f)) return fail(CEMU_ERR_HIP, "peak probe: no elapsed time");
    *fp64_flops_per_s = 2.0 * kFmaChains * (double)fma_iters * (double)threads / (ms_fma * 1e-3);
    const double waves = (double)cus * (kProbeThreads / 64);
    *int8_ops_per_s = 2.0 * 16 * 16 * 64 * kMfmaChains * (double)mfma_iters * waves / (ms_mfma * 1e-3);
    return CEMU_OK;
}

extern "C" int cemu_measure_lds(double *write_bytes_per_s, double *read_bytes_per_s, void *hip_stream)
{
    clear_error();
    if (!write_bytes_per_s || !read_bytes_per_s) return fail(CEMU_ERR_NULL, "NULL result pointer");
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cus <= 0) return fail(CEMU_ERR_HIP, msg("device query", e));
    const size_t threads = (size_t)cus * kProbeThreads;
    void *sink = nullptr;
    if (hipMalloc(&sink, threads * sizeof(double)) != hipSuccess) return fail(CEMU_ERR_OOM, "probe buffer");
    hipStream_t s = (hipStream_t)hip_stream;
    const int iters = 1 << 12;
    float ms_w = 0.f, ms_r = 0.f;
    int rc = CEMU_OK;
    for (int rep = 0; rep < 8 && rc == CEMU_OK; ++rep) {
        float t = 0.f;
        rc = time_launch(s, [&] {
            hipLaunchKernelGGL(lds_write_probe, dim3(cus), dim3(kProbeThreads), 0, s, (unsigned *)sink, iters);
        }, &t);
        if (rc == CEMU_OK && t > 0.f && (ms_w == 0.f || t < ms_w)) ms_w = t;
        if (rc == CEMU_OK)
            rc = time_launch(s, [&] {
                hipLaunchKernelGGL(lds_read_probe, dim3(cus), dim3(kProbeThreads), 0, s, (unsigned *)sink, iters);
            }, &t);
        if (rc == CEMU_OK && t > 0.f && (ms_r == 0.f || t < ms_r)) ms_r = t;
    }
    (void)hipFree(sink);
    if (rc != CEMU_OK) return rc;
    if (!(ms_w > 0.f) || !(ms_r > 0.f)) return fail(CEMU_ERR_HIP, "LDS probe: no elapsed time");
    const double bytes = 8.0 * 16.0 * (double)iters * (double)threads;
    *write_bytes_per_s = bytes / (ms_w * 1e-3);
    *read_bytes_per_s = bytes / (ms_r * 1e-3);
    return CEMU_OK;
}
