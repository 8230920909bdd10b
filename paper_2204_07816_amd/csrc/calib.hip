// calib.hip -- matrix-core calibration: the rate a register-only loop of
// independent MFMA instructions sustains on the device.  The network kernels'
// roofline fractions are quoted against the published dense peaks (2.5
// PFLOP/s BF16, 78.6 TFLOP/s FP64); this loop, which has no memory traffic,
// no LDS and no vector work, shows how much of those peaks the matrix cores
// deliver under full load, and so what the fractions can reach.
#include "nqs_internal.h"

namespace nqs {
namespace {

constexpr int kThreads = 256;
constexpr int kAcc = 16;  // independent accumulators per wave

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;

// Two waves per SIMD with the accumulators in VGPRs (the file is built with
// the VGPR form of the MFMA instructions): with accumulators in AGPRs the
// compiler copied every accumulator out and back on each iteration, and the
// loop measured the copies (1.46 PFLOP/s BF16) instead of the matrix cores.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_rate_f64(double *out, int iters)
{
    double4_t acc[kAcc];
#pragma unroll
    for (int i = 0; i < kAcc; ++i) acc[i] = (double4_t){0, 0, 0, 0};
    const double a = 1.0 + threadIdx.x * 1e-9, b = 1e-3;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kAcc; ++i)
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kAcc; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_rate_bf16(double *out, int iters)
{
    floatx4 acc[kAcc];
#pragma unroll
    for (int i = 0; i < kAcc; ++i) acc[i] = (floatx4){0, 0, 0, 0};
    bf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(1.0f + threadIdx.x * 1e-3f);
        b[i] = (__bf16)0.5f;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < kAcc; ++i)
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < kAcc; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    out[(int64_t)blockIdx.x * kThreads + threadIdx.x] = s;
}

}  // namespace
}  // namespace nqs

extern "C" nqs_status nqs_mfma_rate(int32_t kind, int64_t workgroups, int32_t iters, double *ms,
                                    double *tflops, void *stream)
{
    using namespace nqs;
    if ((kind != 0 && kind != 1) || workgroups < 1 || workgroups > (1 << 20) || iters < 1 ||
        !ms || !tflops)
        return NQS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (stream_capturing(s)) return NQS_E_WORKSPACE;
    double *out = nullptr;
    if (hipMalloc((void **)&out, sizeof(double) * (size_t)workgroups * kThreads) != hipSuccess)
        return NQS_E_NOMEM;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    nqs_status st = NQS_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = NQS_E_HIP;
    for (int rep = 0; rep < 2 && st == NQS_OK; ++rep) {   // the first launch warms up
        (void)hipEventRecord(e0, s);
        if (kind == 0)
            NQS_LAUNCH(k_rate_bf16, dim3((unsigned)workgroups), dim3(kThreads), 0, s, out, iters);
        else
            NQS_LAUNCH(k_rate_f64, dim3((unsigned)workgroups), dim3(kThreads), 0, s, out, iters);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) st = NQS_E_HIP;
    }
    float t = 0.0f;
    if (st == NQS_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = NQS_E_HIP;
    if (st == NQS_OK) {
        const double per = kind == 0 ? 16.0 * 16 * 32 * 2 : 16.0 * 16 * 4 * 2;   // flops per MFMA
        const double flops = (double)workgroups * (kThreads / 64) * iters * kAcc * per;
        *ms = t;
        *tflops = flops / ((double)t * 1e-3) / 1e12;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return st;
}
