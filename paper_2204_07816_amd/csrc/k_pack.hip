// k_pack.hip -- the parameter update of the VMC loop on the device [Sec. 3.2:
// the SR direction updates the weights]: theta <- theta + scale * dtheta on
// the canonical FP64 copy, then every kernel family's packing rebuilt from
// it, so that a whole VMC iteration needs no host round trip and can be
// captured in a graph.  The packings are the ones the host builds when the
// weights are set (same layouts, same FP64 -> FP32 / BF16 roundings), so a
// device update and setting the updated weights from the host give identical
// kernel inputs.
#include <algorithm>

#include "nqs_internal.h"

namespace nqs {
namespace {

constexpr int kThreads = 256;

// theta[i] + scale * d[i] without contraction (product rounded, then sum)
__global__ void k_axpy(double *__restrict__ w, const double *__restrict__ d, double scale,
                       int64_t n)
{
#pragma clang fp contract(off)
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const double p = scale * d[i];
        w[i] = w[i] + p;
    }
}

// w = theta (a kernel rather than a copy call, so that a captured graph holds
// only kernel nodes)
__global__ void k_copy_f64(double *__restrict__ w, const double *__restrict__ theta, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        w[i] = theta[i];
}

// offset of layer l in the canonical vector (layer 1 has one input channel)
__device__ inline int64_t canon_off(int l, int C)
{
    return l == 0 ? 0 : (int64_t)(C * 9 + C) + (int64_t)(l - 1) * (C * C * 9 + C);
}

// vector-path packing: per layer [9][cin][C] then the bias; FP64 and FP32
__global__ void k_pack_vec(const double *__restrict__ w, int K, int C, int64_t P,
                           double *__restrict__ v64, float *__restrict__ v32)
{
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < P;
         q += (int64_t)gridDim.x * kThreads) {
        int l = 0;
        while (l + 1 < K && q >= canon_off(l + 1, C)) ++l;
        const int64_t base = canon_off(l, C);
        const int cin = l == 0 ? 1 : C;
        const int64_t r = q - base;
        double v;
        if (r < (int64_t)9 * cin * C) {
            const int t = (int)(r / ((int64_t)cin * C));
            const int rem = (int)(r - (int64_t)t * cin * C);
            const int ci = rem / C, co = rem - (rem / C) * C;
            v = w[base + ((int64_t)co * cin + ci) * 9 + t];
        } else {
            v = w[base + r];                                // bias: same position
        }
        v64[q] = v;
        v32[q] = (float)v;
    }
}

// backward data pass, layers 2..K: [t'][co][ci] = W[co][ci][8 - t']
__global__ void k_pack_bwd(const double *__restrict__ w, int K, int C, double *__restrict__ bw)
{
    const int64_t per = (int64_t)9 * C * C, n = per * (K - 1);
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kThreads) {
        const int l = 1 + (int)(q / per);
        const int r = (int)(q - (int64_t)(l - 1) * per);
        const int t = r / (C * C), co = (r / C) % C, ci = r % C;
        bw[q] = w[canon_off(l, C) + ((int64_t)co * C + ci) * 9 + (8 - t)];
    }
}

// FP64 -> BF16, round to nearest even: through FP32, with the FP32 value on
// a BF16 midpoint decided against the exact double (no double rounding)
__device__ inline uint16_t bf16_rne_d(double d)
{
    const float f = __double2float_rn(d);
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // NaN
    const uint32_t low = u & 0xffffu;
    uint32_t hi = u >> 16;
    if (low == 0x8000u) {
        const uint32_t lo_b = u & 0xffff0000u, up_b = lo_b + 0x10000u;
        const double mid = 0.5 * ((double)__uint_as_float(lo_b) + (double)__uint_as_float(up_b));
        const double ad = fabs(d), am = fabs(mid);
        if (ad > am)
            hi += 1;
        else if (ad == am)
            hi += (hi & 1);
        return (uint16_t)hi;
    }
    if (low > 0x8000u) hi += 1;
    return (uint16_t)hi;
}

__device__ inline int chan_of_slot_d(int q, int C)
{
    if (C == 32) {
        const int g = q >> 3, r = q & 7;
        return r < 4 ? 4 * g + r : 16 + 4 * g + (r - 4);
    }
    return q;
}

// BF16 A operands of layers 2..K: [l-1][j][h][lane][i]; lane l holds output
// channel 16 h + l % 16 and the 8 reduction elements of lane group l / 16
__global__ void k_pack_mfma(const double *__restrict__ w, int K, int C,
                            uint16_t *__restrict__ wm, uint16_t *__restrict__ wlo)
{
    const int KS = (C == 32) ? 9 : 5, NH = C / 16;
    const int64_t per = (int64_t)KS * NH * 64 * 8, n = per * (K - 1);
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kThreads) {
        const int l = 1 + (int)(q / per);
        int r = (int)(q - (int64_t)(l - 1) * per);
        const int i = r & 7;
        r >>= 3;
        const int lane = r & 63;
        r >>= 6;
        const int h = r % NH, j = r / NH;
        const int g = lane >> 4, co = 16 * h + (lane & 15);
        int tap, ci;
        if (C == 32) {
            tap = j;
            ci = chan_of_slot_d(g * 8 + i, 32);
        } else {
            tap = 2 * j + (g >> 1);
            ci = (g & 1) * 8 + i;
        }
        const double wv = tap <= 8 ? w[canon_off(l, C) + ((int64_t)co * C + ci) * 9 + tap] : 0.0;
        const uint16_t hi = bf16_rne_d(wv);
        wm[q] = hi;
        // split form: lo = bf16(W - hi), the difference exact in FP64
        if (wlo) wlo[q] = bf16_rne_d(wv - (double)__uint_as_float((uint32_t)hi << 16));
    }
}

// layer-1 weights [9][C] and the biases of all layers [K][C], FP32
__global__ void k_pack_l1(const double *__restrict__ w, int K, int C, float *__restrict__ l1)
{
    const int n = 9 * C + K * C;
    for (int q = blockIdx.x * kThreads + threadIdx.x; q < n; q += gridDim.x * kThreads) {
        double v;
        if (q < 9 * C) {
            const int t = q / C, co = q - t * C;
            v = w[co * 9 + t];
        } else {
            const int l = (q - 9 * C) / C, co = (q - 9 * C) - l * C;
            v = w[canon_off(l, C) + (int64_t)C * (l == 0 ? 1 : C) * 9 + co];
        }
        l1[q] = (float)v;
    }
}

int grid_of(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads, 4096));
}

}  // namespace

// every kernel family's packing rebuilt from the canonical vector w_canon
static void device_repack(nqs_ctx *c, hipStream_t s)
{
    const int K = c->K, C = c->C;
    if (const BlockNet *bn = block_net(c)) {   // only the packing of a block network
        bn->pack_device(c, s);
        return;
    }
    NQS_LAUNCH(k_pack_vec, dim3(grid_of(c->P)), dim3(kThreads), 0, s, (const double *)c->w_canon,
               K, C, c->P, c->w_vec64, c->w_vec32);
    if (K > 1)
        NQS_LAUNCH(k_pack_bwd, dim3(grid_of((int64_t)9 * C * C * (K - 1))), dim3(kThreads), 0, s,
                   (const double *)c->w_canon, K, C, c->w_bwd64);
    if (c->dtype == NQS_BF16 || c->dtype == NQS_BF16X3) {
        const int KS = (C == 32) ? 9 : 5;
        NQS_LAUNCH(k_pack_mfma, dim3(grid_of((int64_t)(K - 1) * KS * (C / 16) * 512)),
                   dim3(kThreads), 0, s, (const double *)c->w_canon, K, C, c->w_mfma,
                   c->dtype == NQS_BF16X3 ? c->w_mfma_lo : (uint16_t *)nullptr);
        NQS_LAUNCH(k_pack_l1, dim3(grid_of(9 * C + K * C)), dim3(kThreads), 0, s,
                   (const double *)c->w_canon, K, C, c->w_l1);
    }
}

void device_update_weights(nqs_ctx *c, const double *dtheta, double scale, hipStream_t s)
{
    NQS_LAUNCH(k_axpy, dim3(grid_of(c->P)), dim3(kThreads), 0, s, c->w_canon, dtheta, scale,
               c->P);
    device_repack(c, s);
}

void device_set_weights(nqs_ctx *c, const double *theta, hipStream_t s)
{
    NQS_LAUNCH(k_copy_f64, dim3(grid_of(c->P)), dim3(kThreads), 0, s, c->w_canon, theta, c->P);
    device_repack(c, s);
}

}  // namespace nqs
