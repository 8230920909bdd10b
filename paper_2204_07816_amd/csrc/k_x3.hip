// k_x3.hip -- the split-BF16 (BF16X3) form of the CNN log-amplitude for the
// base pass of the samples and the full recomputation of exchanged
// configurations [Sec. 5.2: periodic 3x3 convolutions, log of a product of
// neurons; Sec. 5.4.1: the network over the exchanged configurations].
//
// Every operand of layers 2..K is carried as hi + lo BF16 (hi = bf16(x),
// lo = bf16(x - hi), |x - hi - lo| <= 2^-16 |x|) and each product as
// hi*hi + hi*lo + lo*hi: three v_mfma_f32_16x16x32_bf16 per tap and output
// half, FP32 accumulation seeded with the bias (the bf16x3 scheme of Henry,
// Tang and Heinecke, 2019).  Layer 1 (one input channel) is FP32 on the vector
// ALU.  Activations are split again after each layer's ln cosh.
//
// One launch per layer over all configurations: the previous layer's plane is
// read from global memory (the activation cache in the base pass, a scratch
// plane in full mode), so no layer has to fit in LDS.  Per output site the
// arithmetic is the incremental cone kernel's -- the same K-step order, the
// same three products in the same order, the same ln cosh and split, the same
// FP64 channel-sum order -- so the cached activations and site sums are
// exactly what the cone kernel computes for the sites an exchange does not
// reach.
//
// Plane layout: [configuration][site][64 BF16]; the 16-byte chunk g (g < 4)
// of a site holds the hi parts of channel slots 8g..8g+7, chunk 4 + g their lo
// parts (slot order of mf::chan_of_slot).
#include <algorithm>

#include "mfma_common.h"

namespace nqs {
namespace {

using mf::bf16x8;
using mf::floatx4;

constexpr int C = 32;
constexpr int KS = 9;
constexpr int NH = 2;
constexpr int kNW = 4;
constexpr int kThreads = kNW * 64;
constexpr int kSite = 2 * C;          // BF16 values per site (hi then lo)

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int wrapi(int a, int L)
{
    a += (a < 0) ? L : 0;
    return a - ((a >= L) ? L : 0);
}

__device__ __forceinline__ uint32_t pack2(uint16_t a, uint16_t b)
{
    return (uint32_t)a | ((uint32_t)b << 16);
}

// Geometry of configuration `cfg`: its sample and, in full mode, the exchanged
// pair (qi = qj = -1 for a sample's own network).
struct X3Args {
    const int8_t *spins;
    int L, K;
    int full;                   // 0: base pass of samples; 1: queue items q0 + cfg
    const uint32_t *queue;
    const int64_t *qlen;
    int64_t q0, M;              // configurations of this launch
    const float *w1;            // layer 1 [9][C], then the biases [K][C] (logical channels)
    const bf16x8 *wa, *wl;      // A operands (hi, lo) of layers 2..K: [k-2][KS][NH][64 lanes]
};

__device__ __forceinline__ bool cfg_live(const X3Args &a, int64_t cfg)
{
    return cfg < a.M && (!a.full || a.q0 + cfg < a.qlen[0]);
}

// Layer 1: one thread per (configuration, site, channel pair m); slots 2m and
// 2m + 1 of chunk m / 4, in the cone kernel's FMA order (bias, taps 0..8).
__global__ void __launch_bounds__(256) k_x3_layer1(X3Args a, uint16_t *out, int64_t out_stride)
{
    const int L = a.L, N = L * L;
    const int64_t total = a.M * N * 16;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * 256) {
        const int m = (int)(t & 15);
        const int64_t ps = t >> 4;
        const int64_t cfg = ps / N;
        const int p = (int)(ps - cfg * N);
        if (!cfg_live(a, cfg)) continue;
        int s = (int)cfg, qi = -1, qj = -1;
        if (a.full) {
            const uint32_t e = a.queue[a.q0 + cfg];
            s = item_sample(e);
            const int b = item_bond(e), tau = b & 3, i = b >> 2;
            qi = i;
            qj = wrapi(i / L + bond_dy(tau), L) * L + wrapi(i % L + bond_dx(tau), L);
        }
        const int8_t *sp = a.spins + (int64_t)s * N;
        const int x = p % L, y = p / L;
        float sv[9];
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) {
            int site = wrapi(y + tp / 3 - 1, L) * L + wrapi(x + tp % 3 - 1, L);
            site = (site == qi) ? qj : ((site == qj) ? qi : site);
            sv[tp] = (float)sp[site];
        }
        const int c0 = mf::chan_of_slot<C>(2 * m), c1 = mf::chan_of_slot<C>(2 * m + 1);
        float z0 = a.w1[9 * C + c0], z1 = a.w1[9 * C + c1];
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) {
            z0 = __builtin_fmaf(a.w1[tp * C + c0], sv[tp], z0);
            z1 = __builtin_fmaf(a.w1[tp * C + c1], sv[tp], z1);
        }
        uint16_t h0, l0, h1, l1;
        mf::split_bf16(mf::ln_cosh_x3(z0), &h0, &l0);
        mf::split_bf16(mf::ln_cosh_x3(z1), &h1, &l1);
        uint16_t *site_out = out + cfg * out_stride + (int64_t)p * kSite;
        *(uint32_t *)(site_out + 2 * m) = pack2(h0, h1);
        *(uint32_t *)(site_out + C + 2 * m) = pack2(l0, l1);
    }
}

// Layer k >= 2: work units of 16 consecutive sites of one configuration, one
// per wave at a time; the wave holds the layer's hi and lo A operands.  The
// last layer writes the per-site FP64 channel sums to hs_out[cfg][site].
__global__ void __launch_bounds__(kThreads) k_x3_conv(X3Args a, int k, const uint16_t *in,
                                                      int64_t in_stride, uint16_t *out,
                                                      int64_t out_stride, double *hs_out)
{
    const int L = a.L, N = L * L;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, n16 = lane & 15;
    const bool last = (k == a.K);
    bf16x8 wh[KS][NH], wl[KS][NH];
    {
        const bf16x8 *bh = a.wa + (int64_t)(k - 2) * KS * NH * 64;
        const bf16x8 *bl = a.wl + (int64_t)(k - 2) * KS * NH * 64;
#pragma unroll
        for (int j = 0; j < KS; ++j)
#pragma unroll
            for (int hh = 0; hh < NH; ++hh) {
                wh[j][hh] = bh[(j * NH + hh) * 64 + lane];
                wl[j][hh] = bl[(j * NH + hh) * 64 + lane];
            }
    }
    floatx4 bias[NH];
#pragma unroll
    for (int hh = 0; hh < NH; ++hh)
#pragma unroll
        for (int r = 0; r < 4; ++r) bias[hh][r] = a.w1[9 * C + (k - 1) * C + 16 * hh + 4 * g + r];

    const int tiles = (N + 15) >> 4;
    const int64_t units = a.M * tiles;
    for (int64_t u = (int64_t)blockIdx.x * kNW + wave; u < units; u += (int64_t)gridDim.x * kNW) {
        const int64_t cfg = u / tiles;
        const int tile = (int)(u - cfg * tiles);
        if (!cfg_live(a, cfg)) continue;       // uniform over the wave
        int p = tile * 16 + n16;
        const bool valid = p < N;
        p = valid ? p : N - 1;
        const int x = p % L, y = p / L;
        const uint16_t *pin = in + cfg * in_stride;
        floatx4 acc[NH];
#pragma unroll
        for (int j = 0; j < KS; ++j) {
            const int q = wrapi(y + j / 3 - 1, L) * L + wrapi(x + j % 3 - 1, L);
            const bf16x8 bh = *(const bf16x8 *)(pin + (int64_t)q * kSite + 8 * g);
            const bf16x8 bl = *(const bf16x8 *)(pin + (int64_t)q * kSite + C + 8 * g);
#pragma unroll
            for (int hh = 0; hh < NH; ++hh) {
                floatx4 c0 = j == 0 ? bias[hh] : acc[hh];
                c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl[j][hh], bh, c0, 0, 0, 0);
                c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh[j][hh], bl, c0, 0, 0, 0);
                acc[hh] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh[j][hh], bh, c0, 0, 0, 0);
            }
        }
        float zv[8], hv[8];
#pragma unroll
        for (int hh = 0; hh < NH; ++hh)
#pragma unroll
            for (int r = 0; r < 4; ++r) zv[hh * 4 + r] = acc[hh][r];
        mf::ln_cosh_x3_n<8>(zv, hv);
        if (!last) {
            uint16_t hi[8], lo[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) mf::split_bf16(hv[r], &hi[r], &lo[r]);
            if (valid) {
                uint16_t *site_out = out + cfg * out_stride + (int64_t)p * kSite;
                const u32x4 ph = {pack2(hi[0], hi[1]), pack2(hi[2], hi[3]), pack2(hi[4], hi[5]),
                                  pack2(hi[6], hi[7])};
                const u32x4 pl = {pack2(lo[0], lo[1]), pack2(lo[2], lo[3]), pack2(lo[4], lo[5]),
                                  pack2(lo[6], lo[7])};
                *(u32x4 *)(site_out + 8 * g) = ph;
                *(u32x4 *)(site_out + C + 8 * g) = pl;
            }
        } else {
            double part = 0.0;
#pragma unroll
            for (int r = 0; r < 8; ++r) part += (double)hv[r];
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            if (g == 0 && valid) hs_out[cfg * N + p] = part;
        }
    }
}

// f[s] = sum_p hs[s][p] (base pass) or dlog[q0 + cfg] = sum_p (hs[cfg][p] -
// hsum[sample][p]) (full mode): one workgroup per configuration, a fixed-order
// tree over the sites.
__global__ void __launch_bounds__(256) k_x3_reduce(X3Args a, const double *hs, const double *hsum,
                                                   double *f_out, double *dlog, int32_t *err)
{
    __shared__ double red[256];
    const int N = a.L * a.L;
    for (int64_t cfg = blockIdx.x; cfg < a.M; cfg += gridDim.x) {
        if (!cfg_live(a, cfg)) continue;
        const double *row = hs + cfg * N;
        const double *base = nullptr;
        if (a.full) base = hsum + (int64_t)item_sample(a.queue[a.q0 + cfg]) * N;
        double v = 0.0;
        for (int p = threadIdx.x; p < N; p += 256) v += a.full ? row[p] - base[p] : row[p];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double t = red[0];
            if (!isfinite(t)) atomicOr(err, kErrNonFinite);
            if (a.full)
                dlog[a.q0 + cfg] = t;
            else
                f_out[cfg] = t;
        }
        __syncthreads();
    }
}

X3Args args_of(const nqs_ctx *c, const int8_t *spins)
{
    X3Args a{};
    a.spins = spins;
    a.L = c->L;
    a.K = c->K;
    a.w1 = c->w_l1;
    a.wa = (const bf16x8 *)c->w_mfma;
    a.wl = (const bf16x8 *)c->w_mfma_lo;
    return a;
}

unsigned grid_for(int64_t work, int per_block, int cap)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + per_block - 1) / per_block, cap));
}

// Layers 1..K of M configurations: layer k's plane is plane(k) (k = 1..K-1),
// the last layer's site sums go to hs.
template <typename PlaneOf>
void run_layers(const nqs_ctx *c, const X3Args &a, PlaneOf plane, int64_t stride, double *hs,
                hipStream_t s)
{
    const int N = c->N;
    NQS_LAUNCH(k_x3_layer1, dim3(grid_for(a.M * N * 16, 256, 65536)), dim3(256), 0, s, a,
               plane(1), stride);
    const int64_t units = a.M * ((N + 15) / 16);
    const unsigned grid = grid_for(units, kNW, c->n_cu * 8);
    for (int k = 2; k <= c->K; ++k)
        NQS_LAUNCH(k_x3_conv, dim3(grid), dim3(kThreads), 0, s, a, k,
                   (const uint16_t *)plane(k - 1), stride, k < c->K ? plane(k) : (uint16_t *)nullptr,
                   stride, hs);
}

}  // namespace

bool x3_supported(const nqs_ctx *c) { return c->C == 32 && c->K >= 2; }

size_t x3_cache_bytes(const nqs_ctx *c, int64_t B)
{
    return (size_t)B * (c->K - 1) * c->N * kSite * sizeof(uint16_t);
}

size_t x3_plane_bytes(const nqs_ctx *c, int64_t M)
{
    return (size_t)M * c->N * kSite * sizeof(uint16_t);
}

size_t x3_sums_bytes(const nqs_ctx *c, int64_t M) { return (size_t)M * c->N * sizeof(double); }

int64_t x3_chunk(const nqs_ctx *c, int64_t work)
{
    const size_t per = 2 * x3_plane_bytes(c, 1) + x3_sums_bytes(c, 1);
    const int64_t m = (int64_t)(((size_t)1 << 30) / per);
    return std::max<int64_t>(1, std::min<int64_t>(m, std::max<int64_t>(work, 1)));
}

void x3_base_forward(const nqs_ctx *c, const int8_t *spins, int B, double *f, double *hsum,
                     void *cache, void *hs_tmp, hipStream_t s)
{
    (void)hs_tmp;
    if (B <= 0) return;
    X3Args a = args_of(c, spins);
    a.full = 0;
    a.M = B;
    uint16_t *cb = (uint16_t *)cache;
    const int64_t layer = (int64_t)c->N * kSite;
    const int64_t stride = (int64_t)(c->K - 1) * layer;
    // the cache holds layer k of sample s at [s][k - 1]
    run_layers(c, a, [&](int k) { return cb + (int64_t)(k - 1) * layer; }, stride, hsum, s);
    NQS_LAUNCH(k_x3_reduce, dim3(grid_for(B, 1, 65536)), dim3(256), 0, s, a, (const double *)hsum,
               (const double *)nullptr, f, (double *)nullptr, c->err);
}

void x3_conn_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                     const int64_t *qlen, int64_t q0, int64_t M, const double *hsum, double *dlog,
                     void *plane_a, void *plane_b, void *hs_tmp, hipStream_t s)
{
    if (M <= 0) return;
    X3Args a = args_of(c, spins);
    a.full = 1;
    a.queue = queue;
    a.qlen = qlen;
    a.q0 = q0;
    a.M = M;
    uint16_t *pa = (uint16_t *)plane_a, *pb = (uint16_t *)plane_b;
    const int64_t stride = (int64_t)c->N * kSite;
    run_layers(c, a, [&](int k) { return (k & 1) ? pa : pb; }, stride, (double *)hs_tmp, s);
    NQS_LAUNCH(k_x3_reduce, dim3(grid_for(M, 1, 65536)), dim3(256), 0, s, a,
               (const double *)hs_tmp, hsum, (double *)nullptr, dlog, c->err);
}

}  // namespace nqs
