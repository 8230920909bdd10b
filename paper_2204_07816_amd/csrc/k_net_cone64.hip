// k_net_cone64.hip -- the exchanged-configuration pass of the ln cosh CNN in
// FP64 by the receptive cone [Sec. 5.4.1: the forwards of the O(L^2)
// exchanged configurations are the hot spot; Sec. 6.3 and Sec. 8: faithful
// ground-state energies need double precision], on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64).
//
// Exchanging the pair (q_i, q_j) changes the spins of a w0 x h0 box, and
// layer k's output (a 3x3 circular convolution and ln cosh) only on R_k, the
// box widened by k sites.  So f(S') - f(S) = sum over the sites p of R_K of
// (sum_c h'_K[p][c] - sum_c h_K[p][c]).
//
// One workgroup of eight waves takes one queue item at a time, over
// XCD-contiguous ranges of the queue.  A square frame of side 2K + 4 (the box
// widened by K + 1) holds in LDS the C FP64 channels of the current layer's
// input; layer k reads it on R_{k+1} and forms R_k as tiles of 16 sites x C
// channels, with the operand layout and MFMA order of the full pass's
// k_conv_mma (K-blocks of 16 channels per tap, 4 channels per K-step), the
// layer's packed taps streamed from memory as B operands two K-blocks ahead.
// The results wait in registers until every wave has read the frame, then
// replace R_k in place, and the ring R_{k+2} \ R_k is filled from the
// sample's activations of layer k, kept by the base pass (cache: h_1 ..
// h_{K-1}, [K-1][B][N][C]).  Layer 1 (one input channel) runs on the vector
// ALU from the exchanged spins with k_layer1's FMA order.  Every neuron
// therefore equals the full recomputation's bit for bit, and the last layer's
// per-site channel sums are taken sequentially over c as the base pass takes
// hsum, so unchanged sites cancel exactly and each site's difference equals
// the full pass's; only the order of the final sum over sites differs.
// Needs 16 or 32 channels, 2 <= K <= 8 and L >= 2K + 4 (the frame does not
// overlap itself on the torus).
#include <algorithm>

#include "nqs_internal.h"

namespace nqs {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kNW = 8;
constexpr int kThreads = kNW * 64;
constexpr int kXcd = 8;
constexpr int kMaxK64 = 8;
// tiles per wave and layer: R_K of a 2 x 2 box has 21 tiles at K = 8
constexpr int kStage = (21 + kNW - 1) / kNW;

struct Cone64Args {
    const int8_t *spins;        // [B][N]
    const uint32_t *queue;
    const int64_t *qlen;
    int64_t cap;
    const double *w;            // layer 1 [9][C] + bias [C]; layer k > 1 [9][C][C] + bias [C]
    const double *cache;        // h_1 .. h_{K-1} of samples b0 ..: [K-1][cB][N][C]
    const double *hsum;         // [B][N]: sum over c of h_K (base pass)
    int64_t cB, b0, nb;         // cache slot stride; samples of this launch
    double *dlog;
    int32_t *err;
    int L, K;
};

__device__ inline int wrapc(int a, int L) { return a < 0 ? a + L : (a >= L ? a - L : a); }

// byte offset of 16-byte chunk c (channels 2c, 2c + 1) of frame site f; the
// C / 2 chunks of a site are rotated by the site index, so lanes reading one
// chunk position of consecutive sites spread over the banks
template <int C>
__device__ inline int fo(int f, int c)
{
    return f * (C * 8) + ((c ^ (f & (C / 2 - 1))) << 4);
}

// one K-block's operands of a tile: A (this lane's 4 channels at its site's
// tap), B (4 K-steps x NB column blocks of W)
template <int C>
struct Ops {
    double2 a[2];
    double b[4][C / 16];
};

template <int C>
__device__ inline void c64_fetch(const unsigned char *fr, const double *wl, int fm, int P, int kq,
                                 int m16, int kb, Ops<C> &o)
{
    constexpr int NB = C / 16;
    const int t = kb / NB, cb = kb - t * NB;
    const int f = fm + (t / 3 - 1) * P + (t - 3 * (t / 3) - 1);
    const int ch = cb * 8 + 2 * kq;                       // chunk of channels cb 16 + 4 kq
    o.a[0] = *(const double2 *)(fr + fo<C>(f, ch));
    o.a[1] = *(const double2 *)(fr + fo<C>(f, ch + 1));
    const double *wt = wl + ((int64_t)t * C + cb * 16 + 4 * kq) * C + m16;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int h = 0; h < NB; ++h) o.b[s][h] = wt[s * C + 16 * h];
}

template <int C>
__device__ inline void c64_mma(const Ops<C> &o, double4_t (&acc)[C / 16])
{
    constexpr int NB = C / 16;
    const double av[4] = {o.a[0].x, o.a[0].y, o.a[1].x, o.a[1].y};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int h = 0; h < NB; ++h)
            acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], o.b[s][h], acc[h], 0, 0, 0);
}

// One tile of layer k (16 sites from frame site fm of this lane's A row):
// h = ln cosh(bias + W (*) input), D element i of column block h: row kq + 4 i,
// channel 16 h + m16.  The K-blocks run in the full pass's order; each
// block's operands are read two blocks before its MFMAs issue (the weights'
// latency from L2 exceeds one block's MFMA time), in three register sets
// that take turns over a loop rolled by three blocks (9 NB is a multiple of 3).
template <int C>
__device__ inline void c64_tile(const unsigned char *fr, const double *wl, const double *bias,
                                int fm, int P, int kq, int m16, double (&out)[C / 16][4])
{
    constexpr int NB = C / 16;
    constexpr int NKB = 9 * NB;
    double4_t acc[NB];
#pragma unroll
    for (int h = 0; h < NB; ++h) {
        const double b = bias[16 * h + m16];
        acc[h] = (double4_t){b, b, b, b};
    }
    Ops<C> o0, o1, o2;
    c64_fetch<C>(fr, wl, fm, P, kq, m16, 0, o0);
    c64_fetch<C>(fr, wl, fm, P, kq, m16, 1, o1);
#pragma unroll 1
    for (int kb = 0; kb < NKB - 3; kb += 3) {
        c64_fetch<C>(fr, wl, fm, P, kq, m16, kb + 2, o2);
        c64_mma<C>(o0, acc);
        c64_fetch<C>(fr, wl, fm, P, kq, m16, kb + 3, o0);
        c64_mma<C>(o1, acc);
        c64_fetch<C>(fr, wl, fm, P, kq, m16, kb + 4, o1);
        c64_mma<C>(o2, acc);
    }
    c64_fetch<C>(fr, wl, fm, P, kq, m16, NKB - 1, o2);
    c64_mma<C>(o0, acc);
    c64_mma<C>(o1, acc);
    c64_mma<C>(o2, acc);
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) out[h][i] = ln_cosh_fwd(acc[h][i]);
}

template <int C>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_net_cone64(Cone64Args a)
{
    constexpr int NB = C / 16;
    constexpr int CHK = C / 2;               // 16-byte chunks per site
    // ring chunks per thread: the largest ring, R_{K+1} \ R_{K-1} of a 2 x 2
    // box, has 16 K + 16 sites
    constexpr int RS = ((16 * kMaxK64 + 16) * CHK + kThreads - 1) / kThreads;
    static_assert(RS <= 5, "ring slots are five named registers");
    extern __shared__ __attribute__((aligned(16))) unsigned char fr[];
    __shared__ double red[kNW];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m16 = lane & 15, kq = lane >> 4;
    const int L = a.L, N = L * L, K = a.K, F = K + 1, P = 2 * K + 4;
    const int64_t n_items = min(a.qlen[0], a.cap);
    const int per_xcd = gridDim.x / kXcd;
    const int xcd = blockIdx.x % kXcd, slot = blockIdx.x / kXcd;
    const int64_t seg = (n_items + kXcd - 1) / kXcd;
    const int64_t u_end = min(n_items, (xcd + 1) * seg);

    for (int64_t u = xcd * seg + slot; u < u_end; u += per_xcd) {
        const uint32_t e = a.queue[u];
        const int s = item_sample(e), b = item_bond(e), tau = b & 3, i0 = b >> 2;
        if (s < a.b0 || s >= a.b0 + a.nb) continue;      // another launch's sample
        const int xi = i0 % L, yi = i0 / L;
        const int qi = i0, qj = wrapc(yi + bond_dy(tau), L) * L + wrapc(xi + bond_dx(tau), L);
        const int ax = xi, ay = (tau == 3) ? wrapc(yi - 1, L) : yi;
        const int w0 = (tau == 1) ? 1 : 2, h0 = (tau == 0) ? 1 : 2;
        const int8_t *sp = a.spins + (int64_t)s * N;
        // lattice site of frame position (fx, fy): ax - F + fx lies in (-L, 2L)
        auto site_of = [&](int fx, int fy) {
            int x = ax - F + fx, y = ay - F + fy;
            x += x < 0 ? L : (x >= L ? -L : 0);
            y += y < 0 ? L : (y >= L ? -L : 0);
            return y * L + x;
        };
        // ring R_{l+2} \ R_l from the cache of layer l: its 4 (w0 + 2l + 4) +
        // 4 (h0 + 2l) sites (two rows above and below R_l at full width, then
        // two columns left and right of it), CHK chunks each; chunk q of the
        // ring goes to this thread's slot q / kThreads (named registers: an
        // array of them would live in scratch).  ring_load reads them,
        // ring_store writes them to the frame.
        double2 rv0, rv1, rv2, rv3, rv4;
        int rd0 = -1, rd1 = -1, rd2 = -1, rd3 = -1, rd4 = -1;
        auto ring_one = [&](int l, int r, double2 &v, int &d) __attribute__((always_inline)) {
            const int W = w0 + 2 * l + 4, H = h0 + 2 * l + 4, hi = h0 + 2 * l;
            const int total = (4 * W + 4 * hi) * CHK;
            const double *src = a.cache + ((int64_t)(l - 1) * a.cB + (s - a.b0)) * N * C;
            const int q = tid + r * kThreads;
            const int rs = q / CHK, c = q - rs * CHK;
            const int band = (rs >= W) + (rs >= 2 * W) + (rs >= 3 * W);
            const int rr = rs - 4 * W, col = rr & 3;
            const bool bands = rs < 4 * W;
            const int px = bands ? rs - band * W : (col < 2 ? col : W - 4 + col);
            const int py = bands ? (band < 2 ? band : H - 4 + band) : 2 + (rr >> 2);
            const bool live = q < total;
            const int fx = F - l - 2 + px, fy = F - l - 2 + py;
            const int site = live ? site_of(fx, fy) : 0;
            v = *(const double2 *)(src + (int64_t)site * C + 2 * c);
            d = live ? fo<C>(fy * P + fx, c) : -1;
        };
        auto ring_load = [&](int l) __attribute__((always_inline)) {
            ring_one(l, 0, rv0, rd0);
            if constexpr (RS > 1) ring_one(l, 1, rv1, rd1);
            if constexpr (RS > 2) ring_one(l, 2, rv2, rd2);
            if constexpr (RS > 3) ring_one(l, 3, rv3, rd3);
            if constexpr (RS > 4) ring_one(l, 4, rv4, rd4);
        };
        auto ring_store = [&]() __attribute__((always_inline)) {
            if (rd0 >= 0) *(double2 *)(fr + rd0) = rv0;
            if constexpr (RS > 1)
                if (rd1 >= 0) *(double2 *)(fr + rd1) = rv1;
            if constexpr (RS > 2)
                if (rd2 >= 0) *(double2 *)(fr + rd2) = rv2;
            if constexpr (RS > 3)
                if (rd3 >= 0) *(double2 *)(fr + rd3) = rv3;
            if constexpr (RS > 4)
                if (rd4 >= 0) *(double2 *)(fr + rd4) = rv4;
        };

        // layer 1 on R_1 from the exchanged spins: thread (site, channel),
        // k_layer1's order (bias, then the taps 0..8) and ln cosh
        {
            const int w1 = w0 + 2, n1 = w1 * (h0 + 2);
            for (int q = tid; q < n1 * C; q += kThreads) {
                const int p = q / C, co = q - p * C;
                const int py = p / w1, px = p - py * w1;
                const int fx = F - 1 + px, fy = F - 1 + py;
                double z = a.w[9 * C + co];
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    int site = site_of(fx + t % 3 - 1, fy + t / 3 - 1);
                    site = (site == qi) ? qj : ((site == qj) ? qi : site);
                    z = fma(a.w[t * C + co], (double)sp[site], z);
                }
                *(double *)(fr + fo<C>(fy * P + fx, co >> 1) + (co & 1) * 8) = ln_cosh_fwd(z);
            }
        }
        ring_load(1);
        ring_store();
        __syncthreads();

        double dl = 0.0;
        for (int k = 2; k <= K; ++k) {
            const double *wl = a.w + 10 * C + (int64_t)(k - 2) * (9 * C * C + C);
            const double *bias = wl + 9 * C * C;
            const int wd = w0 + 2 * k, nl = wd * (h0 + 2 * k);
            const int ntiles = (nl + 15) >> 4;
            const uint32_t mul = ((1u << 20) + wd - 1) / wd;
            auto frame_of = [&](int p) {   // frame site of position p of R_k
                const int v = (int)(((uint32_t)p * mul) >> 20);
                return (F - k + v) * P + (F - k + p - v * wd);
            };
            // this wave's tiles ti = wave + kNW jj, results staged in
            // registers until every wave has read the frame
            double st[kStage][NB][4];
#pragma unroll
            for (int jj = 0; jj < kStage; ++jj) {
                const int ti = wave + kNW * jj;
                if (ti < ntiles)
                    c64_tile<C>(fr, wl, bias, frame_of(min(ti * 16 + m16, nl - 1)), P, kq, m16,
                                st[jj]);
            }
            if (k < K) ring_load(k);
            __syncthreads();                 // every read of the frame for layer k is done
#pragma unroll
            for (int jj = 0; jj < kStage; ++jj) {
                const int ti = wave + kNW * jj;
                if (ti < ntiles)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int p = ti * 16 + kq + 4 * i;
                        if (p < nl) {
                            const int f = frame_of(p);
#pragma unroll
                            for (int h = 0; h < NB; ++h) {
                                const int co = 16 * h + m16;
                                *(double *)(fr + fo<C>(f, co >> 1) + (co & 1) * 8) = st[jj][h][i];
                            }
                        }
                    }
            }
            if (k < K) ring_store();
            __syncthreads();
            if (k == K) {
                // per site of R_K: the channel sum in the base pass's order,
                // minus the base pass's
                const double *hb = a.hsum + (int64_t)s * N;
                for (int p = tid; p < nl; p += kThreads) {
                    const int v = (int)(((uint32_t)p * mul) >> 20);
                    const int f = (F - k + v) * P + (F - k + p - v * wd);
                    double hs = 0.0;
#pragma unroll 8
                    for (int c = 0; c < C; ++c)
                        hs += *(const double *)(fr + fo<C>(f, c >> 1) + (c & 1) * 8);
                    dl += hs - hb[site_of(F - k + p - v * wd, F - k + v)];
                }
            }
        }
        // fixed-order sums over the lanes, then over the waves
        for (int off = 32; off > 0; off >>= 1) dl += __shfl_xor(dl, off);
        if (lane == 0) red[wave] = dl;
        __syncthreads();
        if (tid == 0) {
            double v = 0.0;
            for (int w = 0; w < kNW; ++w) v += red[w];
            if (!isfinite(v)) atomicOr(a.err, kErrNonFinite);
            a.dlog[u] = v;
        }
        __syncthreads();                     // red and the frame are free again
    }
}

}  // namespace

bool cone64_ok(const nqs_ctx *c)
{
    return c->dtype == NQS_FP64 && c->net == kNetLnCosh && (c->C == 16 || c->C == 32) &&
           c->K >= 2 && c->K <= kMaxK64 && c->L >= 2 * c->K + 4;
}

size_t cone64_cache_bytes(const nqs_ctx *c, int64_t cB)
{
    return sizeof(double) * (size_t)(c->K - 1) * (size_t)cB * c->N * c->C;
}

// samples per cache fill: at most 16 GiB of cached activations
int64_t cone64_chunk(const nqs_ctx *c, int64_t B)
{
    const size_t per = cone64_cache_bytes(c, 1);
    const int64_t m = (int64_t)(((size_t)16 << 30) / std::max<size_t>(per, 1));
    return std::max<int64_t>(1, std::min(m, std::max<int64_t>(B, 1)));
}

void cone64_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                    const int64_t *qlen, int64_t cap, const double *cache, int64_t cB, int64_t b0,
                    int64_t nb, const double *hsum, double *dlog, hipStream_t s)
{
    if (cap <= 0 || nb <= 0) return;
    const Cone64Args a{spins, queue, qlen, cap, c->w_vec64, cache, hsum, cB, b0, nb, dlog,
                       c->err, c->L, c->K};
    const int P = 2 * c->K + 4;
    const size_t lds = (size_t)P * P * c->C * sizeof(double);
    // one workgroup of eight waves per CU; a multiple of 8 for the XCD ranges
    const int grid = std::max(kXcd, c->n_cu / kXcd * kXcd);
    if (c->C == 32) {
        (void)hipFuncSetAttribute((const void *)k_net_cone64<32>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        NQS_LAUNCH((k_net_cone64<32>), dim3(grid), dim3(kThreads), lds, s, a);
    } else {
        (void)hipFuncSetAttribute((const void *)k_net_cone64<16>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        NQS_LAUNCH((k_net_cone64<16>), dim3(grid), dim3(kThreads), lds, s, a);
    }
}

}  // namespace nqs
