// k_net_inc.hip -- the exchanged-configuration pass in incremental mode for
// any lattice the incremental method applies to (windows may wrap around the
// torus, 16 or 32 channels) [Sec. 5.4.1: forwards of the network over the
// O(L^2) exchanged configurations are over 95% of the time].  Lattices wide
// enough that no window wraps, with 32 channels, take the faster unwrapped
// form in k_net_cone.hip.
//
// An exchange of the antiparallel pair (i, j) changes layer k of the network
// only on the sites within Chebyshev distance k of i or j.  For every queue
// item the kernel recomputes layer k on the bounding rectangle R_k of that
// cone (clamped to the torus) and takes all other inputs from the activations
// the base pass cached for the sample:
//
//   window W_k = R_{k+1} (LDS)   <- h'_{k-1} on R_{k-1} (previous layer, LDS)
//                                 + h_{k-1} on the ring W_k \ R_{k-1} (cache, HBM/L2)
//   R_k outputs (MFMA, BF16 x BF16 -> FP32) -> ln cosh -> BF16 -> W_{k+1}
//   last layer: dlog += sum_{p in R_K} (sum_c h'_K(p, c) - hs(p))  (FP64)
//
// Geometry is anchored at the exchanged pair, so every window layout, tap
// offset and ring list depends only on the bond type and the layer; the ring
// lists are precomputed per context.  Two LDS windows alternate between
// layers: each output tile is written to the next window as soon as it is
// finished, and one barrier per layer separates the layers.  The ring of the
// next window is fetched into registers before the layer's matrix work and
// stored after it; the next layer's weights are fetched as soon as the last
// MFMA of the layer has issued.  Sites inside a window carry their 16-byte
// chunks XOR-swizzled by site index to spread LDS banks.
#include <algorithm>
#include <vector>

#include "mfma_common.h"

namespace nqs {
namespace {

using mf::bf16x8;
using mf::floatx4;
using mf::Shape;

constexpr int kNW = 4;
constexpr int kXcd = 8;          // XCDs; workgroup b runs on XCD b % kXcd
constexpr int kThreads = kNW * 64;
constexpr int kRingRegs = 2;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // 16-byte chunk

struct IncParams {
    const int8_t *spins;
    int L, K;
    const uint32_t *queue;
    const int64_t *qlen;
    int64_t capacity;
    const bf16x8 *wa;
    const float *w1;
    const float *bias;
    const uint16_t *cache;
    const double *hsum;
    double *dlog;
    int32_t *err;
    const int32_t *ring;       // packed (window index | (du mod L) << 16 | (dv mod L) << 24)
    const int32_t *ring_off;   // [4][K] entry offsets: ring of W_{k+1} for k = 1..K-1
    int win_bytes;             // bytes of one window buffer
};

// Up to kMaxConnJobs lattices (contexts of one network shape) in one launch:
// their queue items form one index space, job after job.
struct IncJobs {
    IncParams job[kMaxConnJobs];
    int n;
};

// a mod L for a in [-L, 2L): every anchor offset of this kernel lies in
// [-(K+2), L) and the incremental mode requires L >= K + 2.
__device__ __forceinline__ int wrap_l(int a, int L)
{
    a += (a < 0) ? L : 0;
    return a - ((a >= L) ? L : 0);
}

// Window sites are padded to one extra 16-byte chunk (80 B for 32 channels,
// 48 B for 16): the 16 sites read by a lane group then start on 16 distinct
// 16-byte bank groups, so the 16-byte LDS loads and stores are conflict-free.
template <int C>
struct Win {
    static constexpr int STRIDE = Shape<C>::PSB + 16;
};

// byte offset of 16-byte chunk c of window site wi
template <int C>
__device__ __forceinline__ int chunk_addr(int wi, int c)
{
    return wi * Win<C>::STRIDE + (c << 4);
}

// Store the CG channels of lane group g (values already BF16-packed in pairs).
template <int C>
__device__ __forceinline__ void store_group(unsigned char *buf, int wi, int g, const uint32_t *pk)
{
    if (C == 32) {
        const u32x4 v = {pk[0], pk[1], pk[2], pk[3]};
        *(u32x4 *)(buf + chunk_addr<C>(wi, g)) = v;
    } else {
        uint2 v = {pk[0], pk[1]};
        *(uint2 *)(buf + chunk_addr<C>(wi, g >> 1) + ((g & 1) << 3)) = v;
    }
}

__device__ __forceinline__ uint32_t pack2(float a, float b)
{
    return (uint32_t)mf::to_bf16(a) | ((uint32_t)mf::to_bf16(b) << 16);
}

template <int C>
struct Ring {
    u32x4 v[kRingRegs];
    int wi[kRingRegs];
};

// Fetch the ring chunks of the next window (first kRingRegs * 256 of them).
template <int C>
__device__ __forceinline__ void ring_fetch(Ring<C> &r, const IncParams &p, int e0, int e1,
                                           int ax, int ay, const uint16_t *layer_cache)
{
    const int L = p.L;
    const int total = (e1 - e0) * Shape<C>::CHUNKS;
    // The loads are issued unconditionally (surplus lanes re-read the first
    // entry) so that the compiler can count outstanding loads exactly and
    // let the layer's matrix work start before they land.
#pragma unroll
    for (int i = 0; i < kRingRegs; ++i) {
        const int q0 = threadIdx.x + i * kThreads;
        const bool live = q0 < total;
        const int q = live ? q0 : 0;
        const int ent = p.ring[e0 + q / Shape<C>::CHUNKS];
        const int c = q % Shape<C>::CHUNKS;
        int x = ax + ((ent >> 16) & 255), y = ay + ((ent >> 24) & 255);
        x -= (x >= L) ? L : 0;
        y -= (y >= L) ? L : 0;
        r.v[i] = *(const u32x4 *)(layer_cache + (int64_t)(y * L + x) * C + c * 8);
        r.wi[i] = live ? (((ent & 0xffff) << 4) | c) : -1;
    }
}

template <int C>
__device__ __forceinline__ void ring_store(const Ring<C> &r, unsigned char *buf, const IncParams &p,
                                           int e0, int e1, int ax, int ay,
                                           const uint16_t *layer_cache)
{
#pragma unroll
    for (int i = 0; i < kRingRegs; ++i)
        if (r.wi[i] >= 0) *(u32x4 *)(buf + chunk_addr<C>(r.wi[i] >> 4, r.wi[i] & 15)) = r.v[i];
    // chunks beyond the prefetched ones (only for large clamped windows)
    const int L = p.L;
    const int total = (e1 - e0) * Shape<C>::CHUNKS;
    for (int q = threadIdx.x + kRingRegs * kThreads; q < total; q += kThreads) {
        const int ent = p.ring[e0 + q / Shape<C>::CHUNKS];
        const int c = q % Shape<C>::CHUNKS;
        int x = ax + ((ent >> 16) & 255), y = ay + ((ent >> 24) & 255);
        x -= (x >= L) ? L : 0;
        y -= (y >= L) ? L : 0;
        *(u32x4 *)(buf + chunk_addr<C>(ent & 0xffff, c)) =
            *(const u32x4 *)(layer_cache + (int64_t)(y * L + x) * C + c * 8);
    }
}

template <int C>
__device__ __forceinline__ void load_weights(bf16x8 (&wa)[Shape<C>::KS][Shape<C>::NH],
                                             const bf16x8 *base, int lane)
{
#pragma unroll
    for (int j = 0; j < Shape<C>::KS; ++j)
#pragma unroll
        for (int hh = 0; hh < Shape<C>::NH; ++hh)
            wa[j][hh] = base[(j * Shape<C>::NH + hh) * 64 + lane];
}

// Matrix work of NT (1 or 2) tiles of one layer: implicit-GEMM MFMA over
// window W_k, then ln cosh and either the BF16 store into the next window
// (inner layers) or the FP64 per-site sums (last layer).  Straight-line code:
// the tap address of every K-step is one add of a precomputed row byte base
// and column byte offset.
template <int C, bool last, int NT>
__device__ __forceinline__ void tile_group(const bf16x8 (&wa)[Shape<C>::KS][Shape<C>::NH],
                                           const float (&bias)[Shape<C>::NH][4],
                                           unsigned char *lds, int cur, int nxt, int t0,
                                           int ntiles, int npos, uint32_t mul, int ex, int wex,
                                           int nex, bool wcx, bool wcy, int L, int K, int ax,
                                           int ay, const double *hsum_s, int g, int n16,
                                           double &fsum)
{
    using S = Shape<C>;
    constexpr int STRIDE = Win<C>::STRIDE;
    const int chunk_b = (C == 32 ? g : (g & 1)) << 4;   // 16-byte chunk this lane group reads
    floatx4 acc[NT][S::NH];
    int pos_u[NT], pos_v[NT];
    bool valid[NT];
    int rowb[NT][3], colb[NT][3];
    double hs_base[NT];
#pragma unroll
    for (int w = 0; w < NT; ++w) {
        const int tile = t0 + w * kNW;
        int p = tile * 16 + n16;
        valid[w] = p < npos;
        if (p >= npos) p = npos - 1;
        const int v = (int)(((uint32_t)p * mul) >> 20);
        const int u = p - __mul24(v, ex);
        pos_u[w] = u;
        pos_v[w] = v;
        // window W_k = R_{k+1} coordinates of the taps (d - 1) around (u, v)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int wv = v + d;
            if (wcy && wv >= L) wv -= L;
            int wu = u + d;
            if (wcx && wu >= L) wu -= L;
            rowb[w][d] = __mul24(wv, wex * STRIDE) + cur + chunk_b;
            colb[w][d] = __mul24(wu, STRIDE);
        }
#pragma unroll
        for (int hh = 0; hh < S::NH; ++hh)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[w][hh][r] = bias[hh][r];
        hs_base[w] = 0.0;
        if (last) {   // unconditional load (clamped position), used by lane group 0
            const int site = wrap_l(ay + v - K, L) * L + wrap_l(ax + u - K, L);
            hs_base[w] = hsum_s[site];
        }
    }
#pragma unroll
    for (int j = 0; j < S::KS; ++j) {
#pragma unroll
        for (int w = 0; w < NT; ++w) {
            int a;
            if (C == 32) {
                a = rowb[w][j / 3] + colb[w][j % 3];
            } else {
                // lane groups 0-1 read tap 2j, groups 2-3 tap 2j+1 (clamped to 8)
                const int ta = 2 * j, tb = (2 * j + 1 > 8) ? 8 : 2 * j + 1;
                const int aa = rowb[w][ta / 3] + colb[w][ta % 3];
                const int ab = rowb[w][tb / 3] + colb[w][tb % 3];
                a = (g >> 1) ? ab : aa;
            }
            const bf16x8 bv = *(const bf16x8 *)(lds + a);
#pragma unroll
            for (int hh = 0; hh < S::NH; ++hh)
                acc[w][hh] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j][hh], bv, acc[w][hh], 0,
                                                                    0, 0);
        }
    }
#pragma unroll
    for (int w = 0; w < NT; ++w) {
        float zv[S::CG], hv[S::CG];
#pragma unroll
        for (int hh = 0; hh < S::NH; ++hh)
#pragma unroll
            for (int r = 0; r < 4; ++r) zv[hh * 4 + r] = acc[w][hh][r];
        mf::ln_cosh_n<S::CG>(zv, hv);
        if (!last) {
            if (valid[w]) {
                uint32_t pk[S::CG / 2];
#pragma unroll
                for (int r = 0; r < S::CG / 2; ++r) pk[r] = pack2(hv[2 * r], hv[2 * r + 1]);
                int wu = pos_u[w] + 2, wv = pos_v[w] + 2;
                if (wu >= L) wu -= L;
                if (wv >= L) wv -= L;
                store_group<C>(lds + nxt, __mul24(wv, nex) + wu, g, pk);
            }
        } else {
            double part = 0.0;
#pragma unroll
            for (int r = 0; r < S::CG; ++r) part += (double)hv[r];
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            if (g == 0 && valid[w]) fsum += part - hs_base[w];
        }
    }
}

// All tiles of one layer owned by this wave, two in flight where possible.
// Instantiated separately for the last layer so that inner layers contain no
// conditional global loads and the compiler's load counting stays exact.
template <int C, bool last>
__device__ __forceinline__ void layer_tiles(const bf16x8 (&wa)[Shape<C>::KS][Shape<C>::NH],
                                            const float (&bias)[Shape<C>::NH][4],
                                            unsigned char *lds, int cur, int nxt,
                                            int ntiles, int npos, uint32_t mul, int ex, int wex,
                                            int nex, bool wcx, bool wcy, int L, int K, int ax,
                                            int ay, const double *hsum_s, int wave, int g, int n16,
                                            double &fsum)
{
    for (int t0 = wave; t0 < ntiles; t0 += 2 * kNW) {
        if (t0 + kNW < ntiles)
            tile_group<C, last, 2>(wa, bias, lds, cur, nxt, t0, ntiles, npos, mul, ex, wex, nex, wcx,
                                   wcy, L, K, ax, ay, hsum_s, g, n16, fsum);
        else
            tile_group<C, last, 1>(wa, bias, lds, cur, nxt, t0, ntiles, npos, mul, ex, wex, nex, wcx,
                                   wcy, L, K, ax, ay, hsum_s, g, n16, fsum);
    }
}

template <int C>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_net_inc(IncJobs jobs)
{
    using S = Shape<C>;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    __shared__ double red[kNW];
    unsigned char *buf0 = lds, *buf1 = lds + jobs.job[0].win_bytes;

    const int K = jobs.job[0].K;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, n16 = lane & 15;
    // first item of each job in the common index space
    int64_t first[kMaxConnJobs + 1];
    first[0] = 0;
#pragma unroll
    for (int j = 0; j < kMaxConnJobs; ++j)
        first[j + 1] = first[j] + (j < jobs.n ? min(jobs.job[j].qlen[0], jobs.job[j].capacity) : 0);
    const int64_t n_units = first[kMaxConnJobs];
    const int64_t wl_stride = (int64_t)S::KS * S::NH * 64;

    auto job_of = [&](int64_t u) {
        int jb = 0;
#pragma unroll
        for (int j = 1; j < kMaxConnJobs; ++j) jb = (u >= first[j]) ? j : jb;
        return jb;
    };
    // XCD-contiguous ranges of the queue: consecutive items (mostly of one
    // sample) stay on one XCD, whose L2 then serves that sample's cache
    const int per_xcd = gridDim.x / kXcd;
    const int xcd = blockIdx.x % kXcd, slot = blockIdx.x / kXcd;
    const int64_t seg = (n_units + kXcd - 1) / kXcd;
    const int64_t u_end = min(n_units, (xcd + 1) * seg);
    bf16x8 wa[S::KS][S::NH];
    if (xcd * seg + slot < u_end)                                                 // layer 2
        load_weights<C>(wa, jobs.job[job_of(xcd * seg + slot)].wa, lane);

    for (int64_t u = xcd * seg + slot; u < u_end; u += per_xcd) {
        const int jb = job_of(u);
        const IncParams &prm = jobs.job[jb];
        const int64_t unit = u - first[jb];
        const int L = prm.L, N = L * L;
        const uint32_t e = prm.queue[unit];
        const int s = item_sample(e);
        const int b = item_bond(e), tau = b & 3, i0 = b >> 2;
        const int xi = i0 % L, yi = i0 / L;
        const int qi = i0, qj = wrap_l(yi + bond_dy(tau), L) * L + wrap_l(xi + bond_dx(tau), L);
        const int ax = xi, ay = (tau == 3) ? wrap_l(yi - 1, L) : yi;
        const int w0 = (tau == 1) ? 1 : 2, h0 = (tau == 0) ? 1 : 2;
        const int8_t *sp = prm.spins + (int64_t)s * N;
        const uint16_t *cache_s = prm.cache + (int64_t)s * (K - 1) * N * C;
        const int *roff = prm.ring_off + tau * K;

        // ---- layer 1 (vector ALU) into W_2 = R_3 in buf0 ----
        {
            Ring<C> ring;
            ring_fetch<C>(ring, prm, roff[0], roff[1], ax, ay, cache_s);
            const int ex1 = min(w0 + 2, L), ey1 = min(h0 + 2, L);
            const int exn = min(w0 + 6, L), eyn = min(h0 + 6, L);
            const int npos = ex1 * ey1;
            for (int q = tid; q < npos * 4; q += kThreads) {
                const int p = q >> 2, gg = q & 3;
                const int u = p % ex1, v = p / ex1;
                const int gx = wrap_l(ax + u - 1, L), gy = wrap_l(ay + v - 1, L);
                float sv[9];
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    int site = wrap_l(gy + t / 3 - 1, L) * L + wrap_l(gx + t % 3 - 1, L);
                    site = (site == qi) ? qj : ((site == qj) ? qi : site);
                    sv[t] = (float)sp[site];
                }
                uint32_t pk[S::CG / 2];
#pragma unroll
                for (int r = 0; r < S::CG; r += 2) {
                    const float h0v = mf::ln_cosh(mf::layer1_z(prm.w1, prm.bias, C,
                                                               mf::chan_of_slot<C>(gg * S::CG + r), sv));
                    const float h1v = mf::ln_cosh(mf::layer1_z(prm.w1, prm.bias, C,
                                                               mf::chan_of_slot<C>(gg * S::CG + r + 1), sv));
                    pk[r / 2] = pack2(h0v, h1v);
                }
                int wu = u + 2, wv = v + 2;
                if (wu >= L) wu -= L;
                if (wv >= L) wv -= L;
                store_group<C>(buf0, wv * exn + wu, gg, pk);
            }
            ring_store<C>(ring, buf0, prm, roff[0], roff[1], ax, ay, cache_s);
        }
        __syncthreads();

        double fsum = 0.0;
        for (int k = 2; k <= K; ++k) {
            const int cur_off = ((k & 1) == 0) ? 0 : prm.win_bytes;
            const int nxt_off = ((k & 1) == 0) ? prm.win_bytes : 0;
            unsigned char *nxt = lds + nxt_off;
            const int ex = min(w0 + 2 * k, L), ey = min(h0 + 2 * k, L);
            const int wex = min(w0 + 2 * k + 2, L), wey = min(h0 + 2 * k + 2, L);
            const bool wcx = wex == L, wcy = wey == L;
            const int nex = min(w0 + 2 * k + 4, L);
            const int npos = ex * ey;
            const int ntiles = (npos + 15) >> 4;
            const uint32_t mul = ((1u << 20) + ex - 1) / ex;
            const bool last = k == K;

            Ring<C> ring;
            if (!last) ring_fetch<C>(ring, prm, roff[k - 1], roff[k], ax, ay,
                                     cache_s + (int64_t)(k - 1) * N * C);
            float bias[S::NH][4];
#pragma unroll
            for (int hh = 0; hh < S::NH; ++hh)
#pragma unroll
                for (int r = 0; r < 4; ++r) bias[hh][r] = prm.bias[(k - 1) * C + 16 * hh + 4 * g + r];

            if (!last)
                layer_tiles<C, false>(wa, bias, lds, cur_off, nxt_off, ntiles, npos, mul, ex, wex, nex, wcx, wcy,
                                      L, K, ax, ay, prm.hsum + (int64_t)s * N, wave, g, n16, fsum);
            else
                layer_tiles<C, true>(wa, bias, lds, cur_off, nxt_off, ntiles, npos, mul, ex, wex, nex, wcx, wcy,
                                     L, K, ax, ay, prm.hsum + (int64_t)s * N, wave, g, n16, fsum);
            // weights of the next layer, or layer 2's of the next item (whose job
            // may differ)
            if (!last)
                load_weights<C>(wa, prm.wa + (int64_t)(k - 1) * wl_stride, lane);
            else if (u + per_xcd < u_end)
                load_weights<C>(wa, jobs.job[job_of(u + per_xcd)].wa, lane);
            if (!last) ring_store<C>(ring, nxt, prm, roff[k - 1], roff[k], ax, ay,
                                     cache_s + (int64_t)(k - 1) * N * C);
            __syncthreads();
        }

        for (int off = 32; off > 0; off >>= 1) fsum += __shfl_xor(fsum, off);
        if (lane == 0) red[wave] = fsum;
        __syncthreads();
        if (tid == 0) {
            double v = 0.0;
            for (int w = 0; w < kNW; ++w) v += red[w];
            if (!isfinite(v)) atomicOr(prm.err, kErrNonFinite);
            prm.dlog[unit] = v;
        }
    }
}

}  // namespace

// Ring lists: for bond type tau and layer k = 1..K-1, the sites of the next
// window W_{k+1} = R_{k+2} outside R_k, as (window index, offset from the
// anchor).  Stored per context; item-independent because the geometry is
// anchored at the exchanged pair.
nqs_status mfma_build_ring_tables(nqs_ctx *c)
{
    const int L = c->L, K = c->K;
    std::vector<int32_t> ent, off((size_t)4 * K, 0);
    for (int tau = 0; tau < 4; ++tau) {
        const int w0 = (tau == 1) ? 1 : 2, h0 = (tau == 0) ? 1 : 2;
        for (int k = 1; k < K; ++k) {
            off[(size_t)tau * K + (k - 1)] = (int32_t)ent.size();
            const int ex = std::min(w0 + 2 * k, L), ey = std::min(h0 + 2 * k, L);
            const int nex = std::min(w0 + 2 * k + 4, L), ney = std::min(h0 + 2 * k + 4, L);
            for (int wv = 0; wv < ney; ++wv)
                for (int wu = 0; wu < nex; ++wu) {
                    const int du = wu - (k + 2), dv = wv - (k + 2);   // offsets from the anchor
                    // inside R_k: anchor offset in [-k, -k + ex) modulo L (a clamped
                    // window spans one period, which R_k's range may straddle)
                    const bool in_x = (ex == L) || (((du + k) % L + L) % L < ex);
                    const bool in_y = (ey == L) || (((dv + k) % L + L) % L < ey);
                    if (in_x && in_y) continue;
                    // anchor offsets stored reduced modulo L (0 <= offset < L <= 64)
                    const int dum = ((du % L) + L) % L, dvm = ((dv % L) + L) % L;
                    ent.push_back((wv * nex + wu) | (dum << 16) | (dvm << 24));
                }
        }
        off[(size_t)tau * K + (K - 1)] = (int32_t)ent.size();
    }
    if (ent.empty()) ent.push_back(0);
    if (c->ring_tab) (void)hipFree(c->ring_tab);
    if (c->ring_off) (void)hipFree(c->ring_off);
    c->ring_tab = nullptr;
    c->ring_off = nullptr;
    if (hipMalloc((void **)&c->ring_tab, ent.size() * 4) != hipSuccess ||
        hipMalloc((void **)&c->ring_off, off.size() * 4) != hipSuccess)
        return NQS_E_NOMEM;
    if (hipMemcpy(c->ring_tab, ent.data(), ent.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->ring_off, off.data(), off.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return NQS_E_HIP;
    return NQS_OK;
}

size_t mfma_inc_lds_bytes(const nqs_ctx *c)
{
    int wmax = 0;
    for (int k = 1; k <= c->K; ++k) {
        const int e = std::min(2 + 2 * k + 2, c->L);   // W_k = R_{k+1}, 2x2 seed
        wmax = std::max(wmax, e * e);
    }
    return (size_t)wmax * (c->C * 2 + 16);   // one window buffer, padded sites
}

void mfma_inc_forward_jobs(const ConnJob *jobs, int n, hipStream_t s)
{
    if (n <= 0) return;
    IncJobs jp{};
    jp.n = n;
    size_t win = 0;
    int64_t total_cap = 0;
    for (int i = 0; i < n; ++i) {
        win = std::max(win, mfma_inc_lds_bytes(jobs[i].c));
        total_cap += jobs[i].capacity;
    }
    for (int i = 0; i < n; ++i) {
        const nqs_ctx *c = jobs[i].c;
        IncParams &p = jp.job[i];
        p.spins = jobs[i].spins;
        p.L = c->L;
        p.K = c->K;
        p.queue = jobs[i].queue;
        p.qlen = jobs[i].qlen;
        p.capacity = jobs[i].capacity;
        p.wa = (const bf16x8 *)c->w_mfma;
        p.w1 = c->w_l1;
        p.bias = c->w_l1 + 9 * c->C;
        p.cache = (const uint16_t *)jobs[i].cache;
        p.hsum = jobs[i].hsum;
        p.dlog = jobs[i].dlog;
        p.err = c->err;
        p.ring = c->ring_tab;
        p.ring_off = c->ring_off;
        p.win_bytes = (int)win;   // one buffer size for every job: the largest window
    }
    if (total_cap <= 0) return;
    const int C = jobs[0].c->C;
    const size_t lds = 2 * win;
    // persistent grid: exactly the workgroups that are resident at once
    const void *fn = C == 32 ? (const void *)k_net_inc<32> : (const void *)k_net_inc<16>;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    // persistent grid of resident workgroups, a multiple of the XCD count
    const int64_t want = std::max<int64_t>((int64_t)jobs[0].c->n_cu * per_cu / kXcd * kXcd, kXcd);
    if (C == 32)
        NQS_LAUNCH((k_net_inc<32>), dim3((unsigned)want), dim3(kThreads), lds, s, jp);
    else
        NQS_LAUNCH((k_net_inc<16>), dim3((unsigned)want), dim3(kThreads), lds, s, jp);
}

void mfma_inc_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                      const int64_t *qlen, int64_t capacity, const double *hsum,
                      const void *cache, double *dlog, hipStream_t s)
{
    const ConnJob j{c, spins, queue, qlen, capacity, hsum, cache, dlog};
    mfma_inc_forward_jobs(&j, 1, s);
}

}  // namespace nqs
