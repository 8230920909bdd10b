// k_net_cone.hip -- the exchanged-configuration pass in incremental mode for
// lattices wide enough that no window of the receptive cone wraps around the
// torus (L >= 2K + 4) and 32 channels: the form taken by the large lattices
// the local energy is dominated by [Sec. 5.4.1].
//
// The method is that of the general incremental kernel: an exchange of the
// antiparallel pair (i, j) changes layer k only on R_k, the bounding
// rectangle of the sites within Chebyshev distance k of i or j; layer k is
// recomputed on R_k from window W_k = R_{k+1} (LDS), which holds layer k-1 of
// this configuration on R_{k-1} and the cached base-pass activations on the
// ring W_k \ R_{k-1}; the last layer adds sum_{p in R_K} (hs'(p) - hs(p)).
// The arithmetic (MFMA K-step order, ln cosh, layer-1 FMA order, BF16
// rounding, FP64 site sums) is the base pass's, so sites the exchange does
// not reach cancel exactly.
//
// What the unwrapped geometry buys:
//  * window W_k is a plain rectangle, stored as four channel planes (plane c
//    holds channels 8c..8c+7 of every site, 16 bytes per site, rows of the
//    window's width).  The 16 lanes of an MFMA lane group read one plane at 16
//    consecutive output positions, so within a row they read 256 contiguous
//    bytes; without padding the two windows of K = 8 take 46 KB, which leaves
//    room for three workgroups per CU.
//  * a tap's LDS address is a per-tile row base plus a compile-time column
//    offset, so the nine reads of a tile cost two adds.
//  * the ring W_{k+1} minus R_k (an annulus two sites wide) is listed per bond
//    type in a small table whose entries are loaded two layers ahead; the
//    ring of W_{k+2} is fetched at the start of layer k and stored at the
//    start of layer k + 1, a whole layer ahead of its use.
//  * layer 1 is spread over all threads (two channels each).
//  * consecutive queue items (mostly of one sample, sharing its cached
//    activations) are kept on one XCD so that its L2 serves the ring reads.
#include <algorithm>
#include <vector>

#include "mfma_common.h"

namespace nqs {
namespace {

using mf::bf16x8;
using mf::floatx4;

constexpr int C = 32;
constexpr int KS = 9;           // K-steps (one tap of 32 channels each)
constexpr int NH = 2;           // 16-channel output halves
constexpr int kRingRegs = 2;
constexpr int kChunk = 16;      // bytes of one 8-channel chunk of a site
constexpr int kXcd = 8;         // XCDs; workgroup b runs on XCD b % kXcd

// The operand form: X = 1 plain BF16; X = 3, 4, 5 split BF16 (hi + lo of
// every operand, three products per tap).  The split form's windows and cache
// hold the lo parts as four more channel planes / chunks, twice the LDS.  Two
// workgroups of four waves per CU keep two configurations in flight (1.5x at
// K = 6 against one of eight): X = 4 where two workgroups' windows fit (K <=
// 7), X = 5 (one frame updated in place, the lo weights in LDS) where two of
// its frames fit (K <= 8), else X = 3, one workgroup of eight waves.
template <int X>
struct Form {
    static constexpr int NW = X == 3 ? 8 : 4;          // waves per workgroup
    static constexpr int kThreads = NW * 64;
    static constexpr int CH = X >= 3 ? 8 : 4;          // 16-byte chunks (planes) per site
    static constexpr int SITE = CH * 8;                // BF16 values per cached site
    static constexpr int WPE = X >= 3 ? 2 : 3;         // waves per SIMD
    // X = 5: the split form in one frame of side 2K + 4 updated in place
    // (outputs staged in registers) with the lo parts of the layer's weights in
    // LDS, so that two workgroups of four waves fit a CU at K <= 8
    static constexpr bool FRAME = X == 5;
};
constexpr int kFrameMaxT = 4;   // tiles per wave of an inner layer in the frame form (K <= 8)
constexpr int kMaxK = 16;
constexpr int kMaxJobs = kMaxConnJobs;
// layer-1 weights in LDS: for each of the 16 channel pairs a thread can own,
// the 9 taps and the bias of both channels (20 floats); then the biases of
// layers 2..K (C floats each)
constexpr int kW1Floats = 16 * 20;
constexpr int kBiasFloats = (kMaxK - 1) * 32;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // 16-byte chunk
typedef float float2v __attribute__((ext_vector_type(2)));

struct ConeParams {
    const int8_t *spins;
    int L, K;
    const uint32_t *queue;
    const int64_t *qlen;
    int64_t capacity;
    const bf16x8 *wa;          // layer k >= 2: [k-2][KS][NH][64 lanes]
    const bf16x8 *wl;          // split form: the lo parts, same layout
    const float *w1;           // layer 1 [9][C]
    const float *bias;         // [K][C]
    const uint16_t *cache;     // base-pass BF16 activations [B][K-1][N][SITE] (slot order;
                               // split form: the 32 hi values, then the 32 lo values)
    const double *hsum;        // base-pass per-site channel sums of layer K [B][N]
    double *dlog;
    int32_t *err;
    int ps_a, ps_b;            // plane strides (bytes) of the even- and odd-layer buffers
    int buf_b;                 // byte offset of the odd-layer buffer (CH planes of ps_a)
    const int32_t *ring;       // ring tables, one entry per site (see ring_chunk)
    // write-back launches only: the configuration S' of every item whose
    // chain has commit[chain] != 0 becomes the chain's base pass (the cone's
    // activations replace the cache and its site sums replace hsum)
    const int32_t *commit;
    uint16_t *cache_w;
    double *hsum_w;
};

// Up to kMaxJobs lattices (contexts of one network shape) in one launch: their
// queue items form one index space, job after job.
struct ConeJobs {
    ConeParams job[kMaxJobs];
    // per job, [tau][k - 1]: first ring-table entry of the ring of W_{k+1};
    // [tau][K - 1]: end
    int ring_off[kMaxJobs][4][kMaxK];
    int n;
};

__device__ __forceinline__ int wrap_l(int a, int L)
{
    a += (a < 0) ? L : 0;
    return a - ((a >= L) ? L : 0);
}

__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    const float2v f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
}

__device__ __forceinline__ uint32_t pack_u16(uint16_t a, uint16_t b)
{
    return (uint32_t)a | ((uint32_t)b << 16);
}

struct Ring {
    u32x4 v[kRingRegs];
    int dst[kRingRegs];        // byte address in the window buffer, -1: none
};

// This thread's ring-table entries (one per prefetched chunk), -1: none.
struct RingTab {
    int ent[kRingRegs];
};

// Table entries of the ring of W_{k+1} (entries [e0, e1) of the table, one
// per site): chunk q = lt + i * kThreads reads entry e0 + q / CH.
template <int X>
__device__ __forceinline__ void ring_tab_load(RingTab &t, const ConeParams &p, bool live, int e0,
                                              int e1, int lt)
{
    using F = Form<X>;
#pragma unroll
    for (int i = 0; i < kRingRegs; ++i) {
        const int q = lt + i * F::kThreads;
        const bool ok = live && q < (e1 - e0) * F::CH;
        const int e = p.ring[ok ? e0 + q / F::CH : 0];
        t.ent[i] = ok ? e : -1;
    }
}

// Chunk c of ring entry `ent` (window index | (du mod L) << 16 | (dv mod L) << 24,
// offsets from the anchor): .x element offset in the layer cache, .y byte
// offset in the window buffer of plane stride ps.
template <int X>
__device__ __forceinline__ int2 ring_chunk(int ent, int c, int ax, int ay, int L, int ps)
{
    uint32_t x = (uint32_t)(ax + ((ent >> 16) & 255));
    uint32_t y = (uint32_t)(ay + ((uint32_t)ent >> 24));
    x = min(x, x - (uint32_t)L);        // x, y < 2L: one conditional period
    y = min(y, y - (uint32_t)L);
    return make_int2((int)(__umul24(y, (uint32_t)L) + x) * Form<X>::SITE + c * 8,
                     (int)__umul24((uint32_t)c, (uint32_t)ps) + (ent & 0xffff) * kChunk);
}

// Issue the loads of the prefetched ring chunks named by `t`.
template <int X>
__device__ __forceinline__ void ring_fetch(Ring &r, const RingTab &t, int lt, int ax, int ay, int L,
                                           int ps, const uint16_t *layer_cache)
{
#pragma unroll
    for (int i = 0; i < kRingRegs; ++i) {
        const bool live = t.ent[i] >= 0;
        const int2 sd = ring_chunk<X>(live ? t.ent[i] : 0, lt % Form<X>::CH, ax, ay, L, ps);
        r.v[i] = *(const u32x4 *)(layer_cache + (uint32_t)sd.x);
        r.dst[i] = live ? sd.y : -1;
    }
}

// Store the fetched chunks, then copy any chunks of entries [e0, e1) beyond
// them directly.
template <int X>
__device__ __forceinline__ void ring_store(const Ring &r, const ConeParams &p, int lt,
                                           unsigned char *buf, int e0, int e1, int ax, int ay,
                                           int L, int ps, const uint16_t *layer_cache)
{
    using F = Form<X>;
#pragma unroll
    for (int i = 0; i < kRingRegs; ++i)
        if (r.dst[i] >= 0) *(u32x4 *)(buf + r.dst[i]) = r.v[i];
    const int total = (e1 - e0) * F::CH;
    for (int q = lt + kRingRegs * F::kThreads; q < total; q += F::kThreads) {
        const int2 sd = ring_chunk<X>(p.ring[e0 + q / F::CH], q % F::CH, ax, ay, L, ps);
        *(u32x4 *)(buf + sd.y) = *(const u32x4 *)(layer_cache + (uint32_t)sd.x);
    }
}

// Weights of one layer (A operands, one 16-byte fragment per lane per
// K-step and half; the split form also the lo parts).
template <int X>
struct Weights {
    bf16x8 hi[KS][NH];
    bf16x8 lo[X >= 3 && X != 5 ? KS : 1][NH];     // the frame form reads them from LDS
};

template <int X>
__device__ __forceinline__ void load_layer(Weights<X> &wt, const ConeParams &p, int k, int lane)
{
    const bf16x8 *base = p.wa + (int64_t)(k - 2) * KS * NH * 64;
#pragma unroll
    for (int j = 0; j < KS; ++j)
#pragma unroll
        for (int hh = 0; hh < NH; ++hh) wt.hi[j][hh] = base[(j * NH + hh) * 64 + lane];
    if (X >= 3 && X != 5) {
        const bf16x8 *bl = p.wl + (int64_t)(k - 2) * KS * NH * 64;
#pragma unroll
        for (int j = 0; j < KS; ++j)
#pragma unroll
            for (int hh = 0; hh < NH; ++hh)
                wt.lo[X >= 3 && X != 5 ? j : 0][hh] = bl[(j * NH + hh) * 64 + lane];
    }
}

// Everything one tile needs (wave-uniform): the tile's first position in R_k
// and the layer geometry.
struct TileArgs {
    int p0, npos, ex;
    uint32_t mul;              // ceil(2^20 / ex): p / ex = (p * mul) >> 20, exact for ex <= 64, p < 66 ex
    int p16;                   // row pitch of W_k in bytes (within a plane)
    int q16;                   // row pitch of W_{k+1} in bytes
    int psc, psn;              // plane strides of the buffers of W_k and W_{k+1}
};

// NT tiles of one layer.  Inner layers store the BF16 activations into
// W_{k+1} (split form: hi into planes 0..3, lo into planes 4..7); the last
// layer accumulates the site sums.
template <int X, bool last, int NT, bool COMMIT>
__device__ __forceinline__ void cone_group(const Weights<X> &wt, const floatx4 (&bias)[NH],
                                           const unsigned char *cur, unsigned char *nxt,
                                           uint16_t *wcache, double *whsum, int k,
                                           const TileArgs (&ta)[NT], int L, int K, int ax, int ay,
                                           const double *hsum_s, int g, int n16, double &fsum,
                                           const unsigned char *wlo = nullptr,
                                           u32x4 *sh = nullptr, u32x4 *sl = nullptr,
                                           int *sa = nullptr)
{
    using F = Form<X>;
    floatx4 acc[NT][NH];
    int ain[NT], aout[NT];
    bool valid[NT];
    double hs_base[NT];
    int site_w[NT];            // lattice site of the output (write-back launches)
#pragma unroll
    for (int w = 0; w < NT; ++w) {
        int p = ta[w].p0 + n16;
        valid[w] = p < ta[w].npos;
        p = valid[w] ? p : ta[w].npos - 1;
        const int v = (int)(((uint32_t)p * ta[w].mul) >> 20);
        const int u = p - __mul24(v, ta[w].ex);
        const int u16 = u * kChunk;
        // tap (dx, dy) of output (u, v) is window site (u + 1 + dx, v + 1 + dy);
        // lane group g reads plane g (and plane 4 + g for the lo parts)
        ain[w] = __mul24(g, ta[w].psc) + __mul24(v, ta[w].p16) + u16;
        // output goes to W_{k+1} site (u + 2, v + 2)
        aout[w] = __mul24(g, ta[w].psn) + __mul24(v + 2, ta[w].q16) + u16 + 2 * kChunk;
        hs_base[w] = 0.0;
        site_w[w] = 0;
        if (last || COMMIT) site_w[w] = wrap_l(ay + v - k, L) * L + wrap_l(ax + u - k, L);
        if (last) hs_base[w] = hsum_s[site_w[w]];
    }
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
#pragma unroll
        for (int w = 0; w < NT; ++w) {
            const unsigned char *row = cur + ain[w] + dy * ta[w].p16;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int j = dy * 3 + dx;
                const bf16x8 bv = *(const bf16x8 *)(row + dx * kChunk);
                if (X >= 3) {
                    // the split form's product order: lo*hi, hi*lo, hi*hi
                    const bf16x8 bl = *(const bf16x8 *)(row + 4 * ta[w].psc + dx * kChunk);
#pragma unroll
                    for (int hh = 0; hh < NH; ++hh) {
                        floatx4 c0 = j == 0 ? bias[hh] : acc[w][hh];
                        bf16x8 wl;
                        if constexpr (Form<X>::FRAME)
                            wl = *(const bf16x8 *)(wlo + (((j * NH + hh) << 6) + (g << 4) + n16) *
                                                             kChunk);
                        else
                            wl = wt.lo[X >= 3 && X != 5 ? j : 0][hh];
                        c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, bv, c0, 0, 0, 0);
                        c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wt.hi[j][hh], bl, c0, 0, 0,
                                                                     0);
                        acc[w][hh] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wt.hi[j][hh], bv,
                                                                             c0, 0, 0, 0);
                    }
                } else {
#pragma unroll
                    for (int hh = 0; hh < NH; ++hh)
                        acc[w][hh] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            wt.hi[j][hh], bv, j == 0 ? bias[hh] : acc[w][hh], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int w = 0; w < NT; ++w) {
        float zv[8], hv[8];
#pragma unroll
        for (int hh = 0; hh < NH; ++hh)
#pragma unroll
            for (int r = 0; r < 4; ++r) zv[hh * 4 + r] = acc[w][hh][r];
        if (X >= 3)
            mf::ln_cosh_x3_n<8>(zv, hv);
        else
            mf::ln_cosh_n<8>(zv, hv);
        if (!last) {
            if (X >= 3) {
                uint16_t hi[8], lo[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) mf::split_bf16(hv[r], &hi[r], &lo[r]);
                const u32x4 ph = {pack_u16(hi[0], hi[1]), pack_u16(hi[2], hi[3]),
                                  pack_u16(hi[4], hi[5]), pack_u16(hi[6], hi[7])};
                const u32x4 pl = {pack_u16(lo[0], lo[1]), pack_u16(lo[2], lo[3]),
                                  pack_u16(lo[4], lo[5]), pack_u16(lo[6], lo[7])};
                if constexpr (Form<X>::FRAME) {
                    // held until every wave has read the frame
                    sh[w] = ph;
                    sl[w] = pl;
                    sa[w] = valid[w] ? aout[w] : -1;
                }
                if (valid[w]) {
                    if constexpr (!Form<X>::FRAME) {
                        *(u32x4 *)(nxt + aout[w]) = ph;
                        *(u32x4 *)(nxt + aout[w] + 4 * ta[w].psn) = pl;
                    }
                    if (COMMIT) {
                        *(u32x4 *)(wcache + site_w[w] * F::SITE + g * 8) = ph;
                        *(u32x4 *)(wcache + site_w[w] * F::SITE + C + g * 8) = pl;
                    }
                }
            } else if (valid[w]) {
                const u32x4 pk = {pack_bf16(hv[0], hv[1]), pack_bf16(hv[2], hv[3]),
                                  pack_bf16(hv[4], hv[5]), pack_bf16(hv[6], hv[7])};
                *(u32x4 *)(nxt + aout[w]) = pk;
                if (COMMIT) *(u32x4 *)(wcache + site_w[w] * F::SITE + g * 8) = pk;
            }
        } else {
            double part = 0.0;
#pragma unroll
            for (int r = 0; r < 8; ++r) part += (double)hv[r];
            part += __shfl_xor(part, 16);
            part += __shfl_xor(part, 32);
            if (g == 0 && valid[w]) {
                fsum += part - hs_base[w];
                if (COMMIT) whsum[site_w[w]] = part;
            }
        }
    }
}

// Waves that work on a layer of ntiles tiles.  Plain form: small layers go to
// two waves, so that the other two need not fetch that layer's weights.  Split
// form (eight waves, three times the matrix work per tile): one tile per wave
// as far as the tiles go.
template <int X>
__device__ __forceinline__ int active_waves(int ntiles)
{
    if (X >= 3) return ntiles < Form<X>::NW ? ntiles : Form<X>::NW;
    return ntiles <= 8 ? 2 : Form<X>::NW;
}

// All tiles of layer k owned by this wave (tiles wave, wave + nw, ...), one at
// a time (the other workgroups / waves of the CU supply the parallelism a
// second tile in flight would), with the layer's weights in `wt`.
// Frame form: fw16 is the frame's row pitch in bytes, wlo the layer's lo
// weights in LDS, and an inner layer's outputs are staged in sh, sl, sa (tile
// wave + n nw in slot n; sa = -1: nothing to store).
template <int X, bool last, bool COMMIT>
__device__ __forceinline__ void cone_layer(const Weights<X> &wt, const float *bs,
                                           const unsigned char *cur, unsigned char *nxt,
                                           uint16_t *wcache, double *whsum, int psc,
                                           int psn, int k, int w0, int h0, int L, int K, int ax,
                                           int ay, const double *hsum_s, int wave, int g, int n16,
                                           double &fsum, int fw16 = 0,
                                           const unsigned char *wlo = nullptr,
                                           u32x4 *sh = nullptr, u32x4 *sl = nullptr,
                                           int *sa = nullptr)
{
    TileArgs a;
    a.ex = w0 + 2 * k;
    a.npos = a.ex * (h0 + 2 * k);
    a.mul = ((1u << 20) + a.ex - 1) / a.ex;
    a.p16 = fw16 ? fw16 : (a.ex + 2) * kChunk;     // W_k = R_{k+1}: width ex + 2
    a.q16 = fw16 ? fw16 : (a.ex + 4) * kChunk;     // W_{k+1}: width ex + 4
    a.psc = psc;
    a.psn = psn;
    const int ntiles = (a.npos + 15) >> 4;
    const int nw = active_waves<X>(ntiles);
    if constexpr (Form<X>::FRAME && !last) {
#pragma unroll
        for (int n = 0; n < kFrameMaxT; ++n) sa[n] = -1;
    }
    if (wave >= nw) return;
    // bias of this lane's output rows 16 hh + 4 g + r
    floatx4 bias[NH];
#pragma unroll
    for (int hh = 0; hh < NH; ++hh)
        bias[hh] = *(const floatx4 *)(bs + (k - 2) * C + 16 * hh + 4 * g);
    if constexpr (Form<X>::FRAME && !last) {
#pragma unroll
        for (int n = 0; n < kFrameMaxT; ++n) {
            const int t = wave + n * nw;
            if (t < ntiles) {
                TileArgs ta[1] = {a};
                ta[0].p0 = t * 16;
                cone_group<X, last, 1, COMMIT>(wt, bias, cur, nxt, wcache, whsum, k, ta, L, K, ax,
                                               ay, hsum_s, g, n16, fsum, wlo, sh + n, sl + n,
                                               sa + n);
            }
        }
        return;
    }
    int t = wave;
    for (; t < ntiles; t += nw) {
        TileArgs ta[1] = {a};
        ta[0].p0 = t * 16;
        cone_group<X, last, 1, COMMIT>(wt, bias, cur, nxt, wcache, whsum, k, ta, L, K, ax, ay,
                                       hsum_s, g, n16, fsum, wlo);
    }
}

// Plain form: three workgroups per CU, 166 VGPRs and 46 KB of LDS (K = 8)
// each.  Split form: two workgroups of four waves per CU (windows, K <= 7; the
// frame form, 73 KB, at K = 8), else one of eight waves.
// NJ: the number of jobs the launch can hold.  COMMIT: write-back launch (one
// job): items whose chain is flagged in commit[] store the activations of
// their cone into the cache and their site sums into hsum, so that the cache
// becomes the base pass of S' (the arithmetic is the base pass's, so the
// values are those a new base pass would give); other items are skipped.
// Reads of the cache (ring, layer k) and writes (R_k, layer k) never meet.
template <int NJ, bool COMMIT, int X>
__global__ void __launch_bounds__(Form<X>::kThreads)
    __attribute__((amdgpu_waves_per_eu(Form<X>::WPE, Form<X>::WPE)))
k_net_cone(ConeJobs jobs)
{
    using F = Form<X>;
    constexpr int kThreads = F::kThreads;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    __shared__ double red[F::NW];

    const int K = jobs.job[0].K;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
    const int g = lane >> 4, n16 = lane & 15;
    // first item of each job in the common index space
    int64_t first[NJ + 1];
    first[0] = 0;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        first[j + 1] = first[j] + (j < jobs.n ? min(jobs.job[j].qlen[0], jobs.job[j].capacity) : 0);
    const int64_t n_units = first[NJ];

    // XCD-contiguous ranges of the queue
    const int per_xcd = gridDim.x / kXcd;
    const int xcd = blockIdx.x % kXcd, slot = blockIdx.x / kXcd;
    const int64_t seg = (n_units + kXcd - 1) / kXcd;
    const int64_t u_end = min(n_units, (xcd + 1) * seg);

    auto job_of = [&](int64_t u) {
        int jb = 0;
#pragma unroll
        for (int j = 1; j < NJ; ++j) jb = (u >= first[j]) ? j : jb;
        return jb;
    };
    Weights<X> wt;
    if (xcd * seg + slot < u_end) load_layer<X>(wt, jobs.job[job_of(xcd * seg + slot)], 2, lane);
    // frame form: the layer's lo weights in LDS after the frame, the next
    // layer's on their way in lpf (chunk q = tid + r kThreads of KS NH 64)
    constexpr int kLoChunks = KS * NH * 64;
    constexpr int kLoSlots = F::FRAME ? (kLoChunks + kThreads - 1) / kThreads : 1;
    unsigned char *wlo = lds + F::CH * (jobs.job[0].ps_a + jobs.job[0].ps_b);
    u32x4 lpf[kLoSlots];
    auto lo_fetch = [&](const ConeParams &pp, int k) {
        const u32x4 *src = reinterpret_cast<const u32x4 *>(pp.wl) + (int64_t)(k - 2) * kLoChunks;
#pragma unroll
        for (int r = 0; r < kLoSlots; ++r) {
            const int q = tid + r * kThreads;
            lpf[r] = src[q < kLoChunks ? q : 0];
        }
    };
    auto lo_store = [&]() {
#pragma unroll
        for (int r = 0; r < kLoSlots; ++r) {
            const int q = tid + r * kThreads;
            if (q < kLoChunks) *(u32x4 *)(wlo + q * kChunk) = lpf[r];
        }
    };
    if constexpr (F::FRAME)
        if (xcd * seg + slot < u_end) lo_fetch(jobs.job[job_of(xcd * seg + slot)], 2);
    float *w1s = reinterpret_cast<float *>(wlo + (F::FRAME ? kLoChunks * kChunk : 0));
    float *bs = w1s + kW1Floats;   // bias of layer k at bs[(k - 2) C]
    int w1_job = -1;   // job whose layer-1 weights w1s holds

    for (int64_t u = xcd * seg + slot; u < u_end; u += per_xcd) {
        const int jb = job_of(u);
        // this job's parameters, read once per configuration
        const ConeParams prm = jobs.job[jb];
        if (jb != w1_job) {
            // every thread has passed the previous configuration's barriers, so
            // nobody still reads the old table
            for (int q = tid; q < kW1Floats; q += kThreads) {
                const int m = q / 20, r = q - 20 * (q / 20);
                const int co = mf::chan_of_slot<C>(2 * m + (r >= 10 ? 1 : 0));
                const int t = r >= 10 ? r - 10 : r;
                w1s[q] = t < 9 ? prm.w1[t * C + co] : prm.bias[co];
            }
            for (int q = tid; q < (K - 1) * C; q += kThreads) bs[q] = prm.bias[C + q];
            __syncthreads();
            w1_job = jb;
        }
        const int *roff_j = jobs.ring_off[jb][0];
        const int64_t unit = u - first[jb];
        const int L = prm.L, N = L * L;
        const uint32_t e = prm.queue[unit];
        const int s = item_sample(e);
        if (COMMIT && prm.commit[s] == 0) continue;   // uniform over the workgroup
        const int b = item_bond(e), tau = b & 3, i0 = b >> 2;
        const int xi = i0 % L, yi = i0 / L;
        const int qi = i0, qj = wrap_l(yi + bond_dy(tau), L) * L + wrap_l(xi + bond_dx(tau), L);
        const int ax = xi, ay = (tau == 3) ? wrap_l(yi - 1, L) : yi;
        const int w0 = (tau == 1) ? 1 : 2, h0 = (tau == 0) ? 1 : 2;
        const int8_t *sp = prm.spins + (int64_t)s * N;
        const int64_t layer_el = (int64_t)N * F::SITE;   // cache values per layer
        const uint16_t *cache_s = prm.cache + (int64_t)s * (K - 1) * layer_el;
        const double *hsum_s = prm.hsum + (int64_t)s * N;
        uint16_t *wcache_s = COMMIT ? prm.cache_w + (int64_t)s * (K - 1) * layer_el : nullptr;
        double *whsum_s = COMMIT ? prm.hsum_w + (int64_t)s * N : nullptr;

        const int *roff = roff_j + tau * kMaxK;

        // ---- layer 1 (vector ALU) into W_2 (buffer A), two channels per thread ----
        RingTab tab;
        {
            ring_tab_load<X>(tab, prm, true, roff[0], roff[1], tid);
            Ring ring;
            ring_fetch<X>(ring, tab, tid, ax, ay, L, prm.ps_a, cache_s);
            ring_tab_load<X>(tab, prm, K >= 3, roff[1], roff[K >= 3 ? 2 : 1], tid);
            const int ex1 = w0 + 2, ey1 = h0 + 2;
            const int pos = tid >> 4, m = tid & 15;
            if (pos < ex1 * ey1) {
                const int u = pos % ex1, v = pos / ex1;
                const int gx = wrap_l(ax + u - 1, L), gy = wrap_l(ay + v - 1, L);
                float sv[9];
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    int site = wrap_l(gy + t / 3 - 1, L) * L + wrap_l(gx + t % 3 - 1, L);
                    site = (site == qi) ? qj : ((site == qj) ? qi : site);
                    sv[t] = (float)sp[site];
                }
                // the base pass's FMA order: bias, then taps 0..8
                const float *wm = w1s + 20 * m;
                float z0 = wm[9], z1 = wm[19];
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    z0 = __builtin_fmaf(wm[t], sv[t], z0);
                    z1 = __builtin_fmaf(wm[10 + t], sv[t], z1);
                }
                // W_2 site (u + 2, v + 2), pitch its width; in the frame form
                // frame site (K + u, K + v), pitch 2K + 4
                const int p2 = F::FRAME ? 2 * K + 4 : ex1 + 4;
                const int o2 = F::FRAME ? K : 2;
                unsigned char *dst =
                    lds + (m >> 2) * prm.ps_a + ((v + o2) * p2 + u + o2) * kChunk + (m & 3) * 4;
                uint16_t *cdst = COMMIT ? wcache_s + (gy * L + gx) * F::SITE + (m >> 2) * 8 +
                                              (m & 3) * 2
                                        : nullptr;
                if (X >= 3) {
                    uint16_t h0u, l0u, h1u, l1u;
                    mf::split_bf16(mf::ln_cosh_x3(z0), &h0u, &l0u);
                    mf::split_bf16(mf::ln_cosh_x3(z1), &h1u, &l1u);
                    *(uint32_t *)dst = pack_u16(h0u, h1u);
                    *(uint32_t *)(dst + 4 * prm.ps_a) = pack_u16(l0u, l1u);
                    if (COMMIT) {
                        *(uint32_t *)cdst = pack_u16(h0u, h1u);
                        *(uint32_t *)(cdst + C) = pack_u16(l0u, l1u);
                    }
                } else {
                    const float h0v = mf::ln_cosh(z0);
                    const float h1v = mf::ln_cosh(z1);
                    *(uint32_t *)dst = pack_bf16(h0v, h1v);
                    if (COMMIT) *(uint32_t *)cdst = pack_bf16(h0v, h1v);
                }
            }
            ring_store<X>(ring, prm, tid, lds, roff[0], roff[1], ax, ay, L, prm.ps_a, cache_s);
            if constexpr (F::FRAME) lo_store();          // layer 2's lo weights
        }
        // ring of W_{k+1}, fetched one layer ahead; its table entries two ahead
        Ring ring;
        ring_fetch<X>(ring, tab, tid, ax, ay, L, F::FRAME ? prm.ps_a : prm.ps_b,
                      cache_s + (K >= 3 ? layer_el : 0));
        ring_tab_load<X>(tab, prm, K >= 4, roff[K >= 4 ? 2 : 0], roff[K >= 4 ? 3 : 0], tid);
        __syncthreads();

        double fsum = 0.0;
        if constexpr (F::FRAME) {
            // one frame: W_k is its sub-square from (K - k, K - k), R_k from
            // (K + 1 - k, K + 1 - k).  A layer's outputs wait in registers
            // until every wave has read W_k, then replace R_k; the ring
            // W_{k+1} \ R_k follows from the cache, and the next layer's lo
            // weights from lpf.
            const int fw = 2 * K + 4, fw16 = fw * kChunk, ps = prm.ps_a;
            for (int k = 2; k <= K; ++k) {
                const unsigned char *cur = lds + (K - k) * (fw + 1) * kChunk;
                unsigned char *nxt = lds + (K - k - 1) * (fw + 1) * kChunk;
                uint16_t *wc = COMMIT ? wcache_s + (int64_t)(k - 1) * layer_el : nullptr;
                if (k < K)
                    lo_fetch(prm, k + 1);
                else if (u + per_xcd < u_end)
                    lo_fetch(jobs.job[job_of(u + per_xcd)], 2);
                u32x4 sh[kFrameMaxT], sl[kFrameMaxT];
                int sa[kFrameMaxT];
                // the tiles run at a raised wave priority, so that when the
                // CU's two workgroups compete for instruction issue, tile work
                // goes first (1% faster at K = 8, bit-identical)
                __builtin_amdgcn_s_setprio(1);
                if (k < K)
                    cone_layer<X, false, COMMIT>(wt, bs, cur, nxt, wc, whsum_s, ps, ps, k, w0, h0,
                                                 L, K, ax, ay, hsum_s, wave, g, n16, fsum, fw16,
                                                 wlo, sh, sl, sa);
                else
                    cone_layer<X, true, COMMIT>(wt, bs, cur, nxt, wc, whsum_s, ps, ps, k, w0, h0,
                                                L, K, ax, ay, hsum_s, wave, g, n16, fsum, fw16,
                                                wlo);
                __builtin_amdgcn_s_setprio(0);
                if (k < K) {
                    const int nt_next = ((w0 + 2 * k + 2) * (h0 + 2 * k + 2) + 15) >> 4;
                    if (wave < active_waves<X>(nt_next)) load_layer<X>(wt, prm, k + 1, lane);
                } else if (u + per_xcd < u_end) {
                    load_layer<X>(wt, jobs.job[job_of(u + per_xcd)], 2, lane);
                }
                __syncthreads();                 // every read of W_k and of its weights is done
                if (k < K) {
#pragma unroll
                    for (int n = 0; n < kFrameMaxT; ++n)
                        if (sa[n] >= 0) {
                            *(u32x4 *)(nxt + sa[n]) = sh[n];
                            *(u32x4 *)(nxt + sa[n] + 4 * ps) = sl[n];
                        }
                    ring_store<X>(ring, prm, tid, lds, roff[k - 1], roff[k], ax, ay, L, ps,
                                  cache_s + (int64_t)(k - 1) * layer_el);
                    lo_store();
                    if (k + 1 < K) {
                        ring_fetch<X>(ring, tab, tid, ax, ay, L, ps,
                                      cache_s + (int64_t)k * layer_el);
                        const bool more = k + 2 < K;
                        ring_tab_load<X>(tab, prm, more, roff[more ? k + 1 : 0],
                                         roff[more ? k + 2 : 0], tid);
                    }
                    __syncthreads();             // W_{k+1} and its lo weights are complete
                }
            }
        } else {
        for (int k = 2; k <= K; ++k) {
            unsigned char *cur = lds + ((k & 1) ? prm.buf_b : 0);
            unsigned char *nxt = lds + ((k & 1) ? 0 : prm.buf_b);
            const int psc = (k & 1) ? prm.ps_b : prm.ps_a;
            const int psn = (k & 1) ? prm.ps_a : prm.ps_b;
            // ring of W_{k+1} into the buffer W_{k-1} occupied, the ring of
            // W_{k+2} on its way, and the table entries of the ring of W_{k+3}
            if (k < K) {
                ring_store<X>(ring, prm, tid, nxt, roff[k - 1], roff[k], ax, ay, L, psn,
                              cache_s + (int64_t)(k - 1) * layer_el);
                if (k + 1 < K) {
                    // W_{k+2} lives in the buffer of W_k
                    ring_fetch<X>(ring, tab, tid, ax, ay, L, psc, cache_s + (int64_t)k * layer_el);
                    const bool more = k + 2 < K;
                    ring_tab_load<X>(tab, prm, more, roff[more ? k + 1 : 0],
                                     roff[more ? k + 2 : 0], tid);
                }
            }
            uint16_t *wc = COMMIT ? wcache_s + (int64_t)(k - 1) * layer_el : nullptr;
            if (k < K)
                cone_layer<X, false, COMMIT>(wt, bs, cur, nxt, wc, whsum_s, psc, psn, k, w0, h0,
                                             L, K, ax, ay, hsum_s, wave, g, n16, fsum);
            else
                cone_layer<X, true, COMMIT>(wt, bs, cur, nxt, wc, whsum_s, psc, psn, k, w0, h0,
                                            L, K, ax, ay, hsum_s, wave, g, n16, fsum);
            // weights of the next layer if this wave works on it; after the last,
            // layer 2's of the next configuration (whose job may differ)
            if (k < K) {
                const int nt_next = ((w0 + 2 * k + 2) * (h0 + 2 * k + 2) + 15) >> 4;
                if (wave < active_waves<X>(nt_next)) load_layer<X>(wt, prm, k + 1, lane);
            } else if (u + per_xcd < u_end) {
                load_layer<X>(wt, jobs.job[job_of(u + per_xcd)], 2, lane);
            }
            __syncthreads();
        }
        }

        for (int off = 32; off > 0; off >>= 1) fsum += __shfl_xor(fsum, off);
        if (lane == 0) red[wave] = fsum;
        __syncthreads();
        if (tid == 0) {
            double v = 0.0;
            for (int w = 0; w < F::NW; ++w) v += red[w];
            if (!isfinite(v)) atomicOr(prm.err, kErrNonFinite);
            prm.dlog[unit] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Lockstep form: G exchanged configurations per workgroup, layer by layer.
//
// The kernel above works on one configuration at a time, so every wave
// re-reads a layer's A operands (18 KB plain, 36 KB split) for every
// configuration it touches: the texture-address unit, not the matrix cores,
// limits it.  Here a workgroup takes G consecutive queue items of one lattice
// (mostly of one sample) and advances them together: each wave loads layer
// k's weights once and works on the tiles of all G cones, so the weight
// traffic per configuration falls by G.
//
// Each item has one frame in LDS, the rectangle R_{K+1} (2K + 4 sites square
// for the largest bond box, CH channel planes of 16 bytes per site); window
// W_k and output R_k of every layer are centred sub-rectangles of it, so a
// layer is updated in place: the waves compute all their tiles of layer k
// into registers, a barrier retires the reads of W_k, then the outputs and
// the ring W_{k+1} \ R_k (prefetched from the sample's cache during the
// compute) are written, and a second barrier opens layer k + 1.  Half the
// LDS of the double-buffered windows is what lets G configurations share a
// workgroup.  The per-site arithmetic (K-step order, products, ln cosh,
// rounding, FP64 site sums) is the base pass's, as in the kernel above.
// ---------------------------------------------------------------------------

constexpr int kLsMaxK = 8;      // frames and register arrays are sized for K <= 8

struct LsJob {
    const int8_t *spins;
    int L;
    const uint32_t *queue;
    const int64_t *qlen;
    int64_t capacity;
    const bf16x8 *wa, *wl;
    const float *w1;            // layer 1 [9][C]
    const float *bias;          // [K][C]
    const uint16_t *cache;
    const double *hsum;
    double *dlog;
    int32_t *err;
};

struct LsJobs {
    LsJob job[kMaxJobs];
    int n, K;
    const int32_t *tab;         // frame ring tables (identical for every job of one K)
    int16_t off[4][kMaxK];      // [tau][k - 1]: first entry of the ring W_{k+1} \ R_k; [tau][K - 1]: end
};

template <int X, int G, int NW>
struct LsShape {
    static constexpr int CH = Form<X>::CH;
    static constexpr int SITE = Form<X>::SITE;
    static constexpr int THREADS = NW * 64;
    static constexpr int TILES_MAX = ((2 * kLsMaxK + 2) * (2 * kLsMaxK + 2) + 15) / 16;
    static constexpr int MAXT = (G * TILES_MAX + NW - 1) / NW;    // tiles per wave and layer
    static constexpr int RING_MAX = 16 * (kLsMaxK - 1) + 32;      // ring sites per item and layer
    static constexpr int MAXR = (G * RING_MAX * CH + THREADS - 1) / THREADS;
};

// one batch item, kept in LDS
struct LsItem {
    int s, tau, ax, ay, qi, qj, live, pad;
    int64_t unit;
};

__device__ __forceinline__ int box_w(int tau) { return tau == 1 ? 1 : 2; }
__device__ __forceinline__ int box_h(int tau) { return tau == 0 ? 1 : 2; }

// Prefix tables of one layer (LDS): first tile and first ring chunk of each
// item, item after item.  Filled by thread 0 for the next layer between the
// layer's two barriers, so no wave reads them while they change.
template <int G>
struct LsTab {
    int tile[G + 1];
    int ring[G + 1];
};

template <int X, int G>
__device__ __forceinline__ void ls_fill_tab(LsTab<G> &t, const LsItem *items, const LsJobs &jobs,
                                            int k, int K)
{
    t.tile[0] = 0;
    t.ring[0] = 0;
    for (int i = 0; i < G; ++i) {
        const LsItem it = items[i];
        const int ex = box_w(it.tau) + 2 * k, ey = box_h(it.tau) + 2 * k;
        t.tile[i + 1] = t.tile[i] + (it.live ? (ex * ey + 15) >> 4 : 0);
        // ring W_{k+1} \ R_k (none after the last layer)
        t.ring[i + 1] = t.ring[i] + ((k < K && it.live)
                                         ? (jobs.off[it.tau][k] - jobs.off[it.tau][k - 1]) * Form<X>::CH
                                         : 0);
    }
}

// item of entry q of a prefix table (q < tab[G])
template <int G>
__device__ __forceinline__ int ls_item_of(const int *tab, int q)
{
    int i = 0;
    for (int j = 1; j < G; ++j) i = (q >= tab[j]) ? j : i;
    return i;
}

template <int X, int G, int NW, int WPE>
__global__ void __launch_bounds__(NW * 64)
    __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
k_net_cone_ls(LsJobs jobs)
{
    using S = LsShape<X, G, NW>;
    using F = Form<X>;
    constexpr int kThreads = S::THREADS;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];

    const int K = jobs.K;
    const int FW = 2 * K + 4;                  // frame width and height (sites)
    const int PB = FW * FW * kChunk;           // bytes of one channel plane of a frame
    const int FB = S::CH * PB;                 // bytes of a frame
    float *w1s = reinterpret_cast<float *>(lds + G * FB);
    float *bs = w1s + kW1Floats;               // bias of layer k at bs[(k - 2) C]
    LsItem *items = reinterpret_cast<LsItem *>(bs + (K - 1) * C);
    double *red = reinterpret_cast<double *>(items + G);     // [NW][G]
    LsTab<G> *tab = reinterpret_cast<LsTab<G> *>(red + NW * G);   // [2]: by layer parity

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, n16 = lane & 15;

    // batches of one job each: job j holds ceil(n_j / G) batches (at most two jobs)
    const int64_t n0 = jobs.n > 0 ? min(jobs.job[0].qlen[0], jobs.job[0].capacity) : 0;
    const int64_t n1 = jobs.n > 1 ? min(jobs.job[1].qlen[0], jobs.job[1].capacity) : 0;
    const int64_t nb0 = (n0 + G - 1) / G;
    const int64_t n_batches = nb0 + (n1 + G - 1) / G;
    const int per_xcd = gridDim.x / kXcd;
    const int xcd = blockIdx.x % kXcd, slot = blockIdx.x / kXcd;
    const int64_t seg = (n_batches + kXcd - 1) / kXcd;
    const int64_t b_end = min(n_batches, (xcd + 1) * seg);

    int w1_job = -1;

    for (int64_t b = xcd * seg + slot; b < b_end; b += per_xcd) {
        const int jb = b >= nb0 ? 1 : 0;
        const LsJob &jp = jobs.job[jb];
        const int L = jp.L, N = L * L;
        const int64_t i0 = (b - (jb ? nb0 : 0)) * G;
        const int64_t n_job = jb ? n1 : n0;
        const int64_t layer_el = (int64_t)N * F::SITE;
        // the previous batch's reads of its frames and tables are retired
        // (it ended with a barrier); load this batch's items and tables
        if (tid < G) {
            LsItem it{};
            const int64_t u = i0 + tid;
            it.live = u < n_job;
            it.unit = u;
            if (it.live) {
                const uint32_t e = jp.queue[u];
                it.s = item_sample(e);
                const int bd = item_bond(e), tau = bd & 3, q0 = bd >> 2;
                const int xi = q0 % L, yi = q0 / L;
                it.tau = tau;
                it.qi = q0;
                it.qj = wrap_l(yi + bond_dy(tau), L) * L + wrap_l(xi + bond_dx(tau), L);
                it.ax = xi;
                it.ay = (tau == 3) ? wrap_l(yi - 1, L) : yi;
            }
            items[tid] = it;
        }
        if (jb != w1_job) {
            for (int q = tid; q < kW1Floats; q += kThreads) {
                const int m = q / 20, r = q - 20 * (q / 20);
                const int co = mf::chan_of_slot<C>(2 * m + (r >= 10 ? 1 : 0));
                const int t = r >= 10 ? r - 10 : r;
                w1s[q] = t < 9 ? jp.w1[t * C + co] : jp.bias[co];
            }
            for (int q = tid; q < (K - 1) * C; q += kThreads) bs[q] = jp.bias[C + q];
            w1_job = jb;
        }
        __syncthreads();
        // ring W_2 \ R_1 (prefix in tab[1].ring) and layer 2's tiles and ring (tab[0])
        if (tid == 0) {
            ls_fill_tab<X, G>(tab[1], items, jobs, 1, K);
            ls_fill_tab<X, G>(tab[0], items, jobs, 2, K);
        }

        // ---- layer 1 (vector ALU) on R_1 of every item, two channels per unit ----
        for (int q = tid; q < G * 256; q += kThreads) {
            const int i = q >> 8, pos = (q >> 4) & 15, m = q & 15;
            const LsItem it = items[i];
            const int w0 = box_w(it.tau), h0 = box_h(it.tau);
            const int ex1 = w0 + 2;
            if (!it.live || pos >= ex1 * (h0 + 2)) continue;
            const int u = pos % ex1, v = pos / ex1;
            const int gx = wrap_l(it.ax + u - 1, L), gy = wrap_l(it.ay + v - 1, L);
            const int8_t *sp = jp.spins + (int64_t)it.s * N;
            float sv[9];
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                int site = wrap_l(gy + t / 3 - 1, L) * L + wrap_l(gx + t % 3 - 1, L);
                site = (site == it.qi) ? it.qj : ((site == it.qj) ? it.qi : site);
                sv[t] = (float)sp[site];
            }
            const float *wm = w1s + 20 * m;
            float z0 = wm[9], z1 = wm[19];
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                z0 = __builtin_fmaf(wm[t], sv[t], z0);
                z1 = __builtin_fmaf(wm[10 + t], sv[t], z1);
            }
            // R_1 sits at frame (K + u, K + v)
            unsigned char *dst =
                lds + i * FB + (m >> 2) * PB + ((K + v) * FW + K + u) * kChunk + (m & 3) * 4;
            if (X >= 3) {
                uint16_t h0u, l0u, h1u, l1u;
                mf::split_bf16(mf::ln_cosh_x3(z0), &h0u, &l0u);
                mf::split_bf16(mf::ln_cosh_x3(z1), &h1u, &l1u);
                *(uint32_t *)dst = pack_u16(h0u, h1u);
                *(uint32_t *)(dst + 4 * PB) = pack_u16(l0u, l1u);
            } else {
                *(uint32_t *)dst = pack_bf16(mf::ln_cosh(z0), mf::ln_cosh(z1));
            }
        }
        __syncthreads();                        // tables visible
        // ring W_2 \ R_1 from the cache of layer 1
        {
            const int *rt = tab[1].ring;
            const int total = rt[G];
            for (int q = tid; q < total; q += kThreads) {
                const int i = ls_item_of<G>(rt, q);
                const LsItem it = items[i];
                const int r = q - rt[i], e = r / S::CH, c = r - e * S::CH;
                const int ent = jobs.tab[jobs.off[it.tau][0] + e];
                const int fx = (ent >> 16) & 255, fy = (uint32_t)ent >> 24;
                const int site = wrap_l(it.ay + fy - K - 1, L) * L + wrap_l(it.ax + fx - K - 1, L);
                *(u32x4 *)(lds + i * FB + c * PB + (ent & 0xffff) * kChunk) =
                    *(const u32x4 *)(jp.cache + (int64_t)it.s * (K - 1) * layer_el +
                                     (int64_t)site * F::SITE + c * 8);
            }
        }
        __syncthreads();

        double fs[G];
#pragma unroll
        for (int i = 0; i < G; ++i) fs[i] = 0.0;

        for (int k = 2; k <= K; ++k) {
            const bool last = (k == K);
            const LsTab<G> &tk = tab[k & 1 ? 1 : 0];
            const int ntiles = tk.tile[G];
            // ring W_{k+1} \ R_k of every item (cache of layer k), in flight
            // during the compute
            u32x4 rv[S::MAXR];
            int rdst[S::MAXR];
            const int rtotal = tk.ring[G];
#pragma unroll
            for (int r = 0; r < S::MAXR; ++r) {
                const int q = tid + r * kThreads;
                rdst[r] = -1;
                if (q < rtotal) {
                    const int i = ls_item_of<G>(tk.ring, q);
                    const LsItem it = items[i];
                    const int rr = q - tk.ring[i], e = rr / S::CH, c = rr - e * S::CH;
                    const int ent = jobs.tab[jobs.off[it.tau][k - 1] + e];
                    const int fx = (ent >> 16) & 255, fy = (uint32_t)ent >> 24;
                    const int site =
                        wrap_l(it.ay + fy - K - 1, L) * L + wrap_l(it.ax + fx - K - 1, L);
                    rv[r] = *(const u32x4 *)(jp.cache + ((int64_t)it.s * (K - 1) + (k - 1)) * layer_el +
                                             (int64_t)site * F::SITE + c * 8);
                    rdst[r] = i * FB + c * PB + (ent & 0xffff) * kChunk;
                }
            }
            // bias of this lane's output rows 16 hh + 4 g + r
            floatx4 bias[NH];
#pragma unroll
            for (int hh = 0; hh < NH; ++hh)
                bias[hh] = *(const floatx4 *)(bs + (k - 2) * C + 16 * hh + 4 * g);

            // this wave's tiles: tile n is T = wave + n NW; per tile the LDS
            // address of tap (0, 0), the output address (-1: not stored) and,
            // in the last layer, the lattice site and item of the output
            int a0[S::MAXT], oaddr[S::MAXT], osite[S::MAXT], oitem[S::MAXT];
#pragma unroll
            for (int n = 0; n < S::MAXT; ++n) {
                const int T = wave + n * NW;
                a0[n] = 0;
                oaddr[n] = -1;
                osite[n] = -1;
                oitem[n] = 0;
                if (T >= ntiles) continue;      // uniform over the wave
                const int i = ls_item_of<G>(tk.tile, T);
                const LsItem it = items[i];
                const int ex = box_w(it.tau) + 2 * k, npos = ex * (box_h(it.tau) + 2 * k);
                int p = (T - tk.tile[i]) * 16 + n16;
                const bool valid = p < npos;
                p = valid ? p : npos - 1;
                // p / ex as (p * ceil(2^20 / ex)) >> 20: exact for ex <= 64, p < 66 ex
                const uint32_t mul = ((1u << 20) + ex - 1) / ex;
                const int v = (int)(((uint32_t)p * mul) >> 20), u = p - v * ex;
                const int fx = K + 1 - k + u, fy = K + 1 - k + v;     // output site in the frame
                a0[n] = i * FB + g * PB + ((fy - 1) * FW + fx - 1) * kChunk;
                if (valid) {
                    oaddr[n] = i * FB + g * PB + (fy * FW + fx) * kChunk;
                    osite[n] = it.s * N + wrap_l(it.ay + fy - K - 1, L) * L +
                               wrap_l(it.ax + fx - K - 1, L);
                }
                oitem[n] = i;
            }
            // taps outermost: the tap's A operands (streamed, the next tap's in
            // flight) against every tile of the wave; per tile and half the
            // accumulation order is the base pass's (bias, then taps 0..8)
            floatx4 acc[S::MAXT][NH];
            const bf16x8 *wbase = jp.wa + (int64_t)(k - 2) * KS * NH * 64 + lane;
            const bf16x8 *lbase = jp.wl + (int64_t)(k - 2) * KS * NH * 64 + lane;
            bf16x8 ah[NH], al[NH], nh[NH], nl[NH];
#pragma unroll
            for (int hh = 0; hh < NH; ++hh) {
                ah[hh] = wbase[hh * 64];
                if (X >= 3) al[hh] = lbase[hh * 64];
            }
#pragma unroll
            for (int j = 0; j < KS; ++j) {
                if (j + 1 < KS) {
#pragma unroll
                    for (int hh = 0; hh < NH; ++hh) {
                        nh[hh] = wbase[((j + 1) * NH + hh) * 64];
                        if (X >= 3) nl[hh] = lbase[((j + 1) * NH + hh) * 64];
                    }
                }
                const int toff = ((j / 3) * FW + (j % 3)) * kChunk;
#pragma unroll
                for (int n = 0; n < S::MAXT; ++n) {
                    if (wave + n * NW >= ntiles) continue;     // uniform
                    const unsigned char *ap = lds + a0[n] + toff;
                    const bf16x8 bv = *(const bf16x8 *)ap;
                    if (X >= 3) {
                        const bf16x8 bl = *(const bf16x8 *)(ap + 4 * PB);
#pragma unroll
                        for (int hh = 0; hh < NH; ++hh) {
                            floatx4 c0 = j == 0 ? bias[hh] : acc[n][hh];
                            c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[hh], bv, c0, 0, 0, 0);
                            c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[hh], bl, c0, 0, 0, 0);
                            acc[n][hh] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[hh], bv, c0, 0,
                                                                                 0, 0);
                        }
                    } else {
#pragma unroll
                        for (int hh = 0; hh < NH; ++hh)
                            acc[n][hh] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                ah[hh], bv, j == 0 ? bias[hh] : acc[n][hh], 0, 0, 0);
                    }
                }
                if (j + 1 < KS) {
#pragma unroll
                    for (int hh = 0; hh < NH; ++hh) {
                        ah[hh] = nh[hh];
                        if (X >= 3) al[hh] = nl[hh];
                    }
                }
            }
            // epilogue: ln cosh, then BF16 (split: hi and lo) held for the
            // in-place store, or the last layer's site sums
            u32x4 oh[S::MAXT], ol[X >= 3 ? S::MAXT : 1];
#pragma unroll
            for (int n = 0; n < S::MAXT; ++n) {
                if (wave + n * NW >= ntiles) continue;         // uniform
                float zv[8], hv[8];
#pragma unroll
                for (int hh = 0; hh < NH; ++hh)
#pragma unroll
                    for (int r = 0; r < 4; ++r) zv[hh * 4 + r] = acc[n][hh][r];
                if (X >= 3)
                    mf::ln_cosh_x3_n<8>(zv, hv);
                else
                    mf::ln_cosh_n<8>(zv, hv);
                if (!last) {
                    if (X >= 3) {
                        uint16_t hi[8], lo[8];
#pragma unroll
                        for (int r = 0; r < 8; ++r) mf::split_bf16(hv[r], &hi[r], &lo[r]);
                        oh[n] = u32x4{pack_u16(hi[0], hi[1]), pack_u16(hi[2], hi[3]),
                                      pack_u16(hi[4], hi[5]), pack_u16(hi[6], hi[7])};
                        ol[X >= 3 ? n : 0] = u32x4{pack_u16(lo[0], lo[1]), pack_u16(lo[2], lo[3]),
                                                   pack_u16(lo[4], lo[5]), pack_u16(lo[6], lo[7])};
                    } else {
                        oh[n] = u32x4{pack_bf16(hv[0], hv[1]), pack_bf16(hv[2], hv[3]),
                                      pack_bf16(hv[4], hv[5]), pack_bf16(hv[6], hv[7])};
                    }
                } else {
                    double part = 0.0;
#pragma unroll
                    for (int r = 0; r < 8; ++r) part += (double)hv[r];
                    part += __shfl_xor(part, 16);
                    part += __shfl_xor(part, 32);
                    if (g == 0 && osite[n] >= 0) {
                        const double d = part - jp.hsum[osite[n]];
                        // item oitem[n]'s sum; compared, not indexed
#pragma unroll
                        for (int q = 0; q < G; ++q) fs[q] += (q == oitem[n]) ? d : 0.0;
                    }
                }
            }
            __syncthreads();                    // every read of W_k and of tab[k] is done
            if (!last) {
                if (tid == 0) ls_fill_tab<X, G>(tab[k & 1 ? 0 : 1], items, jobs, k + 1, K);
#pragma unroll
                for (int n = 0; n < S::MAXT; ++n)
                    if (oaddr[n] >= 0) {
                        *(u32x4 *)(lds + oaddr[n]) = oh[n];
                        if (X >= 3) *(u32x4 *)(lds + oaddr[n] + 4 * PB) = ol[X >= 3 ? n : 0];
                    }
#pragma unroll
                for (int r = 0; r < S::MAXR; ++r)
                    if (rdst[r] >= 0) *(u32x4 *)(lds + rdst[r]) = rv[r];
                __syncthreads();                // W_{k+1} and tab[k + 1] are complete
            }
        }

        // ---- per-item sums: lanes, then waves in a fixed order ----
#pragma unroll
        for (int i = 0; i < G; ++i) {
            double v = fs[i];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) red[wave * G + i] = v;
        }
        __syncthreads();
        if (tid < G) {
            const LsItem it = items[tid];
            if (it.live) {
                double v = 0.0;
                for (int w = 0; w < NW; ++w) v += red[w * G + tid];
                if (!isfinite(v)) atomicOr(jp.err, kErrNonFinite);
                jp.dlog[it.unit] = v;
            }
        }
        // the items, sums, tables and frames of this batch stay in use until here
        __syncthreads();
    }
}

// row pitch (sites) of window W_k for a changed box of width w0: its width
inline int win_pitch(int w0, int k) { return w0 + 2 * k + 2; }

// bytes of one channel plane of window W_k for the largest bond box (2 x 2)
inline int plane_bytes(int k) { return (2 * k + 4) * win_pitch(2, k) * kChunk; }

// One chunk added to every plane stride.  A stride that is a multiple of 256
// bytes (every even layer's, and the frame's, 16 (K + 2)^2 bytes) puts the
// eight chunks of a site, which eight neighbouring lanes store together, and
// the four lane groups' planes of an operand fetch into the same LDS banks.
constexpr int kPlanePad = kChunk;

// plane strides of the even- and odd-layer buffers
inline void plane_strides(int K, int *ps_a, int *ps_b)
{
    *ps_a = *ps_b = 0;
    for (int k = 2; k <= K; ++k) {
        int &ps = (k & 1) ? *ps_b : *ps_a;
        ps = std::max(ps, plane_bytes(k) + kPlanePad);
    }
}

}  // namespace

bool cone_supported(const nqs_ctx *c)
{
    return c->dtype == NQS_BF16 && c->C == 32 && c->K >= 2 && c->L >= 2 * c->K + 4 &&
           mfma_supported(c) && cone_lds_bytes(c) <= 159 * 1024;
}

bool cone_x3_supported(const nqs_ctx *c)
{
    return c->dtype == NQS_BF16X3 && c->C == 32 && c->K >= 2 && c->L >= 2 * c->K + 4 &&
           cone_lds_bytes(c) <= 159 * 1024;
}

size_t cone_lds_bytes(const nqs_ctx *c)
{
    int a, b;
    plane_strides(c->K, &a, &b);
    const int ch = c->dtype == NQS_BF16X3 ? Form<3>::CH : Form<1>::CH;
    return (size_t)ch * (a + b) + sizeof(float) * (kW1Floats + kBiasFloats);
}

// Ring tables of the unwrapped geometry: for bond type tau and k = 1..K-1 the
// sites of W_{k+1} = R_{k+2} outside R_k, as (index in W_{k+1}, whose pitch is
// P_{k+1}) | (offset from the anchor modulo L) << 16 (x) and << 24 (y).
// Ring tables of the lockstep kernel: for bond type tau and k = 1..K-1 the
// sites of W_{k+1} = R_{k+2} outside R_k in frame coordinates (the frame is
// R_{K+1} of the 2 x 2 box, 2K + 4 sites square; R_k of a w0 x h0 box starts
// at K + 1 - k), as frame index | x << 16 | y << 24.
static void ls_tables(int K, std::vector<int32_t> &ent, std::vector<int> &off)
{
    const int FW = 2 * K + 4;
    off.assign((size_t)4 * kMaxK, 0);
    for (int tau = 0; tau < 4; ++tau) {
        const int w0 = (tau == 1) ? 1 : 2, h0 = (tau == 0) ? 1 : 2;
        for (int k = 1; k < K; ++k) {
            off[(size_t)tau * kMaxK + (k - 1)] = (int)ent.size();
            const int r0 = K + 1 - k, w0r = K - 1 - k;
            for (int fy = w0r; fy < w0r + h0 + 2 * k + 4; ++fy)
                for (int fx = w0r; fx < w0r + w0 + 2 * k + 4; ++fx) {
                    if (fx >= r0 && fx < r0 + w0 + 2 * k && fy >= r0 && fy < r0 + h0 + 2 * k)
                        continue;   // R_k
                    ent.push_back((fy * FW + fx) | (fx << 16) | (fy << 24));
                }
        }
        off[(size_t)tau * kMaxK + (K - 1)] = (int)ent.size();
    }
}

// Ring tables of the in-place frame form: cone_tab's entries (the sites of
// W_{k+1} = R_{k+2} outside R_k, with their offsets from the anchor modulo L)
// with the window index replaced by the frame index (frame of side 2K + 4, the
// bond box's anchor at frame site (K + 1, K + 1)).
static void fr_tables(int K, int L, std::vector<int32_t> &ent, std::vector<int> &off)
{
    const int FW = 2 * K + 4, F = K + 1;
    off.assign((size_t)4 * kMaxK, 0);
    for (int tau = 0; tau < 4; ++tau) {
        const int w0 = (tau == 1) ? 1 : 2, h0 = (tau == 0) ? 1 : 2;
        for (int k = 1; k < K; ++k) {
            off[(size_t)tau * kMaxK + (k - 1)] = (int)ent.size();
            const int r0 = F - k, w0r = F - k - 2;
            for (int fy = w0r; fy < w0r + h0 + 2 * k + 4; ++fy)
                for (int fx = w0r; fx < w0r + w0 + 2 * k + 4; ++fx) {
                    if (fx >= r0 && fx < r0 + w0 + 2 * k && fy >= r0 && fy < r0 + h0 + 2 * k)
                        continue;   // R_k
                    const int du = (((fx - F) % L) + L) % L, dv = (((fy - F) % L) + L) % L;
                    ent.push_back((fy * FW + fx) | (du << 16) | (dv << 24));
                }
        }
        off[(size_t)tau * kMaxK + (K - 1)] = (int)ent.size();
    }
}

nqs_status cone_build_ring_tables(nqs_ctx *c)
{
    const int L = c->L, K = c->K;
    if (K <= kLsMaxK) {
        std::vector<int32_t> fe;
        fr_tables(K, L, fe, c->fr_off);
        if (c->fr_tab) (void)hipFree(c->fr_tab);
        c->fr_tab = nullptr;
        if (hipMalloc((void **)&c->fr_tab, std::max<size_t>(fe.size(), 1) * 4) != hipSuccess)
            return NQS_E_NOMEM;
        if (!fe.empty() &&
            hipMemcpy(c->fr_tab, fe.data(), fe.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return NQS_E_HIP;
    }
    if (K <= kLsMaxK) {
        std::vector<int32_t> le;
        ls_tables(K, le, c->ls_off);
        if (c->ls_tab) (void)hipFree(c->ls_tab);
        c->ls_tab = nullptr;
        if (hipMalloc((void **)&c->ls_tab, std::max<size_t>(le.size(), 1) * 4) != hipSuccess)
            return NQS_E_NOMEM;
        if (!le.empty() &&
            hipMemcpy(c->ls_tab, le.data(), le.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return NQS_E_HIP;
    }
    std::vector<int32_t> ent;
    c->cone_off.assign((size_t)4 * kMaxK, 0);
    for (int tau = 0; tau < 4; ++tau) {
        const int w0 = (tau == 1) ? 1 : 2, h0 = (tau == 0) ? 1 : 2;
        for (int k = 1; k < K; ++k) {
            c->cone_off[(size_t)tau * kMaxK + (k - 1)] = (int)ent.size();
            const int ex = w0 + 2 * k, ey = h0 + 2 * k;
            const int pitch = win_pitch(w0, k + 1);
            for (int wv = 0; wv < ey + 4; ++wv)
                for (int wu = 0; wu < ex + 4; ++wu) {
                    if (wu >= 2 && wu < 2 + ex && wv >= 2 && wv < 2 + ey) continue;   // R_k
                    const int du = wu - (k + 2), dv = wv - (k + 2);
                    const int dum = ((du % L) + L) % L, dvm = ((dv % L) + L) % L;
                    ent.push_back((wv * pitch + wu) | (dum << 16) | (dvm << 24));
                }
        }
        c->cone_off[(size_t)tau * kMaxK + (K - 1)] = (int)ent.size();
    }
    if (c->cone_tab) (void)hipFree(c->cone_tab);
    c->cone_tab = nullptr;
    if (hipMalloc((void **)&c->cone_tab, std::max<size_t>(ent.size(), 1) * 4) != hipSuccess)
        return NQS_E_NOMEM;
    if (!ent.empty() &&
        hipMemcpy(c->cone_tab, ent.data(), ent.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return NQS_E_HIP;
    return NQS_OK;
}

template <int NJ, bool COMMIT, int X>
static void cone_launch_x(const ConeJobs &jp, const nqs_ctx *c0, size_t lds, hipStream_t s)
{
    const void *fn = (const void *)k_net_cone<NJ, COMMIT, X>;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, Form<X>::kThreads, lds) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    // persistent grid of resident workgroups, a multiple of the XCD count
    const int64_t want = std::max<int64_t>((int64_t)c0->n_cu * per_cu / kXcd * kXcd, kXcd);
    NQS_LAUNCH((k_net_cone<NJ, COMMIT, X>), dim3((unsigned)want), dim3(Form<X>::kThreads), lds,
               s, jp);
}

// bytes of LDS the lockstep kernel takes for G items
static size_t ls_lds_bytes(int K, int X, int G, int NW)
{
    const size_t FW = 2 * (size_t)K + 4;
    const size_t fb = (X == 3 ? Form<3>::CH : Form<1>::CH) * FW * FW * kChunk;
    return G * fb + sizeof(float) * (kW1Floats + (size_t)(K - 1) * C) + G * sizeof(LsItem) +
           (size_t)NW * G * sizeof(double) + 2 * sizeof(int) * 2 * (G + 1);
}

template <int X, int G, int NW, int WPE>
static bool ls_launch_x(const LsJobs &jp, const nqs_ctx *c0, hipStream_t s)
{
    const size_t lds = ls_lds_bytes(c0->K, X, G, NW);
    if (lds > 160 * 1024) return false;
    const void *fn = (const void *)k_net_cone_ls<X, G, NW, WPE>;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NW * 64, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int64_t want = std::max<int64_t>((int64_t)c0->n_cu * per_cu / kXcd * kXcd, kXcd);
    NQS_LAUNCH((k_net_cone_ls<X, G, NW, WPE>), dim3((unsigned)want), dim3(NW * 64), lds, s, jp);
    return true;
}

// The lockstep kernel's shapes (items per workgroup, waves); variant 0 is the
// default of each form, the autotuner may pick another.
struct LsVariant {
    int G, NW, WPE;
};
const LsVariant kLsPlain[] = {{1, 4, 3}, {2, 8, 2}};
const LsVariant kLsSplit[] = {{1, 4, 2}, {1, 8, 2}};

static bool ls_launch(const ConnJob *jobs, int n, hipStream_t s)
{
    const nqs_ctx *c0 = jobs[0].c;
    if (n > 2 || c0->K > kLsMaxK || c0->ls_tab == nullptr || c0->cone_variant < 0) return false;
    LsJobs jp{};
    jp.n = n;
    jp.K = c0->K;
    jp.tab = c0->ls_tab;
    for (int t = 0; t < 4; ++t)
        for (int k = 0; k < kMaxK; ++k) jp.off[t][k] = (int16_t)c0->ls_off[(size_t)t * kMaxK + k];
    int64_t total_cap = 0;
    for (int i = 0; i < n; ++i) {
        const nqs_ctx *c = jobs[i].c;
        LsJob &p = jp.job[i];
        p.spins = jobs[i].spins;
        p.L = c->L;
        p.queue = jobs[i].queue;
        p.qlen = jobs[i].qlen;
        p.capacity = jobs[i].capacity;
        p.wa = (const bf16x8 *)c->w_mfma;
        p.wl = (const bf16x8 *)c->w_mfma_lo;
        p.w1 = c->w_l1;
        p.bias = c->w_l1 + 9 * C;
        p.cache = (const uint16_t *)jobs[i].cache;
        p.hsum = jobs[i].hsum;
        p.dlog = jobs[i].dlog;
        p.err = c->err;
        total_cap += jobs[i].capacity;
    }
    if (total_cap <= 0) return true;
    const int v = c0->cone_variant;
    if (c0->dtype == NQS_BF16X3) {
        switch (v) {
        case 0: return ls_launch_x<3, 1, 4, 2>(jp, c0, s);
        case 1: return ls_launch_x<3, 1, 8, 2>(jp, c0, s);
        default: return false;
        }
    }
    switch (v) {
    case 0: return ls_launch_x<1, 1, 4, 3>(jp, c0, s);
    case 1: return ls_launch_x<1, 2, 8, 2>(jp, c0, s);
    default: return false;
    }
}

// commit: null for the exchanged-configuration pass; else the write-back
// launch (one job) for the chains flagged in commit[]
static void cone_launch(const ConnJob *jobs, int n, const int32_t *commit, hipStream_t s)
{
    if (n <= 0) return;
    // the lockstep kernel serves the exchanged-configuration pass where its
    // frames fit (K <= 8); write-back launches and deeper networks take the
    // one-configuration kernel
    if (!commit && ls_launch(jobs, n, s)) return;
    // the split form's shape: two four-wave workgroups per CU with their two
    // window buffers where those fit (K <= 7), else with one frame updated in
    // place and the lo weights in LDS where that fits (K <= 8), else one
    // workgroup of eight waves
    const nqs_ctx *c0 = jobs[0].c;
    const size_t tables = sizeof(float) * (kW1Floats + kBiasFloats);
    const size_t wsums = Form<4>::NW * sizeof(double);
    const int FW = 2 * c0->K + 4;
    const size_t frame_ps = (size_t)FW * FW * kChunk + kPlanePad;
    const size_t lo_bytes = (size_t)KS * NH * 64 * kChunk;
    const size_t frame_lds = Form<5>::CH * frame_ps + lo_bytes + tables;
    int split_x = 3;
    if (c0->dtype == NQS_BF16X3) {
        if (2 * (cone_lds_bytes(c0) + wsums) <= 160 * 1024) {
            split_x = 4;
        } else {
            bool frame = c0->K <= kLsMaxK && 2 * (frame_lds + wsums) <= 160 * 1024;
            for (int i = 0; i < n; ++i) frame = frame && jobs[i].c->fr_tab != nullptr;
            if (frame) split_x = 5;
        }
    }
    ConeJobs jp{};
    jp.n = n;
    int64_t total_cap = 0;
    for (int i = 0; i < n; ++i) {
        const nqs_ctx *c = jobs[i].c;
        ConeParams &p = jp.job[i];
        p.spins = jobs[i].spins;
        p.L = c->L;
        p.K = c->K;
        p.queue = jobs[i].queue;
        p.qlen = jobs[i].qlen;
        p.capacity = jobs[i].capacity;
        p.wa = (const bf16x8 *)c->w_mfma;
        p.wl = (const bf16x8 *)c->w_mfma_lo;
        p.w1 = c->w_l1;
        p.bias = c->w_l1 + 9 * C;
        p.cache = (const uint16_t *)jobs[i].cache;
        p.hsum = jobs[i].hsum;
        p.dlog = jobs[i].dlog;
        p.err = c->err;
        if (split_x == 5) {
            p.ring = c->fr_tab;
            for (int t = 0; t < 4; ++t)
                for (int k = 0; k < kMaxK; ++k) jp.ring_off[i][t][k] = c->fr_off[(size_t)t * kMaxK + k];
            p.ps_a = (int)frame_ps;              // one frame: plane stride, no second buffer
            p.ps_b = 0;
            p.buf_b = 0;
        } else {
            p.ring = c->cone_tab;
            for (int t = 0; t < 4; ++t)
                for (int k = 0; k < kMaxK; ++k)
                    jp.ring_off[i][t][k] = c->cone_off[(size_t)t * kMaxK + k];
            plane_strides(c->K, &p.ps_a, &p.ps_b);
            p.buf_b = (c->dtype == NQS_BF16X3 ? Form<3>::CH : Form<1>::CH) * p.ps_a;
        }
        p.commit = commit;
        p.cache_w = (uint16_t *)jobs[i].cache;
        p.hsum_w = const_cast<double *>(jobs[i].hsum);
        total_cap += jobs[i].capacity;
    }
    if (total_cap <= 0) return;
    const size_t lds = split_x == 5 ? frame_lds : cone_lds_bytes(c0);
    // launches of one or two lattices use the two-job instantiation (fewer
    // scalar registers; a one-job instantiation spills)
    if (c0->dtype == NQS_BF16X3) {
        if (split_x == 5) {
            if (commit)
                cone_launch_x<2, true, 5>(jp, c0, lds, s);
            else if (n > 2)
                cone_launch_x<kMaxJobs, false, 5>(jp, c0, lds, s);
            else
                cone_launch_x<2, false, 5>(jp, c0, lds, s);
            return;
        }
        if (split_x == 4) {
            if (commit)
                cone_launch_x<2, true, 4>(jp, c0, lds, s);
            else if (n > 2)
                cone_launch_x<kMaxJobs, false, 4>(jp, c0, lds, s);
            else
                cone_launch_x<2, false, 4>(jp, c0, lds, s);
            return;
        }
        if (commit)
            cone_launch_x<2, true, 3>(jp, c0, lds, s);
        else if (n > 2)
            cone_launch_x<kMaxJobs, false, 3>(jp, c0, lds, s);
        else
            cone_launch_x<2, false, 3>(jp, c0, lds, s);
        return;
    }
    if (commit)
        cone_launch_x<2, true, 1>(jp, c0, lds, s);
    else if (n > 2)
        cone_launch_x<kMaxJobs, false, 1>(jp, c0, lds, s);
    else
        cone_launch_x<2, false, 1>(jp, c0, lds, s);
}

void cone_forward_jobs(const ConnJob *jobs, int n, hipStream_t s) { cone_launch(jobs, n, nullptr, s); }

void cone_commit(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue, const int64_t *qlen,
                 int64_t capacity, double *hsum, void *cache, double *dlog, const int32_t *commit,
                 hipStream_t s)
{
    const ConnJob j{c, spins, queue, qlen, capacity, hsum, cache, dlog};
    cone_launch(&j, 1, commit, s);
}


void cone_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue, const int64_t *qlen,
                  int64_t capacity, const double *hsum, const void *cache, double *dlog,
                  hipStream_t s)
{
    const ConnJob j{c, spins, queue, qlen, capacity, hsum, cache, dlog};
    cone_forward_jobs(&j, 1, s);
}

}  // namespace nqs

namespace nqs {
int cone_variants(const nqs_ctx *c)
{
    if (c->K > kLsMaxK) return 0;
    return c->dtype == NQS_BF16X3 ? (int)(sizeof(kLsSplit) / sizeof(kLsSplit[0]))
                                  : (int)(sizeof(kLsPlain) / sizeof(kLsPlain[0]));
}

void cone_variant_shape(const nqs_ctx *c, int v, int *items, int *waves)
{
    if (v < 0 || v >= cone_variants(c)) {
        // the one-configuration kernel
        *items = 1;
        *waves = 0;
        return;
    }
    const LsVariant t = c->dtype == NQS_BF16X3 ? kLsSplit[v] : kLsPlain[v];
    *items = t.G;
    *waves = t.NW;
}

int cone_variant_of(const nqs_ctx *c, int items, int waves)
{
    for (int v = 0; v < cone_variants(c); ++v) {
        int g, w;
        cone_variant_shape(c, v, &g, &w);
        if (g == items && w == waves) return v;
    }
    return -1;
}
}  // namespace nqs
