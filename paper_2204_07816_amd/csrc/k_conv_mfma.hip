// k_conv_mfma.hip -- BF16 matrix-core form of the CNN log-amplitude for the
// exchanged configurations of the local energy [Sec. 5.4.1: the forward of
// the network over the O(L^2) exchanged configurations takes over 95% of the
// time; Sec. 5.2: periodic 3x3 convolutions, log of a product of neurons].
//
// One fused kernel evaluates a whole network per work item (a sample in the
// base pass, one exchanged configuration S' otherwise):
//
//   * layer 1 (one input channel) on the vector ALU in FP32 from the int8
//     spins with the pair exchanged on the fly;
//   * layers 2..K as implicit GEMMs on v_mfma_f32_16x16x32_bf16: A = 16
//     output channels x 32 reduction elements of the weights (held in VGPRs
//     for the whole layer), B = 32 reduction elements x 16 sites gathered
//     from the activation window in LDS with the periodic wrap folded into
//     the index arithmetic (no padded copy), FP32 accumulation seeded with
//     the bias;
//   * ln cosh in FP32, activations rounded to BF16 (round to nearest even)
//     between layers; the last layer's per-site channel sums in FP64.
//
// Incremental mode: an exchange at sites (i, j) can only change layer k on
// the sites within Chebyshev distance k of i or j.  The kernel recomputes
// layer k on the bounding rectangle R_k of that cone (clamped to the torus)
// and reads every other input from the activations the base pass cached for
// the sample.  f(S') - f(s) = sum_{p in R_K} (hs'(p) - hs(p)) in FP64, with
// hs(p) the base pass's per-site sum, so sites the exchange does not reach
// contribute exactly zero: both passes run the same instruction sequence on
// the same inputs.  Full mode uses R_k = the whole lattice.
//
// Activation layout (LDS window and HBM cache): [site][C] BF16 with the
// channels of a site permuted so that the 16-lane groups of the MFMA output
// write 16 contiguous bytes, and the next layer's B operand reads them back
// as one 16-byte LDS load per lane.  The weight packing absorbs the
// permutation.
#include <algorithm>

#include "mfma_common.h"

namespace nqs {
namespace {

using mf::bf16x8;
using mf::floatx4;
using mf::Shape;

enum { kBase = 0, kFull = 1, kIncr = 2 };

__device__ inline int wrapm(int a, int L) { return ((a % L) + L) % L; }

struct Rect {
    int ox, oy, ex, ey;
};

// Bounding rectangle of the layer-k cone of the exchanged pair, clamped to
// the torus; origin 0 when an extent covers the whole ring.
__device__ inline Rect rect_k(bool full, int x0, int y0, int w0, int h0, int k, int L)
{
    Rect r;
    if (full) {
        r.ox = 0; r.oy = 0; r.ex = L; r.ey = L;
        return r;
    }
    r.ex = min(w0 + 2 * k, L);
    r.ey = min(h0 + 2 * k, L);
    r.ox = (r.ex == L) ? 0 : wrapm(x0 - k, L);
    r.oy = (r.ey == L) ? 0 : wrapm(y0 - k, L);
    return r;
}

// Index of global site (gx, gy) inside rectangle W (caller guarantees it lies in W).
__device__ inline int win_index(const Rect &W, int gx, int gy, int L)
{
    const int u = wrapm(gx - W.ox, L), v = wrapm(gy - W.oy, L);
    return v * W.ex + u;
}

__device__ inline bool in_rect(const Rect &R, int gx, int gy, int L)
{
    return wrapm(gx - R.ox, L) < R.ex && wrapm(gy - R.oy, L) < R.ey;
}

struct Params {
    const int8_t *spins;
    int L, K, B;
    int mode;
    const bf16x8 *wa;        // MFMA A operands, layers 2..K
    const float *w1;         // layer 1 weights [9][C] (logical channels)
    const float *bias;       // [K][C] logical
    // base pass outputs
    uint16_t *cache_out;     // [B][K-1][N][C] bf16 (physical slots)
    double *hsum_out;        // [B][N]
    double *f_out;           // [B]
    // exchanged configurations
    const uint32_t *queue;
    const int64_t *qlen;
    int64_t capacity;
    const uint16_t *cache_in;
    const double *hsum_in;
    double *dlog;
    int32_t *err;
};

// Up to kMaxConnJobs lattices (contexts of one network shape) in one launch of
// an exchanged-configuration mode: their queue items form one index space, job
// after job.  The base pass is always a single job.
struct NetJobs {
    Params job[kMaxConnJobs];
    int n;
};

template <int C, int NW, int MAXT>
__global__ void __launch_bounds__(NW * 64)
k_net(NetJobs jobs)
{
    using S = Shape<C>;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    __shared__ double red[NW];

    const int K = jobs.job[0].K;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, n16 = lane & 15;
    const bool base = jobs.job[0].mode == kBase;
    const bool full = jobs.job[0].mode != kIncr;

    // first item of each job in the common index space
    int64_t first[kMaxConnJobs + 1];
    first[0] = 0;
#pragma unroll
    for (int j = 0; j < kMaxConnJobs; ++j)
        first[j + 1] = first[j] + (j >= jobs.n ? 0
                                               : (base ? jobs.job[j].B
                                                       : min(jobs.job[j].qlen[0], jobs.job[j].capacity)));
    const int64_t n_units = first[kMaxConnJobs];
    for (int64_t u = blockIdx.x; u < n_units; u += gridDim.x) {
        int jb = 0;
#pragma unroll
        for (int j = 1; j < kMaxConnJobs; ++j) jb = (u >= first[j]) ? j : jb;
        const Params &prm = jobs.job[jb];
        const int64_t unit = u - first[jb];
        const int L = prm.L, N = L * L;
        // ---- geometry of the work item ----
        int s, x0 = 0, y0 = 0, w0 = 1, h0 = 1, qi = -1, qj = -1;
        if (base) {
            s = (int)unit;
        } else {
            const uint32_t e = prm.queue[unit];
            s = item_sample(e);
            const int b = item_bond(e), t = b & 3, i = b >> 2;
            const int xi = i % L, yi = i / L;
            qi = i;
            qj = wrapm(yi + bond_dy(t), L) * L + wrapm(xi + bond_dx(t), L);
            x0 = xi;
            w0 = (t == 1) ? 1 : 2;
            h0 = (t == 0) ? 1 : 2;
            y0 = (t == 3) ? wrapm(yi - 1, L) : yi;
        }
        const int8_t *sp = prm.spins + (int64_t)s * N;

        // ---- layer 1 on the vector ALU: outputs on R_1 into window W_2 = R_3 ----
        {
            const Rect R1 = rect_k(full, x0, y0, w0, h0, 1, L);
            const Rect W2 = rect_k(full, x0, y0, w0, h0, K >= 2 ? 3 : 1, L);
            const int npos = R1.ex * R1.ey;
            for (int q = tid; q < npos * 4; q += NW * 64) {
                const int p = q >> 2, gg = q & 3;
                const int gx = (R1.ox + p % R1.ex) % L, gy = (R1.oy + p / R1.ex) % L;
                float sv[9];
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const int yy = wrapm(gy + t / 3 - 1, L), xx = wrapm(gx + t % 3 - 1, L);
                    int site = yy * L + xx;
                    site = (site == qi) ? qj : ((site == qj) ? qi : site);
                    sv[t] = (float)sp[site];
                }
                float h[S::CG];
#pragma unroll
                for (int r = 0; r < S::CG; ++r) {
                    const int co = mf::chan_of_slot<C>(gg * S::CG + r);
                    h[r] = mf::ln_cosh(mf::layer1_z(prm.w1, prm.bias, C, co, sv));
                }
                if (K == 1) continue;  // (single-layer networks are not routed here)
                uint16_t hb[S::CG];
#pragma unroll
                for (int r = 0; r < S::CG; ++r) hb[r] = mf::to_bf16(h[r]);
                const int wi = win_index(W2, gx, gy, L);
                uint16_t *dst = (uint16_t *)(lds + wi * S::PSB) + gg * S::CG;
#pragma unroll
                for (int r = 0; r < S::CG; ++r) dst[r] = hb[r];
                if (base) {
                    uint16_t *cd = prm.cache_out + (((int64_t)s * (K - 1) + 0) * N + gy * L + gx) * C +
                                   gg * S::CG;
#pragma unroll
                    for (int r = 0; r < S::CG; ++r) cd[r] = hb[r];
                }
            }
            if (!full) {
                // ring of W_2 outside R_1 from the cache of layer 1
                const int nw = W2.ex * W2.ey;
                for (int q = tid; q < nw * 4; q += NW * 64) {
                    const int p = q >> 2, gg = q & 3;
                    const int gx = (W2.ox + p % W2.ex) % L, gy = (W2.oy + p / W2.ex) % L;
                    if (in_rect(R1, gx, gy, L)) continue;
                    const uint16_t *src = prm.cache_in +
                                          (((int64_t)s * (K - 1) + 0) * N + gy * L + gx) * C +
                                          gg * S::CG;
                    uint16_t *dst = (uint16_t *)(lds + p * S::PSB) + gg * S::CG;
#pragma unroll
                    for (int r = 0; r < S::CG; ++r) dst[r] = src[r];
                }
            }
        }
        __syncthreads();

        double fsum = 0.0;   // per-lane partial of f (base) or of f(S') - f(s)
        // ---- layers 2..K on the matrix cores ----
        for (int k = 2; k <= K; ++k) {
            const Rect Rk = rect_k(full, x0, y0, w0, h0, k, L);
            const Rect Wk = rect_k(full, x0, y0, w0, h0, k + 1, L);
            const int npos = Rk.ex * Rk.ey;
            const int ntiles = (npos + 15) >> 4;
            // weights of this layer: A operands [KS][NH][64 lanes]
            bf16x8 wa[S::KS][S::NH];
            const bf16x8 *wl = prm.wa + (int64_t)(k - 2) * S::KS * S::NH * 64;
#pragma unroll
            for (int j = 0; j < S::KS; ++j)
#pragma unroll
                for (int hh = 0; hh < S::NH; ++hh) wa[j][hh] = wl[(j * S::NH + hh) * 64 + lane];
            float bias[S::NH][4];
#pragma unroll
            for (int hh = 0; hh < S::NH; ++hh)
#pragma unroll
                for (int r = 0; r < 4; ++r) bias[hh][r] = prm.bias[(k - 1) * C + 16 * hh + 4 * g + r];

            floatx4 acc[MAXT][S::NH];
            int tgx[MAXT], tgy[MAXT];
#pragma unroll
            for (int ti = 0; ti < MAXT; ++ti) {
                const int tile = wave + ti * NW;
#pragma unroll
                for (int hh = 0; hh < S::NH; ++hh)
                    for (int r = 0; r < 4; ++r) acc[ti][hh][r] = bias[hh][r];
                tgx[ti] = -1;
                tgy[ti] = -1;
                if (tile >= ntiles) continue;
                int p = tile * 16 + n16;
                const bool valid = p < npos;
                if (!valid) p = npos - 1;     // compute a duplicate, never stored
                const int u = p % Rk.ex, v = p / Rk.ex;
                const int gx = (Rk.ox + u) % L, gy = (Rk.oy + v) % L;
                if (valid) {
                    tgx[ti] = gx;
                    tgy[ti] = gy;
                }
                // window rows / columns of the three taps in each direction
                int wr[3], wc[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    wr[d] = wrapm(gy + d - 1 - Wk.oy, L) * Wk.ex;
                    wc[d] = wrapm(gx + d - 1 - Wk.ox, L);
                }
#pragma unroll
                for (int j = 0; j < S::KS; ++j) {
                    int tap, chunk;
                    mf::kstep_tap<C>(j, g, &tap, &chunk);
                    const int wi = wr[tap / 3] + wc[tap % 3];
                    const bf16x8 bv = *(const bf16x8 *)(lds + wi * S::PSB + chunk * 16);
#pragma unroll
                    for (int hh = 0; hh < S::NH; ++hh)
                        acc[ti][hh] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j][hh], bv,
                                                                             acc[ti][hh], 0, 0, 0);
                }
            }

            if (k < K) {
                // activations of layer k: ln cosh, BF16, written into the next
                // window W_{k+1} = R_{k+2} (and into the cache in the base pass)
                // once every wave has finished reading window W_k
                const Rect Wn = rect_k(full, x0, y0, w0, h0, k + 2, L);
                __syncthreads();
#pragma unroll
                for (int ti = 0; ti < MAXT; ++ti) {
                    if (tgx[ti] < 0) continue;
                    uint16_t hb[S::CG];
#pragma unroll
                    for (int hh = 0; hh < S::NH; ++hh)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            hb[hh * 4 + r] = mf::to_bf16(mf::ln_cosh(acc[ti][hh][r]));
                    const int wi = win_index(Wn, tgx[ti], tgy[ti], L);
                    uint16_t *dst = (uint16_t *)(lds + wi * S::PSB) + g * S::CG;
#pragma unroll
                    for (int r = 0; r < S::CG; ++r) dst[r] = hb[r];
                    if (base) {
                        uint16_t *cd = prm.cache_out +
                                       (((int64_t)s * (K - 1) + (k - 1)) * N + tgy[ti] * L + tgx[ti]) * C +
                                       g * S::CG;
#pragma unroll
                        for (int r = 0; r < S::CG; ++r) cd[r] = hb[r];
                    }
                }
                if (!full) {
                    const int nw = Wn.ex * Wn.ey;
                    for (int q = tid; q < nw * 4; q += NW * 64) {
                        const int p = q >> 2, gg = q & 3;
                        const int gx = (Wn.ox + p % Wn.ex) % L, gy = (Wn.oy + p / Wn.ex) % L;
                        if (in_rect(Rk, gx, gy, L)) continue;
                        const uint16_t *src =
                            prm.cache_in + (((int64_t)s * (K - 1) + (k - 1)) * N + gy * L + gx) * C +
                            gg * S::CG;
                        uint16_t *dst = (uint16_t *)(lds + p * S::PSB) + gg * S::CG;
#pragma unroll
                        for (int r = 0; r < S::CG; ++r) dst[r] = src[r];
                    }
                }
                __syncthreads();
            } else {
                // last layer: per-site FP64 channel sums
#pragma unroll
                for (int ti = 0; ti < MAXT; ++ti) {
                    double part = 0.0;
#pragma unroll
                    for (int hh = 0; hh < S::NH; ++hh)
#pragma unroll
                        for (int r = 0; r < 4; ++r) part += (double)mf::ln_cosh(acc[ti][hh][r]);
                    part += __shfl_xor(part, 16);
                    part += __shfl_xor(part, 32);
                    if (g == 0 && tgx[ti] >= 0) {
                        const int site = tgy[ti] * L + tgx[ti];
                        if (base) {
                            prm.hsum_out[(int64_t)s * N + site] = part;
                            fsum += part;
                        } else {
                            fsum += part - prm.hsum_in[(int64_t)s * N + site];
                        }
                    }
                }
            }
        }

        // ---- work-item reduction (fixed order) ----
        for (int off = 32; off > 0; off >>= 1) fsum += __shfl_xor(fsum, off);
        if (lane == 0) red[wave] = fsum;
        __syncthreads();
        if (tid == 0) {
            double v = 0.0;
            for (int w = 0; w < NW; ++w) v += red[w];
            if (!isfinite(v)) atomicOr(prm.err, kErrNonFinite);
            if (base)
                prm.f_out[s] = v;
            else
                prm.dlog[unit] = v;
        }
        __syncthreads();
    }
}

struct Variant {
    int nw, maxt;
};

const Variant kVariants[] = {{4, 2}, {4, 4}, {4, 6}, {8, 6}, {8, 11}};

// Smallest (waves, tiles-per-wave) variant that covers the largest layer; for
// the full-recompute exchanged-configuration pass (tuned = true) the
// autotuner's choice when it has made one and it fits.
bool pick_variant(const nqs_ctx *c, bool full, Variant *v, size_t *lds, bool tuned = false)
{
    const int L = c->L, K = c->K;
    int max_pos = 0, max_win = 0;
    for (int k = 1; k <= K + 1; ++k) {
        const int ex = full ? L : std::min(2 + 2 * k, L);
        const int area = ex * ex;
        if (k <= K) max_pos = std::max(max_pos, area);
        max_win = std::max(max_win, area);
    }
    if (full) max_win = L * L;
    const int tiles = (max_pos + 15) / 16;
    if (tuned && c->full_nw > 0) {
        for (const Variant &t : kVariants)
            if (t.nw == c->full_nw && t.maxt == c->full_maxt && t.nw * t.maxt >= tiles) {
                *v = t;
                *lds = (size_t)max_win * c->C * 2;
                if (*lds <= 160 * 1024 - 1024) return true;
            }
    }
    for (const Variant &t : kVariants) {
        if (t.nw * t.maxt >= tiles) {
            *v = t;
            *lds = (size_t)max_win * c->C * 2;
            return *lds <= 160 * 1024 - 1024;
        }
    }
    return false;
}

template <int C>
void launch_variant(const Variant &v, dim3 grid, size_t lds, const NetJobs &p, hipStream_t s)
{
#define NQS_NET(NW, MT)                                                                      \
    if (v.nw == NW && v.maxt == MT) {                                                        \
        hipFuncSetAttribute((const void *)k_net<C, NW, MT>,                                  \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);           \
        NQS_LAUNCH((k_net<C, NW, MT>), grid, dim3(NW * 64), lds, s, p);              \
        return;                                                                              \
    }
    NQS_NET(4, 2)
    NQS_NET(4, 4)
    NQS_NET(4, 6)
    NQS_NET(8, 6)
    NQS_NET(8, 11)
#undef NQS_NET
}

// One launch over jobs [0, n): the variant (waves, tiles per wave, LDS) is the
// one of the largest lattice, which covers the smaller ones.
void launch(const nqs_ctx *const *ctxs, int n, bool full, dim3 grid, const NetJobs &p,
            hipStream_t s)
{
    int big = 0;
    for (int i = 1; i < n; ++i)
        if (ctxs[i]->L > ctxs[big]->L) big = i;
    Variant v;
    size_t lds;
    if (!pick_variant(ctxs[big], full, &v, &lds, n == 1 && full)) return;
    if (ctxs[big]->C == 32)
        launch_variant<32>(v, grid, lds, p, s);
    else
        launch_variant<16>(v, grid, lds, p, s);
}

void launch(const nqs_ctx *c, bool full, dim3 grid, const Params &p, hipStream_t s)
{
    NetJobs jp{};
    jp.job[0] = p;
    jp.n = 1;
    launch(&c, 1, full, grid, jp, s);
}

Params common(const nqs_ctx *c, const int8_t *spins, int mode)
{
    Params p{};
    p.spins = spins;
    p.L = c->L;
    p.K = c->K;
    p.mode = mode;
    p.wa = (const bf16x8 *)c->w_mfma;
    p.w1 = c->w_l1;
    p.bias = c->w_l1 + 9 * c->C;
    p.err = c->err;
    return p;
}

}  // namespace

int mfma_full_variants(const nqs_ctx *c, int *nw, int *maxt, int cap)
{
    // every variant at least as large as the smallest that fits (same LDS)
    Variant d;
    size_t lds;
    if (!pick_variant(c, true, &d, &lds)) return 0;
    int n = 0;
    for (const Variant &t : kVariants)
        if (n < cap && t.nw * t.maxt >= d.nw * d.maxt) {
            nw[n] = t.nw;
            maxt[n] = t.maxt;
            ++n;
        }
    return n;
}

bool mfma_supported(const nqs_ctx *c)
{
    if (!(c->C == 16 || c->C == 32) || c->K < 2) return false;
    Variant v;
    size_t lds;
    return pick_variant(c, true, &v, &lds);
}

bool mfma_inc_supported(const nqs_ctx *c)
{
    // anchor offsets must stay within one period of the torus
    return mfma_supported(c) && c->L >= c->K + 2 && 2 * mfma_inc_lds_bytes(c) <= 160 * 1024 - 1024;
}

int mfma_lds_full_ok(const nqs_ctx *c)
{
    Variant v;
    size_t lds;
    return pick_variant(c, true, &v, &lds) ? 1 : 0;
}

size_t mfma_cache_bytes(const nqs_ctx *c, int64_t B)
{
    return (size_t)B * (c->K - 1) * c->N * c->C * 2;
}

void mfma_base_forward(const nqs_ctx *c, const int8_t *spins, int B, double *f, double *hsum,
                       void *cache, hipStream_t s)
{
    if (B <= 0) return;
    Params p = common(c, spins, kBase);
    p.B = B;
    p.cache_out = (uint16_t *)cache;
    p.hsum_out = hsum;
    p.f_out = f;
    const int grid = std::min(B, c->n_cu * 2);
    launch(c, true, dim3(grid), p, s);
}

void mfma_conn_forward_jobs(nqs_mode mode, const ConnJob *jobs, int n, hipStream_t s)
{
    if (n <= 0) return;
    if (mode == NQS_INCREMENTAL) {
        // lattices the unwrapped-window kernel serves share one launch of it;
        // the others (wrapped windows, 16 channels) one launch of the general
        // kernel: each lattice runs exactly as in its single-lattice call
        ConnJob cone[kMaxConnJobs], rest[kMaxConnJobs];
        int nc = 0, nr = 0;
        for (int i = 0; i < n; ++i) {
            if (cone_supported(jobs[i].c))
                cone[nc++] = jobs[i];
            else
                rest[nr++] = jobs[i];
        }
        if (nc > 0) cone_forward_jobs(cone, nc, s);
        if (nr > 0) mfma_inc_forward_jobs(rest, nr, s);
        return;
    }
    NetJobs jp{};
    jp.n = n;
    const nqs_ctx *ctxs[kMaxConnJobs];
    int64_t total_cap = 0;
    for (int i = 0; i < n; ++i) {
        ctxs[i] = jobs[i].c;
        Params &p = jp.job[i];
        p = common(jobs[i].c, jobs[i].spins, kFull);
        p.queue = jobs[i].queue;
        p.qlen = jobs[i].qlen;
        p.capacity = jobs[i].capacity;
        p.cache_in = (const uint16_t *)jobs[i].cache;
        p.hsum_in = jobs[i].hsum;
        p.dlog = jobs[i].dlog;
        total_cap += jobs[i].capacity;
    }
    if (total_cap <= 0) return;
    const int64_t want = std::min<int64_t>(total_cap, (int64_t)jobs[0].c->n_cu * 2);
    launch(ctxs, n, true, dim3((unsigned)want), jp, s);
}

void mfma_conn_forward(const nqs_ctx *c, nqs_mode mode, const int8_t *spins,
                       const uint32_t *queue, const int64_t *qlen, int64_t capacity,
                       const double *hsum, const void *cache, double *dlog, int *counter,
                       hipStream_t s)
{
    (void)counter;
    if (capacity <= 0) return;
    const ConnJob j{c, spins, queue, qlen, capacity, hsum, cache, dlog};
    mfma_conn_forward_jobs(mode, &j, 1, s);
}

}  // namespace nqs
