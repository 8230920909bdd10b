// k_conv_f64mma.hip -- FP64 matrix-core (v_mfma_f64_16x16x4f64) forms of the
// vector path's convolution layer (layers 2..K) and of the per-sample weight
// gradient, for channel counts 16 and 32.  Arithmetic stays FP64 end to end:
// every output element is an FP64 fused multiply-add chain.  They serve the
// plain FP64 network (base and exchanged configurations alike, so the two
// sides of a log-ratio still run identical arithmetic), the forward pass that
// saves pre-activations, the backward data pass, and the weight gradients
// that form the rows of O [Sec. 3.2].
//
// Operand layout of v_mfma_f64_16x16x4f64 (64 lanes, lane l):
//   A[m][k]: m = l % 16, k = l / 16;  B[k][n]: k = l / 16, n = l % 16;
//   D[m][n] (4 doubles): m = l / 16 + 4 i, n = l % 16.
#include <algorithm>

#include "nqs_internal.h"

namespace nqs {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kMT = 4;            // 16-site M-tiles per wave (64 sites)
constexpr int kNT = 3;            // 16-column N-tiles per weight-gradient wave

__device__ inline int wrapi(int a, int L) { return a < 0 ? a + L : (a >= L ? a - L : a); }

// ln cosh z in FP64, the same form as the vector-ALU layers: expm1/log1p
// below |z| = 1, |z| - ln 2 + log1p(exp(-2|z|)) above.
__device__ inline double ln_cosh_d(double z)
{
    const double a = fabs(z);
    if (a > 1.0) return a - 0.69314718055994530942 + log1p(exp(-2.0 * a));
    const double e = expm1(a);
    return log1p(e * e / (2.0 + 2.0 * e));
}

struct ConvArgs {
    const double *in;        // [M][N][Cin]
    const double *w;         // [9][Cin][Cout]
    const double *bias;      // [Cout] or null
    double *out;             // [M][N][Cout]
    double *zk;              // epi 1: saved z [M][N][Cout]; epi 2: z_{k-1} for tanh
    const int64_t *qlen;     // exchanged-configuration queue length (null: all M live)
    int64_t q_begin;
    int64_t M;
    int L, Cin, epi;
};

// out[m][p][co] = epi(bias[co] + sum_{t, ci} W[t][ci][co] in[m][p + off(t)][ci])
// for 64 sites x COUT channels per wave.  GEMM: M = sites, N = co, K = (t, ci)
// in steps of 4; within a 16-channel block, lane group kq at sub-step s takes
// channel 4 kq + s, so each lane reads 4 consecutive channels of a site.
// epi 0: ln cosh; 1: ln cosh and save z; 2: z * tanh(zk) (backward data pass);
// 3: tanh z (the last layer's delta).
// MODE 1 (CNN1 convolution, COUT = 32): column 16 h + j holds z[2 j + h], so
// one lane holds both inputs of a channel-pair max: out [M][N][16] gets
// max(z[2j], z[2j+1]) (the second only when larger), zk (may be null) the z
// in natural channel order [M][N][32].  MODE 2 (transposed convolutions,
// data gradients): out = z, no activation.  MODE 3 (CNN2 convolution): out
// [M][N][COUT] gets m[c] = max(z[c], z[(c+1) mod COUT]) (the second only
// when larger), zk (may be null) the z; channel c+1 sits in the next lane of
// the same 16-lane row group, or for c = 16 h + 15 in lane 0 of the group
// and the next 16-column tile.
template <int COUT, int MODE = 0>
__global__ void __launch_bounds__(kThreads)
k_conv_mma(ConvArgs a)
{
    constexpr int NH = COUT / 16;
    const int L = a.L, N = L * L, Cin = a.Cin;
    const int lane = threadIdx.x & 63;
    const int m16 = lane & 15, kq = lane >> 4;
    const int ntile = (N + 16 * kMT - 1) / (16 * kMT);
    const int64_t wave_id = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    int64_t live = a.M;
    if (a.qlen) {
        const int64_t left = a.qlen[0] - a.q_begin;
        live = left < 0 ? 0 : (left < a.M ? left : a.M);
    }
    const int64_t plane = wave_id / ntile;
    if (plane >= live) return;
    const int p0 = (int)(wave_id - plane * ntile) * 16 * kMT;
    const double *inp = a.in + plane * (int64_t)N * Cin;

    int sx[kMT], sy[kMT];
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt) {
        int p = p0 + mt * 16 + m16;
        if (p >= N) p = N - 1;
        sy[mt] = p / L;
        sx[mt] = p - sy[mt] * L;
    }
    double4_t acc[kMT][NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
        const double b = a.bias ? a.bias[16 * h + m16] : 0.0;
#pragma unroll
        for (int mt = 0; mt < kMT; ++mt) acc[mt][h] = (double4_t){b, b, b, b};
    }
    for (int t = 0; t < 9; ++t) {
        const int dy = t / 3 - 1, dx = t % 3 - 1;
        int site[kMT];
#pragma unroll
        for (int mt = 0; mt < kMT; ++mt)
            site[mt] = wrapi(sy[mt] + dy, L) * L + wrapi(sx[mt] + dx, L);
        const double *wt = a.w + (int64_t)t * Cin * COUT;
        for (int c0 = 0; c0 < Cin; c0 += 16) {
            const int cb = c0 + 4 * kq;
            double av[kMT][4], bv[4][NH];
#pragma unroll
            for (int mt = 0; mt < kMT; ++mt) {
                const double2 *src = reinterpret_cast<const double2 *>(inp + (int64_t)site[mt] * Cin + cb);
                const double2 u = src[0], v = src[1];
                av[mt][0] = u.x;
                av[mt][1] = u.y;
                av[mt][2] = v.x;
                av[mt][3] = v.y;
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int h = 0; h < NH; ++h) bv[s][h] = wt[(int64_t)(cb + s) * COUT + 16 * h + m16];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
                    for (int h = 0; h < NH; ++h)
                        acc[mt][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt][s], bv[s][h],
                                                                          acc[mt][h], 0, 0, 0);
        }
    }
    const int64_t obase = plane * (int64_t)N * COUT;
    if constexpr (MODE == 1) {
        static_assert(COUT == 32, "channel pairs span the two 16-column tiles");
#pragma unroll
        for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = p0 + mt * 16 + kq + 4 * i;
                if (p >= N) continue;
                const double z0 = acc[mt][0][i], z1 = acc[mt][1][i];
                a.out[plane * (int64_t)N * 16 + (int64_t)p * 16 + m16] = (z1 > z0) ? z1 : z0;
                if (a.zk) {
                    a.zk[obase + (int64_t)p * 32 + 2 * m16] = z0;
                    a.zk[obase + (int64_t)p * 32 + 2 * m16 + 1] = z1;
                }
            }
        return;
    }
    if constexpr (MODE == 3) {
        const int lane_next = (lane & ~15) | ((m16 + 1) & 15);
#pragma unroll
        for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = p0 + mt * 16 + kq + 4 * i;   // same row in lane_next
                double nb[NH];
#pragma unroll
                for (int h = 0; h < NH; ++h) nb[h] = __shfl(acc[mt][h][i], lane_next, 64);
                if (p >= N) continue;
#pragma unroll
                for (int h = 0; h < NH; ++h) {
                    const double z0 = acc[mt][h][i];
                    const double z1 = m16 < 15 ? nb[h] : nb[(h + 1) % NH];
                    const int64_t o = obase + (int64_t)p * COUT + 16 * h + m16;
                    a.out[o] = (z1 > z0) ? z1 : z0;
                    if (a.zk) a.zk[o] = z0;
                }
            }
        return;
    }
    if constexpr (MODE == 2) {
#pragma unroll
        for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = p0 + mt * 16 + kq + 4 * i;
                if (p >= N) continue;
#pragma unroll
                for (int h = 0; h < NH; ++h)
                    a.out[obase + (int64_t)p * COUT + 16 * h + m16] = acc[mt][h][i];
            }
        return;
    }
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int p = p0 + mt * 16 + kq + 4 * i;
            if (p >= N) continue;
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                const int64_t o = obase + (int64_t)p * COUT + 16 * h + m16;
                const double z = acc[mt][h][i];
                if (a.epi >= 2) {
                    // one tanh call site: epi 3 writes tanh z, epi 2 z tanh(zk)
                    const double th = tanh(a.epi == 3 ? z : a.zk[o]);
                    a.out[o] = a.epi == 3 ? th : z * th;
                } else {
                    if (a.epi == 1) a.zk[o] = z;
                    a.out[o] = ln_cosh_d(z);
                }
            }
        }
}

// Weight and bias gradients of one layer with C input and output channels,
// per sample:  dW[co][ci][t] = sum_p delta[p][co] h[p + off(t)][ci],
//              db[co] = sum_p delta[p][co].
// GEMM over sites: M = co (C), N = (t, ci) (9C columns, ci fastest, so a
// 16-column tile never straddles two taps), K = sites in steps of 4.  A wave
// owns all C output channels and kNT consecutive column tiles of one sample.
// TRANS (a transposed convolution u[co][p] = sum V[ci][co][t] h[p - off(t)][ci]):
// dV[ci][co][t] = sum_p delta[p][co] h[p - off(t)][ci], stored input channel
// first; the bias gradient as before.
template <typename OT, int C, bool TRANS = false>
__global__ void __launch_bounds__(kThreads)
k_wgrad_mma(const double *__restrict__ hin, const double *__restrict__ delta, int L, int B,
            int64_t P, int64_t woff, OT *__restrict__ O)
{
    constexpr int NH = C / 16;
    constexpr int NTILE = 9 * C / 16;
    constexpr int WPS = (NTILE + kNT - 1) / kNT;   // waves per sample
    const int N = L * L;
    const int lane = threadIdx.x & 63;
    const int m16 = lane & 15, kq = lane >> 4;
    const int64_t wave_id = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int64_t s = wave_id / WPS;
    if (s >= B) return;
    const int wg = (int)(wave_id - s * WPS);
    const double *dl = delta + s * (int64_t)N * C;
    const double *hs = hin + s * (int64_t)N * C;

    int tdy[kNT], tdx[kNT], tci[kNT];
    bool tok[kNT];
#pragma unroll
    for (int j = 0; j < kNT; ++j) {
        const int tile = wg * kNT + j;
        tok[j] = tile < NTILE;
        const int col = (tok[j] ? tile : 0) * 16;
        const int t = col / C;
        tdy[j] = TRANS ? 1 - t / 3 : t / 3 - 1;
        tdx[j] = TRANS ? 1 - t % 3 : t % 3 - 1;
        tci[j] = col % C + m16;
    }
    double4_t acc[NH][kNT];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int j = 0; j < kNT; ++j) acc[h][j] = (double4_t){0, 0, 0, 0};
    double dbp[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) dbp[h] = 0.0;

    // operands of K-step p0 (sites p0 .. p0 + 3; this lane's site p = p0 + kq
    // at (y, x)); a column tile past the last one reads tile 0's column and
    // is never stored
    auto fetch = [&](int p, int y, int x, double (&av)[NH], double (&bv)[kNT]) {
#pragma unroll
        for (int h = 0; h < NH; ++h) av[h] = dl[(int64_t)p * C + 16 * h + m16];
#pragma unroll
        for (int j = 0; j < kNT; ++j) {
            const int r = wrapi(y + tdy[j], L) * L + wrapi(x + tdx[j], L);
            bv[j] = hs[(int64_t)r * C + tci[j]];
        }
    };
    const int y0 = kq / L, x0 = kq - (kq / L) * L;
    int y = y0, x = x0;                        // site of position p0 + kq
    double av[NH], bv[kNT];
    fetch(kq, y, x, av, bv);
    // the operands of step p0 + 4 are fetched while the matrix cores work on
    // p0 (the last step fetches step 0's again, unused, so that the loop has
    // no branch)
    for (int p0 = 0; p0 < N; p0 += 4) {
        int xn = x + 4, yn = y;                // L >= 4: at most one row end
        if (xn >= L) {
            xn -= L;
            ++yn;
        }
        const bool more = p0 + 4 < N;
        double an[NH], bn[kNT];
        fetch(more ? p0 + 4 + kq : kq, more ? yn : y0, more ? xn : x0, an, bn);
#pragma unroll
        for (int h = 0; h < NH; ++h) dbp[h] += av[h];
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int j = 0; j < kNT; ++j)
                acc[h][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h], bv[j], acc[h][j], 0, 0, 0);
#pragma unroll
        for (int h = 0; h < NH; ++h) av[h] = an[h];
#pragma unroll
        for (int j = 0; j < kNT; ++j) bv[j] = bn[j];
        x = xn;
        y = yn;
    }
    OT *o = O + s * P + woff;
    // D element i of this lane: co = 16 h + kq + 4 i, column ci = tci[j]
#pragma unroll
    for (int j = 0; j < kNT; ++j) {
        if (!tok[j]) continue;
        const int t = (wg * kNT + j) * 16 / C;
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = 16 * h + kq + 4 * i;
                const int64_t idx = TRANS ? ((int64_t)tci[j] * C + co) * 9 + t
                                          : ((int64_t)co * C + tci[j]) * 9 + t;
                o[idx] = (OT)acc[h][j][i];
            }
    }
    if (wg == 0) {
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            double v = dbp[h];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (kq == 0) o[(int64_t)C * C * 9 + 16 * h + m16] = (OT)v;
        }
    }
}

}  // namespace

bool f64mma_conv_ok(int Cin, int Cout) { return (Cin == 16 || Cin == 32) && (Cout == 16 || Cout == 32); }

void f64mma_conv(const nqs_ctx *c, const double *in, int64_t M, int Cin, int Cout,
                 const double *w, const double *bias, double *out, int epi, double *zk,
                 const int64_t *qlen, int64_t q_begin, hipStream_t s)
{
    if (M <= 0) return;
    ConvArgs a{in, w, bias, out, zk, qlen, q_begin, M, c->L, Cin, epi};
    const int64_t ntile = (c->N + 16 * kMT - 1) / (16 * kMT);
    const int64_t blocks = (M * ntile + kThreads / 64 - 1) / (kThreads / 64);
    if (Cout == 32)
        NQS_LAUNCH((k_conv_mma<32>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
    else
        NQS_LAUNCH((k_conv_mma<16>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
}

// CNN1 with 16 channels: the convolution 16 -> 32 with the channel-pair max
// in the epilogue (packed columns, see MODE 1), and the transposed
// convolution 16 -> 16 as a convolution with flipped, transposed taps.
void f64mma_cnn1_conv(const nqs_ctx *c, const double *in, int64_t M, const double *w,
                      const double *bias, double *out, double *zsave, const int64_t *qlen,
                      int64_t q_begin, hipStream_t s)
{
    if (M <= 0) return;
    ConvArgs a{in, w, bias, out, zsave, qlen, q_begin, M, c->L, 16, 0};
    const int64_t ntile = (c->N + 16 * kMT - 1) / (16 * kMT);
    const int64_t blocks = (M * ntile + kThreads / 64 - 1) / (kThreads / 64);
    NQS_LAUNCH((k_conv_mma<32, 1>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
}

void f64mma_cnn1_convt(const nqs_ctx *c, const double *in, int64_t M, const double *w,
                       const double *bias, double *out, const int64_t *qlen, int64_t q_begin,
                       hipStream_t s)
{
    if (M <= 0) return;
    ConvArgs a{in, w, bias, out, nullptr, qlen, q_begin, M, c->L, 16, 0};
    const int64_t ntile = (c->N + 16 * kMT - 1) / (16 * kMT);
    const int64_t blocks = (M * ntile + kThreads / 64 - 1) / (kThreads / 64);
    NQS_LAUNCH((k_conv_mma<16, 2>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
}

// plain convolution Cin (16 or 32) -> 16 with no bias and no activation
// (the data gradients of the CNN1 backward)
void f64mma_cnn1_plain(const nqs_ctx *c, const double *in, int64_t M, int Cin, const double *w,
                       double *out, hipStream_t s)
{
    if (M <= 0) return;
    ConvArgs a{in, w, nullptr, out, nullptr, nullptr, 0, M, c->L, Cin, 0};
    const int64_t ntile = (c->N + 16 * kMT - 1) / (16 * kMT);
    const int64_t blocks = (M * ntile + kThreads / 64 - 1) / (kThreads / 64);
    NQS_LAUNCH((k_conv_mma<16, 2>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
}

// CNN2 convolution C -> C with the stride-one channel max in the epilogue
// (MODE 3): m into out, z into zsave (may be null)
void f64mma_cnn2_conv(const nqs_ctx *c, const double *in, int64_t M, const double *w,
                      const double *bias, double *out, double *zsave, const int64_t *qlen,
                      int64_t q_begin, hipStream_t s)
{
    if (M <= 0) return;
    ConvArgs a{in, w, bias, out, zsave, qlen, q_begin, M, c->L, c->C, 0};
    const int64_t ntile = (c->N + 16 * kMT - 1) / (16 * kMT);
    const int64_t blocks = (M * ntile + kThreads / 64 - 1) / (kThreads / 64);
    if (c->C == 32)
        NQS_LAUNCH((k_conv_mma<32, 3>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
    else
        NQS_LAUNCH((k_conv_mma<16, 3>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
}

// convolution Cin -> Cout (16 or 32) with an optional bias and no activation
// (MODE 2): transposed convolutions as convolutions with flipped, transposed
// taps, and the data gradients of the backward
void f64mma_linear(const nqs_ctx *c, const double *in, int64_t M, int Cin, int Cout,
                   const double *w, const double *bias, double *out, const int64_t *qlen,
                   int64_t q_begin, hipStream_t s)
{
    if (M <= 0) return;
    ConvArgs a{in, w, bias, out, nullptr, qlen, q_begin, M, c->L, Cin, 0};
    const int64_t ntile = (c->N + 16 * kMT - 1) / (16 * kMT);
    const int64_t blocks = (M * ntile + kThreads / 64 - 1) / (kThreads / 64);
    if (Cout == 32)
        NQS_LAUNCH((k_conv_mma<32, 2>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
    else
        NQS_LAUNCH((k_conv_mma<16, 2>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
}

bool f64mma_wgrad_ok(int C) { return C == 16 || C == 32; }

namespace {
template <bool TRANS>
void wgrad_launch(const nqs_ctx *c, const double *hin, const double *delta, int B, int64_t woff,
                  void *O, nqs_dtype odt, hipStream_t s)
{
    const int C = c->C;
    const int wps = (9 * C / 16 + kNT - 1) / kNT;
    const int64_t blocks = ((int64_t)B * wps + kThreads / 64 - 1) / (kThreads / 64);
    const dim3 g((unsigned)blocks), b(kThreads);
    if (C == 32) {
        if (odt == NQS_FP32)
            NQS_LAUNCH((k_wgrad_mma<float, 32, TRANS>), g, b, 0, s, hin, delta, c->L, B, c->P, woff, (float *)O);
        else
            NQS_LAUNCH((k_wgrad_mma<double, 32, TRANS>), g, b, 0, s, hin, delta, c->L, B, c->P, woff, (double *)O);
    } else {
        if (odt == NQS_FP32)
            NQS_LAUNCH((k_wgrad_mma<float, 16, TRANS>), g, b, 0, s, hin, delta, c->L, B, c->P, woff, (float *)O);
        else
            NQS_LAUNCH((k_wgrad_mma<double, 16, TRANS>), g, b, 0, s, hin, delta, c->L, B, c->P, woff, (double *)O);
    }
}
}  // namespace

void f64mma_wgrad(const nqs_ctx *c, const double *hin, const double *delta, int B, int64_t woff,
                  void *O, nqs_dtype odt, hipStream_t s, bool trans)
{
    if (B <= 0) return;
    if (trans)
        wgrad_launch<true>(c, hin, delta, B, woff, O, odt, s);
    else
        wgrad_launch<false>(c, hin, delta, B, woff, O, odt, s);
}

}  // namespace nqs
