// k_conv_f64mma.hip -- FP64 matrix-core (v_mfma_f64_16x16x4f64) forms of the
// vector path's convolution layer (layers 2..K) and of the per-sample weight
// gradient, for channel counts 16 and 32.  Arithmetic stays FP64 end to end:
// every output element is an FP64 fused multiply-add chain.  They serve the
// plain FP64 network (base and exchanged configurations alike, so the two
// sides of a log-ratio still run identical arithmetic), the forward pass that
// saves tanh of the pre-activations, the backward data pass, and the weight gradients
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


struct ConvArgs {
    const double *in;        // [M][N][Cin]
    const double *w;         // [9][Cin][Cout]
    const double *bias;      // [Cout] or null
    double *out;             // [M][N][Cout]
    double *zk;              // epi 1: saved tanh z [M][N][Cout]; epi 2: tanh z_{k-1}; MODE 1, 3: z
    const int64_t *qlen;     // exchanged-configuration queue length (null: all M live)
    int64_t q_begin;
    int64_t M;
    int L, Cin, epi;
};

// out[m][p][co] = epi(bias[co] + sum_{t, ci} W[t][ci][co] in[m][p + off(t)][ci])
// for 64 sites x COUT channels per wave.  GEMM: M = sites, N = co, K = (t, ci)
// in steps of 4; within a 16-channel block, lane group kq at sub-step s takes
// channel 4 kq + s, so each lane reads 4 consecutive channels of a site.
// epi 0: ln cosh; 1: ln cosh and save tanh z in zk; 2: z * zk (backward data
// pass, zk the saved tanh); 3: tanh z (the last layer's delta).
// MODE 1 (CNN1 convolution, COUT = 32): column 16 h + j holds z[2 j + h], so
// one lane holds both inputs of a channel-pair max: out [M][N][16] gets
// max(z[2j], z[2j+1]) (the second only when larger), zk (may be null) the z
// in natural channel order [M][N][32].  MODE 2 (transposed convolutions,
// data gradients): out = z, no activation.  MODE 3 (CNN2 convolution): out
// [M][N][COUT] gets m[c] = max(z[c], z[(c+1) mod COUT]) (the second only
// when larger), zk (may be null) the z; channel c+1 sits in the next lane of
// the same 16-lane row group, or for c = 16 h + 15 in lane 0 of the group
// and the next 16-column tile.
template <int COUT, int MODE, int CIN>
__global__ void __launch_bounds__(kThreads)
k_conv_mma(ConvArgs a)
{
    constexpr int NH = COUT / 16;
    constexpr int NCB = CIN / 16;               // 16-channel K-blocks per tap
    constexpr int NSTEP = 9 * NCB;
    const int L = a.L, N = L * L;
    const int lane = threadIdx.x & 63;
    const int m16 = lane & 15, kq = lane >> 4;
    const int64_t wave_id = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    int64_t live = a.M;
    if (a.qlen) {
        const int64_t left = a.qlen[0] - a.q_begin;
        live = left < 0 ? 0 : (left < a.M ? left : a.M);
    }
    // The planes' sites form one index space g = plane * N + p, tiled in runs
    // of 16 kMT that may span two planes, so no lattice size leaves part of a
    // tile idle; planes are contiguous, so element (g, c) of any [M][N][X]
    // array sits at g X + c.
    const int64_t total = live * N;
    const int64_t g0 = wave_id * 16 * kMT;
    if (g0 >= total) return;
    const double *inr[kMT];          // this lane's A-row plane
    int sx[kMT], sy[kMT];
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt) {
        int64_t g = g0 + mt * 16 + m16;
        if (g >= total) g = total - 1;
        const int64_t pl = g / N;
        const int p = (int)(g - pl * N);
        inr[mt] = a.in + pl * (int64_t)N * CIN;
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
    // operands of K-block kb (tap t = kb / NCB, channels c0 .. c0 + 15): this
    // lane's 4 consecutive input channels at each of its kMT sites, and the
    // 4 x NH weights of its column
    auto fetch = [&](int kb, double (&av)[kMT][4], double (&bv)[4][NH]) {
        const int t = kb / NCB, c0 = (kb - t * NCB) * 16;
        const int dy = t / 3 - 1, dx = t % 3 - 1;
        const int cb = c0 + 4 * kq;
#pragma unroll
        for (int mt = 0; mt < kMT; ++mt) {
            const int site = wrapi(sy[mt] + dy, L) * L + wrapi(sx[mt] + dx, L);
            const double2 *src = reinterpret_cast<const double2 *>(inr[mt] + (int64_t)site * CIN + cb);
            const double2 u = src[0], v = src[1];
            av[mt][0] = u.x;
            av[mt][1] = u.y;
            av[mt][2] = v.x;
            av[mt][3] = v.y;
        }
        const double *wt = a.w + ((int64_t)t * CIN + cb) * COUT + m16;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int h = 0; h < NH; ++h) bv[s][h] = wt[s * COUT + 16 * h];
    };
    auto mma = [&](const double (&av)[kMT][4], const double (&bv)[4][NH]) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
                for (int h = 0; h < NH; ++h)
                    acc[mt][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt][s], bv[s][h],
                                                                      acc[mt][h], 0, 0, 0);
    };
    // (fetching the next K-block's operands before this one's MFMAs, in
    // registers, measured no faster: three waves per SIMD hide the latency)
    for (int kb = 0; kb < NSTEP; ++kb) {
        double av[kMT][4], bv[4][NH];
        fetch(kb, av, bv);
        mma(av, bv);
    }
    // D element i of tile mt in this lane: site g0 + 16 mt + kq + 4 i, column
    // 16 h + m16
    if constexpr (MODE == 1) {
        static_assert(COUT == 32, "channel pairs span the two 16-column tiles");
#pragma unroll
        for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t g = g0 + mt * 16 + kq + 4 * i;
                if (g >= total) continue;
                const double z0 = acc[mt][0][i], z1 = acc[mt][1][i];
                a.out[g * 16 + m16] = (z1 > z0) ? z1 : z0;
                if (a.zk) {
                    a.zk[g * 32 + 2 * m16] = z0;
                    a.zk[g * 32 + 2 * m16 + 1] = z1;
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
                const int64_t g = g0 + mt * 16 + kq + 4 * i;   // same row in lane_next
                double nb[NH];
#pragma unroll
                for (int h = 0; h < NH; ++h) nb[h] = __shfl(acc[mt][h][i], lane_next, 64);
                if (g >= total) continue;
#pragma unroll
                for (int h = 0; h < NH; ++h) {
                    const double z0 = acc[mt][h][i];
                    const double z1 = m16 < 15 ? nb[h] : nb[(h + 1) % NH];
                    const int64_t o = g * COUT + 16 * h + m16;
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
                const int64_t g = g0 + mt * 16 + kq + 4 * i;
                if (g >= total) continue;
#pragma unroll
                for (int h = 0; h < NH; ++h) a.out[g * COUT + 16 * h + m16] = acc[mt][h][i];
            }
        return;
    }
    if (a.epi == 2) {
        // backward data pass: z times the saved tanh of the layer below
#pragma unroll
        for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t g = g0 + mt * 16 + kq + 4 * i;
                if (g >= total) continue;
#pragma unroll
                for (int h = 0; h < NH; ++h) {
                    const int64_t o = g * COUT + 16 * h + m16;
                    a.out[o] = acc[mt][h][i] * a.zk[o];
                }
            }
        return;
    }
    // The transcendental epilogues run in two phases: z leaves the
    // accumulators first, then each element is re-read (by the lane that
    // wrote it) and transformed in a rolled loop, so no accumulator is live
    // across the math library's code.
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t g = g0 + mt * 16 + kq + 4 * i;
            if (g >= total) continue;
#pragma unroll
            for (int h = 0; h < NH; ++h) a.out[g * COUT + 16 * h + m16] = acc[mt][h][i];
        }
#pragma unroll 1
    for (int e = 0; e < kMT * 4 * NH; ++e) {
        const int mt = e / (4 * NH), i = (e / NH) % 4, h = e % NH;
        const int64_t g = g0 + mt * 16 + kq + 4 * i;
        if (g >= total) continue;
        const int64_t o = g * COUT + 16 * h + m16;
        const double z = a.out[o];
        if (a.epi == 3) {
            a.out[o] = tanh(z);
        } else if (a.epi == 1) {
            double th;
            a.out[o] = ln_cosh_tanh(z, &th);
            a.zk[o] = th;
        } else {
            a.out[o] = ln_cosh_fwd(z);
        }
    }
}

// Weight and bias gradients of one layer with C input and output channels,
// per sample:  dW[co][ci][t] = sum_p delta[p][co] h[p + off(t)][ci],
//              db[co] = sum_p delta[p][co].
// GEMM over sites: M = co (C), N = (t, ci) (9C columns, ci fastest, so a
// 16-column tile never straddles two taps), K = sites in steps of 4.  A
// column group of kNT consecutive 16-column tiles of one sample is shared by
// two waves of a workgroup, one per half of the site range; the second half's
// partial sums pass through LDS and the first adds them (lo + hi, a fixed
// order), so rows stay deterministic.  A workgroup holds two column groups
// (one idle pair when a sample has an odd number of groups).
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
    constexpr int WPS = (NTILE + kNT - 1) / kNT;   // column groups per sample
    constexpr int GPS = (WPS + 1) / 2;             // workgroups per sample
    constexpr int NRED = NH * kNT * 4 + NH;        // partials per lane
    __shared__ double red[2][NRED][64];
    const int N = L * L;
    const int lane = threadIdx.x & 63;
    const int m16 = lane & 15, kq = lane >> 4;
    const int w = threadIdx.x >> 6, cgl = w >> 1, kh = w & 1;
    const int64_t s = blockIdx.x / GPS;            // the grid holds B * GPS workgroups
    const int wg = (int)(blockIdx.x - s * GPS) * 2 + cgl;
    const bool active = wg < WPS;
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
    // this wave's half of the sites, [pb, pe), both multiples of 4 (N is)
    const int mid = (N / 2) & ~3;
    const int pb = kh ? mid : 0, pe = kh ? N : mid;
    if (active && pb < pe) {
        const int y0 = (pb + kq) / L, x0 = (pb + kq) - ((pb + kq) / L) * L;
        int y = y0, x = x0;                    // site of position p0 + kq
        double av[NH], bv[kNT];
        fetch(pb + kq, y, x, av, bv);
        // the operands of step p0 + 4 are fetched while the matrix cores work
        // on p0 (the last step fetches the first step's again, unused, so that
        // the loop has no branch)
        for (int p0 = pb; p0 < pe; p0 += 4) {
            int xn = x + 4, yn = y;            // L >= 4: at most one row end
            if (xn >= L) {
                xn -= L;
                ++yn;
            }
            const bool more = p0 + 4 < pe;
            double an[NH], bn[kNT];
            fetch(more ? p0 + 4 + kq : pb + kq, more ? yn : y0, more ? xn : x0, an, bn);
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
    }
    // the second half hands its partial sums to the first
    if (kh == 1) {
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int j = 0; j < kNT; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i) red[cgl][(h * kNT + j) * 4 + i][lane] = acc[h][j][i];
#pragma unroll
        for (int h = 0; h < NH; ++h) red[cgl][NH * kNT * 4 + h][lane] = dbp[h];
    }
    __syncthreads();
    if (kh == 1 || !active) return;
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int j = 0; j < kNT; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[h][j][i] += red[cgl][(h * kNT + j) * 4 + i][lane];
#pragma unroll
    for (int h = 0; h < NH; ++h) dbp[h] += red[cgl][NH * kNT * 4 + h][lane];
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

// one launch of k_conv_mma<COUT, MODE, Cin> over M planes
template <int COUT, int MODE>
void conv_launch(const nqs_ctx *c, const ConvArgs &a, hipStream_t s)
{
    const int64_t tiles = (a.M * c->N + 16 * kMT - 1) / (16 * kMT);
    const int64_t blocks = (tiles + kThreads / 64 - 1) / (kThreads / 64);
    if (a.Cin == 32)
        NQS_LAUNCH((k_conv_mma<COUT, MODE, 32>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
    else
        NQS_LAUNCH((k_conv_mma<COUT, MODE, 16>), dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
}

void f64mma_conv(const nqs_ctx *c, const double *in, int64_t M, int Cin, int Cout,
                 const double *w, const double *bias, double *out, int epi, double *zk,
                 const int64_t *qlen, int64_t q_begin, hipStream_t s)
{
    if (M <= 0) return;
    ConvArgs a{in, w, bias, out, zk, qlen, q_begin, M, c->L, Cin, epi};
    if (Cout == 32)
        conv_launch<32, 0>(c, a, s);
    else
        conv_launch<16, 0>(c, a, s);
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
    conv_launch<32, 1>(c, a, s);
}

void f64mma_cnn1_convt(const nqs_ctx *c, const double *in, int64_t M, const double *w,
                       const double *bias, double *out, const int64_t *qlen, int64_t q_begin,
                       hipStream_t s)
{
    if (M <= 0) return;
    ConvArgs a{in, w, bias, out, nullptr, qlen, q_begin, M, c->L, 16, 0};
    conv_launch<16, 2>(c, a, s);
}

// plain convolution Cin (16 or 32) -> 16 with no bias and no activation
// (the data gradients of the CNN1 backward)
void f64mma_cnn1_plain(const nqs_ctx *c, const double *in, int64_t M, int Cin, const double *w,
                       double *out, hipStream_t s)
{
    if (M <= 0) return;
    ConvArgs a{in, w, nullptr, out, nullptr, nullptr, 0, M, c->L, Cin, 0};
    conv_launch<16, 2>(c, a, s);
}

// CNN2 convolution C -> C with the stride-one channel max in the epilogue
// (MODE 3): m into out, z into zsave (may be null)
void f64mma_cnn2_conv(const nqs_ctx *c, const double *in, int64_t M, const double *w,
                      const double *bias, double *out, double *zsave, const int64_t *qlen,
                      int64_t q_begin, hipStream_t s)
{
    if (M <= 0) return;
    ConvArgs a{in, w, bias, out, zsave, qlen, q_begin, M, c->L, c->C, 0};
    if (c->C == 32)
        conv_launch<32, 3>(c, a, s);
    else
        conv_launch<16, 3>(c, a, s);
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
    if (Cout == 32)
        conv_launch<32, 2>(c, a, s);
    else
        conv_launch<16, 2>(c, a, s);
}

bool f64mma_wgrad_ok(int C) { return C == 16 || C == 32; }

namespace {
template <bool TRANS>
void wgrad_launch(const nqs_ctx *c, const double *hin, const double *delta, int B, int64_t woff,
                  void *O, nqs_dtype odt, hipStream_t s)
{
    const int C = c->C;
    const int wps = (9 * C / 16 + kNT - 1) / kNT;            // column groups per sample
    const int64_t blocks = (int64_t)B * ((wps + 1) / 2);       // two groups per workgroup
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
