// k_cnn1.hip -- the CNN1 network family [Sec. 5.2: blocks of a 2D
// convolution, a 1D max-pooling and a transposed convolution, padded by the
// periodic boundary; the wave-function coefficient is the product of the
// output neurons], in FP64.
//
// The block figure is not available, so the block is read as
//   z = a + W (*) h          3x3 circular convolution, c_in -> 2C channels
//   m[c] = max(z[2c], z[2c+1])             max-pool of window 2 over channels
//   u = v + V (*)^T m        3x3 circular transposed convolution, stride 1,
//                            u[co][p] = v[co] + sum V[ci][co][ky][kx] m[ci][p - (ky-1, kx-1)]
// with h = spins for the first block and u of the block below otherwise;
// log|psi_net| = sum log|u_K| and sign(psi_net) = prod sign(u_K).
// Canonical parameter order per block: W[2C][c_in][3][3], a[2C],
// V[C][C][3][3] (input channel first), v[C].
//
// With 16 channels the FP64 matrix cores (v_mfma_f64_16x16x4f64,
// k_conv_f64mma.hip) run every transposed convolution, as a convolution with
// flipped, transposed taps (V[ci][co][8 - t]), and the convolutions 16 -> 32
// of blocks 2.., with the channel-pair max in their epilogue.  The first
// convolution (one input channel) stays on the vector ALU.  The packing,
// built on the device from the canonical vector:
//   block 1: [9][16][16] transposed taps, [16] bias (2320 doubles);
//   block k >= 2: [9][16][32] convolution taps, column 16 h + j holding
//   channel 2 j + h, [32] its bias in the same column order, then the
//   transposed part as for block 1 (6960 doubles);
// then for the backward's data gradients, also convolutions on the matrix
// cores: per block [9][16][16] taps V[ci][co][t] read as [t][co][ci] (the
// gradient through the transposed convolution), then per block k >= 2
// [9][32][16] taps W[co][ci][8 - t] read as [t][co][ci] (the gradient
// through the convolution).
//
// Planes are NHWC ([plane][site][channel]) in HBM.  The forward serves the
// samples (base planes) and the exchanged configurations of the local
// energy (one plane per queue item, the pair exchanged as the spins are
// read), recomputed in full.  The backward gives O = d log|psi| / d theta per
// sample: 1/u at the output, then per block the transposed convolution's
// weight gradients, its data gradient routed through the max to the larger
// input (the first on a tie), the convolution's weight gradients and its
// data gradient.  Every weight gradient is a fixed-order sum over the sites
// of one sample, so rows are deterministic.
#include <algorithm>

#include "nqs_internal.h"

namespace nqs {
namespace {

constexpr int kThreads = 256;

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ inline int wrapc(int a, int L) { return a < 0 ? a + L : (a >= L ? a - L : a); }

// canonical sizes with 16 channels
constexpr int kMC = 16;
constexpr int kConvT = kMC * kMC * 9;                  // V: 2304
constexpr int kConv1 = 2 * kMC * 9;                    // W of block 1 (c_in = 1): 288
constexpr int kConvK = 2 * kMC * kMC * 9;              // W of blocks 2..: 4608
constexpr int kBlock1 = kConv1 + 2 * kMC + kConvT + kMC;          // 2640
constexpr int kBlockK = kConvK + 2 * kMC + kConvT + kMC;          // blocks 2..: 6960
constexpr int kPackFirst = kConvT + kMC;                          // packed block 1: 2320
constexpr int kPackBlock = kBlockK;         // packed block k >= 2: same count, reordered
static_assert(kBlock1 == 2640 && kPackFirst == 2320 && kPackBlock == 6960, "packing sizes");

// offsets of block k's parameters in the canonical vector
struct Cnn1Block {
    int64_t W, a, V, v;
    int cin;
};

Cnn1Block block_of(int C, int k)
{
    int64_t off = 0;
    for (int l = 0; l < k; ++l) {
        const int ci = (l == 0) ? 1 : C;
        off += (int64_t)2 * C * ci * 9 + 2 * C + (int64_t)C * C * 9 + C;
    }
    Cnn1Block b;
    b.cin = (k == 0) ? 1 : C;
    b.W = off;
    b.a = b.W + (int64_t)2 * C * b.cin * 9;
    b.V = b.a + 2 * C;
    b.v = b.V + (int64_t)C * C * 9;
    return b;
}

// planes of a launch: samples (queue null) or queue items q_begin + m
struct C1Planes {
    const uint32_t *queue;
    int64_t q_begin;
    const int64_t *qlen;
};

__device__ inline int64_t c1_live(const C1Planes &pm, int64_t M)
{
    if (!pm.queue) return M;
    const int64_t left = pm.qlen[0] - pm.q_begin;
    return left < 0 ? 0 : (left < M ? left : M);
}

// sample of plane m and the exchanged pair (-1, -1 for a sample plane)
__device__ inline void c1_origin(const C1Planes &pm, int64_t m, int L, int *s, int *qi, int *qj)
{
    if (!pm.queue) {
        *s = (int)m;
        *qi = -1;
        *qj = -1;
        return;
    }
    const uint32_t e = pm.queue[pm.q_begin + m];
    const int b = item_bond(e), i = b >> 2, t = b & 3;
    const int x = i % L, y = i / L;
    *s = item_sample(e);
    *qi = i;
    *qj = wrapc(y + bond_dy(t), L) * L + wrapc(x + bond_dx(t), L);
}

// Convolution and max-pool of the first block (one input channel, the
// spins) with 16 channels: thread (plane, site) reads its 9 spins once and
// forms all 32 z and 16 pooled m; the taps and biases sit in LDS.  Same
// arithmetic order per output as k_c1_conv (bias, then taps 0..8).
__global__ void __launch_bounds__(kThreads)
k_c1_conv_first(const int8_t *__restrict__ spins, C1Planes pm, int64_t M, int L,
                const double *__restrict__ W, const double *__restrict__ a,
                double *__restrict__ mout, double *__restrict__ zsave)
{
    __shared__ double ws[2 * kMC * 9], as[2 * kMC];
    for (int q = threadIdx.x; q < 2 * kMC * 9; q += kThreads) ws[q] = W[q];
    for (int q = threadIdx.x; q < 2 * kMC; q += kThreads) as[q] = a[q];
    __syncthreads();
    const int N = L * L;
    const int64_t total = c1_live(pm, M) * N;
    for (int64_t mp = (int64_t)blockIdx.x * kThreads + threadIdx.x; mp < total;
         mp += (int64_t)gridDim.x * kThreads) {
        const int64_t m = mp / N;
        const int p = (int)(mp - m * N);
        const int x = p % L, y = p / L;
        int s, qi, qj;
        c1_origin(pm, m, L, &s, &qi, &qj);
        const int8_t *sp = spins + (int64_t)s * N;
        double h[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            int q = wrapc(y + t / 3 - 1, L) * L + wrapc(x + t % 3 - 1, L);
            q = (q == qi) ? qj : ((q == qj) ? qi : q);
            h[t] = (double)sp[q];
        }
#pragma unroll 4
        for (int c = 0; c < kMC; ++c) {
            double z0 = as[2 * c], z1 = as[2 * c + 1];
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                z0 = fma(ws[(2 * c) * 9 + t], h[t], z0);
                z1 = fma(ws[(2 * c + 1) * 9 + t], h[t], z1);
            }
            mout[mp * kMC + c] = (z1 > z0) ? z1 : z0;
            if (zsave) {
                zsave[mp * 2 * kMC + 2 * c] = z0;
                zsave[mp * 2 * kMC + 2 * c + 1] = z1;
            }
        }
    }
}

// Convolution and max-pool of one block: thread (plane, site, c) forms
// z[2c], z[2c+1] and m[c].  in: [M][N][cin] (null: the spins of the plane).
__global__ void __launch_bounds__(kThreads)
k_c1_conv(const int8_t *__restrict__ spins, C1Planes pm, int64_t M, int L, int C, int cin,
          const double *__restrict__ in, const double *__restrict__ W,
          const double *__restrict__ a, double *__restrict__ mout, double *__restrict__ zsave)
{
    const int N = L * L;
    const int64_t total = c1_live(pm, M) * N * C;
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * kThreads) {
        const int c = (int)(g % C);
        const int64_t mp = g / C;
        const int64_t m = mp / N;
        const int p = (int)(mp - m * N);
        const int x = p % L, y = p / L;
        double z0 = a[2 * c], z1 = a[2 * c + 1];
        const double *w0 = W + (int64_t)(2 * c) * cin * 9;
        const double *w1 = w0 + (int64_t)cin * 9;
        if (!in) {
            int s, qi, qj;
            c1_origin(pm, m, L, &s, &qi, &qj);
            const int8_t *sp = spins + (int64_t)s * N;
            for (int t = 0; t < 9; ++t) {
                int q = wrapc(y + t / 3 - 1, L) * L + wrapc(x + t % 3 - 1, L);
                q = (q == qi) ? qj : ((q == qj) ? qi : q);
                const double h = (double)sp[q];
                z0 = fma(w0[t], h, z0);
                z1 = fma(w1[t], h, z1);
            }
        } else {
            for (int t = 0; t < 9; ++t) {
                const int q = wrapc(y + t / 3 - 1, L) * L + wrapc(x + t % 3 - 1, L);
                const double *hq = in + (m * N + q) * cin;
                for (int ci = 0; ci < cin; ++ci) {
                    z0 = fma(w0[ci * 9 + t], hq[ci], z0);
                    z1 = fma(w1[ci * 9 + t], hq[ci], z1);
                }
            }
        }
        mout[mp * C + c] = (z1 > z0) ? z1 : z0;
        if (zsave) {
            zsave[mp * 2 * C + 2 * c] = z0;
            zsave[mp * 2 * C + 2 * c + 1] = z1;
        }
    }
}

// Transposed convolution of one block: thread (plane, site, co).
__global__ void __launch_bounds__(kThreads)
k_c1_convt(C1Planes pm, int64_t M, int L, int C, const double *__restrict__ min_,
           const double *__restrict__ V, const double *__restrict__ v, double *__restrict__ uout)
{
    const int N = L * L;
    const int64_t total = c1_live(pm, M) * N * C;
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * kThreads) {
        const int co = (int)(g % C);
        const int64_t mp = g / C;
        const int64_t m = mp / N;
        const int p = (int)(mp - m * N);
        const int x = p % L, y = p / L;
        double u = v[co];
        for (int t = 0; t < 9; ++t) {
            const int q = wrapc(y - t / 3 + 1, L) * L + wrapc(x - t % 3 + 1, L);
            const double *mq = min_ + (m * N + q) * C;
            for (int ci = 0; ci < C; ++ci) u = fma(V[((int64_t)ci * C + co) * 9 + t], mq[ci], u);
        }
        uout[mp * C + co] = u;
    }
}

// Per plane: f = sum log|u| (fixed reduction tree) and the parity of the
// negative neurons.  Sample planes write f and the network sign (and
// multiply it into sign_pub when given); item planes write
// dlog = f' - f(sample) and the sign ratio.
__global__ void __launch_bounds__(kThreads)
k_c1_final(C1Planes pm, int64_t M, int NC, const double *__restrict__ u, double *__restrict__ f,
           int8_t *__restrict__ sgn, int8_t *__restrict__ sign_pub,
           const double *__restrict__ fbase, const int8_t *__restrict__ sbase, int32_t *err)
{
    __shared__ double red[kThreads];
    __shared__ int neg[kThreads];
    const int64_t m = blockIdx.x;
    if (m >= c1_live(pm, M)) return;
    const double *um = u + m * NC;
    double acc = 0.0;
    int n = 0;
    for (int q = threadIdx.x; q < NC; q += kThreads) {
        acc += log(fabs(um[q]));
        n += (um[q] < 0.0);
    }
    red[threadIdx.x] = acc;
    neg[threadIdx.x] = n;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[threadIdx.x] += red[threadIdx.x + off];
            neg[threadIdx.x] += neg[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double fm = red[0];
        const int8_t sm = (neg[0] & 1) ? -1 : 1;
        if (!isfinite(fm)) atomicOr(err, kErrNonFinite);
        if (!pm.queue) {
            f[m] = fm;
            sgn[m] = sm;
            if (sign_pub) sign_pub[m] = (int8_t)(sign_pub[m] * sm);
        } else {
            const int s = item_sample(pm.queue[pm.q_begin + m]);
            f[m] = fm - fbase[s];
            sgn[m] = (int8_t)(sm * sbase[s]);
        }
    }
}

// ---- backward ----

__global__ void k_c1_ginit(const double *__restrict__ u, int64_t n, double *__restrict__ g)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        g[i] = 1.0 / u[i];
}

// Weight and bias gradients of one block into the O rows.
//   transposed (T = 1): O[V + (ci C + co) 9 + t] = sum_p g[p][co] m[p - off t][ci],
//                       m from the saved z of the block; O[v + co] = sum_p g[p][co]
//   convolution (T = 0): O[W + (co cin + ci) 9 + t] = sum_p gz[p][co] h[p + off t][ci],
//                       h = spins (first block) or u of the block below;
//                       O[a + co] = sum_p gz[p][co]
template <typename OT>
__global__ void __launch_bounds__(kThreads)
k_c1_wgrad(int nb, int L, int C, int T, int nco, int cin, const double *__restrict__ g,
           const double *__restrict__ z, const double *__restrict__ h,
           const int8_t *__restrict__ spins, int64_t offw, int64_t offb, int64_t P,
           OT *__restrict__ O)
{
    const int N = L * L;
    const int nw = nco * cin * 9;         // weights, then nco biases
    const int per = nw + nco;
    const int64_t total = (int64_t)nb * per;
    for (int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * kThreads) {
        const int b = (int)(id / per);
        const int r = (int)(id - (int64_t)b * per);
        const double *gb = g + (int64_t)b * N * nco;
        double acc = 0.0;
        int64_t dst;
        if (r >= nw) {
            const int co = r - nw;
            for (int p = 0; p < N; ++p) acc += gb[(int64_t)p * nco + co];
            dst = offb + co;
        } else if (T) {
            // r = (ci C + co) 9 + t
            const int t = r % 9, cc = r / 9, co = cc % C, ci = cc / C;
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            const double *zb = z + (int64_t)b * N * 2 * C;
            for (int p = 0; p < N; ++p) {
                const int q = wrapc(p / L - dy, L) * L + wrapc(p % L - dx, L);
                const double z0 = zb[(int64_t)q * 2 * C + 2 * ci];
                const double z1 = zb[(int64_t)q * 2 * C + 2 * ci + 1];
                acc = fma(gb[(int64_t)p * nco + co], (z1 > z0) ? z1 : z0, acc);
            }
            dst = offw + r;
        } else {
            // r = (co cin + ci) 9 + t
            const int t = r % 9, cc = r / 9, ci = cc % cin, co = cc / cin;
            const int dy = t / 3 - 1, dx = t % 3 - 1;
            for (int p = 0; p < N; ++p) {
                const int q = wrapc(p / L + dy, L) * L + wrapc(p % L + dx, L);
                const double hv = h ? h[((int64_t)b * N + q) * cin + ci]
                                    : (double)spins[(int64_t)b * N + q];
                acc = fma(gb[(int64_t)p * nco + co], hv, acc);
            }
            dst = offw + r;
        }
        O[(int64_t)b * P + dst] = (OT)acc;
    }
}

// dL/dm of the transposed convolution, routed through the max:
// gm[q][ci] = sum_{co,t} V[ci][co][t] g[q + off t][co]; gz[q][2ci + a] = gm
// for the larger input a (first on a tie), 0 for the other.
__global__ void __launch_bounds__(kThreads)
k_c1_gmax(int nb, int L, int C, const double *__restrict__ g, const double *__restrict__ V,
          const double *__restrict__ z, double *__restrict__ gz)
{
    const int N = L * L;
    const int64_t total = (int64_t)nb * N * C;
    for (int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * kThreads) {
        const int ci = (int)(id % C);
        const int64_t bq = id / C;
        const int64_t b = bq / N;
        const int q = (int)(bq - b * N);
        const int x = q % L, y = q / L;
        double gm = 0.0;
        for (int t = 0; t < 9; ++t) {
            const int p = wrapc(y + t / 3 - 1, L) * L + wrapc(x + t % 3 - 1, L);
            const double *gp = g + (b * N + p) * C;
            for (int co = 0; co < C; ++co) gm = fma(V[((int64_t)ci * C + co) * 9 + t], gp[co], gm);
        }
        const double z0 = z[bq * 2 * C + 2 * ci], z1 = z[bq * 2 * C + 2 * ci + 1];
        const bool second = z1 > z0;
        gz[bq * 2 * C + 2 * ci] = second ? 0.0 : gm;
        gz[bq * 2 * C + 2 * ci + 1] = second ? gm : 0.0;
    }
}

// Weight and bias gradients of blocks 2.. with 16 channels on the FP64 matrix
// cores, per sample: a GEMM over the sites (K, steps of 4) with rows = output
// channels co (A = the gradient at the block's output, 16 per tile) and
// columns = (tap t, input channel ci), one 16-column tile per tap.
//   TRANS = false (convolution 16 -> 32): rows gz[p][co] (2 tiles),
//     columns h[p + off t][ci]; dW[co][ci][t] at offw, da[co] at offb;
//   TRANS = true (transposed convolution): rows g[p][co] (1 tile), columns
//     m[p - off t][ci] with m = max(z[2ci], z[2ci+1]) re-formed from the
//     saved z; dV[ci][co][t] at offw, dv[co] at offb.
// One wave per (sample, 3 taps); three waves per sample.  Fixed summation
// order, so rows are deterministic.
template <typename OT, bool TRANS>
__global__ void __launch_bounds__(kThreads)
k_c1_wgrad_mma(int nb, int L, const double *__restrict__ grad, const double *__restrict__ src,
               int64_t offw, int64_t offb, int64_t P, OT *__restrict__ O)
{
    constexpr int NH = TRANS ? 1 : 2;           // 16-row tiles of output channels
    constexpr int NCO = 16 * NH;
    constexpr int NT = 3;                       // taps per wave
    const int N = L * L;
    const int lane = threadIdx.x & 63;
    const int m16 = lane & 15, kq = lane >> 4;
    const int64_t wave_id = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int64_t b = wave_id / 3;
    if (b >= nb) return;
    const int t0 = (int)(wave_id - b * 3) * NT;
    const double *gb = grad + b * (int64_t)N * NCO;
    const double *sb = src + b * (int64_t)N * (TRANS ? 2 * kMC : kMC);
    const int sg = TRANS ? -1 : 1;
    double4_t acc[NH][NT];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[h][j] = (double4_t){0, 0, 0, 0};
    double dbp[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) dbp[h] = 0.0;
    for (int p0 = 0; p0 < N; p0 += 4) {
        const int p = p0 + kq, y = p / L, x = p - (p / L) * L;
        double av[NH], bv[NT];
#pragma unroll
        for (int h = 0; h < NH; ++h) av[h] = gb[(int64_t)p * NCO + 16 * h + m16];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int t = t0 + j;
            const int r = wrapc(y + sg * (t / 3 - 1), L) * L + wrapc(x + sg * (t % 3 - 1), L);
            if (TRANS) {
                const double z0 = sb[(int64_t)r * 2 * kMC + 2 * m16];
                const double z1 = sb[(int64_t)r * 2 * kMC + 2 * m16 + 1];
                bv[j] = (z1 > z0) ? z1 : z0;
            } else {
                bv[j] = sb[(int64_t)r * kMC + m16];
            }
        }
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            dbp[h] += av[h];
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[h][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h], bv[j], acc[h][j], 0, 0, 0);
        }
    }
    OT *o = O + b * P;
    // D element i of this lane: row co = 16 h + kq + 4 i, column ci = m16 at tap t0 + j
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = 16 * h + kq + 4 * i, ci = m16, t = t0 + j;
                const int64_t idx = TRANS ? ((int64_t)ci * kMC + co) * 9 + t
                                          : ((int64_t)co * kMC + ci) * 9 + t;
                o[offw + idx] = (OT)acc[h][j][i];
            }
    if (t0 == 0) {
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            double v = dbp[h];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (kq == 0) o[offb + 16 * h + m16] = (OT)v;
        }
    }
}

// the max's routing of dL/dm (gm [nb][N][C], computed on the matrix cores)
// into dL/dz: gz[q][2ci + a] = gm for the larger input a (first on a tie)
__global__ void __launch_bounds__(kThreads)
k_c1_route(int64_t n, int C, const double *__restrict__ gm, const double *__restrict__ z,
           double *__restrict__ gz)
{
    for (int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x; id < n;
         id += (int64_t)gridDim.x * kThreads) {
        const int ci = (int)(id % C);
        const int64_t bq = id / C;
        const double z0 = z[bq * 2 * C + 2 * ci], z1 = z[bq * 2 * C + 2 * ci + 1];
        const bool second = z1 > z0;
        gz[bq * 2 * C + 2 * ci] = second ? 0.0 : gm[id];
        gz[bq * 2 * C + 2 * ci + 1] = second ? gm[id] : 0.0;
    }
}

// dL/dh of the convolution: gh[q][ci] = sum_{co,t} W[co][ci][t] gz[q - off t][co]
__global__ void __launch_bounds__(kThreads)
k_c1_gdata(int nb, int L, int C, const double *__restrict__ gz, const double *__restrict__ W,
           double *__restrict__ gh)
{
    const int N = L * L;
    const int64_t total = (int64_t)nb * N * C;
    for (int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * kThreads) {
        const int ci = (int)(id % C);
        const int64_t bq = id / C;
        const int64_t b = bq / N;
        const int q = (int)(bq - b * N);
        const int x = q % L, y = q / L;
        double acc = 0.0;
        for (int t = 0; t < 9; ++t) {
            const int p = wrapc(y - t / 3 + 1, L) * L + wrapc(x - t % 3 + 1, L);
            const double *gp = gz + (b * N + p) * 2 * C;
            for (int co = 0; co < 2 * C; ++co)
                acc = fma(W[((int64_t)co * C + ci) * 9 + t], gp[co], acc);
        }
        gh[bq * C + ci] = acc;
    }
}


// offsets of block k's canonical V and W (c_in = 1 for k = 0, else 16)
__host__ __device__ inline int64_t canon_V(int k)
{
    return k == 0 ? kConv1 + 2 * kMC : kBlock1 + (int64_t)(k - 1) * kBlockK + kConvK + 2 * kMC;
}
__host__ __device__ inline int64_t canon_W(int k) { return kBlock1 + (int64_t)(k - 1) * kBlockK; }
__host__ __device__ inline int64_t fwd_pack_size(int Kb)
{
    return kPackFirst + (int64_t)(Kb - 1) * kPackBlock;
}
// backward packing: gradient through V of block k, and through W of block k >= 1
__host__ __device__ inline int64_t bwd_gm_off(int Kb, int k) { return fwd_pack_size(Kb) + (int64_t)k * kConvT; }
__host__ __device__ inline int64_t bwd_gd_off(int Kb, int k)
{
    return fwd_pack_size(Kb) + (int64_t)Kb * kConvT + (int64_t)(k - 1) * kConvK;
}

// backward packing entry q (0 <= q < Kb kConvT + (Kb - 1) kConvK)
__device__ inline double bwd_pack_value(const double *w, int Kb, int64_t q)
{
    if (q < (int64_t)Kb * kConvT) {
        const int k = (int)(q / kConvT), r = (int)(q - (int64_t)k * kConvT);
        const int ci = r % kMC, co = (r / kMC) % kMC, t = r / (kMC * kMC);
        return w[canon_V(k) + ((int64_t)ci * kMC + co) * 9 + t];
    }
    q -= (int64_t)Kb * kConvT;
    const int k = 1 + (int)(q / kConvK), r = (int)(q - (int64_t)(k - 1) * kConvK);
    const int ci = r % kMC, co = (r / kMC) % (2 * kMC), t = r / (2 * kMC * kMC);
    return w[canon_W(k) + ((int64_t)co * kMC + ci) * 9 + (8 - t)];
}

__global__ void k_c1_pack(const double *__restrict__ w, int Kb, double *__restrict__ out)
{
    const int64_t nf = fwd_pack_size(Kb);
    const int64_t n = nf + (int64_t)Kb * kConvT + (int64_t)(Kb - 1) * kConvK;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kThreads) {
        double val;
        if (q >= nf) {
            out[q] = bwd_pack_value(w, Kb, q - nf);
            continue;
        }
        if (q < kPackFirst) {
            // block 1: canonical W at 0, a at kConv1, V, then v
            const int64_t V = kConv1 + 2 * kMC, v = V + kConvT;
            const int r = (int)q;
            if (r < kConvT) {
                const int co = r % kMC, ci = (r / kMC) % kMC, t = r / (kMC * kMC);
                val = w[V + ((int64_t)ci * kMC + co) * 9 + (8 - t)];
            } else {
                val = w[v + (r - kConvT)];
            }
            out[q] = val;
            continue;
        }
        const int k = 1 + (int)((q - kPackFirst) / kPackBlock);
        int r = (int)(q - kPackFirst - (int64_t)(k - 1) * kPackBlock);
        // canonical offsets of block k (c_in = 16): W, a, V, v
        const int64_t W = kBlock1 + (int64_t)(k - 1) * kBlockK;
        const int64_t a = W + kConvK, V = a + 2 * kMC, v = V + kConvT;
        if (r < kConvK) {
            // [t][ci][n], column n = 16 h + j holds output channel 2 j + h
            const int n = r % (2 * kMC), ci = (r / (2 * kMC)) % kMC, t = r / (2 * kMC * kMC);
            const int co = 2 * (n % kMC) + n / kMC;
            val = w[W + ((int64_t)co * kMC + ci) * 9 + t];
        } else if ((r -= kConvK) < 2 * kMC) {
            val = w[a + 2 * (r % kMC) + r / kMC];
        } else if ((r -= 2 * kMC) < kConvT) {
            const int co = r % kMC, ci = (r / kMC) % kMC, t = r / (kMC * kMC);
            val = w[V + ((int64_t)ci * kMC + co) * 9 + (8 - t)];
        } else {
            val = w[v + (r - kConvT)];
        }
        out[q] = val;
    }
}

int grid_of(const nqs_ctx *c, int64_t work)
{
    const int64_t b = (work + kThreads - 1) / kThreads;
    const int64_t cap = (int64_t)std::max(c->n_cu, 1) * 16;
    return (int)std::max<int64_t>(1, std::min(b, cap));
}

bool mfma_blocks(const nqs_ctx *c) { return c->C == kMC; }

// one block over M planes: h (null for the first block: the spins) -> m
// (pooled, into mbuf) -> u; zsave (may be null) keeps z
void block_forward(const nqs_ctx *c, int k, const int8_t *spins, C1Planes pm, int64_t M,
                   const double *h, double *mbuf, double *u, double *zsave, hipStream_t s)
{
    const int L = c->L, C = c->C;
    const int64_t work = M * c->N * C;
    const Cnn1Block o = block_of(C, k);
    const bool mm = mfma_blocks(c);
    // packed transposed taps and bias of this block (matrix-core path)
    const double *pt = nullptr;
    if (mm)
        pt = k == 0 ? c->w_vec64
                    : c->w_vec64 + kPackFirst + (int64_t)(k - 1) * kPackBlock + kConvK + 2 * kMC;
    if (k > 0 && mm) {
        const double *pk = pt - (kConvK + 2 * kMC);
        f64mma_cnn1_conv(c, h, M, pk, pk + kConvK, mbuf, zsave, pm.qlen, pm.q_begin, s);
    } else {
        if (k == 0 && mm)
            NQS_LAUNCH(k_c1_conv_first, dim3(grid_of(c, M * c->N)), dim3(kThreads), 0, s, spins,
                       pm, M, L, (const double *)c->w_canon + o.W,
                       (const double *)c->w_canon + o.a, mbuf, zsave);
        else
            NQS_LAUNCH(k_c1_conv, dim3(grid_of(c, work)), dim3(kThreads), 0, s, spins, pm, M, L,
                       C, o.cin, h, (const double *)c->w_canon + o.W,
                       (const double *)c->w_canon + o.a, mbuf, zsave);
    }
    if (mm) {
        f64mma_cnn1_convt(c, mbuf, M, pt, pt + kConvT, u, pm.qlen, pm.q_begin, s);
    } else {
        NQS_LAUNCH(k_c1_convt, dim3(grid_of(c, work)), dim3(kThreads), 0, s, pm, M, L, C,
                   (const double *)mbuf, (const double *)c->w_canon + o.V,
                   (const double *)c->w_canon + o.v, u);
    }
}

// the blocks over M planes: the result u of the last block ends in pa
void blocks_forward(const nqs_ctx *c, const int8_t *spins, C1Planes pm, int64_t M, double *pa,
                    double *pb, hipStream_t s)
{
    for (int k = 0; k < c->K; ++k)
        block_forward(c, k, spins, pm, M, k == 0 ? nullptr : pa, pb, pa, nullptr, s);
}

// ---- exchanged configurations by the receptive cone ----
//
// Exchanging the pair (q_i, q_j) changes the spins of a w0 x h0 box.  Number
// the stencils l = 1 .. 2K (block b's convolution is layer 2b - 1, its
// transposed convolution layer 2b, each 3x3 on the torus): the output of
// layer l differs from the sample's only on R_l, the box widened by l sites.
// So log|psi(S')| - log|psi(S)| = sum over R_2K of log|u'_K| - log|u_K|, and
// the sign ratio is the parity of the change in negative neurons on R_2K.
//
// One workgroup of 12 waves (three per SIMD) per queue item.  A square
// frame of side 4K + 4 (the box
// widened by F = 2K + 1) holds in LDS the 16 FP64 channels of the current
// layer's input; layer l reads the frame on R_{l+1} and forms R_l as tiles of
// 16 sites x 16 channels on v_mfma_f64_16x16x4f64, with the operand layout,
// packed taps and MFMA order of the full pass (k_conv_mma), so every neuron
// of the cone is bit-identical to the full recomputation's; the layer's taps
// sit in LDS after the frame, laid out so that each lane reads its four B
// operands of a tap and column block as 32 contiguous bytes.  The results wait
// in registers until every wave has read the frame, then replace R_l in
// place, and the ring R_{l+2} \ R_l is filled from the sample's activations
// of layer l, kept by the base pass (cache: [2K-1][B][N][16], m_1, u_1, m_2,
// ..., m_K; then per site the sum of log|u_K| over the channels, [B][N]
// FP64, and the count of negative u_K, [B][N] int32).  Each wave fetches the
// ring and the next layer's taps as soon as its tiles are done, so the loads
// run while the other waves finish; the stores follow the barrier.  On the
// last layer each neuron of R_2K adds log|u'| and the region's sites
// subtract their base sums.  Layer 1 (one input channel) runs on the vector
// ALU from the exchanged spins, with the full pass's FMA order.  Needs 16
// channels, K <= 6 (the register staging; the ring fits 3 chunks per
// thread) and L >= 4K + 4 (the frame does not overlap itself).
// Per site of the last layer's output u [M][N][16]: the sum of log|u| over
// the channels and the count of negative neurons.
__global__ void __launch_bounds__(kThreads)
k_c1_site_sums(const double *__restrict__ u, int64_t n_sites, double *__restrict__ slog,
               int *__restrict__ nneg)
{
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n_sites;
         q += (int64_t)gridDim.x * kThreads) {
        const double *v = u + q * kMC;
        double acc = 0.0;
        int n = 0;
#pragma unroll
        for (int c = 0; c < kMC; ++c) {
            acc += log(fabs(v[c]));
            n += v[c] < 0.0;
        }
        slog[q] = acc;
        nneg[q] = n;
    }
}

constexpr int kConeMaxK = 6;
constexpr int kConeNW = 12;
constexpr int kConeThreads = kConeNW * 64;
constexpr int kConeStage = 3;   // staged tiles per wave: R_11 has 36 tiles at K = 6
constexpr int kConeTapSlots = (9 * 2 * 256 + kConeThreads - 1) / kConeThreads;   // taps per thread

struct C1ConeArgs {
    const int8_t *spins;        // [B][N]
    const uint32_t *queue;
    const int64_t *qlen;
    int64_t cap;
    const double *wpack;        // the forward's packed taps
    const double *w1;           // block 1, canonical: W [32][9], then a [32]
    const double *cache;        // [2K-1][B][N][16], then slog [B][N], then nneg (int32) [B][N]
    int64_t B;
    double *dlog;
    int8_t *isign;
    int32_t *err;
    int L, K;
};

// byte offset of 16-byte chunk c (channels 2c, 2c + 1) of frame site f; the
// chunks of a site are rotated by f mod 8, so 8 lanes reading one chunk
// position of 8 consecutive sites hit 8 different bank groups
__device__ inline int fr_off(int f, int c) { return f * 128 + ((c ^ (f & 7)) << 4); }

// packed taps of layer l: W[t][ci][col] (ncol columns) and its bias
__device__ inline const double *c1_layer_taps(const double *wp, int l, int *ncol)
{
    const int k = (l - 1) >> 1;                      // 0-based block
    const double *blk = k == 0 ? wp : wp + kPackFirst + (int64_t)(k - 1) * kPackBlock;
    if (l & 1) {                                     // convolution of block k >= 1
        *ncol = 2 * kMC;
        return blk;
    }
    *ncol = kMC;                                     // transposed convolution
    return k == 0 ? blk : blk + kConvK + 2 * kMC;
}

// A layer's taps in LDS: wl[((t NH + h) 64 + lane) 4 + s] = W[t][4 kq + s][16 h + m16]
// (lane = 16 kq + m16), at most kConeTapSlots entries per thread (q = tid + r kConeThreads),
// fetched into tv (entries beyond the layer's: not stored), and its bias
struct C1Taps {
    double tv[kConeTapSlots];
    double bias[2];
    int total;
};

__device__ inline void c1_taps_fetch(C1Taps &tp, const double *wp, int l, int tid, int m16)
{
    int ncol;
    const double *wt = c1_layer_taps(wp, l, &ncol);
    const int nh = ncol >> 4;
    tp.total = 9 * nh * 256;
#pragma unroll
    for (int r = 0; r < kConeTapSlots; ++r) {
        const int q = min(tid + r * kConeThreads, tp.total - 1);
        const int sub = q & 3, ln = (q >> 2) & 63, th = q >> 8;
        const int t = th / nh, h = th - t * nh;
        tp.tv[r] = wt[(t * kMC + 4 * (ln >> 4) + sub) * ncol + 16 * h + (ln & 15)];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) tp.bias[h] = wt[9 * kMC * ncol + 16 * min(h, nh - 1) + m16];
}

__device__ inline void c1_taps_store(const C1Taps &tp, double *wl, int tid)
{
#pragma unroll
    for (int r = 0; r < kConeTapSlots; ++r)
        if (tid + r * kConeThreads < tp.total) wl[tid + r * kConeThreads] = tp.tv[r];
}

// One tile: fm = frame site of this lane's A row; D element i: row kq + 4 i,
// column 16 h + m16; the taps and K-steps in the full pass's order (fully
// unrolled: the compiler reads the operands of all taps ahead).
template <int NH>
__device__ inline void c1_tile(const unsigned char *fr, const double *wl, int fm, int P,
                               int lane, const double (&bias)[2], double4_t (&acc)[2])
{
    const int kq = lane >> 4;
#pragma unroll
    for (int h = 0; h < NH; ++h) acc[h] = (double4_t){bias[h], bias[h], bias[h], bias[h]};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int f = fm + (t / 3 - 1) * P + (t % 3 - 1);
        const double2 u0 = *(const double2 *)(fr + fr_off(f, 2 * kq));
        const double2 u1 = *(const double2 *)(fr + fr_off(f, 2 * kq + 1));
        const double av[4] = {u0.x, u0.y, u1.x, u1.y};
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const double2 *wp = (const double2 *)(wl + ((t * NH + h) * 64 + lane) * 4);
            const double2 w0 = wp[0], w1 = wp[1];
            const double bv[4] = {w0.x, w0.y, w1.x, w1.y};
#pragma unroll
            for (int sub = 0; sub < 4; ++sub)
                acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[sub], bv[sub], acc[h], 0, 0, 0);
        }
    }
}

__global__ void __launch_bounds__(kConeThreads) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_c1_cone(C1ConeArgs a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char fr[];
    __shared__ double red[kConeNW];
    __shared__ int nred[kConeNW];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m16 = lane & 15, kq = lane >> 4;
    const int L = a.L, N = L * L, K = a.K, F = 2 * K + 1, P = 4 * K + 4;
    const int64_t n_items = min(a.qlen[0], a.cap);
    // XCD-contiguous ranges of the queue (the grid is a multiple of 8)
    const int per_xcd = gridDim.x / 8;
    const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
    const int64_t seg = (n_items + 7) / 8;
    const int64_t u_end = min(n_items, (xcd + 1) * seg);
    double *wl = reinterpret_cast<double *>(fr + (size_t)P * P * 128);   // the layer's taps

    for (int64_t u = xcd * seg + slot; u < u_end; u += per_xcd) {
        const uint32_t e = a.queue[u];
        const int s = item_sample(e), b = item_bond(e), tau = b & 3, i0 = b >> 2;
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
        // ring R_{l+2} \ R_l of the frame: its 4 (w0 + 2l + 4) + 4 (h0 + 2l)
        // sites (two rows above and below R_l, full width, then two columns
        // left and right of it) in 8 chunks each, chunk q = tid + r kConeThreads
        // (at most 4 per thread): values from the cache of layer l, offsets
        // in the frame (-1: none)
        double2 rv0, rv1, rv2;
        int rd0, rd1, rd2;   // 3 x 768 >= 1664 ring chunks (K = 6)
        auto ring_fetch = [&](int l) {
            const int W = w0 + 2 * l + 4, H = h0 + 2 * l + 4, hi = h0 + 2 * l;
            const int total = (4 * W + 4 * hi) * 8;
            const double *src = a.cache + ((int64_t)(l - 1) * a.B + s) * N * kMC;
            auto one = [&](int q, double2 &v, int &d) {
                const int rs = q >> 3, c = q & 7;
                const int band = (rs >= W) + (rs >= 2 * W) + (rs >= 3 * W);
                const int rr = rs - 4 * W, col = rr & 3;
                const bool bands = rs < 4 * W;
                const int px = bands ? rs - band * W : (col < 2 ? col : W - 4 + col);
                const int py = bands ? (band < 2 ? band : H - 4 + band) : 2 + (rr >> 2);
                const bool live = q < total;
                const int fx = F - l - 2 + px, fy = F - l - 2 + py;
                const int site = live ? site_of(fx, fy) : 0;
                v = *(const double2 *)(src + (int64_t)site * kMC + 2 * c);
                d = live ? fr_off(fy * P + fx, c) : -1;
            };
            one(tid, rv0, rd0);
            one(tid + kConeThreads, rv1, rd1);
            one(tid + 2 * kConeThreads, rv2, rd2);
        };
        auto ring_store = [&]() {
            if (rd0 >= 0) *(double2 *)(fr + rd0) = rv0;
            if (rd1 >= 0) *(double2 *)(fr + rd1) = rv1;
            if (rd2 >= 0) *(double2 *)(fr + rd2) = rv2;
        };
        C1Taps tp;
        ring_fetch(1);
        c1_taps_fetch(tp, a.wpack, 2, tid, m16);

        // layer 1 on R_1 from the exchanged spins: thread (site, pooled channel j)
        {
            const int w1 = w0 + 2, n1 = w1 * (h0 + 2);
            if (tid < n1 * kMC) {
                const int p = tid >> 4, j = tid & 15;
                const int py = p / w1, px = p - py * w1;
                const int fx = F - 1 + px, fy = F - 1 + py;
                double z0 = a.w1[2 * kMC * 9 + 2 * j], z1 = a.w1[2 * kMC * 9 + 2 * j + 1];
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    int q = site_of(fx + t % 3 - 1, fy + t / 3 - 1);
                    q = (q == qi) ? qj : ((q == qj) ? qi : q);
                    const double hv = (double)sp[q];
                    z0 = fma(a.w1[(2 * j) * 9 + t], hv, z0);
                    z1 = fma(a.w1[(2 * j + 1) * 9 + t], hv, z1);
                }
                *(double *)(fr + fr_off(fy * P + fx, j >> 1) + (j & 1) * 8) = (z1 > z0) ? z1 : z0;
            }
        }
        ring_store();
        c1_taps_store(tp, wl, tid);
        double bias[2] = {tp.bias[0], tp.bias[1]};
        __syncthreads();

        double dl = 0.0;
        int dneg = 0;
        for (int l = 2; l <= 2 * K; ++l) {
            const bool conv = l & 1;
            const int wd = w0 + 2 * l, hd = h0 + 2 * l, nl = wd * hd;
            const int ntiles = (nl + 15) >> 4;
            const uint32_t mul = ((1u << 20) + wd - 1) / wd;
            auto frame_of = [&](int p) {   // frame site of position p of R_l
                const int v = (int)(((uint32_t)p * mul) >> 20);
                return (F - l + v) * P + (F - l + p - v * wd);
            };
            // last layer: the base sums of this thread's sites of R_2K (loads
            // issued before the matrix work)
            double bsum = 0.0;
            int bneg = 0;
            if (l == 2 * K) {
                const double *slog = a.cache + (int64_t)(2 * K - 1) * a.B * N * kMC + (int64_t)s * N;
                const int *nneg = reinterpret_cast<const int *>(
                                      a.cache + (int64_t)(2 * K - 1) * a.B * N * kMC + a.B * N) +
                                  (int64_t)s * N;
#pragma unroll
                for (int r = 0; r < (676 + kConeThreads - 1) / kConeThreads; ++r) {
                    const int p = tid + r * kConeThreads;
                    if (p < nl) {
                        const int v = (int)(((uint32_t)p * mul) >> 20);
                        const int site = site_of(F - l + p - v * wd, F - l + v);
                        bsum += slog[site];
                        bneg += nneg[site];
                    }
                }
            }
            double st[kConeStage][4];
            // the result of this wave's j-th tile (ti = wave + 8 j): staged, or
            // on the last layer its log|u'| and negative neurons
            auto take = [&](int j, int ti, const double (&out)[4]) {
                if (l < 2 * K) {
#pragma unroll
                    for (int jj = 0; jj < kConeStage; ++jj)
                        if (jj == j)
#pragma unroll
                            for (int i = 0; i < 4; ++i) st[jj][i] = out[i];
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (ti * 16 + kq + 4 * i >= nl) continue;
                        dl += log(fabs(out[i]));
                        dneg += out[i] < 0.0;
                    }
                }
            };
            int j = 0;
            for (int ti = wave; ti < ntiles; ti += kConeNW, ++j) {
                const int fm = frame_of(min(ti * 16 + m16, nl - 1));
                double4_t acc[2];
                double out[4];
                if (conv) {
                    c1_tile<2>(fr, wl, fm, P, lane, bias, acc);
#pragma unroll
                    for (int i = 0; i < 4; ++i) out[i] = (acc[1][i] > acc[0][i]) ? acc[1][i] : acc[0][i];
                } else {
                    c1_tile<1>(fr, wl, fm, P, lane, bias, acc);
#pragma unroll
                    for (int i = 0; i < 4; ++i) out[i] = acc[0][i];
                }
                take(j, ti, out);
            }
            if (l == 2 * K) {
                dl -= bsum;
                dneg -= bneg;
                break;
            }
            // this wave's tiles are done: the ring of W_{l+1} and the next
            // layer's taps on their way while the other waves finish
            ring_fetch(l);
            c1_taps_fetch(tp, a.wpack, l + 1, tid, m16);
            __syncthreads();                 // every read of the frame and taps for layer l is done
            j = 0;
            for (int ti = wave; ti < ntiles; ti += kConeNW, ++j) {
#pragma unroll
                for (int jj = 0; jj < kConeStage; ++jj)
                    if (jj == j)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int p = ti * 16 + kq + 4 * i;
                            if (p < nl)
                                *(double *)(fr + fr_off(frame_of(p), m16 >> 1) + (m16 & 1) * 8) =
                                    st[jj][i];
                        }
            }
            ring_store();
            c1_taps_store(tp, wl, tid);
            bias[0] = tp.bias[0];
            bias[1] = tp.bias[1];
            __syncthreads();
        }
        // fixed-order sums over the lanes, then over the waves
        for (int off = 32; off > 0; off >>= 1) {
            dl += __shfl_xor(dl, off);
            dneg += __shfl_xor(dneg, off);
        }
        if (lane == 0) {
            red[wave] = dl;
            nred[wave] = dneg;
        }
        __syncthreads();
        if (tid == 0) {
            double v = 0.0;
            int n = 0;
            for (int w = 0; w < kConeNW; ++w) {
                v += red[w];
                n += nred[w];
            }
            if (!isfinite(v)) atomicOr(a.err, kErrNonFinite);
            a.dlog[u] = v;
            a.isign[u] = (n & 1) ? (int8_t)-1 : (int8_t)1;
        }
        __syncthreads();                     // red and the frame are free again
    }
}

}  // namespace

int64_t cnn1_params(int Kb, int C)
{
    int64_t p = 0;
    for (int k = 0; k < Kb; ++k)
        p += (int64_t)2 * C * (k == 0 ? 1 : C) * 9 + 2 * C + (int64_t)C * C * 9 + C;
    return p;
}

size_t cnn1_plane_bytes(const nqs_ctx *c, int64_t planes)
{
    return sizeof(double) * (size_t)planes * c->N * c->C;
}

int64_t cnn1_chunk(const nqs_ctx *c, int64_t work)
{
    int64_t m = (int64_t)(((size_t)1 << 30) / cnn1_plane_bytes(c, 1));
    m = std::max<int64_t>(1, std::min<int64_t>(m, 65535));
    return std::min(m, std::max<int64_t>(work, 1));
}

void cnn1_base_forward(const nqs_ctx *c, const int8_t *spins, int B, double *f, int8_t *sgn,
                       int8_t *sign_pub, void *pa, void *pb, hipStream_t s)
{
    if (B <= 0) return;
    const C1Planes pm{nullptr, 0, nullptr};
    blocks_forward(c, spins, pm, B, (double *)pa, (double *)pb, s);
    NQS_LAUNCH(k_c1_final, dim3(B), dim3(kThreads), 0, s, pm, (int64_t)B, c->N * c->C,
               (const double *)pa, f, sgn, sign_pub, (const double *)nullptr,
               (const int8_t *)nullptr, c->err);
}

void cnn1_conn_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                       const int64_t *qlen, int64_t q0, int64_t M, const double *fbase,
                       const int8_t *sbase, double *dlog, int8_t *isign, void *pa, void *pb,
                       hipStream_t s)
{
    if (M <= 0) return;
    const C1Planes pm{queue, q0, qlen};
    blocks_forward(c, spins, pm, M, (double *)pa, (double *)pb, s);
    NQS_LAUNCH(k_c1_final, dim3((unsigned)M), dim3(kThreads), 0, s, pm, M, c->N * c->C,
               (const double *)pa, dlog + q0, isign + q0, (int8_t *)nullptr, fbase, sbase,
               c->err);
}

bool cnn1_cone_ok(const nqs_ctx *c)
{
    return c->net == kNetCnn1 && c->C == kMC && c->K >= 1 && c->K <= kConeMaxK &&
           c->L >= 4 * c->K + 4;
}

// stencils 1 .. 2K-1 [2K-1][B][N][16], then slog [B][N] FP64, nneg [B][N] int32
size_t cnn1_cache_bytes(const nqs_ctx *c, int64_t B)
{
    const size_t bn = (size_t)B * c->N;
    return sizeof(double) * ((size_t)(2 * c->K - 1) * bn * kMC + bn) + sizeof(int) * bn;
}

void cnn1_base_forward_cached(const nqs_ctx *c, const int8_t *spins, int nb, double *f,
                              int8_t *sgn, void *pa, void *pb, double *cache, int64_t B,
                              int64_t b0, hipStream_t s)
{
    if (nb <= 0) return;
    const C1Planes pm{nullptr, 0, nullptr};
    const size_t plane = (size_t)c->N * kMC, bytes = sizeof(double) * plane * nb;
    double *u = (double *)pa, *m = (double *)pb;
    for (int k = 0; k < c->K; ++k) {
        block_forward(c, k, spins, pm, nb, k == 0 ? nullptr : u, m, u, nullptr, s);
        (void)hipMemcpyAsync(cache + ((size_t)(2 * k) * B + b0) * plane, m, bytes,
                             hipMemcpyDeviceToDevice, s);
        if (k + 1 < c->K)
            (void)hipMemcpyAsync(cache + ((size_t)(2 * k + 1) * B + b0) * plane, u, bytes,
                                 hipMemcpyDeviceToDevice, s);
    }
    // the last layer: per-site sums of log|u| and negative counts
    double *slog = cache + (size_t)(2 * c->K - 1) * B * plane;
    int *nneg = reinterpret_cast<int *>(slog + (size_t)B * c->N);
    const int64_t sites = (int64_t)nb * c->N;
    NQS_LAUNCH(k_c1_site_sums, dim3(grid_of(c, sites)), dim3(kThreads), 0, s, (const double *)u,
               sites, slog + (size_t)b0 * c->N, nneg + (size_t)b0 * c->N);
    NQS_LAUNCH(k_c1_final, dim3(nb), dim3(kThreads), 0, s, pm, (int64_t)nb, c->N * c->C,
               (const double *)u, f, sgn, (int8_t *)nullptr, (const double *)nullptr,
               (const int8_t *)nullptr, c->err);
}

void cnn1_cone_forward(const nqs_ctx *c, const int8_t *spins, int64_t B, const uint32_t *queue,
                       const int64_t *qlen, int64_t cap, const double *cache, double *dlog,
                       int8_t *isign, hipStream_t s)
{
    if (cap <= 0) return;
    const C1ConeArgs a{spins, queue, qlen,     cap,   c->w_vec64, c->w_canon,
                       cache,  B,     dlog,     isign, c->err,     c->L,
                       c->K};
    const int P = 4 * c->K + 4;
    const size_t lds = (size_t)P * P * 128 + sizeof(double) * kConvK;   // frame, taps
    (void)hipFuncSetAttribute((const void *)k_c1_cone, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    // one workgroup of twelve waves per CU (LDS); a multiple of 8 for the XCD
    // ranges
    const int grid = std::max(8, c->n_cu / 8 * 8);
    NQS_LAUNCH(k_c1_cone, dim3(grid), dim3(kConeThreads), lds, s, a);
}

size_t cnn1_packed_doubles(const nqs_ctx *c)
{
    return mfma_blocks(c) ? (size_t)(fwd_pack_size(c->K) + (int64_t)c->K * kConvT +
                                     (int64_t)(c->K - 1) * kConvK)
                          : 0;
}

void cnn1_pack_device(const nqs_ctx *c, hipStream_t s)
{
    if (!mfma_blocks(c)) return;
    const int64_t n = (int64_t)cnn1_packed_doubles(c);
    NQS_LAUNCH(k_c1_pack, dim3(grid_of(c, n)), dim3(kThreads), 0, s,
               (const double *)c->w_canon, c->K, c->w_vec64);
}

size_t cnn1_deriv_bytes_per_sample(const nqs_ctx *c)
{
    // saved z (K * 2C), saved u (K * C), pooled m, g, gh (C each), gz (2C)
    return sizeof(double) * (size_t)c->N * c->C * (3 * (size_t)c->K + 5);
}

void cnn1_deriv_planes(const nqs_ctx *c, int *zp, int *hp, int *wp)
{
    *zp = 2 * c->K;      // z of every block (2C channels)
    *hp = c->K;          // u of every block
    *wp = 5;             // m, g, gh, gz (2C)
}

void cnn1_deriv_rows(const nqs_ctx *c, const int8_t *spins, int nb, double *zsave,
                     double *usave, double *work, void *O, nqs_dtype odt, hipStream_t s)
{
    const int L = c->L, C = c->C, N = c->N, K = c->K;
    const int64_t plane = (int64_t)nb * N * C;
    double *mbuf = work, *g = work + plane, *gh = work + 2 * plane, *gz = work + 3 * plane;
    const C1Planes pm{nullptr, 0, nullptr};
    const double *w = c->w_canon;
    // forward with every block's z and u kept
    for (int k = 0; k < K; ++k)
        block_forward(c, k, spins, pm, nb, k == 0 ? nullptr : usave + (int64_t)(k - 1) * plane,
                      mbuf, usave + (int64_t)k * plane, zsave + (int64_t)k * 2 * plane, s);
    NQS_LAUNCH(k_c1_ginit, dim3(grid_of(c, plane)), dim3(kThreads), 0, s,
               (const double *)(usave + (int64_t)(K - 1) * plane), plane, g);
    for (int k = K - 1; k >= 0; --k) {
        const Cnn1Block o = block_of(C, k);
        const double *zk = zsave + (int64_t)k * 2 * plane;
        const double *hk = k == 0 ? nullptr : usave + (int64_t)(k - 1) * plane;
        const int64_t wt = (int64_t)nb * (C * C * 9 + C);
        const int64_t wc = (int64_t)nb * (2 * C * o.cin * 9 + 2 * C);
        const dim3 gmm((unsigned)(((int64_t)nb * 3 + kThreads / 64 - 1) / (kThreads / 64)));
        if (mfma_blocks(c)) {
            if (odt == NQS_FP32)
                NQS_LAUNCH((k_c1_wgrad_mma<float, true>), gmm, dim3(kThreads), 0, s, nb, L,
                           (const double *)g, zk, o.V, o.v, c->P, (float *)O);
            else
                NQS_LAUNCH((k_c1_wgrad_mma<double, true>), gmm, dim3(kThreads), 0, s, nb, L,
                           (const double *)g, zk, o.V, o.v, c->P, (double *)O);
        } else if (odt == NQS_FP32) {
            NQS_LAUNCH(k_c1_wgrad<float>, dim3(grid_of(c, wt)), dim3(kThreads), 0, s, nb, L, C,
                       1, C, C, (const double *)g, zk, (const double *)nullptr, spins, o.V, o.v,
                       c->P, (float *)O);
        } else {
            NQS_LAUNCH(k_c1_wgrad<double>, dim3(grid_of(c, wt)), dim3(kThreads), 0, s, nb, L, C,
                       1, C, C, (const double *)g, zk, (const double *)nullptr, spins, o.V, o.v,
                       c->P, (double *)O);
        }
        if (mfma_blocks(c)) {
            // dL/dm = V-convolution of g on the matrix cores (into mbuf), then the max
            f64mma_cnn1_plain(c, g, nb, kMC, c->w_vec64 + bwd_gm_off(K, k), mbuf, s);
            NQS_LAUNCH(k_c1_route, dim3(grid_of(c, plane)), dim3(kThreads), 0, s, plane, C,
                       (const double *)mbuf, zk, gz);
        } else {
            NQS_LAUNCH(k_c1_gmax, dim3(grid_of(c, plane)), dim3(kThreads), 0, s, nb, L, C,
                       (const double *)g, w + o.V, zk, gz);
        }
        if (mfma_blocks(c) && k > 0) {
            if (odt == NQS_FP32)
                NQS_LAUNCH((k_c1_wgrad_mma<float, false>), gmm, dim3(kThreads), 0, s, nb, L,
                           (const double *)gz, hk, o.W, o.a, c->P, (float *)O);
            else
                NQS_LAUNCH((k_c1_wgrad_mma<double, false>), gmm, dim3(kThreads), 0, s, nb, L,
                           (const double *)gz, hk, o.W, o.a, c->P, (double *)O);
        } else if (odt == NQS_FP32) {
            NQS_LAUNCH(k_c1_wgrad<float>, dim3(grid_of(c, wc)), dim3(kThreads), 0, s, nb, L, C,
                       0, 2 * C, o.cin, (const double *)gz, (const double *)nullptr, hk, spins,
                       o.W, o.a, c->P, (float *)O);
        } else {
            NQS_LAUNCH(k_c1_wgrad<double>, dim3(grid_of(c, wc)), dim3(kThreads), 0, s, nb, L, C,
                       0, 2 * C, o.cin, (const double *)gz, (const double *)nullptr, hk, spins,
                       o.W, o.a, c->P, (double *)O);
        }
        if (k > 0) {
            if (mfma_blocks(c))
                f64mma_cnn1_plain(c, gz, nb, 2 * kMC, c->w_vec64 + bwd_gd_off(K, k), gh, s);
            else
                NQS_LAUNCH(k_c1_gdata, dim3(grid_of(c, plane)), dim3(kThreads), 0, s, nb, L, C,
                           (const double *)gz, w + o.W, gh);
            std::swap(g, gh);
        }
    }
}

}  // namespace nqs
