// k_cnn2.hip -- the CNN2 network family [Sec. 5.2: CNN1's building block
// behind an embedding of the site states, the max-pooling taken at stride
// one with the first neurons copied after the last, a final convolution to
// one channel, and the product of its neurons as the wave-function
// coefficient], in FP64, for the t-J model [Sec. 6.1].
//
// The block figure is not available, so the network is read as
//   h0[p][c] = E[e(s_p)][c]       e = 0 hole, 1 up, 2 down   (C channels)
//   z = a + W (*) h               3x3 circular convolution C -> C
//   m[c] = max(z[c], z[(c+1) mod C])      window 2, stride 1 over channels
//   u = v + V (*)^T m             3x3 circular transposed convolution C -> C,
//                                 u[co][p] = v[co] + sum V[ci][co][t] m[ci][p - off t]
//   y[p] = b + sum F[c][t] u_K[p + off t][c]                 (one channel)
// log|psi_net| = sum_p log|y_p| and sign(psi_net) = prod_p sign(y_p).
// Canonical parameter order: E[3][C]; per block W[C][C][3][3], a[C],
// V[C][C][3][3] (input channel first), v[C]; then F[C][3][3], b.
//
// C is 16 or 32: every convolution of the blocks runs on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64, k_conv_f64mma.hip) -- the convolution with
// the stride-one channel max in its epilogue (the neighbouring channel is one
// lane over, read with a cross-lane shuffle), the transposed convolution as a
// convolution with flipped, transposed taps, and in the backward both data
// gradients and all weight gradients.  The embedding, the final one-channel
// convolution with its log|y| reduction, the max's gradient routing and the
// embedding's gradient run on the vector ALU.  Every reduction has a fixed
// order, so the base and the exchanged configurations run identical
// arithmetic and rows of O are deterministic.
//
// Packing, built on the device from the canonical vector, per block k
// (kPackBlock doubles):
//   [9][C][C] convolution taps W[co][ci][t] read as [t][ci][co], a[C],
//   [9][C][C] transposed taps V[ci][co][8 - t] read as [t][ci][co], v[C],
//   [9][C][C] taps of the gradient through V: V[ci][co][t] read as [t][co][ci],
//   [9][C][C] taps of the gradient through W: W[co][ci][8 - t] read as [t][co][ci].
// Planes are NHWC ([plane][site][channel]) in HBM.
#include <algorithm>

#include "nqs_internal.h"

namespace nqs {
namespace {

constexpr int kThreads = 256;

__device__ inline int wrap2(int a, int L) { return a < 0 ? a + L : (a >= L ? a - L : a); }

__host__ __device__ inline int64_t pack_block(int C) { return 36 * (int64_t)C * C + 2 * C; }
__host__ __device__ inline int64_t canon_W(int C, int k)
{
    return 3 * (int64_t)C + (int64_t)k * (18 * (int64_t)C * C + 2 * C);
}
__host__ __device__ inline int64_t canon_F(int C, int Kb) { return canon_W(C, Kb); }

// planes of a launch: samples (queue null) or queue items q_begin + m
struct C2Planes {
    const uint32_t *queue;
    int64_t q_begin;
    const int64_t *qlen;
};

__device__ inline int64_t c2_live(const C2Planes &pm, int64_t M)
{
    if (!pm.queue) return M;
    const int64_t left = pm.qlen[0] - pm.q_begin;
    return left < 0 ? 0 : (left < M ? left : M);
}

// sample of plane m and the exchanged pair (-1, -1 for a sample plane)
__device__ inline void c2_origin(const C2Planes &pm, int64_t m, int L, int *s, int *qi, int *qj)
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
    *qj = wrap2(y + bond_dy(t), L) * L + wrap2(x + bond_dx(t), L);
}

__device__ inline int state_row(int8_t v) { return v == 0 ? 0 : (v > 0 ? 1 : 2); }

// h0[m][p][c] = E[e(s'_p)][c], s' the plane's configuration (the pair
// exchanged for a queue item)
__global__ void __launch_bounds__(kThreads)
k_c2_embed(const int8_t *__restrict__ spins, C2Planes pm, int64_t M, int L, int C,
           const double *__restrict__ E, double *__restrict__ out)
{
    const int N = L * L;
    const int64_t total = c2_live(pm, M) * N * C;
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * kThreads) {
        const int c = (int)(g % C);
        const int64_t mp = g / C;
        const int64_t m = mp / N;
        int p = (int)(mp - m * N);
        int s, qi, qj;
        c2_origin(pm, m, L, &s, &qi, &qj);
        p = (p == qi) ? qj : ((p == qj) ? qi : p);
        out[g] = E[state_row(spins[(int64_t)s * N + p]) * C + c];
    }
}

// Per plane: y[p] = b + sum_{t,c} F[c][t] u[p + off t][c] (bias, then taps
// 0..8, channels in order), f = sum log|y| (fixed reduction tree) and the
// parity of the negative y.  Sample planes write f and the network sign (and
// multiply it into sign_pub when given) or, with yout, keep y; item planes
// write dlog = f' - f(sample) and the sign ratio.  F [C][9] and b sit in LDS.
__global__ void __launch_bounds__(kThreads)
k_c2_final(C2Planes pm, int64_t M, int L, int C, const double *__restrict__ u,
           const double *__restrict__ Fw, double *__restrict__ f, int8_t *__restrict__ sgn,
           int8_t *__restrict__ sign_pub, const double *__restrict__ fbase,
           const int8_t *__restrict__ sbase, double *__restrict__ yout, int32_t *err)
{
    __shared__ double fs[9 * 32 + 1];
    __shared__ double red[kThreads];
    __shared__ int neg[kThreads];
    for (int q = threadIdx.x; q <= 9 * C; q += kThreads) fs[q] = Fw[q];
    __syncthreads();
    const int64_t m = blockIdx.x;
    if (m >= c2_live(pm, M)) return;
    const int N = L * L;
    const double *um = u + m * (int64_t)N * C;
    double acc = 0.0;
    int n = 0;
    for (int p = threadIdx.x; p < N; p += kThreads) {
        const int x = p % L, y = p / L;
        double yv = fs[9 * C];
        for (int t = 0; t < 9; ++t) {
            const int q = wrap2(y + t / 3 - 1, L) * L + wrap2(x + t % 3 - 1, L);
            const double *uq = um + (int64_t)q * C;
            for (int c = 0; c < C; ++c) yv = fma(fs[c * 9 + t], uq[c], yv);
        }
        if (yout) yout[m * N + p] = yv;
        acc += log(fabs(yv));
        n += (yv < 0.0);
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
            if (f) f[m] = fm;
            if (sgn) sgn[m] = sm;
            if (sign_pub) sign_pub[m] = (int8_t)(sign_pub[m] * sm);
        } else {
            const int s = item_sample(pm.queue[pm.q_begin + m]);
            f[m] = fm - fbase[s];
            sgn[m] = (int8_t)(sm * sbase[s]);
        }
    }
}

// ---- backward ----

// Final convolution's parameter gradients per sample, with g_y = 1 / y:
//   O[F + c 9 + t] = sum_p g_y[p] u[p + off t][c],  O[F + 9C] = sum_p g_y[p].
template <typename OT>
__global__ void __launch_bounds__(kThreads)
k_c2_final_wgrad(int nb, int L, int C, const double *__restrict__ yv,
                 const double *__restrict__ u, int64_t offF, int64_t P, OT *__restrict__ O)
{
    const int N = L * L;
    const int per = 9 * C + 1;
    const int64_t total = (int64_t)nb * per;
    for (int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * kThreads) {
        const int b = (int)(id / per);
        const int r = (int)(id - (int64_t)b * per);
        const double *yb = yv + (int64_t)b * N;
        double acc = 0.0;
        if (r == 9 * C) {
            for (int p = 0; p < N; ++p) acc += 1.0 / yb[p];
        } else {
            const int c = r / 9, t = r % 9, dy = t / 3 - 1, dx = t % 3 - 1;
            const double *ub = u + (int64_t)b * N * C;
            for (int p = 0; p < N; ++p) {
                const int q = wrap2(p / L + dy, L) * L + wrap2(p % L + dx, L);
                acc = fma(1.0 / yb[p], ub[(int64_t)q * C + c], acc);
            }
        }
        O[(int64_t)b * P + offF + r] = (OT)acc;
    }
}

// dL/du_K[q][c] = sum_t F[c][t] / y[q - off t]
__global__ void __launch_bounds__(kThreads)
k_c2_final_gdata(int nb, int L, int C, const double *__restrict__ yv,
                 const double *__restrict__ Fw, double *__restrict__ g)
{
    const int N = L * L;
    const int64_t total = (int64_t)nb * N * C;
    for (int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * kThreads) {
        const int c = (int)(id % C);
        const int64_t bq = id / C;
        const int64_t b = bq / N;
        const int q = (int)(bq - b * N);
        const int x = q % L, y = q / L;
        double acc = 0.0;
        for (int t = 0; t < 9; ++t) {
            const int p = wrap2(y - t / 3 + 1, L) * L + wrap2(x - t % 3 + 1, L);
            acc = fma(Fw[c * 9 + t], 1.0 / yv[b * N + p], acc);
        }
        g[id] = acc;
    }
}

// the stride-one max's routing of dL/dm into dL/dz: z[c] is the first input
// of m[c] (taken unless z[c+1] is larger) and the second of m[c-1] (taken
// when larger than z[c-1])
__global__ void __launch_bounds__(kThreads)
k_c2_route(int64_t n, int C, const double *__restrict__ gm, const double *__restrict__ z,
           double *__restrict__ gz)
{
    for (int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x; id < n;
         id += (int64_t)gridDim.x * kThreads) {
        const int c = (int)(id % C);
        const int64_t base = id - c;
        const int cn = c + 1 == C ? 0 : c + 1, cp = c == 0 ? C - 1 : c - 1;
        const double zc = z[id];
        double g = 0.0;
        if (!(z[base + cn] > zc)) g += gm[id];
        if (zc > z[base + cp]) g += gm[base + cp];
        gz[id] = g;
    }
}

// embedding rows: O[e C + c] = sum over the sites p in state e of g[p][c]
template <typename OT>
__global__ void __launch_bounds__(kThreads)
k_c2_embed_grad(int nb, int L, int C, const int8_t *__restrict__ spins,
                const double *__restrict__ g, int64_t P, OT *__restrict__ O)
{
    const int N = L * L;
    const int64_t total = (int64_t)nb * 3 * C;
    for (int64_t id = (int64_t)blockIdx.x * kThreads + threadIdx.x; id < total;
         id += (int64_t)gridDim.x * kThreads) {
        const int b = (int)(id / (3 * C));
        const int r = (int)(id - (int64_t)b * 3 * C);
        const int e = r / C, c = r % C;
        const int8_t *sb = spins + (int64_t)b * N;
        const double *gb = g + (int64_t)b * N * C;
        double acc = 0.0;
        for (int p = 0; p < N; ++p)
            if (state_row(sb[p]) == e) acc += gb[(int64_t)p * C + c];
        O[(int64_t)b * P + r] = (OT)acc;
    }
}

__global__ void k_c2_pack(const double *__restrict__ w, int Kb, int C, double *__restrict__ out)
{
    const int64_t per = pack_block(C), CC9 = 9 * (int64_t)C * C;
    const int64_t n = (int64_t)Kb * per;
    for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kThreads) {
        const int k = (int)(q / per);
        int64_t r = q - (int64_t)k * per;
        const int64_t W = canon_W(C, k), a = W + CC9, V = a + C, v = V + CC9;
        double val;
        if (r < CC9) {                         // [t][ci][co] = W[co][ci][t]
            const int co = (int)(r % C), ci = (int)((r / C) % C), t = (int)(r / (C * C));
            val = w[W + ((int64_t)co * C + ci) * 9 + t];
        } else if ((r -= CC9) < C) {
            val = w[a + r];
        } else if ((r -= C) < CC9) {           // [t][ci][co] = V[ci][co][8 - t]
            const int co = (int)(r % C), ci = (int)((r / C) % C), t = (int)(r / (C * C));
            val = w[V + ((int64_t)ci * C + co) * 9 + (8 - t)];
        } else if ((r -= CC9) < C) {
            val = w[v + r];
        } else if ((r -= C) < CC9) {           // [t][co][ci] = V[ci][co][t]
            const int ci = (int)(r % C), co = (int)((r / C) % C), t = (int)(r / (C * C));
            val = w[V + ((int64_t)ci * C + co) * 9 + t];
        } else {                               // [t][co][ci] = W[co][ci][8 - t]
            r -= CC9;
            const int ci = (int)(r % C), co = (int)((r / C) % C), t = (int)(r / (C * C));
            val = w[W + ((int64_t)co * C + ci) * 9 + (8 - t)];
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

// packed pieces of block k
struct Packed {
    const double *conv, *a, *convt, *v, *gm, *gd;
};

Packed packed(const nqs_ctx *c, int k)
{
    const int C = c->C;
    const int64_t CC9 = 9 * (int64_t)C * C;
    const double *b = c->w_vec64 + (int64_t)k * pack_block(C);
    return Packed{b, b + CC9, b + CC9 + C, b + 2 * CC9 + C, b + 2 * CC9 + 2 * C,
                  b + 3 * CC9 + 2 * C};
}

// the blocks over M planes from the embedding: h (h0, then each block's u),
// m, z: per block the convolution with the max (m, and z when zsave) and the
// transposed convolution (u).  With saves (the backward), h0 / m_k / z_k /
// u_k go to their own planes; otherwise u ends in pa and pb holds m.
void blocks_forward(const nqs_ctx *c, const int8_t *spins, C2Planes pm, int64_t M, double *pa,
                    double *pb, double *zsave, double *msave, double *hsave, hipStream_t s)
{
    const int C = c->C, L = c->L;
    const int64_t plane = M * c->N * C;
    double *h0 = hsave ? hsave : pa;
    NQS_LAUNCH(k_c2_embed, dim3(grid_of(c, plane)), dim3(kThreads), 0, s, spins, pm, M, L, C,
               (const double *)c->w_canon, h0);
    for (int k = 0; k < c->K; ++k) {
        const Packed pk = packed(c, k);
        const double *h = hsave ? hsave + (int64_t)k * plane : pa;
        double *m = msave ? msave + (int64_t)2 * k * plane : pb;
        double *z = zsave ? zsave + (int64_t)2 * k * plane : nullptr;
        double *u = hsave ? hsave + (int64_t)(k + 1) * plane : pa;
        f64mma_cnn2_conv(c, h, M, pk.conv, pk.a, m, z, pm.qlen, pm.q_begin, s);
        f64mma_linear(c, m, M, C, C, pk.convt, pk.v, u, pm.qlen, pm.q_begin, s);
    }
}

}  // namespace

bool cnn2_supported(int Kb, int C) { return Kb >= 1 && (C == 16 || C == 32); }

int64_t cnn2_params(int Kb, int C)
{
    return 3 * (int64_t)C + (int64_t)Kb * (18 * (int64_t)C * C + 2 * C) + 9 * (int64_t)C + 1;
}

size_t cnn2_plane_bytes(const nqs_ctx *c, int64_t planes)
{
    return sizeof(double) * (size_t)planes * c->N * c->C;
}

int64_t cnn2_chunk(const nqs_ctx *c, int64_t work)
{
    int64_t m = (int64_t)(((size_t)1 << 30) / cnn2_plane_bytes(c, 1));
    m = std::max<int64_t>(1, std::min<int64_t>(m, 65535));
    return std::min(m, std::max<int64_t>(work, 1));
}

void cnn2_base_forward(const nqs_ctx *c, const int8_t *spins, int B, double *f, int8_t *sgn,
                       int8_t *sign_pub, void *pa, void *pb, hipStream_t s)
{
    if (B <= 0) return;
    const C2Planes pm{nullptr, 0, nullptr};
    blocks_forward(c, spins, pm, B, (double *)pa, (double *)pb, nullptr, nullptr, nullptr, s);
    NQS_LAUNCH(k_c2_final, dim3(B), dim3(kThreads), 0, s, pm, (int64_t)B, c->L, c->C,
               (const double *)pa, (const double *)c->w_canon + canon_F(c->C, c->K), f, sgn,
               sign_pub, (const double *)nullptr, (const int8_t *)nullptr, (double *)nullptr,
               c->err);
}

void cnn2_conn_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                       const int64_t *qlen, int64_t q0, int64_t M, const double *fbase,
                       const int8_t *sbase, double *dlog, int8_t *isign, void *pa, void *pb,
                       hipStream_t s)
{
    if (M <= 0) return;
    const C2Planes pm{queue, q0, qlen};
    blocks_forward(c, spins, pm, M, (double *)pa, (double *)pb, nullptr, nullptr, nullptr, s);
    NQS_LAUNCH(k_c2_final, dim3((unsigned)M), dim3(kThreads), 0, s, pm, M, c->L, c->C,
               (const double *)pa, (const double *)c->w_canon + canon_F(c->C, c->K), dlog + q0,
               isign + q0, (int8_t *)nullptr, fbase, sbase, (double *)nullptr, c->err);
}

size_t cnn2_packed_doubles(const nqs_ctx *c) { return (size_t)c->K * pack_block(c->C); }

void cnn2_pack_device(const nqs_ctx *c, hipStream_t s)
{
    const int64_t n = (int64_t)cnn2_packed_doubles(c);
    NQS_LAUNCH(k_c2_pack, dim3(grid_of(c, n)), dim3(kThreads), 0, s, (const double *)c->w_canon,
               c->K, c->C, c->w_vec64);
}

void cnn2_deriv_planes(const nqs_ctx *c, int *zp, int *hp, int *wp)
{
    *zp = 2 * c->K;      // z and m of every block
    *hp = c->K + 1;      // h0 and u of every block
    *wp = 4;             // g, dL/dm, dL/dz, y
}

void cnn2_deriv_rows(const nqs_ctx *c, const int8_t *spins, int nb, double *zsave,
                     double *hsave, double *work, void *O, nqs_dtype odt, hipStream_t s)
{
    const int L = c->L, C = c->C, N = c->N, K = c->K;
    const int64_t plane = (int64_t)nb * N * C;
    double *g = work, *gm = work + plane, *gz = work + 2 * plane, *yv = work + 3 * plane;
    const C2Planes pm{nullptr, 0, nullptr};
    // forward with h0, every block's z, m and u kept (m_k right after z_k)
    blocks_forward(c, spins, pm, nb, nullptr, nullptr, zsave, zsave + plane, hsave, s);
    const double *Fw = (const double *)c->w_canon + canon_F(C, K);
    NQS_LAUNCH(k_c2_final, dim3((unsigned)nb), dim3(kThreads), 0, s, pm, (int64_t)nb, L, C,
               (const double *)(hsave + (int64_t)K * plane), Fw, (double *)nullptr,
               (int8_t *)nullptr, (int8_t *)nullptr, (const double *)nullptr,
               (const int8_t *)nullptr, yv, c->err);
    const int64_t nf = (int64_t)nb * (9 * C + 1);
    if (odt == NQS_FP32)
        NQS_LAUNCH(k_c2_final_wgrad<float>, dim3(grid_of(c, nf)), dim3(kThreads), 0, s, nb, L, C,
                   (const double *)yv, (const double *)(hsave + (int64_t)K * plane),
                   canon_F(C, K), c->P, (float *)O);
    else
        NQS_LAUNCH(k_c2_final_wgrad<double>, dim3(grid_of(c, nf)), dim3(kThreads), 0, s, nb, L,
                   C, (const double *)yv, (const double *)(hsave + (int64_t)K * plane),
                   canon_F(C, K), c->P, (double *)O);
    NQS_LAUNCH(k_c2_final_gdata, dim3(grid_of(c, plane)), dim3(kThreads), 0, s, nb, L, C,
               (const double *)yv, Fw, g);
    for (int k = K - 1; k >= 0; --k) {
        const Packed pk = packed(c, k);
        const double *zk = zsave + (int64_t)2 * k * plane;
        const double *mk = zk + plane;
        const double *hk = hsave + (int64_t)k * plane;
        const int64_t W = canon_W(C, k), V = W + 9 * (int64_t)C * C + C;
        // the transposed convolution: dV, dv, then dL/dm through V
        f64mma_wgrad(c, mk, g, nb, V, O, odt, s, true);
        f64mma_linear(c, g, nb, C, C, pk.gm, nullptr, gm, nullptr, 0, s);
        NQS_LAUNCH(k_c2_route, dim3(grid_of(c, plane)), dim3(kThreads), 0, s, plane, C,
                   (const double *)gm, zk, gz);
        // the convolution: dW, da, then dL/dh through W into g
        f64mma_wgrad(c, hk, gz, nb, W, O, odt, s, false);
        f64mma_linear(c, gz, nb, C, C, pk.gd, nullptr, g, nullptr, 0, s);
    }
    const int64_t ne = (int64_t)nb * 3 * C;
    if (odt == NQS_FP32)
        NQS_LAUNCH(k_c2_embed_grad<float>, dim3(grid_of(c, ne)), dim3(kThreads), 0, s, nb, L, C,
                   spins, (const double *)g, c->P, (float *)O);
    else
        NQS_LAUNCH(k_c2_embed_grad<double>, dim3(grid_of(c, ne)), dim3(kThreads), 0, s, nb, L, C,
                   spins, (const double *)g, c->P, (double *)O);
}

}  // namespace nqs
