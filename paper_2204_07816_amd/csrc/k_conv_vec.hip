// k_conv_vec.hip -- vector-ALU (FP64 / FP32) network kernels: the plain form
// of the CNN log-amplitude [Sec. 5.2: periodic 3x3 convolutions, log of a
// product of neurons] evaluated by full recomputation for every exchanged
// configuration [Sec. 5.4.1], and the hand-written backward pass that gives
// the per-sample log-derivatives O_k [Sec. 3.2].
//
// Work is organised layer by layer over a batch of "planes" (one plane per
// sample or per exchanged configuration) resident in HBM, NHWC layout
// ([plane][site][channel], channel fastest).  Each layer kernel keeps the
// layer's weights in LDS ([tap][c_in][c_out]) and lets every thread produce
// CPT output channels of one site, so every activation load feeds CPT FMAs.
// The per-site channel sums of the last layer are taken in FP64; the
// log-ratio of an exchanged configuration is sum_sites (hs'(p) - hs(p)),
// which is exactly zero on sites the exchange does not reach because both
// sides are produced by identical arithmetic.
#include "nqs_internal.h"

namespace nqs {
namespace {

constexpr int kThreads = 256;

__device__ inline int wrapi(int a, int L) { return a < 0 ? a + L : (a >= L ? a - L : a); }

// ln cosh z: FP64 in the shared branch-free form; FP32 with e = expm1(|z|),
// cosh|z| - 1 = e^2 / (2 (1 + e)), so ln cosh z = log1p(e^2 / (2 + 2e)) keeps
// full relative precision at small |z|, and for |z| > 1 the form
// |z| - ln 2 + log1p(exp(-2|z|)) avoids overflow.
__device__ inline double ln_cosh(double z) { return ln_cosh_fwd(z); }
__device__ inline float ln_cosh(float z)
{
    const float a = fabsf(z);
    if (a > 1.0f) return a - 0.693147180559945f + log1pf(expf(-2.0f * a));
    const float e = expm1f(a);
    return log1pf(e * e / (2.0f + 2.0f * e));
}

// Spin of site q in the configuration of a plane: the sample's spins, with
// the pair (qi, qj) exchanged when the plane is an exchanged configuration.
__device__ inline int spin_at(const int8_t *sp, int q, int qi, int qj)
{
    const int src = (q == qi) ? qj : ((q == qj) ? qi : q);
    return sp[src];
}

struct PlaneMap {
    const uint32_t *queue;   // null: plane m is sample m (no exchange)
    int64_t q_begin;
    const int64_t *qlen;     // device queue length (items at or past it are skipped)
};

inline int grid_for(int64_t work, const nqs_ctx *c)
{
    int64_t b = (work + kThreads - 1) / kThreads;
    int64_t cap = (int64_t)c->n_cu * 8;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

// Number of planes of this launch that hold real work.
__device__ inline int64_t live_planes(const PlaneMap &pm, int64_t M)
{
    if (!pm.queue) return M;
    const int64_t left = pm.qlen[0] - pm.q_begin;
    return left < 0 ? 0 : (left < M ? left : M);
}

__device__ inline void plane_origin(const PlaneMap &pm, int64_t m, int L, int *sample, int *qi,
                                    int *qj)
{
    if (!pm.queue) {
        *sample = (int)m;
        *qi = -1;
        *qj = -1;
        return;
    }
    const uint32_t e = pm.queue[pm.q_begin + m];
    const int b = item_bond(e);
    const int i = b >> 2, t = b & 3;
    const int x = i % L, y = i / L;
    *sample = item_sample(e);
    *qi = i;
    *qj = wrapi(y + bond_dy(t), L) * L + wrapi(x + bond_dx(t), L);
}

// Layer 1 (one input channel): out[m][p][co] = g(b[co] + sum_t W1[t][co] s(p + t)).
// W1 packed [9][C] then bias [C].  Each thread produces CPT consecutive
// channels of one site, so a site's spin gathers serve CPT channels and a
// wave's stores cover contiguous memory.
template <typename T, int CPT>
__global__ void __launch_bounds__(kThreads)
k_layer1(const int8_t *__restrict__ spins, PlaneMap pm, int64_t M, int L, int C,
         const T *__restrict__ w1, T *__restrict__ out, double *__restrict__ zsave)
{
    extern __shared__ unsigned char smem_raw[];
    T *w = reinterpret_cast<T *>(smem_raw);
    for (int q = threadIdx.x; q < 10 * C; q += kThreads) w[q] = w1[q];
    __syncthreads();
    const int N = L * L;
    const int groups = C / CPT;
    const int64_t total = live_planes(pm, M) * N * groups;
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * kThreads) {
        const int64_t mp = g / groups;
        const int co0 = (int)(g - mp * groups) * CPT;
        const int64_t m = mp / N;
        const int p = (int)(mp - m * N);
        int s, qi, qj;
        plane_origin(pm, m, L, &s, &qi, &qj);
        const int8_t *sp = spins + (int64_t)s * N;
        const int x = p % L, y = p / L;
        T sv[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = wrapi(y + t / 3 - 1, L), xx = wrapi(x + t % 3 - 1, L);
            sv[t] = (T)spin_at(sp, yy * L + xx, qi, qj);
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int co = co0 + j;
            T z = w[9 * C + co];
#pragma unroll
            for (int t = 0; t < 9; ++t) z = fma(w[t * C + co], sv[t], z);
            if (zsave) {
                double th;
                out[mp * C + co] = (T)ln_cosh_tanh((double)z, &th);
                zsave[mp * C + co] = th;
            } else {
                out[mp * C + co] = ln_cosh(z);
            }
        }
    }
}

template <typename T>
void layer1_launch(const nqs_ctx *c, const int8_t *spins, PlaneMap pm, int64_t M, const T *w1,
                   T *out, double *zsave, hipStream_t s)
{
    const int C = c->C;
    const int64_t sites = M * c->N;
    const size_t lds = sizeof(T) * 10 * C;
    if (C % 8 == 0)
        NQS_LAUNCH((k_layer1<T, 8>), dim3(grid_for(sites * (C / 8), c)), dim3(kThreads), lds, s,
                   spins, pm, M, c->L, C, w1, out, zsave);
    else if (C % 4 == 0)
        NQS_LAUNCH((k_layer1<T, 4>), dim3(grid_for(sites * (C / 4), c)), dim3(kThreads), lds, s,
                   spins, pm, M, c->L, C, w1, out, zsave);
    else
        NQS_LAUNCH((k_layer1<T, 1>), dim3(grid_for(sites * C, c)), dim3(kThreads), lds, s,
                   spins, pm, M, c->L, C, w1, out, zsave);
}

// Layers 2..K and the backward data pass: out[m][p][co] = epi(bias[co] +
// sum_{t, ci} W[t][ci][co] in[m][p + off(t)][ci]).  epi: 0 = ln cosh,
// 1 = ln cosh and save tanh z to zk[m][p][co], 2 = multiply by zk[m][p][co]
// (the saved tanh; no bias), 3 = tanh z (the last layer's delta, d ln cosh z
// / dz).  Saved values are laid out [layer][plane][site][channel].
template <typename T, int CPT>
__global__ void __launch_bounds__(kThreads)
k_layer(const T *__restrict__ in, int64_t M, int L, int Cin, int Cout,
        const T *__restrict__ wl, const T *__restrict__ bias, T *__restrict__ out, int epi,
        double *__restrict__ zk, PlaneMap pm)
{
    extern __shared__ unsigned char smem_raw[];
    T *w = reinterpret_cast<T *>(smem_raw);
    const int nw = 9 * Cin * Cout;
    for (int q = threadIdx.x; q < nw; q += kThreads) w[q] = wl[q];
    __syncthreads();
    const int N = L * L;
    const int groups = Cout / CPT;
    const int64_t total = live_planes(pm, M) * N * groups;
    for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * kThreads) {
        const int cg = (int)(g % groups);
        const int64_t mp = g / groups;
        const int64_t m = mp / N;
        const int p = (int)(mp - m * N);
        const int x = p % L, y = p / L;
        const int co0 = cg * CPT;
        T acc[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) acc[j] = bias ? bias[co0 + j] : (T)0;
        const T *inm = in + m * (int64_t)N * Cin;
        for (int t = 0; t < 9; ++t) {
            const int yy = wrapi(y + t / 3 - 1, L), xx = wrapi(x + t % 3 - 1, L);
            const T *src = inm + (int64_t)(yy * L + xx) * Cin;
            const T *wt = w + t * Cin * Cout + co0;
            for (int ci = 0; ci < Cin; ++ci) {
                const T v = src[ci];
#pragma unroll
                for (int j = 0; j < CPT; ++j) acc[j] = fma(wt[ci * Cout + j], v, acc[j]);
            }
        }
        T *o = out + mp * Cout + co0;
        if (epi == 3) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) o[j] = (T)tanh((double)acc[j]);
        } else if (epi == 2) {
            const double *zp = zk + mp * Cout + co0;
#pragma unroll
            for (int j = 0; j < CPT; ++j) o[j] = acc[j] * (T)zp[j];
        } else if (epi == 1) {
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                double th;
                o[j] = (T)ln_cosh_tanh((double)acc[j], &th);
                zk[mp * Cout + co0 + j] = th;
            }
        } else {
#pragma unroll
            for (int j = 0; j < CPT; ++j) o[j] = ln_cosh(acc[j]);
        }
    }
}

// Per-site FP64 channel sums of the last layer, then per plane either
// f = sum_p hs(p) and hsum = hs (samples) or dlog = sum_p (hs(p) - hsum(p))
// (exchanged configurations).  One block per plane, fixed reduction order.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_final(const T *__restrict__ hK, int64_t M, int N, int C, PlaneMap pm, int L,
        double *__restrict__ f, double *__restrict__ hsum_out, const double *__restrict__ hsum_in,
        double *__restrict__ dlog, int32_t *err)
{
    __shared__ double red[kThreads];
    const int64_t m = blockIdx.x;
    if (m >= live_planes(pm, M)) return;
    int s, qi, qj;
    plane_origin(pm, m, L, &s, &qi, &qj);
    double acc = 0.0;
    for (int p = threadIdx.x; p < N; p += kThreads) {
        const T *h = hK + (m * N + p) * C;
        double hs = 0.0;
        for (int c = 0; c < C; ++c) hs += (double)h[c];
        if (pm.queue) {
            acc += hs - hsum_in[(int64_t)s * N + p];
        } else {
            hsum_out[m * N + p] = hs;
            acc += hs;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double v = red[0];
        if (!isfinite(v)) atomicOr(err, kErrNonFinite);
        if (pm.queue)
            dlog[pm.q_begin + m] = v;
        else
            f[m] = v;
    }
}

// Per-sample weight and bias gradients of one layer:
//   dW[co][ci][t] = sum_p delta[p][co] h_in[p + off(t)][ci],  db[co] = sum_p delta[p][co].
// h_in is the spin image (k = 0) or the activations h_{k-1} [B][N][C].
template <typename OT>
__global__ void __launch_bounds__(kThreads)
k_wgrad(const int8_t *__restrict__ spins, const double *__restrict__ hprev,
        const double *__restrict__ delta, int L, int C, int k, int64_t P, int64_t woff,
        OT *__restrict__ O)
{
    const int s = blockIdx.x;
    const int N = L * L;
    const int Cin = (k == 0) ? 1 : C;
    const double *dl = delta + (int64_t)s * N * C;
    const double *zp = (k == 0) ? nullptr : hprev + (int64_t)s * N * C;
    const int8_t *sp = spins + (int64_t)s * N;
    OT *o = O + (int64_t)s * P + woff;
    const int pairs = C * Cin;
    for (int q = threadIdx.x; q < pairs; q += kThreads) {
        const int co = q / Cin, ci = q % Cin;
        double g[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) g[t] = 0.0;
        for (int p = 0; p < N; ++p) {
            const double d = dl[(int64_t)p * C + co];
            const int x = p % L, y = p / L;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int r = wrapi(y + t / 3 - 1, L) * L + wrapi(x + t % 3 - 1, L);
                const double h = zp ? zp[(int64_t)r * C + ci] : (double)sp[r];
                g[t] = fma(d, h, g[t]);
            }
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) o[(co * Cin + ci) * 9 + t] = (OT)g[t];
    }
    for (int co = threadIdx.x; co < C; co += kThreads) {
        double db = 0.0;
        for (int p = 0; p < N; ++p) db += dl[(int64_t)p * C + co];
        o[C * Cin * 9 + co] = (OT)db;
    }
}

// Layer-1 weight and bias gradients (one input channel), one sample per block:
//   dW1[co][t] = sum_p delta[p][co] s(p + off(t)),  db1[co] = sum_p delta[p][co].
// Thread (part, co) sums the sites p = part (mod nparts); the parts are then
// added in a fixed order, so the result is deterministic.
template <typename OT>
__global__ void __launch_bounds__(kThreads)
k_wgrad1(const int8_t *__restrict__ spins, const double *__restrict__ delta, int L, int C,
         int64_t P, int64_t woff, OT *__restrict__ O)
{
    __shared__ double red[10][kThreads];
    const int s = blockIdx.x, N = L * L;
    const int nparts = kThreads / C;
    const int co = threadIdx.x % C, part = threadIdx.x / C;
    double g[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) g[j] = 0.0;
    if (part < nparts) {
        const double *dl = delta + (int64_t)s * N * C;
        const int8_t *sp = spins + (int64_t)s * N;
        for (int p = part; p < N; p += nparts) {
            const double d = dl[(int64_t)p * C + co];
            const int x = p % L, y = p / L;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int r = wrapi(y + t / 3 - 1, L) * L + wrapi(x + t % 3 - 1, L);
                g[t] = fma(d, (double)sp[r], g[t]);
            }
            g[9] += d;
        }
    }
#pragma unroll
    for (int j = 0; j < 10; ++j) red[j][threadIdx.x] = g[j];
    __syncthreads();
    OT *o = O + (int64_t)s * P + woff;
    for (int q = threadIdx.x; q < 10 * C; q += kThreads) {
        const int c2 = q / 10, j = q - 10 * (q / 10);
        double v = 0.0;
        for (int pt = 0; pt < nparts; ++pt) v += red[j][pt * C + c2];
        if (j < 9)
            o[c2 * 9 + j] = (OT)v;
        else
            o[9 * C + c2] = (OT)v;
    }
}

// delta_K = tanh(z_K)  (d f / d h_K = 1, d ln cosh z / dz = tanh z)
// the last layer's delta when it is layer 1: the saved tanh z
__global__ void k_delta_last(const double *__restrict__ thK, int64_t total,
                             double *__restrict__ delta)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x)
        delta[g] = thK[g];
}

template <typename T>
const T *layer_w(const nqs_ctx *c, int k);
template <>
const double *layer_w<double>(const nqs_ctx *c, int k)
{
    // packing: layer 1 [9][C] + bias[C]; layer k>1 [9][C][C] + bias[C]
    if (k == 0) return c->w_vec64;
    int64_t off = 10 * (int64_t)c->C;
    for (int l = 1; l < k; ++l) off += 9 * (int64_t)c->C * c->C + c->C;
    return c->w_vec64 + off;
}
template <>
const float *layer_w<float>(const nqs_ctx *c, int k)
{
    if (k == 0) return c->w_vec32;
    int64_t off = 10 * (int64_t)c->C;
    for (int l = 1; l < k; ++l) off += 9 * (int64_t)c->C * c->C + c->C;
    return c->w_vec32 + off;
}

template <typename T>
void layer_launch(const nqs_ctx *c, const T *in, int64_t M, int Cin, int Cout, const T *wl,
                  const T *bias, T *out, int epi, double *zk, PlaneMap pm, hipStream_t s)
{
    if constexpr (sizeof(T) == sizeof(double)) {
        if (f64mma_conv_ok(Cin, Cout)) {
            f64mma_conv(c, in, M, Cin, Cout, wl, bias, out, epi, zk, pm.queue ? pm.qlen : nullptr,
                        pm.q_begin, s);
            return;
        }
    }
    const size_t lds = sizeof(T) * 9 * (size_t)Cin * Cout;
    const int N = c->N;
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void *)k_layer<T, 8>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipFuncSetAttribute((const void *)k_layer<T, 4>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipFuncSetAttribute((const void *)k_layer<T, 1>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    if (Cout % 8 == 0) {
        NQS_LAUNCH((k_layer<T, 8>), dim3(grid_for(M * N * (Cout / 8), c)), dim3(kThreads),
                           lds, s, in, M, c->L, Cin, Cout, wl, bias, out, epi, zk, pm);
    } else if (Cout % 4 == 0) {
        NQS_LAUNCH((k_layer<T, 4>), dim3(grid_for(M * N * (Cout / 4), c)), dim3(kThreads),
                           lds, s, in, M, c->L, Cin, Cout, wl, bias, out, epi, zk, pm);
    } else {
        NQS_LAUNCH((k_layer<T, 1>), dim3(grid_for(M * N * Cout, c)), dim3(kThreads), lds,
                           s, in, M, c->L, Cin, Cout, wl, bias, out, epi, zk, pm);
    }
}

// Forward through all layers for M planes; returns the plane holding h_K.
template <typename T>
T *forward_planes(const nqs_ctx *c, const int8_t *spins, PlaneMap pm, int64_t M, T *pa, T *pb,
                  hipStream_t s)
{
    const int N = c->N, C = c->C;
    const T *w1 = layer_w<T>(c, 0);
    layer1_launch<T>(c, spins, pm, M, w1, pa, nullptr, s);
    T *cur = pa, *nxt = pb;
    for (int k = 1; k < c->K; ++k) {
        const T *wl = layer_w<T>(c, k);
        layer_launch<T>(c, cur, M, C, C, wl, wl + 9 * C * C, nxt, 0, nullptr, pm, s);
        T *t = cur;
        cur = nxt;
        nxt = t;
    }
    return cur;
}

template <typename T>
void base_forward_t(const nqs_ctx *c, const int8_t *spins, int B, double *f, double *hsum,
                    void *plane_a, void *plane_b, hipStream_t s)
{
    PlaneMap pm{nullptr, 0, nullptr};
    T *hK = forward_planes<T>(c, spins, pm, B, (T *)plane_a, (T *)plane_b, s);
    NQS_LAUNCH((k_final<T>), dim3(B), dim3(kThreads), 0, s, hK, (int64_t)B, c->N, c->C,
                       pm, c->L, f, hsum, (const double *)nullptr, (double *)nullptr, c->err);
}

template <typename T>
void conn_forward_t(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                    const int64_t *qlen, int64_t q_begin, int64_t q_count, const double *hsum,
                    double *dlog, void *plane_a, void *plane_b, hipStream_t s)
{
    PlaneMap pm{queue, q_begin, qlen};
    T *hK = forward_planes<T>(c, spins, pm, q_count, (T *)plane_a, (T *)plane_b, s);
    NQS_LAUNCH((k_final<T>), dim3((unsigned)q_count), dim3(kThreads), 0, s, hK, q_count,
                       c->N, c->C, pm, c->L, (double *)nullptr, (double *)nullptr, hsum, dlog,
                       c->err);
}

}  // namespace

size_t vec_plane_bytes(const nqs_ctx *c, int64_t items)
{
    const size_t el = (c->dtype == NQS_FP32) ? sizeof(float) : sizeof(double);
    return el * (size_t)items * c->N * c->C;
}

void vec_base_forward(const nqs_ctx *c, const int8_t *spins, int B, double *f, double *hsum,
                      void *plane_a, void *plane_b, hipStream_t s)
{
    if (B <= 0) return;
    if (c->dtype == NQS_FP32)
        base_forward_t<float>(c, spins, B, f, hsum, plane_a, plane_b, s);
    else
        base_forward_t<double>(c, spins, B, f, hsum, plane_a, plane_b, s);
}

void vec_base_forward_cached(const nqs_ctx *c, const int8_t *spins, int nb, double *f,
                             double *hsum, void *plane, double *cache, int64_t cB, hipStream_t s)
{
    if (nb <= 0) return;
    // the same launches as the plain FP64 base pass, with h_1 .. h_{K-1}
    // written into their cache slots and h_K into the plane
    const PlaneMap pm{nullptr, 0, nullptr};
    const int C = c->C;
    const int64_t slot = cB * c->N * C;
    double *h = cache;
    layer1_launch<double>(c, spins, pm, nb, layer_w<double>(c, 0), h, nullptr, s);
    for (int k = 1; k < c->K; ++k) {
        const double *wl = layer_w<double>(c, k);
        double *out = (k + 1 < c->K) ? h + slot : (double *)plane;
        layer_launch<double>(c, h, nb, C, C, wl, wl + 9 * C * C, out, 0, nullptr, pm, s);
        h = out;
    }
    NQS_LAUNCH((k_final<double>), dim3(nb), dim3(kThreads), 0, s, (const double *)h, (int64_t)nb,
               c->N, C, pm, c->L, f, hsum, (const double *)nullptr, (double *)nullptr, c->err);
}

void vec_conn_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                      const int64_t *qlen, int64_t q_begin, int64_t q_count, const double *hsum,
                      double *dlog, void *plane_a, void *plane_b, hipStream_t s)
{
    if (q_count <= 0) return;
    if (c->dtype == NQS_FP32)
        conn_forward_t<float>(c, spins, queue, qlen, q_begin, q_count, hsum, dlog, plane_a,
                              plane_b, s);
    else
        conn_forward_t<double>(c, spins, queue, qlen, q_begin, q_count, hsum, dlog, plane_a,
                               plane_b, s);
}

void vec_deriv_forward(const nqs_ctx *c, const int8_t *spins, int B, double *zsave,
                       double *hsave, double *delta_last, hipStream_t s)
{
    if (B <= 0) return;
    const int N = c->N, C = c->C, K = c->K;
    const int64_t layer = (int64_t)B * N * C;
    const PlaneMap pm{nullptr, 0, nullptr};
    layer1_launch<double>(c, spins, pm, B, layer_w<double>(c, 0), hsave, zsave, s);
    if (K == 1) {
        NQS_LAUNCH(k_delta_last, dim3(grid_for(layer, c)), dim3(kThreads), 0, s, zsave, layer,
                   delta_last);
        return;
    }
    for (int k = 1; k < K; ++k) {
        const double *wl = layer_w<double>(c, k);
        const double *in = hsave + (int64_t)(k - 1) * layer;
        if (k < K - 1)
            layer_launch<double>(c, in, B, C, C, wl, wl + 9 * C * C, hsave + (int64_t)k * layer,
                                 1, zsave + (int64_t)k * layer, pm, s);
        else
            layer_launch<double>(c, in, B, C, C, wl, wl + 9 * C * C, delta_last, 3, nullptr, pm,
                                 s);
    }
}

void vec_backward(const nqs_ctx *c, const int8_t *spins, int B, const double *zsave,
                  const double *hsave, double *delta_a, double *delta_b, void *O, nqs_dtype odt,
                  hipStream_t s)
{
    if (B <= 0) return;
    const int N = c->N, C = c->C, K = c->K;
    const int64_t layer = (int64_t)B * N * C;   // one layer of saved tanh z or h: [B][N][C]
    double *cur = delta_a, *nxt = delta_b;
    std::vector<int64_t> woff(K);   // layer offsets in the canonical parameter vector
    int64_t off = 0;
    for (int k = 0; k < K; ++k) {
        woff[k] = off;
        off += (int64_t)C * (k == 0 ? 1 : C) * 9 + C;
    }
    for (int k = K - 1; k >= 0; --k) {
        if (k == 0) {
            if (odt == NQS_FP32)
                NQS_LAUNCH((k_wgrad1<float>), dim3(B), dim3(kThreads), 0, s, spins, cur, c->L, C,
                           c->P, woff[0], (float *)O);
            else
                NQS_LAUNCH((k_wgrad1<double>), dim3(B), dim3(kThreads), 0, s, spins, cur, c->L,
                           C, c->P, woff[0], (double *)O);
            break;
        }
        const double *hprev = hsave + (int64_t)(k - 1) * layer;
        if (f64mma_wgrad_ok(C))
            f64mma_wgrad(c, hprev, cur, B, woff[k], O, odt, s);
        else if (odt == NQS_FP32)
            NQS_LAUNCH((k_wgrad<float>), dim3(B), dim3(kThreads), 0, s, spins, hprev, cur,
                       c->L, C, k, c->P, woff[k], (float *)O);
        else
            NQS_LAUNCH((k_wgrad<double>), dim3(B), dim3(kThreads), 0, s, spins, hprev, cur,
                       c->L, C, k, c->P, woff[k], (double *)O);
        // delta_{k-1} = (W_k^T * delta_k) o tanh(z_{k-1}): a forward-shaped
        // convolution with flipped taps and transposed weights, no bias
        int64_t boff = 0;
        for (int l = 1; l < k; ++l) boff += 9 * (int64_t)C * C;
        layer_launch<double>(c, cur, B, C, C, c->w_bwd64 + boff, nullptr, nxt, 2,
                             const_cast<double *>(zsave + (int64_t)(k - 1) * layer),
                             PlaneMap{nullptr, 0, nullptr}, s);
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
}

}  // namespace nqs
