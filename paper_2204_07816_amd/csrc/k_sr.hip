// k_sr.hip -- stochastic reconfiguration [Sec. 3.2: SR gradients and
// covariance give the parameter update delta; Sec. 5.4.1 "Distributed SR
// computation"].  The paper forms the [R, R] covariance and factorises it;
// here the same system
//     (S + lambda I) x = F,  S = Obar^T Obar / Ns,  F = Obar^T (E - Ebar) / Ns,
// Obar = O - mean(O), is solved by conjugate gradient with S applied
// matrix-free as two streaming passes over O per iteration (HBM bound).
// O is read as FP32 or FP64; every product, sum and dot is FP64.  Scalars
// (alpha, beta, r.r) stay on the device, so the solve never synchronises
// with the host and can be captured in a graph.  All reductions are two-stage
// with a fixed order (deterministic).  One iteration is five launches: Obar p,
// the partial column sums of Obar^T u, then three kernels that each finish the
// previous one's reduction themselves (see k_ap_dot).
#include <algorithm>

#include "nqs_internal.h"

namespace nqs {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxChunks = 64;

struct SrCtl {
    double rr, ff, alpha, beta, mean, var;
    double rrv[2];   // r.r at the start of iteration it, in slot it & 1
    int done, it;
};

__device__ inline double ld(const float *p, int64_t i) { return (double)p[i]; }
__device__ inline double ld(const double *p, int64_t i) { return p[i]; }

__device__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// 16-byte vectors of O: VW consecutive elements (4 FP32 or 2 FP64)
template <typename OT, int VW> struct Vec;
template <> struct Vec<float, 4> {
    typedef float4 T;
    static __device__ inline void get(const float *q, double (&o)[4])
    {
        const float4 v = *reinterpret_cast<const float4 *>(q);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
};
template <> struct Vec<double, 2> {
    static __device__ inline void get(const double *q, double (&o)[2])
    {
        const double2 v = *reinterpret_cast<const double2 *>(q);
        o[0] = v.x; o[1] = v.y;
    }
};
template <typename OT> struct Vec<OT, 1> {
    static __device__ inline void get(const OT *q, double (&o)[1]) { o[0] = (double)q[0]; }
};

// part[c][p] = sum_{s in chunk c} (O[s][p] - sub[p]) * wt[s]   (sub / wt may be null)
// Each thread owns VW consecutive columns (one 16-byte load per row when
// P is a multiple of VW); every column still sums its rows in order.
template <typename OT, int VW>
__global__ void __launch_bounds__(kThreads)
k_colsum(const OT *__restrict__ O, int64_t B, int64_t P, const double *__restrict__ sub,
         const double *__restrict__ wt, int64_t rows_per_chunk, double *__restrict__ part,
         const SrCtl *ctl)
{
    if (ctl && ctl->done) return;
    const int64_t p = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * VW;
    if (p >= P) return;
    const int64_t s0 = (int64_t)blockIdx.y * rows_per_chunk;
    const int64_t s1 = min(B, s0 + rows_per_chunk);
    double m[VW], acc[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) {
        m[q] = sub ? sub[p + q] : 0.0;
        acc[q] = 0.0;
    }
    for (int64_t s = s0; s < s1; ++s) {
        double o[VW];
        Vec<OT, VW>::get(O + s * P + p, o);
        const double ws = wt ? wt[s] : 1.0;
#pragma unroll
        for (int q = 0; q < VW; ++q) acc[q] = fma(o[q] - m[q], ws, acc[q]);
    }
#pragma unroll
    for (int q = 0; q < VW; ++q) part[(int64_t)blockIdx.y * P + p + q] = acc[q];
}

// out[p] = scale * sum_c part[c][p] (+ lam * v[p])
__global__ void k_colsum_final(const double *__restrict__ part, int nchunk, int64_t P,
                               double scale, double lam, const double *__restrict__ v,
                               double *__restrict__ out, const SrCtl *ctl)
{
    if (ctl && ctl->done) return;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) acc += part[(int64_t)c * P + p];
    out[p] = acc * scale + (v ? lam * v[p] : 0.0);
}

// u[s] = sum_p (O[s][p] - obar[p]) v[p]: kRows rows per block, each thread
// taking VW consecutive elements per step (16-byte loads of O); the FP64
// vectors obar and v are read once per step for all the block's rows.  Each
// row's sum has the same order whatever the number of rows per block.
constexpr int kRows = 4;

template <typename OT, int VW>
__global__ void __launch_bounds__(kThreads)
k_rowdot(const OT *__restrict__ O, int64_t nrows, int64_t P, const double *__restrict__ obar,
         const double *__restrict__ v, double *__restrict__ u, const SrCtl *ctl)
{
    __shared__ double sh[kRows][kThreads];
    if (ctl->done) return;
    const int64_t s0 = (int64_t)blockIdx.x * kRows;
    const int nr = (int)min((int64_t)kRows, nrows - s0);
    double acc[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) acc[r] = 0.0;
    for (int64_t p = (int64_t)threadIdx.x * VW; p < P; p += (int64_t)kThreads * VW) {
        double ob[VW], vv[VW];
#pragma unroll
        for (int q = 0; q < VW; ++q) {
            ob[q] = obar[p + q];
            vv[q] = v[p + q];
        }
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            if (r >= nr) break;
            double o[VW];
            Vec<OT, VW>::get(O + (s0 + r) * P + p, o);
#pragma unroll
            for (int q = 0; q < VW; ++q) acc[r] = fma(o[q] - ob[q], vv[q], acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r) sh[r][threadIdx.x] = acc[r];
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
#pragma unroll
            for (int r = 0; r < kRows; ++r) sh[r][threadIdx.x] += sh[r][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x < nr) u[s0 + threadIdx.x] = sh[threadIdx.x][0];
}

// launches of the two streaming passes, 16-byte loads when P allows them
template <typename OT>
constexpr int vec_width() { return 16 / (int)sizeof(OT); }

template <typename OT>
void launch_colsum(dim3 grid_rows, int64_t P, hipStream_t s, const OT *O, int64_t B,
                   const double *sub, const double *wt, int64_t rpc, double *part,
                   const SrCtl *ctl)
{
    constexpr int VW = vec_width<OT>();
    if (P % VW == 0) {
        const dim3 g((unsigned)((P / VW + kThreads - 1) / kThreads), grid_rows.y);
        NQS_LAUNCH((k_colsum<OT, VW>), g, dim3(kThreads), 0, s, O, B, P, sub, wt, rpc, part, ctl);
    } else {
        const dim3 g((unsigned)((P + kThreads - 1) / kThreads), grid_rows.y);
        NQS_LAUNCH((k_colsum<OT, 1>), g, dim3(kThreads), 0, s, O, B, P, sub, wt, rpc, part, ctl);
    }
}

template <typename OT>
void launch_rowdot(int64_t nrows, int64_t P, hipStream_t s, const OT *O, const double *obar,
                   const double *v, double *u, const SrCtl *ctl)
{
    constexpr int VW = vec_width<OT>();
    const dim3 g((unsigned)((nrows + kRows - 1) / kRows));
    if (P % VW == 0)
        NQS_LAUNCH((k_rowdot<OT, VW>), g, dim3(kThreads), 0, s, O, nrows, P, obar, v, u, ctl);
    else
        NQS_LAUNCH((k_rowdot<OT, 1>), g, dim3(kThreads), 0, s, O, nrows, P, obar, v, u, ctl);
}

// partial dot products a.b, one value per block
__global__ void __launch_bounds__(kThreads)
k_dot_part(const double *__restrict__ a, const double *__restrict__ b, int64_t n,
           double *__restrict__ part, const SrCtl *ctl)
{
    __shared__ double sh[kThreads];
    if (ctl && ctl->done) return;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        acc = fma(a[i], b[i], acc);
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// stage 2 of the initial r.r: rr = ff = value; done if ff == 0
__global__ void __launch_bounds__(kThreads)
k_dot_final(const double *__restrict__ part, int nparts, SrCtl *ctl)
{
    __shared__ double sh[kThreads];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kThreads) acc += part[i];
    acc = block_sum(acc, sh);
    if (threadIdx.x != 0) return;
    ctl->rr = acc;
    ctl->rrv[0] = acc;
    ctl->ff = acc;
    ctl->it = 0;
    ctl->done = !(acc > 0.0);
}

// One CG iteration after Ap's partial column sums, in three launches whose
// final reductions are repeated by every block that needs them (the same
// fixed-order sum in every block, so every block sees the same value):
//   k_ap_dot:     Ap = scale * sum_c part[c] + lam p, and per block sum p.Ap;
//   k_update_xr2: alpha = r.r / p.Ap; x += alpha p, r -= alpha Ap, and per
//                 block sum r.r (p.Ap <= 0: stop without updating);
//   k_update_p2:  beta = r.r_new / r.r; p = r + beta p; block 0 records r.r,
//                 counts the iteration and stops once ||r|| <= 1e-30 ||F||.
// r.r of iteration `it` lives in slot it & 1, so block 0 can write the next
// one while the other blocks still read the current one.
__device__ double sum_parts(const double *part, int n, double *sh)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) acc += part[i];
    return block_sum(acc, sh);
}

__global__ void __launch_bounds__(kThreads)
k_ap_dot(const double *__restrict__ part, int nchunk, int64_t P, double scale, double lam,
         const double *__restrict__ p, double *__restrict__ ap, double *__restrict__ pap_part,
         const SrCtl *ctl)
{
    __shared__ double sh[kThreads];
    if (ctl->done) return;
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    double d = 0.0;
    if (i < P) {
        double acc = 0.0;
        for (int c = 0; c < nchunk; ++c) acc += part[(int64_t)c * P + i];
        const double v = acc * scale + lam * p[i];
        ap[i] = v;
        d = p[i] * v;
    }
    d = block_sum(d, sh);
    if (threadIdx.x == 0) pap_part[blockIdx.x] = d;
}

__global__ void __launch_bounds__(kThreads)
k_update_xr2(double *__restrict__ x, double *__restrict__ r, const double *__restrict__ p,
             const double *__restrict__ ap, int64_t n, const double *__restrict__ pap_part,
             int nparts, double *__restrict__ rr_part, SrCtl *ctl, int it)
{
    __shared__ double sh[kThreads];
    if (ctl->done) return;
    const double pap = sum_parts(pap_part, nparts, sh);
    if (!(pap > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) ctl->done = 1;
        return;
    }
    const double a = ctl->rrv[it & 1] / pap;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        x[i] = fma(a, p[i], x[i]);
        const double ri = fma(-a, ap[i], r[i]);
        r[i] = ri;
        acc = fma(ri, ri, acc);
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) rr_part[blockIdx.x] = acc;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->alpha = a;
}

__global__ void __launch_bounds__(kThreads)
k_update_p2(double *__restrict__ p, const double *__restrict__ r, int64_t n,
            const double *__restrict__ rr_part, int nparts, SrCtl *ctl, int it)
{
    __shared__ double sh[kThreads];
    if (ctl->done) return;
    const double rr_new = sum_parts(rr_part, nparts, sh);
    const double b = rr_new / ctl->rrv[it & 1];
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        p[i] = fma(b, p[i], r[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->rrv[(it + 1) & 1] = rr_new;
        ctl->rr = rr_new;
        ctl->beta = b;
        ctl->it = it + 1;
        // converged far beyond FP64 resolution: ||r|| <= 1e-30 ||F||
        if (!(rr_new > ctl->ff * 1e-60)) ctl->done = 1;
    }
}

// x = 0, r = p = F
__global__ void k_init(double *__restrict__ x, double *__restrict__ r, double *__restrict__ p,
                       const double *__restrict__ F, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = 0.0;
        r[i] = F[i];
        p[i] = F[i];
    }
}

// mean / variance of e, and d = e - mean
__global__ void __launch_bounds__(1024)
k_center(const double *__restrict__ e, int64_t B, double *__restrict__ d, SrCtl *ctl)
{
    __shared__ double sh[1024];
    double acc = 0.0;
    for (int64_t s = threadIdx.x; s < B; s += 1024) acc += e[s];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    const double mean = sh[0] / (double)B;
    __syncthreads();
    acc = 0.0;
    for (int64_t s = threadIdx.x; s < B; s += 1024) {
        const double v = e[s] - mean;
        d[s] = v;
        acc += v * v;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ctl->mean = mean;
        ctl->var = sh[0] / (double)B;
        ctl->done = 0;
        ctl->it = 0;
    }
}

__global__ void k_stats_out(const SrCtl *ctl, double *stats)
{
    stats[0] = ctl->mean;
    stats[1] = ctl->var;
    stats[2] = ctl->ff > 0.0 ? sqrt(ctl->rr / ctl->ff) : 0.0;
    stats[3] = (double)ctl->it;
}

struct SrLayout {
    int64_t nchunk, rows_per_chunk, ndot;
    int64_t nblk;   // blocks of kThreads covering P (partials of p.Ap and r.r)
    size_t off_obar, off_F, off_r, off_p, off_ap, off_d, off_u, off_part, off_dot, off_pap,
        off_rrp, off_ctl, total;
};

SrLayout layout(int64_t B, int64_t P)
{
    SrLayout l;
    l.nchunk = std::min<int64_t>(kMaxChunks, std::max<int64_t>(1, (B + 63) / 64));
    l.rows_per_chunk = (B + l.nchunk - 1) / l.nchunk;
    l.ndot = 512;
    l.nblk = std::max<int64_t>(1, (P + kThreads - 1) / kThreads);
    size_t off = 0;
    auto take = [&](size_t n) {
        size_t o = off;
        off += (n * sizeof(double) + 255) & ~(size_t)255;
        return o;
    };
    l.off_obar = take(P);
    l.off_F = take(P);
    l.off_r = take(P);
    l.off_p = take(P);
    l.off_ap = take(P);
    l.off_d = take(B);
    l.off_u = take(B);
    l.off_part = take((size_t)l.nchunk * P);
    l.off_dot = take(l.ndot);
    l.off_pap = take(l.nblk);
    l.off_rrp = take(l.nblk);
    l.off_ctl = take(sizeof(SrCtl) / sizeof(double) + 1);
    l.total = off;
    return l;
}

// The rest of CG iteration `it` once Ap's partial column sums are in `part`.
void cg_tail(const SrLayout &l, int64_t P, double invB, double lam, double *x, double *r,
             double *p, double *ap, const double *part, unsigned char *w, SrCtl *ctl, int it,
             hipStream_t s)
{
    double *pap = (double *)(w + l.off_pap), *rrp = (double *)(w + l.off_rrp);
    const unsigned nb = (unsigned)l.nblk;
    NQS_LAUNCH(k_ap_dot, dim3(nb), dim3(kThreads), 0, s, part, (int)l.nchunk, P, invB, lam,
               (const double *)p, ap, pap, (const SrCtl *)ctl);
    NQS_LAUNCH(k_update_xr2, dim3(nb), dim3(kThreads), 0, s, x, r, (const double *)p,
               (const double *)ap, P, (const double *)pap, (int)nb, rrp, ctl, it);
    NQS_LAUNCH(k_update_p2, dim3(nb), dim3(kThreads), 0, s, p, (const double *)r, P,
               (const double *)rrp, (int)nb, ctl, it);
}

template <typename OT>
void sr_solve_t(const OT *O, const double *e, int64_t B, int64_t P, double lam, int n_iter,
                double *x, double *stats, unsigned char *w, hipStream_t s)
{
    const SrLayout l = layout(B, P);
    double *obar = (double *)(w + l.off_obar), *F = (double *)(w + l.off_F);
    double *r = (double *)(w + l.off_r), *p = (double *)(w + l.off_p);
    double *ap = (double *)(w + l.off_ap), *d = (double *)(w + l.off_d);
    double *u = (double *)(w + l.off_u), *part = (double *)(w + l.off_part);
    double *dot = (double *)(w + l.off_dot);
    SrCtl *ctl = (SrCtl *)(w + l.off_ctl);
    const dim3 cgrid((unsigned)((P + kThreads - 1) / kThreads), (unsigned)l.nchunk);
    const unsigned vgrid = (unsigned)std::min<int64_t>(1024, (P + kThreads - 1) / kThreads);
    const unsigned fgrid = (unsigned)((P + kThreads - 1) / kThreads);
    const double invB = 1.0 / (double)B;

    NQS_LAUNCH(k_center, dim3(1), dim3(1024), 0, s, e, B, d, ctl);
    // column means
    launch_colsum<OT>(cgrid, P, s, O, B, (const double *)nullptr, (const double *)nullptr,
                      l.rows_per_chunk, part, (const SrCtl *)nullptr);
    NQS_LAUNCH(k_colsum_final, dim3(fgrid), dim3(kThreads), 0, s, part, (int)l.nchunk, P,
                       invB, 0.0, (const double *)nullptr, obar, (const SrCtl *)nullptr);
    // F = Obar^T (E - Ebar) / B
    launch_colsum<OT>(cgrid, P, s, O, B, obar, d, l.rows_per_chunk, part,
                      (const SrCtl *)nullptr);
    NQS_LAUNCH(k_colsum_final, dim3(fgrid), dim3(kThreads), 0, s, part, (int)l.nchunk, P,
                       invB, 0.0, (const double *)nullptr, F, (const SrCtl *)nullptr);
    NQS_LAUNCH(k_init, dim3(vgrid), dim3(kThreads), 0, s, x, r, p, F, P);
    NQS_LAUNCH(k_dot_part, dim3((unsigned)l.ndot), dim3(kThreads), 0, s, r, r, P, dot,
                       (const SrCtl *)nullptr);
    NQS_LAUNCH(k_dot_final, dim3(1), dim3(kThreads), 0, s, dot, (int)l.ndot, ctl);
    for (int it = 0; it < n_iter; ++it) {
        // Ap = Obar^T (Obar p) / B + lambda p
        launch_rowdot<OT>(B, P, s, O, obar, p, u, ctl);
        launch_colsum<OT>(cgrid, P, s, O, B, obar, u, l.rows_per_chunk, part, ctl);
        cg_tail(l, P, invB, lam, x, r, p, ap, part, w, ctl, it, s);
    }
    if (stats) NQS_LAUNCH(k_stats_out, dim3(1), dim3(1), 0, s, ctl, stats);
}


// The same solve with O never held whole: rows [r0, r0 + nb) of O are
// produced on demand into a buffer of `chunk` rows by `rows` (which recomputes
// them from the samples).  chunk is a multiple of the reduction row block, so
// each block's partial column sums see exactly the rows, in exactly the order,
// of the stored-O solve, and the results are the same bit for bit.  One pass
// over O needs nc = ceil(B / chunk) chunks; a pass starts with the chunk left
// in the buffer by the previous one, so an iteration recomputes 2 (nc - 1)
// chunks.
template <typename OT>
void sr_solve_rows_t(const SrRows &rows, OT *obuf, int64_t chunk, const double *e, int64_t B,
                     int64_t P, double lam, int n_iter, double *x, double *stats,
                     unsigned char *w, hipStream_t s)
{
    const SrLayout l = layout(B, P);
    double *obar = (double *)(w + l.off_obar), *F = (double *)(w + l.off_F);
    double *r = (double *)(w + l.off_r), *p = (double *)(w + l.off_p);
    double *ap = (double *)(w + l.off_ap), *d = (double *)(w + l.off_d);
    double *u = (double *)(w + l.off_u), *part = (double *)(w + l.off_part);
    double *dot = (double *)(w + l.off_dot);
    SrCtl *ctl = (SrCtl *)(w + l.off_ctl);
    const int64_t rpc = l.rows_per_chunk;
    const int64_t nc = (B + chunk - 1) / chunk;
    const unsigned vgrid = (unsigned)std::min<int64_t>(1024, (P + kThreads - 1) / kThreads);
    const unsigned fgrid = (unsigned)((P + kThreads - 1) / kThreads);
    const double invB = 1.0 / (double)B;
    int64_t resident = -1;   // chunk whose rows are in obuf

    // one pass over all chunks: fn(r0, nb) sees rows [r0, r0 + nb) in obuf
    auto pass = [&](auto &&fn) {
        int64_t order0 = resident >= 0 ? resident : 0;
        for (int64_t i = 0; i < nc; ++i) {
            const int64_t ci = (order0 + i) % nc;
            const int64_t r0 = ci * chunk;
            const int nb = (int)std::min<int64_t>(chunk, B - r0);
            if (ci != resident) {
                rows(r0, nb, obuf, s);
                resident = ci;
            }
            fn(r0, nb);
        }
    };
    // partial column sums of rows [r0, r0 + nb) into their reduction blocks
    auto colsum = [&](int64_t r0, int nb, const double *sub, const double *wt, const SrCtl *c) {
        const dim3 g(fgrid, (unsigned)((nb + rpc - 1) / rpc));
        launch_colsum<OT>(g, P, s, (const OT *)obuf, (int64_t)nb, sub, wt ? wt + r0 : wt, rpc,
                          part + (r0 / rpc) * P, c);
    };

    NQS_LAUNCH(k_center, dim3(1), dim3(1024), 0, s, e, B, d, ctl);
    pass([&](int64_t r0, int nb) {
        colsum(r0, nb, (const double *)nullptr, (const double *)nullptr, (const SrCtl *)nullptr);
    });
    NQS_LAUNCH(k_colsum_final, dim3(fgrid), dim3(kThreads), 0, s, part, (int)l.nchunk, P, invB,
               0.0, (const double *)nullptr, obar, (const SrCtl *)nullptr);
    pass([&](int64_t r0, int nb) { colsum(r0, nb, obar, d, (const SrCtl *)nullptr); });
    NQS_LAUNCH(k_colsum_final, dim3(fgrid), dim3(kThreads), 0, s, part, (int)l.nchunk, P, invB,
               0.0, (const double *)nullptr, F, (const SrCtl *)nullptr);
    NQS_LAUNCH(k_init, dim3(vgrid), dim3(kThreads), 0, s, x, r, p, F, P);
    NQS_LAUNCH(k_dot_part, dim3((unsigned)l.ndot), dim3(kThreads), 0, s, r, r, P, dot,
               (const SrCtl *)nullptr);
    NQS_LAUNCH(k_dot_final, dim3(1), dim3(kThreads), 0, s, dot, (int)l.ndot, ctl);
    for (int it = 0; it < n_iter; ++it) {
        pass([&](int64_t r0, int nb) {
            launch_rowdot<OT>(nb, P, s, (const OT *)obuf, obar, p, u + r0, ctl);
        });
        pass([&](int64_t r0, int nb) { colsum(r0, nb, obar, u, ctl); });
        cg_tail(l, P, invB, lam, x, r, p, ap, part, w, ctl, it, s);
    }
    if (stats) NQS_LAUNCH(k_stats_out, dim3(1), dim3(1), 0, s, ctl, stats);
}

}  // namespace

size_t sr_workspace_bytes(int64_t B, int64_t P) { return layout(B, P).total; }

void launch_sr_solve(const void *O, nqs_dtype odt, const double *e_loc, int64_t B, int64_t P,
                     double lambda, int n_iter, double *x, double *stats, void *work,
                     hipStream_t s)
{
    if (odt == NQS_FP32)
        sr_solve_t<float>((const float *)O, e_loc, B, P, lambda, n_iter, x, stats,
                          (unsigned char *)work, s);
    else
        sr_solve_t<double>((const double *)O, e_loc, B, P, lambda, n_iter, x, stats,
                           (unsigned char *)work, s);
}

int64_t sr_row_block(int64_t B) { return layout(B, 1).rows_per_chunk; }

void launch_sr_solve_rows(const SrRows &rows, void *obuf, int64_t chunk, nqs_dtype odt,
                          const double *e_loc, int64_t B, int64_t P, double lambda, int n_iter,
                          double *x, double *stats, void *work, hipStream_t s)
{
    if (odt == NQS_FP32)
        sr_solve_rows_t<float>(rows, (float *)obuf, chunk, e_loc, B, P, lambda, n_iter, x, stats,
                               (unsigned char *)work, s);
    else
        sr_solve_rows_t<double>(rows, (double *)obuf, chunk, e_loc, B, P, lambda, n_iter, x,
                                stats, (unsigned char *)work, s);
}

}  // namespace nqs
