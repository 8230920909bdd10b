// k_energy.hip -- FP64 reductions of the local energy [Sec. 5.4.1]:
//   E_loc(s) = E_diag(s) + sum_{S'} (J_b / 2) mu_b exp(f(S') - f(s)),
// mu_b = M(S')/M(s) (Marshall ratio), one block per sample with a fixed
// reduction tree (deterministic), and the batch mean / variance used by the
// stochastic reconfiguration [Sec. 3.2].
#include "nqs_internal.h"

namespace nqs {
namespace {

constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads)
k_energy_reduce(const int64_t *__restrict__ offsets, const uint32_t *__restrict__ queue,
                const double *__restrict__ dlog, const double *__restrict__ ediag, double J1,
                double J2, int marshall, double *__restrict__ e_loc, int32_t *err)
{
    __shared__ double red[kThreads];
    const int s = blockIdx.x;
    const int64_t q0 = offsets[s], q1 = offsets[s + 1];
    double acc = 0.0;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kThreads) {
        const int t = item_bond(queue[q]) & 3;
        const double half_j = 0.5 * (t < 2 ? J1 : J2);
        // J1 pairs join the two sublattices: the Marshall ratio is -1
        const double mu = (marshall && t < 2) ? -1.0 : 1.0;
        acc += half_j * mu * exp(dlog[q]);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double e = ediag[s] + red[0];
        if (!isfinite(e)) atomicOr(err, kErrNonFinite);
        e_loc[s] = e;
    }
}

constexpr int kStatThreads = 1024;

__global__ void __launch_bounds__(kStatThreads)
k_energy_stats(const double *__restrict__ e, int B, double *__restrict__ stats)
{
    __shared__ double red[kStatThreads];
    double acc = 0.0;
    for (int s = threadIdx.x; s < B; s += kStatThreads) acc += e[s];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kStatThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    const double mean = red[0] / (double)B;
    __syncthreads();
    acc = 0.0;
    for (int s = threadIdx.x; s < B; s += kStatThreads) {
        const double d = e[s] - mean;
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int off = kStatThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stats[0] = mean;
        stats[1] = red[0] / (double)B;
    }
}

}  // namespace

void launch_energy_reduce(const nqs_ctx *c, int B, const int64_t *offsets, const uint32_t *queue,
                          const double *dlog, const double *ediag, double *e_loc, int32_t *err,
                          hipStream_t s)
{
    if (B <= 0) return;
    NQS_LAUNCH(k_energy_reduce, dim3(B), dim3(kThreads), 0, s, offsets, queue, dlog,
                       ediag, c->J1, c->J2, c->marshall, e_loc, err);
}

void launch_energy_stats(const double *e_loc, int B, double *stats, hipStream_t s)
{
    NQS_LAUNCH(k_energy_stats, dim3(1), dim3(kStatThreads), 0, s, e_loc, B, stats);
}

}  // namespace nqs
