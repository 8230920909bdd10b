// k_energy.hip -- FP64 reductions of the local energy [Sec. 5.4.1]:
//   E_loc(s) = E_diag(s) + sum_{S'} (J_b / 2) mu_b exp(f(S') - f(s)),
// mu_b = M(S')/M(s) (Marshall ratio), one block per sample with a fixed
// reduction tree (deterministic), and the batch mean / variance used by the
// stochastic reconfiguration [Sec. 3.2].
//
// t-J model [Sec. 6.1, Eq. tJ]: an entry is a spin exchange (<S'|H|S> = J/2)
// or a hop (<S'|H|S> = -t (-1)^n, n the electrons strictly between the two
// sites in the site order: the Jordan-Wigner string of the fermion encoding).
// The block first scans the sample's occupations into a prefix count in LDS,
// so every entry reads n as a difference of two prefix values.
#include "nqs_internal.h"

namespace nqs {
namespace {

constexpr int kThreads = 256;

__global__ void __launch_bounds__(kThreads)
k_energy_reduce(const int64_t *__restrict__ offsets, const uint32_t *__restrict__ queue,
                const double *__restrict__ dlog, const int8_t *__restrict__ isign,
                const double *__restrict__ ediag, double J1, double J2, int marshall,
                double *__restrict__ e_loc, int32_t *err)
{
    __shared__ double red[kThreads];
    const int s = blockIdx.x;
    const int64_t q0 = offsets[s], q1 = offsets[s + 1];
    double acc = 0.0;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kThreads) {
        const int t = item_bond(queue[q]) & 3;
        const double half_j = 0.5 * (t < 2 ? J1 : J2);
        // J1 pairs join the two sublattices: the Marshall ratio is -1
        double mu = (marshall && t < 2) ? -1.0 : 1.0;
        if (isign) mu *= (double)isign[q];      // the network's own sign ratio
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

constexpr int kMaxSites = 64 * 64;

__global__ void __launch_bounds__(kThreads)
k_energy_reduce_tj(const int8_t *__restrict__ spins, int L, const int64_t *__restrict__ offsets,
                   const uint32_t *__restrict__ queue, const double *__restrict__ dlog,
                   const int8_t *__restrict__ isign, const double *__restrict__ ediag,
                   double t_hop, double J, int marshall, double *__restrict__ e_loc, int32_t *err)
{
    __shared__ uint16_t pre[kMaxSites + 1];   // pre[k] = electrons on sites 0 .. k-1
    __shared__ int scan[kThreads];
    __shared__ double red[kThreads];
    const int s = blockIdx.x, N = L * L;
    const int8_t *sp = spins + (int64_t)s * N;
    const int chunk = (N + kThreads - 1) / kThreads;
    const int c0 = min(N, (int)threadIdx.x * chunk), c1 = min(N, c0 + chunk);
    int cnt = 0;
    for (int k = c0; k < c1; ++k) cnt += (sp[k] != 0);
    scan[threadIdx.x] = cnt;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        const int add = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
        __syncthreads();
        scan[threadIdx.x] += add;
        __syncthreads();
    }
    int run = scan[threadIdx.x] - cnt;
    for (int k = c0; k < c1; ++k) {
        pre[k] = (uint16_t)run;
        run += (sp[k] != 0);
    }
    if (threadIdx.x == kThreads - 1) pre[N] = (uint16_t)scan[kThreads - 1];
    __syncthreads();

    const int64_t q0 = offsets[s], q1 = offsets[s + 1];
    double acc = 0.0;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kThreads) {
        const int b = item_bond(queue[q]);
        const int i = b >> 2, t = b & 3, x = i % L, y = i / L;
        const int yj = y + bond_dy(t), xj = x + bond_dx(t);
        const int j = (yj < 0 ? yj + L : (yj >= L ? yj - L : yj)) * L + (xj >= L ? xj - L : xj);
        const int a = sp[i], c = sp[j];
        double coef;
        if (a * c == -1) {
            // exchange moves an up spin to the other sublattice: Marshall ratio -1
            coef = (marshall ? -0.5 : 0.5) * J;
        } else {
            const int lo = min(i, j), hi = max(i, j);
            const int n = (int)pre[hi] - (int)pre[lo + 1];
            const double h = (n & 1) ? t_hop : -t_hop;
            // an up electron changes sublattice: Marshall ratio -1
            coef = (marshall && a + c > 0) ? -h : h;
        }
        if (isign) coef *= (double)isign[q];      // the network's own sign ratio
        acc += coef * exp(dlog[q]);
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

void launch_energy_reduce(const nqs_ctx *c, const int8_t *spins, int B, const int64_t *offsets,
                          const uint32_t *queue, const double *dlog, const int8_t *isign,
                          const double *ediag, double *e_loc, int32_t *err, hipStream_t s)
{
    if (B <= 0) return;
    if (c->model == kModelTJ)
        NQS_LAUNCH(k_energy_reduce_tj, dim3(B), dim3(kThreads), 0, s, spins, c->L, offsets,
                   queue, dlog, isign, ediag, c->t_hop, c->J1, c->marshall, e_loc, err);
    else
        NQS_LAUNCH(k_energy_reduce, dim3(B), dim3(kThreads), 0, s, offsets, queue, dlog,
                   isign, ediag, c->J1, c->J2, c->marshall, e_loc, err);
}

void launch_energy_stats(const double *e_loc, int B, double *stats, hipStream_t s)
{
    NQS_LAUNCH(k_energy_stats, dim3(1), dim3(kStatThreads), 0, s, e_loc, B, stats);
}

}  // namespace nqs
