// k_mcmc.hip -- Metropolis sampling of |psi|^2 by pair exchanges [Sec. 3.2:
// the walkers sample configurations with probability |psi|^2; Sec. 5.4.1:
// many independent chains, each proposal an exchanged configuration whose
// log-amplitude difference is what the local energy also needs].
//
// One step of every chain (one chain per sample of the batch):
//   propose: bond id from the caller's random integer (uniform over the bonds
//            of the Hamiltonian, canonical order), queue item (chain, bond);
//   ratio:   f(S') - f(S) by the exchanged-configuration pass of the local
//            energy (a parallel pair gives S' = S and exactly 0);
//   accept:  an antiparallel pair is exchanged when u < exp(2 (f(S') - f(S))),
//            u the caller's uniform number in [0, 1).
// The proposal is symmetric (the reverse move picks the same bond), so the
// chain satisfies detailed balance for |psi|^2.
#include <algorithm>

#include "nqs_internal.h"

namespace nqs {
namespace {

constexpr int kThreads = 256;

// Bond id of proposal r: r mod (N * ntypes) = site * ntypes + type index,
// types {0, 1} (J1) and/or {2, 3} (J2) as the couplings are non-zero.
__device__ __host__ inline int proposal_bond(uint32_t r, int N, int j1, int j2)
{
    const int ntypes = 2 * (j1 + j2);
    const int q = (int)(r % (uint32_t)(N * ntypes));
    const int i = q / ntypes, k = q - i * ntypes;
    const int t = j1 ? k : 2 + k;
    return 4 * i + t;
}

__global__ void __launch_bounds__(kThreads)
k_mcmc_propose(const uint32_t *__restrict__ rnd, int B, int N, int j1, int j2,
               uint32_t *__restrict__ queue, int64_t *__restrict__ qlen)
{
    const int s = blockIdx.x * kThreads + threadIdx.x;
    if (s == 0) qlen[0] = B;
    if (s >= B) return;
    queue[s] = pack_item(s, proposal_bond(rnd[s], N, j1, j2));
}

__global__ void __launch_bounds__(kThreads)
k_mcmc_accept(int8_t *__restrict__ spins, int B, int L, const uint32_t *__restrict__ queue,
              const double *__restrict__ dlog, const double *__restrict__ u,
              int32_t *__restrict__ accepted)
{
    const int s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= B) return;
    const int b = item_bond(queue[s]);
    const int i = b >> 2, t = b & 3;
    const int x = i % L, y = i / L;
    int xj = x + bond_dx(t), yj = y + bond_dy(t);
    xj = xj < 0 ? xj + L : (xj >= L ? xj - L : xj);
    yj = yj < 0 ? yj + L : (yj >= L ? yj - L : yj);
    const int j = yj * L + xj;
    int8_t *sp = spins + (int64_t)s * L * L;
    const int8_t si = sp[i], sj = sp[j];
    if (si != sj && u[s] < exp(2.0 * dlog[s])) {
        sp[i] = sj;
        sp[j] = si;
        if (accepted) accepted[s] += 1;
    }
}

}  // namespace

void launch_mcmc_propose(const nqs_ctx *c, int B, const uint32_t *rnd, uint32_t *queue,
                         int64_t *qlen, hipStream_t s)
{
    const int grid = std::max(1, (B + kThreads - 1) / kThreads);
    NQS_LAUNCH(k_mcmc_propose, dim3(grid), dim3(kThreads), 0, s, rnd, B, c->N,
               c->J1 != 0.0 ? 1 : 0, c->J2 != 0.0 ? 1 : 0, queue, qlen);
}

void launch_mcmc_accept(const nqs_ctx *c, int8_t *spins, int B, const uint32_t *queue,
                        const double *dlog, const double *u, int32_t *accepted, hipStream_t s)
{
    const int grid = std::max(1, (B + kThreads - 1) / kThreads);
    NQS_LAUNCH(k_mcmc_accept, dim3(grid), dim3(kThreads), 0, s, spins, B, c->L, queue, dlog, u,
               accepted);
}

}  // namespace nqs
