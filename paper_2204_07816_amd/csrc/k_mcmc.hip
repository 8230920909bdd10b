// k_mcmc.hip -- Metropolis sampling of |psi|^2 by pair exchanges [Sec. 3.2:
// the walkers sample configurations with probability |psi|^2; Sec. 5.4.1:
// many independent chains, each proposal an exchanged configuration whose
// log-amplitude difference is what the local energy also needs].
//
// One step of every chain (one chain per sample of the batch):
//   propose: bond id from the caller's random integer (uniform over the bonds
//            of the Hamiltonian, canonical order), queue item (chain, bond);
//   ratio:   f(S') - f(S) by the exchanged-configuration pass of the local
//            energy (a pair of equal values gives S' = S and exactly 0);
//   accept:  a pair of different values (antiparallel spins; t-J also an
//            electron and a hole) is exchanged when u < exp(2 (f(S') - f(S))),
//            u the caller's uniform number in [0, 1).
// Where the incremental cone kernel serves, the base pass is taken once and
// then kept current: accepted chains run a write-back pass of the cone kernel
// (their cone's activations and site sums replace the cached ones, which is
// what a new base pass would give) before their pairs are exchanged.
// The proposal is symmetric (the reverse move picks the same bond), so the
// chain satisfies detailed balance for |psi|^2.
#include <algorithm>

#include "nqs_internal.h"

namespace nqs {
namespace {

constexpr int kThreads = 256;

// Bond id of proposal r: r mod (N * ntypes) = site * ntypes + type index,
// types {0, 1} (nearest neighbours) and/or {2, 3} (next-nearest) as the
// bonds of each class carry terms (t-J: nearest neighbours only).
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

// Sites of the pair of queue item e in chain s.
__device__ inline void item_pair(uint32_t e, int L, int *i, int *j)
{
    const int b = item_bond(e);
    const int i0 = b >> 2, t = b & 3;
    const int x = i0 % L, y = i0 / L;
    int xj = x + bond_dx(t), yj = y + bond_dy(t);
    xj = xj < 0 ? xj + L : (xj >= L ? xj - L : xj);
    yj = yj < 0 ? yj + L : (yj >= L ? yj - L : yj);
    *i = i0;
    *j = yj * L + xj;
}

// flag[s] = 1 when chain s accepts its proposal (the pair's values differ
// and u < exp(2 dlog)); with apply, the pair is exchanged at once.
__global__ void __launch_bounds__(kThreads)
k_mcmc_decide(int8_t *__restrict__ spins, int B, int L, const uint32_t *__restrict__ queue,
              const double *__restrict__ dlog, const double *__restrict__ u,
              int32_t *__restrict__ flag, int32_t *__restrict__ accepted, int apply)
{
    const int s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= B) return;
    int i, j;
    item_pair(queue[s], L, &i, &j);
    int8_t *sp = spins + (int64_t)s * L * L;
    const int8_t si = sp[i], sj = sp[j];
    const int ok = (si != sj && u[s] < exp(2.0 * dlog[s])) ? 1 : 0;
    if (flag) flag[s] = ok;
    if (ok) {
        if (apply) {
            sp[i] = sj;
            sp[j] = si;
        }
        if (accepted) accepted[s] += 1;
    }
}

// exchange the pairs of the flagged chains
__global__ void __launch_bounds__(kThreads)
k_mcmc_apply(int8_t *__restrict__ spins, int B, int L, const uint32_t *__restrict__ queue,
             const int32_t *__restrict__ flag)
{
    const int s = blockIdx.x * kThreads + threadIdx.x;
    if (s >= B || !flag[s]) return;
    int i, j;
    item_pair(queue[s], L, &i, &j);
    int8_t *sp = spins + (int64_t)s * L * L;
    const int8_t si = sp[i];
    sp[i] = sp[j];
    sp[j] = si;
}

}  // namespace

void launch_mcmc_propose(const nqs_ctx *c, int B, const uint32_t *rnd, uint32_t *queue,
                         int64_t *qlen, hipStream_t s)
{
    const int grid = std::max(1, (B + kThreads - 1) / kThreads);
    NQS_LAUNCH(k_mcmc_propose, dim3(grid), dim3(kThreads), 0, s, rnd, B, c->N,
               nn_moves(c) ? 1 : 0, nnn_moves(c) ? 1 : 0, queue, qlen);
}

void launch_mcmc_decide(const nqs_ctx *c, int8_t *spins, int B, const uint32_t *queue,
                        const double *dlog, const double *u, int32_t *flag, int32_t *accepted,
                        bool apply, hipStream_t s)
{
    const int grid = std::max(1, (B + kThreads - 1) / kThreads);
    NQS_LAUNCH(k_mcmc_decide, dim3(grid), dim3(kThreads), 0, s, spins, B, c->L, queue, dlog, u,
               flag, accepted, apply ? 1 : 0);
}

void launch_mcmc_apply(const nqs_ctx *c, int8_t *spins, int B, const uint32_t *queue,
                       const int32_t *flag, hipStream_t s)
{
    const int grid = std::max(1, (B + kThreads - 1) / kThreads);
    NQS_LAUNCH(k_mcmc_apply, dim3(grid), dim3(kThreads), 0, s, spins, B, c->L, queue, flag);
}

}  // namespace nqs
