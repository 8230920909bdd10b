// k_lattice.hip -- integer stage of the local energy [Sec. 5.4.1, hotspot
// energy calculation]: every antiparallel nearest / next-nearest pair of a
// sampled configuration yields one exchanged configuration S' with
// <S'|H|S> = J/2, and the diagonal part is sum_b J_b s_i s_j / 4 [Sec. 6.1].
//
// t-J model [Sec. 6.1, Eq. tJ]: site values +1 / -1 / 0 (hole), nearest-
// neighbour bonds only.  A pair of antiparallel electrons gives a spin
// exchange (J != 0) and an electron next to a hole a hop (t != 0); both are
// the pair's values exchanged, so the same queue entries and network passes
// serve.  Diagonal part: J (s_i s_j - |s_i| |s_j|) / 4 per bond, i.e. -J/2
// per antiparallel pair.
//
// Kernels: per-sample bond counts + diagonal energy + spin validation, a
// single-block exclusive scan into queue offsets, and the queue fill that
// writes (sample, bond) entries in canonical bond order.  All integer work,
// deterministic, bit-exact.
#include "nqs_internal.h"

namespace nqs {
namespace {

constexpr int kThreads = 256;

__device__ inline int wrapi(int a, int L) { return a < 0 ? a + L : (a >= L ? a - L : a); }

// Block-wide exclusive scan of one int64 per thread; returns the prefix and
// writes the block total into *total (all threads).
template <int NT>
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *sh, int64_t *total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        int64_t add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t incl = sh[t];
    *total = sh[NT - 1];
    __syncthreads();
    return incl - v;
}

// Which pairs give a queue entry: values differ, and the term they would
// use has a non-zero coefficient.  Spin model: J1 / J2 by bond class.
// t-J: nearest-neighbour only, exchange (J != 0) or hop (t != 0).
struct BondRule {
    int use_j1, use_j2, tj, use_hop;
    __device__ bool active(int t, int a, int b) const
    {
        if (a == b) return false;
        if (!tj) return t < 2 ? use_j1 : use_j2;
        if (t >= 2) return false;
        return (a != 0 && b != 0) ? use_j1 : use_hop;
    }
};

__global__ void __launch_bounds__(kThreads)
k_bond_count(const int8_t *__restrict__ spins, int L, double J1, double J2, BondRule rule,
             int32_t *__restrict__ counts, double *__restrict__ ediag, int32_t *err)
{
    const int s = blockIdx.x;
    const int N = L * L;
    const int8_t *sp = spins + (int64_t)s * N;
    // n1 / n2: antiparallel J1 / J2 pairs; nq: pairs that give a queue entry
    int n1 = 0, n2 = 0, nq = 0, bad = 0;
    for (int i = threadIdx.x; i < N; i += kThreads) {
        const int x = i % L, y = i / L;
        const int si = sp[i];
        bad |= rule.tj ? (si < -1 || si > 1) : (si != 1 && si != -1);
        // t = 0..3: (x+1,y), (x,y+1), (x+1,y+1), (x+1,y-1)
        const int xp = wrapi(x + 1, L), yp = wrapi(y + 1, L), ym = wrapi(y - 1, L);
        const int nb[4] = {sp[y * L + xp], sp[yp * L + x], sp[yp * L + xp], sp[ym * L + xp]};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int anti = (si * nb[t] == -1);
            if (t < 2) n1 += anti; else n2 += anti;
            nq += rule.active(t, si, nb[t]);
        }
    }
    __shared__ int red[4][kThreads];
    red[0][threadIdx.x] = n1;
    red[1][threadIdx.x] = n2;
    red[2][threadIdx.x] = nq;
    red[3][threadIdx.x] = bad;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
            red[2][threadIdx.x] += red[2][threadIdx.x + off];
            red[3][threadIdx.x] |= red[3][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int a1 = red[0][0], a2 = red[1][0];
        counts[s] = red[2][0];
        if (rule.tj)   // -J/2 per antiparallel nearest-neighbour pair
            ediag[s] = (J1 / 4.0) * (double)(-2 * a1);
        else           // sum over the 2N bonds of one class of s_i s_j = (2N - a) - a
            ediag[s] = (J1 / 4.0) * (double)(2 * N - 2 * a1) +
                       (J2 / 4.0) * (double)(2 * N - 2 * a2);
        if (red[3][0]) atomicOr(err, kErrSpin);
    }
}

constexpr int kScanThreads = 1024;

__global__ void __launch_bounds__(kScanThreads)
k_scan(const int32_t *__restrict__ counts, int B, int64_t *__restrict__ offsets,
       int64_t *__restrict__ qlen)
{
    __shared__ int64_t sh[kScanThreads];
    const int chunk = (B + kScanThreads - 1) / kScanThreads;
    const int b0 = min(B, (int)threadIdx.x * chunk), b1 = min(B, b0 + chunk);
    int64_t local = 0;
    for (int b = b0; b < b1; ++b) local += counts[b];
    int64_t total;
    int64_t run = block_exclusive_scan<kScanThreads>(local, sh, &total);
    for (int b = b0; b < b1; ++b) {
        offsets[b] = run;
        run += counts[b];
    }
    if (threadIdx.x == 0) {
        offsets[B] = total;
        qlen[0] = total;
    }
}

__global__ void __launch_bounds__(kThreads)
k_queue_fill(const int8_t *__restrict__ spins, int L, BondRule rule,
             const int64_t *__restrict__ offsets, uint32_t *__restrict__ queue)
{
    __shared__ int64_t sh[kThreads];
    const int s = blockIdx.x;
    const int N = L * L;
    const int nb = 4 * N;
    const int8_t *sp = spins + (int64_t)s * N;
    const int chunk = (nb + kThreads - 1) / kThreads;
    const int b0 = min(nb, (int)threadIdx.x * chunk), b1 = min(nb, b0 + chunk);
    auto active = [&](int b) -> bool {
        const int i = b >> 2, t = b & 3;
        const int x = i % L, y = i / L;
        const int j = wrapi(y + bond_dy(t), L) * L + wrapi(x + bond_dx(t), L);
        return rule.active(t, sp[i], sp[j]);
    };
    int64_t cnt = 0;
    for (int b = b0; b < b1; ++b) cnt += active(b);
    int64_t total;
    int64_t pos = offsets[s] + block_exclusive_scan<kThreads>(cnt, sh, &total);
    for (int b = b0; b < b1; ++b)
        if (active(b)) queue[pos++] = pack_item(s, b);
}

__global__ void k_queue_expand(const int8_t *__restrict__ spins, int L, int tj,
                               const uint32_t *__restrict__ queue, const int64_t *__restrict__ qlen,
                               int64_t capacity, int marshall, int32_t *__restrict__ bond_ids,
                               int8_t *__restrict__ mu)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = min(qlen[0], capacity);
    if (q >= n) return;
    const uint32_t e = queue[q];
    const int b = item_bond(e);
    bond_ids[q] = b;
    // Exchanging an antiparallel pair between the two sublattices (J1 bond)
    // changes the number of up spins on sublattice A by one; a J2 pair lies
    // on one sublattice and leaves it unchanged.  t-J: an up electron moving
    // to the other sublattice changes the count too, a down electron not.
    int flips = (b & 3) < 2;
    if (tj) {
        const int i = b >> 2, t = b & 3, x = i % L, y = i / L;
        const int j = wrapi(y + bond_dy(t), L) * L + wrapi(x + bond_dx(t), L);
        const int8_t *sp = spins + (int64_t)item_sample(e) * L * L;
        const int a = sp[i], c = sp[j];
        flips = (a * c == -1) || (a + c > 0);
    }
    mu[q] = (int8_t)((marshall && flips) ? -1 : 1);
}

// Marshall sign (-1)^{#up spins on sublattice (x+y) even} of every sample.
__global__ void __launch_bounds__(kThreads)
k_marshall(const int8_t *__restrict__ spins, int L, int marshall, int tj,
           int8_t *__restrict__ sign, int32_t *err)
{
    const int s = blockIdx.x;
    const int N = L * L;
    const int8_t *sp = spins + (int64_t)s * N;
    int ups = 0, bad = 0;
    for (int i = threadIdx.x; i < N; i += kThreads) {
        const int v = sp[i];
        bad |= tj ? (v < -1 || v > 1) : (v != 1 && v != -1);
        ups += (((i % L) + (i / L)) % 2 == 0) && v > 0;
    }
    __shared__ int red[2][kThreads];
    red[0][threadIdx.x] = ups;
    red[1][threadIdx.x] = bad;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] |= red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (sign) sign[s] = (int8_t)((marshall && (red[0][0] & 1)) ? -1 : 1);
        if (red[1][0]) atomicOr(err, kErrSpin);
    }
}

BondRule rule_of(const nqs_ctx *c)
{
    const int tj = c->model == kModelTJ;
    return BondRule{c->J1 != 0.0 ? 1 : 0, (!tj && c->J2 != 0.0) ? 1 : 0, tj,
                    (tj && c->t_hop != 0.0) ? 1 : 0};
}

}  // namespace

void launch_marshall(const nqs_ctx *c, const int8_t *spins, int B, int8_t *sign, hipStream_t s)
{
    if (B <= 0) return;
    NQS_LAUNCH(k_marshall, dim3(B), dim3(kThreads), 0, s, spins, c->L, c->marshall,
               c->model == kModelTJ ? 1 : 0, sign, c->err);
}

void launch_bond_count(const nqs_ctx *c, const int8_t *spins, int B, int32_t *counts,
                       double *ediag, hipStream_t s)
{
    if (B <= 0) return;
    NQS_LAUNCH(k_bond_count, dim3(B), dim3(kThreads), 0, s, spins, c->L, c->J1, c->J2,
               rule_of(c), counts, ediag, c->err);
}

void launch_scan(const int32_t *counts, int B, int64_t *offsets, int64_t *qlen, hipStream_t s)
{
    NQS_LAUNCH(k_scan, dim3(1), dim3(kScanThreads), 0, s, counts, B, offsets, qlen);
}

void launch_queue_fill(const nqs_ctx *c, const int8_t *spins, int B, const int64_t *offsets,
                       uint32_t *queue, hipStream_t s)
{
    if (B <= 0) return;
    NQS_LAUNCH(k_queue_fill, dim3(B), dim3(kThreads), 0, s, spins, c->L, rule_of(c), offsets,
               queue);
}

void launch_queue_expand(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                         const int64_t *qlen, int64_t capacity, int32_t *bond_ids, int8_t *mu,
                         hipStream_t s)
{
    if (capacity <= 0) return;
    const int64_t blocks = (capacity + 255) / 256;
    NQS_LAUNCH(k_queue_expand, dim3((unsigned)blocks), dim3(256), 0, s, spins, c->L,
               c->model == kModelTJ ? 1 : 0, queue, qlen, capacity, c->marshall, bond_ids, mu);
}

}  // namespace nqs
