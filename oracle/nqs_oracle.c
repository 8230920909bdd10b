/*
 * nqs_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see
 * nqs_oracle.h).  Loaded only by tests/, the smoke check and the benchmark's
 * CPU-baseline leg.
 *
 * Each function below follows a passage of arxiv 2204.07816:
 *   - Hamiltonian: Sec. 6.1, Eq. (J1J2), J1 = 1, J2 = 0.5; spin operators
 *     S = sigma/2 (reading: per-site energies near -0.50 printed in Sec. 7.3-7.4
 *     fix the spin-1/2 normalisation).
 *   - wave function |Psi> = sum_S W(S)|S>: Sec. 3.2, Eq. (psi); sign rule of
 *     Table 1, read as the Marshall sign on sublattice (x+y) even.
 *   - local energy E_loc(S) = sum_S' W(S')/W(S) <S'|H|S>, S' = S with one
 *     antiparallel nearest or next-nearest pair exchanged: Sec. 5.4.1
 *     ("Hotspot energy calculation").
 *   - CNN with periodic (PBC) padding and a product of neurons as output:
 *     Sec. 5.2; the layer shape (3x3 conv, ln cosh, sum pool) is the
 *     configuration this library is checked on.
 *   - CNN1 (Sec. 5.2: convolution, 1D max-pooling, transposed convolution,
 *     product of neurons) in the reading stated in nqs_oracle.h; its
 *     hyper-parameters are in a missing figure, so the architecture itself
 *     is parity unpinned against the paper (the functions are pinned
 *     against torch's conv2d / conv_transpose2d / autograd and the exact
 *     diagonalisation).
 *   - CNN2 (Sec. 5.2: CNN1's block behind an embedding of the site states,
 *     the max-pooling at stride one with the first channel copied after the
 *     last, a final convolution to one channel, product of neurons) in the
 *     reading stated in nqs_oracle.h; parity unpinned against the paper for
 *     the same reason (pinned against torch, symmetries and the t-J exact
 *     diagonalisation).
 *   - t-J model: Sec. 6.1, Eq. (tJ), with the fermions encoded by the
 *     Jordan-Wigner transformation along the site order i = y*L + x.
 *   - O_loc = per-sample log-derivative and the SR update: Sec. 3.2 and
 *     Sec. 5.4.1 ("Distributed SR computation"), solved here by CG with an
 *     absolute diagonal shift, 1/Ns normalisation, x0 = 0.
 *
 * Pins (tests/test_oracle_*.py): closed forms of the Neel / stripe /
 * ferromagnet connected lists and diagonal energies; Marshall theorem on the
 * exact 4x4 J2 = 0 ground state; exhaustive <psi|H|psi>/<psi|psi> on 4x4;
 * zero variance of E_loc for the exact eigenvector; translation and spin-flip
 * invariance; torch-CPU circular conv2d for the forward; central finite
 * differences and torch autograd for O; numpy dense solve for SR.  t-J:
 * an exact diagonalisation built from fermion creation / annihilation
 * operators (itself pinned by free-fermion spectra and by the no-hole
 * reduction to the Heisenberg model) gives E_loc = E0 on every configuration
 * of its ground state and <psi|H|psi> for a CNN amplitude.
 */
#include "nqs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* lattice                                                              */
/* ------------------------------------------------------------------ */

static int wrap(int a, int L) { return ((a % L) + L) % L; }

int64_t oracle_num_params(int K, int C)
{
    if (K < 1 || C < 1) return 0;
    int64_t p = (int64_t)C * 1 * 9 + C;                     /* layer 1: 1 -> C */
    p += (int64_t)(K - 1) * ((int64_t)C * C * 9 + C);       /* layers 2..K     */
    return p;
}

int oracle_marshall_sign(int L, const int8_t *spins)
{
    int ups_on_a = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x)
            if (((x + y) % 2 == 0) && spins[y * L + x] > 0) ++ups_on_a;
    return (ups_on_a % 2 == 0) ? 1 : -1;
}

int oracle_bond_sites(int L, int b, int *site_i, int *site_j)
{
    int i = b / 4, t = b % 4;
    int x = i % L, y = i / L;
    int dx = 0, dy = 0, cls = 1;
    switch (t) {
    case 0: dx = 1; dy = 0; cls = 1; break;   /* nearest, +x        */
    case 1: dx = 0; dy = 1; cls = 1; break;   /* nearest, +y        */
    case 2: dx = 1; dy = 1; cls = 2; break;   /* next-nearest, +x+y */
    default: dx = 1; dy = -1; cls = 2; break; /* next-nearest, +x-y */
    }
    *site_i = i;
    *site_j = wrap(y + dy, L) * L + wrap(x + dx, L);
    return cls;
}

/* ------------------------------------------------------------------ */
/* Hamiltonian: connected configurations and diagonal part              */
/* ------------------------------------------------------------------ */

void oracle_connected(int L, double J1, double J2, const int8_t *spins,
                      int32_t *count, int32_t *bond_ids, int8_t *mu,
                      double *e_diag)
{
    const int N = L * L;
    int8_t *flipped = (int8_t *)malloc((size_t)N);
    int n = 0;
    double diag = 0.0;
    int m0 = oracle_marshall_sign(L, spins);
    for (int b = 0; b < 4 * N; ++b) {
        int si, sj;
        int cls = oracle_bond_sites(L, b, &si, &sj);
        double J = (cls == 1) ? J1 : J2;
        /* diagonal: J S^z_i S^z_j = J s_i s_j / 4 */
        diag += J * (double)spins[si] * (double)spins[sj] / 4.0;
        if (J != 0.0 && spins[si] != spins[sj]) {
            memcpy(flipped, spins, (size_t)N);
            flipped[si] = spins[sj];
            flipped[sj] = spins[si];
            bond_ids[n] = b;
            mu[n] = (int8_t)(oracle_marshall_sign(L, flipped) * m0);
            ++n;
        }
    }
    *count = n;
    *e_diag = diag;
    free(flipped);
}

/* ------------------------------------------------------------------ */
/* CNN forward: plain loops, channel-major activations                  */
/* ------------------------------------------------------------------ */

/* ln cosh z.  Near 0 use cosh z - 1 = 2 sinh^2(z/2), which keeps full relative
 * precision of the z^2/2 leading term; for |z| > 1 use
 * |z| + log1p(exp(-2|z|)) - ln 2, which cannot overflow.                   */
static double ln_cosh(double z)
{
    double a = fabs(z);
    if (a <= 1.0) {
        double sh = sinh(0.5 * a);
        return log1p(2.0 * sh * sh);
    }
    return a + log1p(exp(-2.0 * a)) - M_LN2;
}

/* offsets of layer k's weights and biases in the canonical vector */
static void layer_offsets(int K, int C, int k, int64_t *w_off, int64_t *b_off,
                          int *cin)
{
    int64_t off = 0;
    for (int l = 0; l < k; ++l) {
        int ci = (l == 0) ? 1 : C;
        off += (int64_t)C * ci * 9 + C;
    }
    *cin = (k == 0) ? 1 : C;
    *w_off = off;
    *b_off = off + (int64_t)C * (*cin) * 9;
}

/* one circular 3x3 cross-correlation layer: z[co][y][x] */
static void conv_layer(int L, int cin, int cout, const double *W, const double *bias,
                       const double *h_in, double *z_out)
{
    for (int co = 0; co < cout; ++co)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                double acc = bias[co];
                for (int ci = 0; ci < cin; ++ci)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            int yy = wrap(y + ky - 1, L), xx = wrap(x + kx - 1, L);
                            acc += W[((co * cin + ci) * 3 + ky) * 3 + kx] *
                                   h_in[(ci * L + yy) * L + xx];
                        }
                z_out[(co * L + y) * L + x] = acc;
            }
}

/* forward pass; if zs != NULL, stores every pre-activation z_k (k = 1..K)
 * as zs[(k-1)*C*N ...] for the backward pass.  Returns f = sum h_K.        */
static double cnn_forward(int L, int K, int C, const double *w, const int8_t *spins,
                          double *h_a, double *h_b, double *zs)
{
    const int N = L * L;
    for (int i = 0; i < N; ++i) h_a[i] = (double)spins[i];
    double *h_in = h_a, *h_out = h_b;
    for (int k = 0; k < K; ++k) {
        int64_t wo, bo;
        int cin;
        layer_offsets(K, C, k, &wo, &bo, &cin);
        conv_layer(L, cin, C, w + wo, w + bo, h_in, h_out);
        if (zs) memcpy(zs + (size_t)k * C * N, h_out, sizeof(double) * (size_t)C * N);
        for (int q = 0; q < C * N; ++q) h_out[q] = ln_cosh(h_out[q]);
        double *t = h_in; h_in = h_out; h_out = t;
    }
    double f = 0.0;                        /* sum pool: c, then y, then x */
    for (int q = 0; q < C * N; ++q) f += h_in[q];
    return f;
}

static int threads_or_default(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

void oracle_log_psi(int L, int K, int C, const double *w, const int8_t *spins,
                    int64_t B, double *log_abs, int8_t *sign, int nthreads)
{
    const int N = L * L;
    int nt = threads_or_default(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        double *ha = (double *)malloc(sizeof(double) * (size_t)C * N);
        double *hb = (double *)malloc(sizeof(double) * (size_t)C * N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < B; ++s) {
            const int8_t *sp = spins + s * N;
            log_abs[s] = cnn_forward(L, K, C, w, sp, ha, hb, NULL);
            if (sign) sign[s] = (int8_t)oracle_marshall_sign(L, sp);
        }
        free(ha);
        free(hb);
    }
}

/* ------------------------------------------------------------------ */
/* Local energy                                                         */
/* ------------------------------------------------------------------ */

typedef struct {
    int L, K, C;
    const double *w;
    const double *log_abs_tab;
    const int8_t *sign_tab;
} amp_src;

/* amplitude of a configuration: log|psi| and sign */
static void amplitude(const amp_src *a, const int8_t *spins, double *h_a, double *h_b,
                      double *log_abs, int *sign)
{
    if (a->w) {
        *log_abs = cnn_forward(a->L, a->K, a->C, a->w, spins, h_a, h_b, NULL);
        *sign = oracle_marshall_sign(a->L, spins);
    } else {
        int64_t idx = 0;
        const int N = a->L * a->L;
        for (int i = 0; i < N; ++i)
            if (spins[i] > 0) idx |= ((int64_t)1 << i);
        *log_abs = a->log_abs_tab[idx];
        *sign = a->sign_tab[idx];
    }
}

static double local_energy_one(const amp_src *a, double J1, double J2,
                               const int8_t *spins, int8_t *work, double *h_a, double *h_b)
{
    const int L = a->L, N = L * L;
    double f0;
    int m0;
    amplitude(a, spins, h_a, h_b, &f0, &m0);
    double e = 0.0;
    for (int b = 0; b < 4 * N; ++b) {
        int si, sj;
        int cls = oracle_bond_sites(L, b, &si, &sj);
        double J = (cls == 1) ? J1 : J2;
        e += J * (double)spins[si] * (double)spins[sj] / 4.0;    /* <S|H|S>     */
        if (J == 0.0 || spins[si] == spins[sj]) continue;
        memcpy(work, spins, (size_t)N);                         /* S' = S^b    */
        work[si] = spins[sj];
        work[sj] = spins[si];
        double f1;
        int m1;
        amplitude(a, work, h_a, h_b, &f1, &m1);
        /* <S'|H|S> = J/2 for the exchanged pair; W(S')/W(S) */
        e += (J / 2.0) * (double)(m1 * m0) * exp(f1 - f0);
    }
    return e;
}

static void local_energy_batch(const amp_src *a, double J1, double J2,
                               const int8_t *spins, int64_t B, double *e_loc, int nthreads)
{
    const int N = a->L * a->L;
    const int C = a->C > 0 ? a->C : 1;
    int nt = threads_or_default(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        int8_t *work = (int8_t *)malloc((size_t)N);
        double *ha = (double *)malloc(sizeof(double) * (size_t)C * N);
        double *hb = (double *)malloc(sizeof(double) * (size_t)C * N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < B; ++s)
            e_loc[s] = local_energy_one(a, J1, J2, spins + s * N, work, ha, hb);
        free(work);
        free(ha);
        free(hb);
    }
}

void oracle_local_energy(int L, double J1, double J2, int K, int C,
                         const double *w, const int8_t *spins, int64_t B,
                         double *e_loc, int nthreads)
{
    amp_src a = {L, K, C, w, NULL, NULL};
    local_energy_batch(&a, J1, J2, spins, B, e_loc, nthreads);
}

void oracle_local_energy_table(int L, double J1, double J2,
                               const double *log_abs_tab, const int8_t *sign_tab,
                               const int8_t *spins, int64_t B, double *e_loc,
                               int nthreads)
{
    amp_src a = {L, 0, 0, NULL, log_abs_tab, sign_tab};
    local_energy_batch(&a, J1, J2, spins, B, e_loc, nthreads);
}

/* ------------------------------------------------------------------ */
/* t-J model (Sec. 6.1, Eq. tJ)                                         */
/* ------------------------------------------------------------------ */
/* A site holds an up electron (+1), a down electron (-1) or a hole (0); no
 * site is doubly occupied.  The fermion modes are ordered site by site along
 * i = y*L + x (the one-dimensional order of the Jordan-Wigner encoding, Sec.
 * 6.1), and a basis state is the product of its creation operators in that
 * order.  Only nearest-neighbour bonds (t = 0, 1) carry terms:
 *   - J (S_i.S_j - n_i n_j / 4): diagonal J (s_i s_j - |s_i| |s_j|) / 4, and
 *     for an antiparallel pair the spin exchange with <S'|H|S> = +J/2 (the
 *     two Jordan-Wigner strings of the exchange cancel);
 *   - -t sum_sigma (c+_{i sigma} c_{j sigma} + h.c.): an electron next to a
 *     hole moves onto it, <S'|H|S> = -t (-1)^{n}, n the number of electrons
 *     on the sites strictly between i and j in the site order (the
 *     Jordan-Wigner string of the hop).                                   */

static int jw_string_sign(const int8_t *spins, int i, int j)
{
    int lo = i < j ? i : j, hi = i < j ? j : i, n = 0;
    for (int k = lo + 1; k < hi; ++k) n += (spins[k] != 0);
    return (n % 2 == 0) ? 1 : -1;
}

static int valid_tj_spin(int v) { return v == 1 || v == -1 || v == 0; }

/* <S'|H|S> of the nearest-neighbour pair (si, sj) of S, or 0 when the pair
 * has no off-diagonal term (equal values, or a zero coupling).             */
static double tj_offdiag(double t, double J, const int8_t *spins, int si, int sj)
{
    int a = spins[si], b = spins[sj];
    if (a == b) return 0.0;
    if (a != 0 && b != 0) return J / 2.0;                     /* exchange */
    return -t * (double)jw_string_sign(spins, si, sj);        /* hop      */
}

static double tj_diag_bond(double J, int a, int b)
{
    return J * ((double)a * (double)b / 4.0 - (double)(a != 0) * (double)(b != 0) / 4.0);
}

void oracle_tj_connected(int L, double t, double J, const int8_t *spins,
                         int32_t *count, int32_t *bond_ids, int8_t *mu,
                         double *hval, double *e_diag)
{
    const int N = L * L;
    int8_t *moved = (int8_t *)malloc((size_t)N);
    int n = 0;
    double diag = 0.0;
    int m0 = oracle_marshall_sign(L, spins);
    for (int b = 0; b < 4 * N; ++b) {
        int si, sj;
        if (oracle_bond_sites(L, b, &si, &sj) != 1) continue;
        diag += tj_diag_bond(J, spins[si], spins[sj]);
        double h = tj_offdiag(t, J, spins, si, sj);
        if (h == 0.0) continue;
        memcpy(moved, spins, (size_t)N);
        moved[si] = spins[sj];
        moved[sj] = spins[si];
        bond_ids[n] = b;
        mu[n] = (int8_t)(oracle_marshall_sign(L, moved) * m0);
        hval[n] = h;
        ++n;
    }
    *count = n;
    *e_diag = diag;
    free(moved);
}

/* tabulated amplitudes of the t-J configurations: key = sum_i c_i 4^i with
 * c = 0 hole, 1 up, 2 down (N <= 31); keys sorted ascending.              */
typedef struct {
    int64_t n;
    const int64_t *keys;
    const double *log_abs;
    const int8_t *sign;
} tj_table;

static int64_t tj_key(int N, const int8_t *spins)
{
    int64_t k = 0;
    for (int i = N - 1; i >= 0; --i) {
        int c = spins[i] > 0 ? 1 : (spins[i] < 0 ? 2 : 0);
        k = 4 * k + c;
    }
    return k;
}

/* 1 and the amplitude when the configuration is in the table, else 0 */
static int tj_lookup(const tj_table *tab, int N, const int8_t *spins, double *log_abs, int *sign)
{
    int64_t key = tj_key(N, spins), lo = 0, hi = tab->n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (tab->keys[mid] == key) {
            *log_abs = tab->log_abs[mid];
            *sign = tab->sign[mid];
            return 1;
        }
        if (tab->keys[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return 0;
}

/* E_loc(S) = sum_<ij> J (s_i s_j - |s_i||s_j|)/4 + sum_S' <S'|H|S> W(S')/W(S)
 * over the nearest-neighbour pairs with an off-diagonal term.  W from the
 * CNN (w != NULL, Marshall sign) or from the table.                       */
static double tj_local_energy_one(int L, int K, int C, const double *w, const tj_table *tab,
                                  double t, double J, const int8_t *spins, int8_t *work,
                                  double *h_a, double *h_b)
{
    const int N = L * L;
    double f0 = 0.0;
    int m0 = 1;
    if (w) {
        f0 = cnn_forward(L, K, C, w, spins, h_a, h_b, NULL);
        m0 = oracle_marshall_sign(L, spins);
    } else if (!tj_lookup(tab, N, spins, &f0, &m0) || m0 == 0) {
        return NAN;                                  /* W(S) = 0: undefined */
    }
    double e = 0.0;
    for (int b = 0; b < 4 * N; ++b) {
        int si, sj;
        if (oracle_bond_sites(L, b, &si, &sj) != 1) continue;
        e += tj_diag_bond(J, spins[si], spins[sj]);
        double h = tj_offdiag(t, J, spins, si, sj);
        if (h == 0.0) continue;
        memcpy(work, spins, (size_t)N);
        work[si] = spins[sj];
        work[sj] = spins[si];
        double f1;
        int m1;
        if (w) {
            f1 = cnn_forward(L, K, C, w, work, h_a, h_b, NULL);
            m1 = oracle_marshall_sign(L, work);
        } else if (!tj_lookup(tab, N, work, &f1, &m1)) {
            continue;                                /* W(S') = 0 */
        }
        e += h * (double)(m1 * m0) * exp(f1 - f0);
    }
    return e;
}

static void tj_local_energy_batch(int L, int K, int C, const double *w, const tj_table *tab,
                                  double t, double J, const int8_t *spins, int64_t B,
                                  double *e_loc, int nthreads)
{
    const int N = L * L;
    const int Cb = C > 0 ? C : 1;
    int nt = threads_or_default(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        int8_t *work = (int8_t *)malloc((size_t)N);
        double *ha = (double *)malloc(sizeof(double) * (size_t)Cb * N);
        double *hb = (double *)malloc(sizeof(double) * (size_t)Cb * N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < B; ++s)
            e_loc[s] = tj_local_energy_one(L, K, C, w, tab, t, J, spins + s * N, work, ha, hb);
        free(work);
        free(ha);
        free(hb);
    }
}

int oracle_tj_check(int L, const int8_t *spins, int64_t B)
{
    for (int64_t q = 0; q < B * (int64_t)L * L; ++q)
        if (!valid_tj_spin(spins[q])) return 0;
    return 1;
}

void oracle_tj_local_energy(int L, double t, double J, int K, int C, const double *w,
                            const int8_t *spins, int64_t B, double *e_loc, int nthreads)
{
    tj_local_energy_batch(L, K, C, w, NULL, t, J, spins, B, e_loc, nthreads);
}

void oracle_tj_local_energy_table(int L, double t, double J, int64_t n_tab, const int64_t *keys,
                                  const double *log_abs_tab, const int8_t *sign_tab,
                                  const int8_t *spins, int64_t B, double *e_loc, int nthreads)
{
    tj_table tab = {n_tab, keys, log_abs_tab, sign_tab};
    tj_local_energy_batch(L, 0, 0, NULL, &tab, t, J, spins, B, e_loc, nthreads);
}

/* ------------------------------------------------------------------ */
/* CNN1 (Sec. 5.2): blocks of convolution, 1D max-pooling, transposed    */
/* convolution; output the product of the neurons                        */
/* ------------------------------------------------------------------ */
/* Reading (the block figure is missing): block k maps c_in channels
 * (1 for the spins, else C) to C channels by
 *   z[co][p]  = a[co] + sum_{ci,ky,kx} W[co][ci][ky][kx] h[ci][p + (ky-1, kx-1)]   (co < 2C)
 *   m[c][p]   = max(z[2c][p], z[2c+1][p])          (1D max-pool over channel pairs)
 *   u[co][p]  = v[co] + sum_{ci,ky,kx} V[ci][co][ky][kx] m[ci][p - (ky-1, kx-1)]
 *               (transposed convolution, stride 1)
 * with every lattice index taken mod L (padding by the periodic boundary).
 * psi_net = prod_{c,p} u_K[c][p]: log|psi| = sum log|u_K|, sign = prod sign(u_K).
 * Canonical order per block: W, a, V, v.                                 */

int64_t oracle_cnn1_num_params(int Kb, int C)
{
    if (Kb < 1 || C < 1) return 0;
    int64_t p = 0;
    for (int k = 0; k < Kb; ++k) {
        int cin = (k == 0) ? 1 : C;
        p += (int64_t)2 * C * cin * 9 + 2 * C + (int64_t)C * C * 9 + C;
    }
    return p;
}

typedef struct {
    int64_t W, a, V, v;   /* offsets of one block's parameters */
    int cin;
} cnn1_block;

static cnn1_block cnn1_offsets(int C, int k)
{
    cnn1_block o;
    int64_t off = 0;
    for (int l = 0; l < k; ++l) {
        int ci = (l == 0) ? 1 : C;
        off += (int64_t)2 * C * ci * 9 + 2 * C + (int64_t)C * C * 9 + C;
    }
    o.cin = (k == 0) ? 1 : C;
    o.W = off;
    o.a = o.W + (int64_t)2 * C * o.cin * 9;
    o.V = o.a + 2 * C;
    o.v = o.V + (int64_t)C * C * 9;
    return o;
}

/* one block: h [cin][N] -> z [2C][N], m [C][N], u [C][N] */
static void cnn1_block_forward(int L, int C, const double *w, cnn1_block o, const double *h,
                               double *z, double *m, double *u)
{
    const int N = L * L;
    for (int co = 0; co < 2 * C; ++co)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                double acc = w[o.a + co];
                for (int ci = 0; ci < o.cin; ++ci)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx)
                            acc += w[o.W + ((co * o.cin + ci) * 3 + ky) * 3 + kx] *
                                   h[ci * N + wrap(y + ky - 1, L) * L + wrap(x + kx - 1, L)];
                z[co * N + y * L + x] = acc;
            }
    for (int c = 0; c < C; ++c)
        for (int p = 0; p < N; ++p) {
            double z0 = z[(2 * c) * N + p], z1 = z[(2 * c + 1) * N + p];
            m[c * N + p] = (z1 > z0) ? z1 : z0;
        }
    for (int co = 0; co < C; ++co)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                double acc = w[o.v + co];
                for (int ci = 0; ci < C; ++ci)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx)
                            acc += w[o.V + ((ci * C + co) * 3 + ky) * 3 + kx] *
                                   m[ci * N + wrap(y - ky + 1, L) * L + wrap(x - kx + 1, L)];
                u[co * N + y * L + x] = acc;
            }
}

/* forward of all blocks; zs / us (may be NULL) keep every block's z and u.
 * Returns log|psi_net|; *neg = number of negative output neurons.       */
static double cnn1_forward(int L, int Kb, int C, const double *w, const int8_t *spins,
                           double *hin, double *z, double *m, double *u, double *zs, double *us,
                           int *neg)
{
    const int N = L * L;
    for (int i = 0; i < N; ++i) hin[i] = (double)spins[i];
    const double *h = hin;
    for (int k = 0; k < Kb; ++k) {
        cnn1_block o = cnn1_offsets(C, k);
        double *zk = zs ? zs + (size_t)k * 2 * C * N : z;
        double *uk = us ? us + (size_t)k * C * N : u;
        cnn1_block_forward(L, C, w, o, h, zk, m, uk);
        if (!us) {                       /* the next block reads u from hin */
            memcpy(hin, uk, sizeof(double) * (size_t)C * N);
            h = hin;
        } else {
            h = uk;
        }
    }
    const double *uK = us ? us + (size_t)(Kb - 1) * C * N : hin;
    double f = 0.0;
    int n = 0;
    for (int q = 0; q < C * N; ++q) {
        f += log(fabs(uK[q]));
        n += (uK[q] < 0.0);
    }
    *neg = n;
    return f;
}

typedef struct {
    double *hin, *z, *m, *u;
} cnn1_bufs;

static void cnn1_bufs_alloc(cnn1_bufs *b, int L, int C)
{
    size_t n = (size_t)L * L * (size_t)C;
    b->hin = (double *)malloc(sizeof(double) * n);
    b->z = (double *)malloc(sizeof(double) * 2 * n);
    b->m = (double *)malloc(sizeof(double) * n);
    b->u = (double *)malloc(sizeof(double) * n);
}

static void cnn1_bufs_free(cnn1_bufs *b)
{
    free(b->hin);
    free(b->z);
    free(b->m);
    free(b->u);
}

/* psi = M(s)^marshall * prod u_K: log|psi| and sign */
static double cnn1_amplitude(int L, int Kb, int C, const double *w, int marshall,
                             const int8_t *spins, cnn1_bufs *b, int *sign)
{
    int neg;
    double f = cnn1_forward(L, Kb, C, w, spins, b->hin, b->z, b->m, b->u, NULL, NULL, &neg);
    int sg = (neg % 2 == 0) ? 1 : -1;
    if (marshall) sg *= oracle_marshall_sign(L, spins);
    *sign = sg;
    return f;
}

void oracle_cnn1_log_psi(int L, int Kb, int C, const double *w, int marshall,
                         const int8_t *spins, int64_t B, double *log_abs, int8_t *sign,
                         int nthreads)
{
    const int N = L * L;
    int nt = threads_or_default(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        cnn1_bufs b;
        cnn1_bufs_alloc(&b, L, C);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < B; ++s) {
            int sg;
            log_abs[s] = cnn1_amplitude(L, Kb, C, w, marshall, spins + s * N, &b, &sg);
            if (sign) sign[s] = (int8_t)sg;
        }
        cnn1_bufs_free(&b);
    }
}

void oracle_cnn1_local_energy(int L, double J1, double J2, int Kb, int C, const double *w,
                              int marshall, const int8_t *spins, int64_t B, double *e_loc,
                              int nthreads)
{
    const int N = L * L;
    int nt = threads_or_default(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        cnn1_bufs b;
        cnn1_bufs_alloc(&b, L, C);
        int8_t *work = (int8_t *)malloc((size_t)N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < B; ++s) {
            const int8_t *sp = spins + s * N;
            int m0;
            double f0 = cnn1_amplitude(L, Kb, C, w, marshall, sp, &b, &m0);
            double e = 0.0;
            for (int bd = 0; bd < 4 * N; ++bd) {
                int si, sj;
                int cls = oracle_bond_sites(L, bd, &si, &sj);
                double J = (cls == 1) ? J1 : J2;
                e += J * (double)sp[si] * (double)sp[sj] / 4.0;
                if (J == 0.0 || sp[si] == sp[sj]) continue;
                memcpy(work, sp, (size_t)N);
                work[si] = sp[sj];
                work[sj] = sp[si];
                int m1;
                double f1 = cnn1_amplitude(L, Kb, C, w, marshall, work, &b, &m1);
                e += (J / 2.0) * (double)(m1 * m0) * exp(f1 - f0);
            }
            e_loc[s] = e;
        }
        free(work);
        cnn1_bufs_free(&b);
    }
}

/* O[p] = d log|psi| / d theta_p by reverse mode through the blocks; the
 * max routes its gradient to the larger input (the first on a tie).      */
static void cnn1_log_deriv_one(int L, int Kb, int C, const double *w, const int8_t *spins,
                               double *O, double *zs, double *us, cnn1_bufs *b,
                               double *gu, double *gm, double *gz, double *gh)
{
    const int N = L * L;
    int neg;
    cnn1_forward(L, Kb, C, w, spins, b->hin, b->z, b->m, b->u, zs, us, &neg);
    const double *uK = us + (size_t)(Kb - 1) * C * N;
    for (int q = 0; q < C * N; ++q) gu[q] = 1.0 / uK[q];
    for (int k = Kb - 1; k >= 0; --k) {
        cnn1_block o = cnn1_offsets(C, k);
        const double *zk = zs + (size_t)k * 2 * C * N;
        /* block input h and the pooled m */
        double *h = b->hin;
        if (k == 0) {
            for (int i = 0; i < N; ++i) h[i] = (double)spins[i];
        } else {
            memcpy(h, us + (size_t)(k - 1) * C * N, sizeof(double) * (size_t)C * N);
        }
        double *m = b->m;
        for (int c = 0; c < C; ++c)
            for (int p = 0; p < N; ++p) {
                double z0 = zk[(2 * c) * N + p], z1 = zk[(2 * c + 1) * N + p];
                m[c * N + p] = (z1 > z0) ? z1 : z0;
            }
        /* transposed convolution: dV, dv, and dL/dm */
        for (int ci = 0; ci < C; ++ci)
            for (int co = 0; co < C; ++co)
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx) {
                        double acc = 0.0;
                        for (int y = 0; y < L; ++y)
                            for (int x = 0; x < L; ++x)
                                acc += gu[co * N + y * L + x] *
                                       m[ci * N + wrap(y - ky + 1, L) * L + wrap(x - kx + 1, L)];
                        O[o.V + ((ci * C + co) * 3 + ky) * 3 + kx] = acc;
                    }
        for (int co = 0; co < C; ++co) {
            double acc = 0.0;
            for (int p = 0; p < N; ++p) acc += gu[co * N + p];
            O[o.v + co] = acc;
        }
        for (int ci = 0; ci < C; ++ci)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    double acc = 0.0;
                    for (int co = 0; co < C; ++co)
                        for (int ky = 0; ky < 3; ++ky)
                            for (int kx = 0; kx < 3; ++kx)
                                acc += w[o.V + ((ci * C + co) * 3 + ky) * 3 + kx] *
                                       gu[co * N + wrap(y + ky - 1, L) * L + wrap(x + kx - 1, L)];
                    gm[ci * N + y * L + x] = acc;
                }
        /* max over channel pairs */
        for (int c = 0; c < C; ++c)
            for (int p = 0; p < N; ++p) {
                double z0 = zk[(2 * c) * N + p], z1 = zk[(2 * c + 1) * N + p];
                int second = (z1 > z0);
                gz[(2 * c) * N + p] = second ? 0.0 : gm[c * N + p];
                gz[(2 * c + 1) * N + p] = second ? gm[c * N + p] : 0.0;
            }
        /* convolution: dW, da, and dL/dh for the block below */
        for (int co = 0; co < 2 * C; ++co)
            for (int ci = 0; ci < o.cin; ++ci)
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx) {
                        double acc = 0.0;
                        for (int y = 0; y < L; ++y)
                            for (int x = 0; x < L; ++x)
                                acc += gz[co * N + y * L + x] *
                                       h[ci * N + wrap(y + ky - 1, L) * L + wrap(x + kx - 1, L)];
                        O[o.W + ((co * o.cin + ci) * 3 + ky) * 3 + kx] = acc;
                    }
        for (int co = 0; co < 2 * C; ++co) {
            double acc = 0.0;
            for (int p = 0; p < N; ++p) acc += gz[co * N + p];
            O[o.a + co] = acc;
        }
        if (k > 0) {
            for (int ci = 0; ci < C; ++ci)
                for (int y = 0; y < L; ++y)
                    for (int x = 0; x < L; ++x) {
                        double acc = 0.0;
                        for (int co = 0; co < 2 * C; ++co)
                            for (int ky = 0; ky < 3; ++ky)
                                for (int kx = 0; kx < 3; ++kx)
                                    acc += w[o.W + ((co * C + ci) * 3 + ky) * 3 + kx] *
                                           gz[co * N + wrap(y - ky + 1, L) * L + wrap(x - kx + 1, L)];
                        gh[ci * N + y * L + x] = acc;
                    }
            memcpy(gu, gh, sizeof(double) * (size_t)C * N);
        }
    }
}

void oracle_cnn1_log_deriv(int L, int Kb, int C, const double *w, const int8_t *spins,
                           int64_t B, double *O, int nthreads)
{
    const int N = L * L;
    const int64_t P = oracle_cnn1_num_params(Kb, C);
    int nt = threads_or_default(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        cnn1_bufs b;
        cnn1_bufs_alloc(&b, L, C);
        size_t cn = (size_t)C * N;
        double *zs = (double *)malloc(sizeof(double) * 2 * cn * Kb);
        double *us = (double *)malloc(sizeof(double) * cn * Kb);
        double *gu = (double *)malloc(sizeof(double) * cn);
        double *gm = (double *)malloc(sizeof(double) * cn);
        double *gz = (double *)malloc(sizeof(double) * 2 * cn);
        double *gh = (double *)malloc(sizeof(double) * cn);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < B; ++s)
            cnn1_log_deriv_one(L, Kb, C, w, spins + s * N, O + s * P, zs, us, &b, gu, gm, gz, gh);
        free(zs);
        free(us);
        free(gu);
        free(gm);
        free(gz);
        free(gh);
        cnn1_bufs_free(&b);
    }
}

/* t-J local energy (Sec. 6.1, Eq. tJ) with the CNN1 amplitude: the terms of
 * tj_connected, each weighted by psi(S')/psi(s) including the network's sign. */
void oracle_tj_cnn1_local_energy(int L, double t, double J, int Kb, int C, const double *w,
                                 int marshall, const int8_t *spins, int64_t B, double *e_loc,
                                 int nthreads)
{
    const int N = L * L;
    int nt = threads_or_default(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        cnn1_bufs b;
        cnn1_bufs_alloc(&b, L, C);
        int8_t *work = (int8_t *)malloc((size_t)N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < B; ++s) {
            const int8_t *sp = spins + s * N;
            int m0;
            double f0 = cnn1_amplitude(L, Kb, C, w, marshall, sp, &b, &m0);
            double e = 0.0;
            for (int bd = 0; bd < 4 * N; ++bd) {
                int si, sj;
                if (oracle_bond_sites(L, bd, &si, &sj) != 1) continue;
                e += tj_diag_bond(J, sp[si], sp[sj]);
                double h = tj_offdiag(t, J, sp, si, sj);
                if (h == 0.0) continue;
                memcpy(work, sp, (size_t)N);
                work[si] = sp[sj];
                work[sj] = sp[si];
                int m1;
                double f1 = cnn1_amplitude(L, Kb, C, w, marshall, work, &b, &m1);
                e += h * (double)(m1 * m0) * exp(f1 - f0);
            }
            e_loc[s] = e;
        }
        free(work);
        cnn1_bufs_free(&b);
    }
}

/* ------------------------------------------------------------------ */
/* CNN2 (Sec. 5.2): CNN1's blocks behind an embedding of the site        */
/* states, with a max-pool of stride one; a final convolution to one     */
/* channel; output the product of the neurons                            */
/* ------------------------------------------------------------------ */
/* Reading (the block figure is missing): the state of site p selects an
 * embedding row, e = 0 for a hole, 1 for an up and 2 for a down electron,
 *   h0[c][p] = E[e(s_p)][c]                                   (C channels)
 * and every block maps C channels to C channels:
 *   z[co][p] = a[co] + sum_{ci,ky,kx} W[co][ci][ky][kx] h[ci][p + (ky-1, kx-1)]
 *   m[c][p]  = max(z[c][p], z[(c+1) mod C][p])
 *              (window 2 over the channels, stride 1; the last window takes
 *               the first channel, copied after the last)
 *   u[co][p] = v[co] + sum_{ci,ky,kx} V[ci][co][ky][kx] m[ci][p - (ky-1, kx-1)]
 * then y[p] = b + sum_{c,ky,kx} F[c][ky][kx] u_K[c][p + (ky-1, kx-1)] and
 * psi_net = prod_p y[p].  Lattice indices wrap mod L (the spatial padding
 * copies the first rows and columns after the last).
 * Canonical order: E[3][C]; per block W[C][C][3][3], a[C], V[C][C][3][3]
 * (input channel first), v[C]; then F[C][3][3], b.                      */

int64_t oracle_cnn2_num_params(int Kb, int C)
{
    if (Kb < 1 || C < 1) return 0;
    return (int64_t)3 * C + (int64_t)Kb * (18 * (int64_t)C * C + 2 * C) + 9 * (int64_t)C + 1;
}

typedef struct {
    int64_t W, a, V, v;
} cnn2_block;

static cnn2_block cnn2_offsets(int C, int k)
{
    cnn2_block o;
    o.W = (int64_t)3 * C + (int64_t)k * (18 * (int64_t)C * C + 2 * C);
    o.a = o.W + (int64_t)9 * C * C;
    o.V = o.a + C;
    o.v = o.V + (int64_t)9 * C * C;
    return o;
}

static int64_t cnn2_final_offset(int Kb, int C) { return cnn2_offsets(C, Kb).W; }

static int cnn2_class(int8_t s) { return s == 0 ? 0 : (s > 0 ? 1 : 2); }

/* one block: h [C][N] -> z [C][N], m [C][N], u [C][N] */
static void cnn2_block_forward(int L, int C, const double *w, cnn2_block o, const double *h,
                               double *z, double *m, double *u)
{
    const int N = L * L;
    for (int co = 0; co < C; ++co)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                double acc = w[o.a + co];
                for (int ci = 0; ci < C; ++ci)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx)
                            acc += w[o.W + ((co * C + ci) * 3 + ky) * 3 + kx] *
                                   h[ci * N + wrap(y + ky - 1, L) * L + wrap(x + kx - 1, L)];
                z[co * N + y * L + x] = acc;
            }
    for (int c = 0; c < C; ++c)
        for (int p = 0; p < N; ++p) {
            double z0 = z[c * N + p], z1 = z[((c + 1) % C) * N + p];
            m[c * N + p] = (z1 > z0) ? z1 : z0;
        }
    for (int co = 0; co < C; ++co)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                double acc = w[o.v + co];
                for (int ci = 0; ci < C; ++ci)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx)
                            acc += w[o.V + ((ci * C + co) * 3 + ky) * 3 + kx] *
                                   m[ci * N + wrap(y - ky + 1, L) * L + wrap(x - kx + 1, L)];
                u[co * N + y * L + x] = acc;
            }
}

/* the final convolution C -> 1: y [N] from u [C][N] */
static void cnn2_final(int L, int C, const double *w, int64_t fo, const double *u, double *yv)
{
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            double acc = w[fo + 9 * C];
            for (int c = 0; c < C; ++c)
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx)
                        acc += w[fo + (c * 3 + ky) * 3 + kx] *
                               u[c * L * L + wrap(y + ky - 1, L) * L + wrap(x + kx - 1, L)];
            yv[y * L + x] = acc;
        }
}

typedef struct {
    double *h0, *z, *m, *u, *y;   /* h0, y: one sample; z, m, u: Kb blocks each */
} cnn2_state;

static void cnn2_state_alloc(cnn2_state *st, int L, int Kb, int C)
{
    size_t cn = (size_t)L * L * C;
    st->h0 = (double *)malloc(sizeof(double) * cn);
    st->z = (double *)malloc(sizeof(double) * cn * Kb);
    st->m = (double *)malloc(sizeof(double) * cn * Kb);
    st->u = (double *)malloc(sizeof(double) * cn * Kb);
    st->y = (double *)malloc(sizeof(double) * (size_t)L * L);
}

static void cnn2_state_free(cnn2_state *st)
{
    free(st->h0);
    free(st->z);
    free(st->m);
    free(st->u);
    free(st->y);
}

/* forward of one configuration, keeping every block's z, m, u */
static void cnn2_forward(int L, int Kb, int C, const double *w, const int8_t *spins,
                         cnn2_state *st)
{
    const int N = L * L;
    const size_t cn = (size_t)C * N;
    for (int c = 0; c < C; ++c)
        for (int p = 0; p < N; ++p) st->h0[c * N + p] = w[cnn2_class(spins[p]) * C + c];
    for (int k = 0; k < Kb; ++k) {
        const double *h = (k == 0) ? st->h0 : st->u + (size_t)(k - 1) * cn;
        cnn2_block_forward(L, C, w, cnn2_offsets(C, k), h, st->z + (size_t)k * cn,
                           st->m + (size_t)k * cn, st->u + (size_t)k * cn);
    }
    cnn2_final(L, C, w, cnn2_final_offset(Kb, C), st->u + (size_t)(Kb - 1) * cn, st->y);
}

/* psi = M(s)^marshall * prod_p y[p]: log|psi| and sign */
static double cnn2_amplitude(int L, int Kb, int C, const double *w, int marshall,
                             const int8_t *spins, cnn2_state *st, int *sign)
{
    cnn2_forward(L, Kb, C, w, spins, st);
    double f = 0.0;
    int neg = 0;
    for (int p = 0; p < L * L; ++p) {
        f += log(fabs(st->y[p]));
        neg += (st->y[p] < 0.0);
    }
    int sg = (neg % 2 == 0) ? 1 : -1;
    if (marshall) sg *= oracle_marshall_sign(L, spins);
    *sign = sg;
    return f;
}

void oracle_cnn2_log_psi(int L, int Kb, int C, const double *w, int marshall,
                         const int8_t *spins, int64_t B, double *log_abs, int8_t *sign,
                         int nthreads)
{
    const int N = L * L;
    int nt = threads_or_default(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        cnn2_state st;
        cnn2_state_alloc(&st, L, Kb, C);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < B; ++s) {
            int sg;
            log_abs[s] = cnn2_amplitude(L, Kb, C, w, marshall, spins + s * N, &st, &sg);
            if (sign) sign[s] = (int8_t)sg;
        }
        cnn2_state_free(&st);
    }
}

/* t-J local energy (Sec. 6.1, Eq. tJ) with the CNN2 amplitude: the terms of
 * tj_connected, each weighted by psi(S')/psi(s) including the network's sign. */
void oracle_tj_cnn2_local_energy(int L, double t, double J, int Kb, int C, const double *w,
                                 int marshall, const int8_t *spins, int64_t B, double *e_loc,
                                 int nthreads)
{
    const int N = L * L;
    int nt = threads_or_default(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        cnn2_state st;
        cnn2_state_alloc(&st, L, Kb, C);
        int8_t *work = (int8_t *)malloc((size_t)N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < B; ++s) {
            const int8_t *sp = spins + s * N;
            int m0;
            double f0 = cnn2_amplitude(L, Kb, C, w, marshall, sp, &st, &m0);
            double e = 0.0;
            for (int bd = 0; bd < 4 * N; ++bd) {
                int si, sj;
                if (oracle_bond_sites(L, bd, &si, &sj) != 1) continue;
                e += tj_diag_bond(J, sp[si], sp[sj]);
                double h = tj_offdiag(t, J, sp, si, sj);
                if (h == 0.0) continue;
                memcpy(work, sp, (size_t)N);
                work[si] = sp[sj];
                work[sj] = sp[si];
                int m1;
                double f1 = cnn2_amplitude(L, Kb, C, w, marshall, work, &st, &m1);
                e += h * (double)(m1 * m0) * exp(f1 - f0);
            }
            e_loc[s] = e;
        }
        free(work);
        cnn2_state_free(&st);
    }
}

/* O[p] = d log|psi| / d theta_p by reverse mode: dlog|psi|/dy = 1/y, then
 * the final convolution, the blocks from the last to the first, and the
 * embedding rows.  m[c] = max(z[c], z[c+1]) passes its gradient to z[c]
 * unless z[c+1] is strictly larger.                                       */
static void cnn2_log_deriv_one(int L, int Kb, int C, const double *w, const int8_t *spins,
                               double *O, cnn2_state *st, double *gu, double *gm, double *gz,
                               double *gh)
{
    const int N = L * L;
    const size_t cn = (size_t)C * N;
    cnn2_forward(L, Kb, C, w, spins, st);
    /* final convolution */
    const int64_t fo = cnn2_final_offset(Kb, C);
    const double *uK = st->u + (size_t)(Kb - 1) * cn;
    for (int c = 0; c < C; ++c)
        for (int ky = 0; ky < 3; ++ky)
            for (int kx = 0; kx < 3; ++kx) {
                double acc = 0.0;
                for (int y = 0; y < L; ++y)
                    for (int x = 0; x < L; ++x)
                        acc += (1.0 / st->y[y * L + x]) *
                               uK[c * N + wrap(y + ky - 1, L) * L + wrap(x + kx - 1, L)];
                O[fo + (c * 3 + ky) * 3 + kx] = acc;
            }
    {
        double acc = 0.0;
        for (int p = 0; p < N; ++p) acc += 1.0 / st->y[p];
        O[fo + 9 * C] = acc;
    }
    for (int c = 0; c < C; ++c)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                double acc = 0.0;
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx)
                        acc += w[fo + (c * 3 + ky) * 3 + kx] /
                               st->y[wrap(y - ky + 1, L) * L + wrap(x - kx + 1, L)];
                gu[c * N + y * L + x] = acc;
            }
    for (int k = Kb - 1; k >= 0; --k) {
        cnn2_block o = cnn2_offsets(C, k);
        const double *zk = st->z + (size_t)k * cn;
        const double *mk = st->m + (size_t)k * cn;
        const double *h = (k == 0) ? st->h0 : st->u + (size_t)(k - 1) * cn;
        /* transposed convolution: dV, dv, and dL/dm */
        for (int ci = 0; ci < C; ++ci)
            for (int co = 0; co < C; ++co)
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx) {
                        double acc = 0.0;
                        for (int y = 0; y < L; ++y)
                            for (int x = 0; x < L; ++x)
                                acc += gu[co * N + y * L + x] *
                                       mk[ci * N + wrap(y - ky + 1, L) * L + wrap(x - kx + 1, L)];
                        O[o.V + ((ci * C + co) * 3 + ky) * 3 + kx] = acc;
                    }
        for (int co = 0; co < C; ++co) {
            double acc = 0.0;
            for (int p = 0; p < N; ++p) acc += gu[co * N + p];
            O[o.v + co] = acc;
        }
        for (int ci = 0; ci < C; ++ci)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    double acc = 0.0;
                    for (int co = 0; co < C; ++co)
                        for (int ky = 0; ky < 3; ++ky)
                            for (int kx = 0; kx < 3; ++kx)
                                acc += w[o.V + ((ci * C + co) * 3 + ky) * 3 + kx] *
                                       gu[co * N + wrap(y + ky - 1, L) * L + wrap(x + kx - 1, L)];
                    gm[ci * N + y * L + x] = acc;
                }
        /* the stride-one max: z[c] feeds m[c] (first input) and m[c-1]
         * (second input) */
        for (int c = 0; c < C; ++c) {
            const int cn1 = (c + 1) % C, cp1 = (c + C - 1) % C;
            for (int p = 0; p < N; ++p) {
                double g = 0.0;
                if (!(zk[cn1 * N + p] > zk[c * N + p])) g += gm[c * N + p];
                if (zk[c * N + p] > zk[cp1 * N + p]) g += gm[cp1 * N + p];
                gz[c * N + p] = g;
            }
        }
        /* convolution: dW, da, and dL/dh */
        for (int co = 0; co < C; ++co)
            for (int ci = 0; ci < C; ++ci)
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx) {
                        double acc = 0.0;
                        for (int y = 0; y < L; ++y)
                            for (int x = 0; x < L; ++x)
                                acc += gz[co * N + y * L + x] *
                                       h[ci * N + wrap(y + ky - 1, L) * L + wrap(x + kx - 1, L)];
                        O[o.W + ((co * C + ci) * 3 + ky) * 3 + kx] = acc;
                    }
        for (int co = 0; co < C; ++co) {
            double acc = 0.0;
            for (int p = 0; p < N; ++p) acc += gz[co * N + p];
            O[o.a + co] = acc;
        }
        for (int ci = 0; ci < C; ++ci)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    double acc = 0.0;
                    for (int co = 0; co < C; ++co)
                        for (int ky = 0; ky < 3; ++ky)
                            for (int kx = 0; kx < 3; ++kx)
                                acc += w[o.W + ((co * C + ci) * 3 + ky) * 3 + kx] *
                                       gz[co * N + wrap(y - ky + 1, L) * L + wrap(x - kx + 1, L)];
                    gh[ci * N + y * L + x] = acc;
                }
        memcpy(gu, gh, sizeof(double) * cn);
    }
    /* embedding rows: dE[e][c] = sum over the sites in state e */
    for (int e = 0; e < 3; ++e)
        for (int c = 0; c < C; ++c) {
            double acc = 0.0;
            for (int p = 0; p < N; ++p)
                if (cnn2_class(spins[p]) == e) acc += gu[c * N + p];
            O[e * C + c] = acc;
        }
}

void oracle_cnn2_log_deriv(int L, int Kb, int C, const double *w, const int8_t *spins,
                           int64_t B, double *O, int nthreads)
{
    const int N = L * L;
    const int64_t P = oracle_cnn2_num_params(Kb, C);
    int nt = threads_or_default(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        cnn2_state st;
        cnn2_state_alloc(&st, L, Kb, C);
        size_t cn = (size_t)C * N;
        double *gu = (double *)malloc(sizeof(double) * cn);
        double *gm = (double *)malloc(sizeof(double) * cn);
        double *gz = (double *)malloc(sizeof(double) * cn);
        double *gh = (double *)malloc(sizeof(double) * cn);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < B; ++s)
            cnn2_log_deriv_one(L, Kb, C, w, spins + s * N, O + s * P, &st, gu, gm, gz, gh);
        free(gu);
        free(gm);
        free(gz);
        free(gh);
        cnn2_state_free(&st);
    }
}

/* ------------------------------------------------------------------ */
/* Log-derivatives by reverse-mode chain rule                           */
/* ------------------------------------------------------------------ */

static void log_deriv_one(int L, int K, int C, const double *w, const int8_t *spins,
                          double *O, double *zs, double *h_a, double *h_b,
                          double *delta, double *grad_in)
{
    const int N = L * L;
    cnn_forward(L, K, C, w, spins, h_a, h_b, zs);
    /* dF/dh_K = 1, dh/dz = tanh z */
    const double *zK = zs + (size_t)(K - 1) * C * N;
    for (int q = 0; q < C * N; ++q) delta[q] = tanh(zK[q]);
    for (int k = K - 1; k >= 0; --k) {
        int64_t wo, bo;
        int cin;
        layer_offsets(K, C, k, &wo, &bo, &cin);
        const double *W = w + wo;
        /* input activations of layer k: spins, or ln cosh of z_{k-1} */
        double *h_prev = h_a;
        if (k == 0) {
            for (int i = 0; i < N; ++i) h_prev[i] = (double)spins[i];
        } else {
            const double *zp = zs + (size_t)(k - 1) * C * N;
            for (int q = 0; q < C * N; ++q) h_prev[q] = ln_cosh(zp[q]);
        }
        /* weight and bias gradients */
        for (int co = 0; co < C; ++co) {
            double db = 0.0;
            for (int p = 0; p < N; ++p) db += delta[co * N + p];
            O[bo + co] = db;
            for (int ci = 0; ci < cin; ++ci)
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx) {
                        double g = 0.0;
                        for (int y = 0; y < L; ++y)
                            for (int x = 0; x < L; ++x) {
                                int yy = wrap(y + ky - 1, L), xx = wrap(x + kx - 1, L);
                                g += delta[(co * L + y) * L + x] *
                                     h_prev[(ci * L + yy) * L + xx];
                            }
                        O[wo + ((co * cin + ci) * 3 + ky) * 3 + kx] = g;
                    }
        }
        if (k == 0) break;
        /* gradient w.r.t. the layer input (transposed circular conv) */
        memset(grad_in, 0, sizeof(double) * (size_t)cin * N);
        for (int co = 0; co < C; ++co)
            for (int ci = 0; ci < cin; ++ci)
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx) {
                        double wv = W[((co * cin + ci) * 3 + ky) * 3 + kx];
                        for (int y = 0; y < L; ++y)
                            for (int x = 0; x < L; ++x) {
                                int yy = wrap(y + ky - 1, L), xx = wrap(x + kx - 1, L);
                                grad_in[(ci * L + yy) * L + xx] +=
                                    wv * delta[(co * L + y) * L + x];
                            }
                    }
        const double *zp = zs + (size_t)(k - 1) * C * N;
        for (int q = 0; q < cin * N; ++q) delta[q] = grad_in[q] * tanh(zp[q]);
    }
}

void oracle_log_deriv(int L, int K, int C, const double *w, const int8_t *spins,
                      int64_t B, double *O, int nthreads)
{
    const int N = L * L;
    const int64_t P = oracle_num_params(K, C);
    int nt = threads_or_default(nthreads);
    (void)nt;
#pragma omp parallel num_threads(nt)
    {
        double *zs = (double *)malloc(sizeof(double) * (size_t)K * C * N);
        double *ha = (double *)malloc(sizeof(double) * (size_t)C * N);
        double *hb = (double *)malloc(sizeof(double) * (size_t)C * N);
        double *dl = (double *)malloc(sizeof(double) * (size_t)C * N);
        double *gi = (double *)malloc(sizeof(double) * (size_t)C * N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < B; ++s)
            log_deriv_one(L, K, C, w, spins + s * N, O + s * P, zs, ha, hb, dl, gi);
        free(zs);
        free(ha);
        free(hb);
        free(dl);
        free(gi);
    }
}

/* ------------------------------------------------------------------ */
/* Rounding-error sensitivities (test support for reduced-precision     */
/* evaluations of the network)                                          */
/* ------------------------------------------------------------------ */

/* Every layer of one configuration kept, channel-major [k][c][p], k = 0..K-1
 * standing for layers 1..K:
 *   z  pre-activation;  h = ln cosh z;
 *   a  = |b| + sum |W| |h_in| (the magnitude an accumulation of z runs over);
 *   g  = d f / d h_k (reverse mode; g = 1 on the last layer, whose values
 *        are summed directly);
 *   d  = d f / d z_k = g tanh z_k.                                          */
typedef struct {
    double *z, *h, *a, *g, *d;
} sens_layers;

static void sens_alloc(sens_layers *s, int K, int C, int N)
{
    const size_t n = (size_t)K * C * N;
    s->z = (double *)malloc(sizeof(double) * n);
    s->h = (double *)malloc(sizeof(double) * n);
    s->a = (double *)malloc(sizeof(double) * n);
    s->g = (double *)malloc(sizeof(double) * n);
    s->d = (double *)malloc(sizeof(double) * n);
}

static void sens_free(sens_layers *s)
{
    free(s->z); free(s->h); free(s->a); free(s->g); free(s->d);
}

/* magnitude of a 3x3 circular accumulation: |b| + sum |W| |h_in|           */
static void conv_layer_abs(int L, int cin, int cout, const double *W, const double *bias,
                           const double *h_in, double *a_out)
{
    for (int co = 0; co < cout; ++co)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                double acc = fabs(bias[co]);
                for (int ci = 0; ci < cin; ++ci)
                    for (int ky = 0; ky < 3; ++ky)
                        for (int kx = 0; kx < 3; ++kx) {
                            int yy = wrap(y + ky - 1, L), xx = wrap(x + kx - 1, L);
                            acc += fabs(W[((co * cin + ci) * 3 + ky) * 3 + kx]) *
                                   fabs(h_in[(ci * L + yy) * L + xx]);
                        }
                a_out[(co * L + y) * L + x] = acc;
            }
}

/* forward (keeping every layer) and reverse pass of one configuration;
 * returns f.  h0: N scratch values for the spins as the first input.      */
static double sens_pass(int L, int K, int C, const double *w, const int8_t *spins,
                        sens_layers *s, double *h0)
{
    const int N = L * L;
    const size_t plane = (size_t)C * N;
    for (int i = 0; i < N; ++i) h0[i] = (double)spins[i];
    for (int k = 0; k < K; ++k) {
        int64_t wo, bo;
        int cin;
        layer_offsets(K, C, k, &wo, &bo, &cin);
        const double *hin = (k == 0) ? h0 : s->h + (size_t)(k - 1) * plane;
        conv_layer(L, cin, C, w + wo, w + bo, hin, s->z + (size_t)k * plane);
        conv_layer_abs(L, cin, C, w + wo, w + bo, hin, s->a + (size_t)k * plane);
        for (size_t q = 0; q < plane; ++q)
            s->h[(size_t)k * plane + q] = ln_cosh(s->z[(size_t)k * plane + q]);
    }
    double f = 0.0;
    for (size_t q = 0; q < plane; ++q) f += s->h[(size_t)(K - 1) * plane + q];
    /* reverse: g_K = 1; d_k = g_k tanh z_k; g_{k-1} = W_k^T (*) d_k        */
    for (size_t q = 0; q < plane; ++q) s->g[(size_t)(K - 1) * plane + q] = 1.0;
    for (int k = K - 1; k >= 0; --k) {
        double *g = s->g + (size_t)k * plane, *d = s->d + (size_t)k * plane;
        const double *z = s->z + (size_t)k * plane;
        for (size_t q = 0; q < plane; ++q) d[q] = g[q] * tanh(z[q]);
        if (k == 0) break;
        int64_t wo, bo;
        int cin;
        layer_offsets(K, C, k, &wo, &bo, &cin);
        const double *W = w + wo;
        double *gp = s->g + (size_t)(k - 1) * plane;
        memset(gp, 0, sizeof(double) * plane);
        for (int co = 0; co < C; ++co)
            for (int ci = 0; ci < cin; ++ci)
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx) {
                        const double wv = W[((co * cin + ci) * 3 + ky) * 3 + kx];
                        for (int y = 0; y < L; ++y)
                            for (int x = 0; x < L; ++x) {
                                int yy = wrap(y + ky - 1, L), xx = wrap(x + kx - 1, L);
                                gp[(ci * L + yy) * L + xx] += wv * d[(co * L + y) * L + x];
                            }
                    }
    }
    return f;
}

void oracle_sens_layers(int L, int K, int C, const double *w, const int8_t *spins,
                        double *z, double *h, double *a, double *g, double *d)
{
    const int N = L * L;
    const size_t n = (size_t)K * C * N;
    sens_layers s;
    sens_alloc(&s, K, C, N);
    double *h0 = (double *)malloc(sizeof(double) * (size_t)N);
    sens_pass(L, K, C, w, spins, &s, h0);
    memcpy(z, s.z, sizeof(double) * n);
    memcpy(h, s.h, sizeof(double) * n);
    memcpy(a, s.a, sizeof(double) * n);
    memcpy(g, s.g, sizeof(double) * n);
    memcpy(d, s.d, sizeof(double) * n);
    free(h0);
    sens_free(&s);
}

/* Adds one value's coefficient to the sums: inside the changed region the
 * two evaluations round independently (two terms), outside it they share
 * one rounded value, which enters with the difference of the sensitivities. */
static void sens_term(double vp, double v, double cp, double c, double *s1, double *s2)
{
    if (vp != v) {
        const double t1 = fabs(cp * vp), t2 = fabs(c * v);
        *s1 += t1 + t2;
        *s2 += t1 * t1 + t2 * t2;
    } else {
        const double t = fabs((cp - c) * v);
        *s1 += t;
        *s2 += t * t;
    }
}

void oracle_dlog_sens(int L, int K, int C, const double *w, const int8_t *spins, int64_t B,
                      const int32_t *item_sample, const int32_t *item_bond, int64_t M,
                      double *out, int nthreads)
{
    const int N = L * L;
    const size_t plane = (size_t)C * N;
    int nt = threads_or_default(nthreads);
    (void)nt;
    (void)B;
#pragma omp parallel num_threads(nt)
    {
        sens_layers s0, s1;
        sens_alloc(&s0, K, C, N);
        sens_alloc(&s1, K, C, N);
        double *h0 = (double *)malloc(sizeof(double) * (size_t)N);
        int8_t *sp = (int8_t *)malloc((size_t)N);
#pragma omp for schedule(dynamic, 1)
        for (int64_t m = 0; m < M; ++m) {
            const int8_t *sb = spins + (int64_t)item_sample[m] * N;
            double *o = out + m * 6;
            const double f0 = sens_pass(L, K, C, w, sb, &s0, h0);
            if (item_bond[m] < 0) {
                /* the configuration itself: every value rounds once         */
                double act1 = 0, act2 = 0, acc1 = 0, acc2 = 0, lc1 = 0;
                for (int k = 0; k < K; ++k)
                    for (size_t q = 0; q < plane; ++q) {
                        const size_t i = (size_t)k * plane + q;
                        const double th = fabs(s0.g[i] * s0.h[i]);
                        const double tz = fabs(s0.d[i]) * s0.a[i];
                        if (k < K - 1) { act1 += th; act2 += th * th; }
                        acc1 += tz; acc2 += tz * tz;
                        lc1 += th;
                    }
                o[0] = f0; o[1] = act1; o[2] = sqrt(act2); o[3] = acc1; o[4] = lc1;
                o[5] = sqrt(acc2);
                continue;
            }
            int si, sj;
            oracle_bond_sites(L, item_bond[m], &si, &sj);
            memcpy(sp, sb, (size_t)N);
            sp[si] = sb[sj];
            sp[sj] = sb[si];
            const double f1 = sens_pass(L, K, C, w, sp, &s1, h0);
            double act1 = 0, act2 = 0, acc1 = 0, acc2 = 0, lc1 = 0, lc2 = 0;
            for (int k = 0; k < K; ++k)
                for (size_t q = 0; q < plane; ++q) {
                    const size_t i = (size_t)k * plane + q;
                    if (k < K - 1) sens_term(s1.h[i], s0.h[i], s1.g[i], s0.g[i], &act1, &act2);
                    sens_term(s1.h[i], s0.h[i], s1.g[i], s0.g[i], &lc1, &lc2);
                    /* z: the accumulation's error scales with a, not |z|     */
                    if (s1.z[i] != s0.z[i]) {
                        const double t1 = fabs(s1.d[i]) * s1.a[i], t2 = fabs(s0.d[i]) * s0.a[i];
                        acc1 += t1 + t2;
                        acc2 += t1 * t1 + t2 * t2;
                    } else {
                        const double t = fabs(s1.d[i] - s0.d[i]) * s0.a[i];
                        acc1 += t;
                        acc2 += t * t;
                    }
                }
            o[0] = f1 - f0; o[1] = act1; o[2] = sqrt(act2); o[3] = acc1; o[4] = lc1;
            o[5] = sqrt(acc2);
        }
        free(sp);
        free(h0);
        sens_free(&s0);
        sens_free(&s1);
    }
}

/* ------------------------------------------------------------------ */
/* Statistics and stochastic reconfiguration                            */
/* ------------------------------------------------------------------ */

void oracle_energy_stats(const double *e_loc, int64_t B, double *stats)
{
    double m = 0.0;
    for (int64_t s = 0; s < B; ++s) m += e_loc[s];
    m /= (double)B;
    double v = 0.0;
    for (int64_t s = 0; s < B; ++s) v += (e_loc[s] - m) * (e_loc[s] - m);
    stats[0] = m;
    stats[1] = v / (double)B;
}

static double dot(const double *a, const double *b, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* column means of O */
static void col_mean(const double *O, int64_t B, int64_t P, double *obar)
{
    for (int64_t p = 0; p < P; ++p) obar[p] = 0.0;
    for (int64_t s = 0; s < B; ++s)
        for (int64_t p = 0; p < P; ++p) obar[p] += O[s * P + p];
    for (int64_t p = 0; p < P; ++p) obar[p] /= (double)B;
}

/* y = (Obar^T Obar / B + lambda) v, Obar = O - obar, applied without forming S */
static void apply_s(const double *O, const double *obar, int64_t B, int64_t P,
                    double lambda, const double *v, double *y, double *u)
{
    for (int64_t s = 0; s < B; ++s) {
        double acc = 0.0;
        for (int64_t p = 0; p < P; ++p) acc += (O[s * P + p] - obar[p]) * v[p];
        u[s] = acc;
    }
    for (int64_t p = 0; p < P; ++p) y[p] = 0.0;
    for (int64_t s = 0; s < B; ++s)
        for (int64_t p = 0; p < P; ++p) y[p] += (O[s * P + p] - obar[p]) * u[s];
    for (int64_t p = 0; p < P; ++p) y[p] = y[p] / (double)B + lambda * v[p];
}

static void force_vector(const double *O, const double *obar, const double *e, int64_t B,
                         int64_t P, double *F)
{
    double m = 0.0;
    for (int64_t s = 0; s < B; ++s) m += e[s];
    m /= (double)B;
    for (int64_t p = 0; p < P; ++p) F[p] = 0.0;
    for (int64_t s = 0; s < B; ++s)
        for (int64_t p = 0; p < P; ++p) F[p] += (O[s * P + p] - obar[p]) * (e[s] - m);
    for (int64_t p = 0; p < P; ++p) F[p] /= (double)B;
}

void oracle_sr_apply(const double *O, int64_t B, int64_t P, double lambda,
                     const double *v, double *y)
{
    double *obar = (double *)malloc(sizeof(double) * (size_t)P);
    double *u = (double *)malloc(sizeof(double) * (size_t)B);
    col_mean(O, B, P, obar);
    apply_s(O, obar, B, P, lambda, v, y, u);
    free(obar);
    free(u);
}

void oracle_sr_cg(const double *O, const double *e_loc, int64_t B, int64_t P,
                  double lambda, int n_iter, double *x, double *stats)
{
    double *obar = (double *)malloc(sizeof(double) * (size_t)P);
    double *F = (double *)malloc(sizeof(double) * (size_t)P);
    double *r = (double *)malloc(sizeof(double) * (size_t)P);
    double *p = (double *)malloc(sizeof(double) * (size_t)P);
    double *Ap = (double *)malloc(sizeof(double) * (size_t)P);
    double *u = (double *)malloc(sizeof(double) * (size_t)B);
    col_mean(O, B, P, obar);
    force_vector(O, obar, e_loc, B, P, F);
    for (int64_t i = 0; i < P; ++i) { x[i] = 0.0; r[i] = F[i]; p[i] = F[i]; }
    double rr = dot(r, r, P);
    const double ff = rr;
    int it = 0;
    /* Early exit only once the recursive residual is 1e-30 of ||F|| (far below
     * FP64 resolution of x): past that point r.r and p.Ap underflow.        */
    const double stop = ff * 1e-60;
    for (; it < n_iter && rr > stop; ++it) {
        apply_s(O, obar, B, P, lambda, p, Ap, u);
        double pap = dot(p, Ap, P);
        if (!(pap > 0.0)) break;
        double alpha = rr / pap;
        for (int64_t i = 0; i < P; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
        double rr_new = dot(r, r, P);
        double beta = rr_new / rr;
        for (int64_t i = 0; i < P; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
    }
    stats[0] = ff > 0.0 ? sqrt(rr / ff) : 0.0;
    stats[1] = (double)it;
    free(obar); free(F); free(r); free(p); free(Ap); free(u);
}

int oracle_sr_dense(const double *O, const double *e_loc, int64_t B, int64_t P,
                    double lambda, double *x)
{
    double *obar = (double *)malloc(sizeof(double) * (size_t)P);
    double *F = (double *)malloc(sizeof(double) * (size_t)P);
    double *A = (double *)malloc(sizeof(double) * (size_t)P * P);
    col_mean(O, B, P, obar);
    force_vector(O, obar, e_loc, B, P, F);
    /* A = Obar^T Obar / B + lambda I */
    for (int64_t i = 0; i < P; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            double acc = 0.0;
            for (int64_t s = 0; s < B; ++s)
                acc += (O[s * P + i] - obar[i]) * (O[s * P + j] - obar[j]);
            acc /= (double)B;
            if (i == j) acc += lambda;
            A[i * P + j] = acc;
            A[j * P + i] = acc;
        }
    /* Cholesky A = G G^T, lower triangle in place */
    int ok = 0;
    for (int64_t j = 0; j < P && ok == 0; ++j) {
        double d = A[j * P + j];
        for (int64_t k = 0; k < j; ++k) d -= A[j * P + k] * A[j * P + k];
        if (d <= 0.0) { ok = -1; break; }
        d = sqrt(d);
        A[j * P + j] = d;
        for (int64_t i = j + 1; i < P; ++i) {
            double v = A[i * P + j];
            for (int64_t k = 0; k < j; ++k) v -= A[i * P + k] * A[j * P + k];
            A[i * P + j] = v / d;
        }
    }
    if (ok == 0) {
        /* forward then backward substitution */
        for (int64_t i = 0; i < P; ++i) {
            double v = F[i];
            for (int64_t k = 0; k < i; ++k) v -= A[i * P + k] * x[k];
            x[i] = v / A[i * P + i];
        }
        for (int64_t i = P - 1; i >= 0; --i) {
            double v = x[i];
            for (int64_t k = i + 1; k < P; ++k) v -= A[k * P + i] * x[k];
            x[i] = v / A[i * P + i];
        }
    }
    free(obar); free(F); free(A);
    return ok;
}
