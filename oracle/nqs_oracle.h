/*
 * nqs_oracle.h -- plain FP64 CPU oracle for CNN variational Monte Carlo of the
 * spin-1/2 J1-J2 Heisenberg model on an L x L periodic square lattice
 * (arxiv 2204.07816).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no source, header, table or helper with the GPU
 * path under paper_2204_07816_amd/.
 *
 * Everything is written from the definitions in the paper, in the plainest
 * form: no blocking, no incremental updates, full recomputation of every
 * connected configuration, channel-major [C][L][L] activations, FP64 only.
 *
 * Conventions (shared *interface* with the GPU library, independent code):
 *   - spins: int8, +1/-1 (t-J: also 0 for a hole), layout [y][x],
 *     site i = y*L + x                                                (Sec. 5.4.1, spin image)
 *   - H = J1 sum_<ij> S_i.S_j + J2 sum_<<ij>> S_i.S_j,  S = sigma/2   (Sec. 6.1, Eq. J1J2)
 *   - psi(s) = M(s) * exp(f(s)),  M = Marshall sign (-1)^{#up spins on sublattice A},
 *     A = {(x+y) even}; f = CNN log-amplitude                         (Sec. 3.2 Eq. psi, Table 1 "sign rule")
 *   - CNN: K layers of 3x3 circular cross-correlation, bias, ln cosh after
 *     every layer, sum over sites and channels.                       (Sec. 5.2, product of neurons)
 *   - weights: FP64, canonical order, layer by layer W_k[co][ci][ky][kx]
 *     then b_k[co]; layer 1 has ci = 1, the others ci = C.
 *
 * The pins that check every function are listed at the top of nqs_oracle.c
 * and exercised by tests/test_oracle_*.py.
 */
#ifndef NQS_ORACLE_H
#define NQS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* number of CNN parameters for K layers of C channels (layer 1: 1 -> C). */
int64_t oracle_num_params(int K, int C);

/* Marshall sign of one configuration: +1 or -1.                 */
int oracle_marshall_sign(int L, const int8_t *spins);

/* The two sites of canonical bond b = 4*i + t (t: 0 (x+1,y), 1 (x,y+1),
 * 2 (x+1,y+1), 3 (x+1,y-1), all mod L).  Returns the coupling class:
 * 1 for a nearest-neighbour pair, 2 for a next-nearest pair.            */
int oracle_bond_sites(int L, int b, int *site_i, int *site_j);

/* Connected configurations of one sample: for every bond with J_b != 0 and
 * antiparallel spins, in increasing bond id.  Writes count, bond ids,
 * the Marshall ratio M(s^b)/M(s) (computed from the two full configurations)
 * and the diagonal energy sum_b J_b s_i s_j / 4.  bond_ids and mu must hold
 * 4*L*L entries.                                                        */
void oracle_connected(int L, double J1, double J2, const int8_t *spins,
                      int32_t *count, int32_t *bond_ids, int8_t *mu,
                      double *e_diag);

/* CNN log-amplitude f(s) for B samples; nthreads <= 0 means all.        */
void oracle_log_psi(int L, int K, int C, const double *w, const int8_t *spins,
                    int64_t B, double *log_abs, int8_t *sign, int nthreads);

/* Local energy E_loc(s) = sum_b J_b s_i s_j/4
 *   + sum_{b antiparallel, J_b != 0} (J_b/2) psi(s^b)/psi(s),
 * psi(s^b) by full recomputation of the network.                         */
void oracle_local_energy(int L, double J1, double J2, int K, int C,
                         const double *w, const int8_t *spins, int64_t B,
                         double *e_loc, int nthreads);

/* Same local energy with an arbitrary tabulated wave function: the amplitude
 * of configuration s is sign_tab[idx] * exp(log_abs_tab[idx]), idx = sum_i
 * [s_i = +1] 2^i.  Only for N = L*L <= 24.                              */
void oracle_local_energy_table(int L, double J1, double J2,
                               const double *log_abs_tab, const int8_t *sign_tab,
                               const int8_t *spins, int64_t B, double *e_loc,
                               int nthreads);

/* t-J model [Sec. 6.1, Eq. tJ]: site values +1 (up electron), -1 (down
 * electron), 0 (hole); nearest-neighbour bonds only; fermion modes ordered
 * site by site along i = y*L + x (Jordan-Wigner order).
 *   H = -t sum_<ij>,sigma (c+_i c_j + h.c.) + J sum_<ij> (S_i.S_j - n_i n_j / 4)
 * psi(s) = M(s) exp(f(s)) as for the spin model (M counts up electrons on
 * sublattice A).  oracle_tj_check: 1 when every value is -1, 0 or +1.     */
int oracle_tj_check(int L, const int8_t *spins, int64_t B);

/* Connected configurations of one t-J sample in increasing bond id: every
 * nearest-neighbour pair with an off-diagonal term (antiparallel electrons
 * and J != 0: exchange, <S'|H|S> = J/2; an electron next to a hole and
 * t != 0: hop, <S'|H|S> = -t (-1)^{electrons strictly between the two sites
 * in the site order}).  Writes count, bond ids, the Marshall ratio
 * M(S')/M(s), the matrix element hval and the diagonal energy
 * sum_<ij> J (s_i s_j - |s_i||s_j|) / 4.  Arrays hold 4*L*L entries.     */
void oracle_tj_connected(int L, double t, double J, const int8_t *spins,
                         int32_t *count, int32_t *bond_ids, int8_t *mu,
                         double *hval, double *e_diag);

/* t-J local energy with the CNN amplitude (full recomputation of every S'). */
void oracle_tj_local_energy(int L, double t, double J, int K, int C, const double *w,
                            const int8_t *spins, int64_t B, double *e_loc, int nthreads);

/* Same with a tabulated wave function: configuration s has amplitude
 * sign_tab[k] exp(log_abs_tab[k]) when keys[k] = sum_i c_i 4^i (c = 0 hole,
 * 1 up, 2 down), keys sorted ascending, N <= 31; a configuration missing
 * from the table has amplitude 0 (E_loc of such an s is NaN).            */
void oracle_tj_local_energy_table(int L, double t, double J, int64_t n_tab, const int64_t *keys,
                                  const double *log_abs_tab, const int8_t *sign_tab,
                                  const int8_t *spins, int64_t B, double *e_loc, int nthreads);

/* CNN1 [Sec. 5.2: blocks of a 2D convolution, a 1D max-pooling and a
 * transposed convolution, periodic padding, output the product of the
 * neurons].  The block figure is missing, so the architecture is parity
 * unpinned against the paper; the reading implemented here:
 * block k maps c_in (1, then C) channels to C by
 *   z = a + W (*) h        3x3 circular convolution, c_in -> 2C, W[2C][c_in][3][3]
 *   m[c] = max(z[2c], z[2c+1])             max-pool of window 2 over channels
 *   u = v + V (*)^T m      3x3 circular transposed convolution, stride 1,
 *                          C -> C, V[C_in][C_out][3][3]:
 *                          u[co][p] = v[co] + sum V[ci][co][ky][kx] m[ci][p - (ky-1, kx-1)]
 * and psi = M(s)^marshall prod_{c,p} u_K[c][p] (so log|psi| = sum log|u_K|
 * and the network carries a sign).  Canonical order per block: W, a, V, v. */
int64_t oracle_cnn1_num_params(int Kb, int C);
void oracle_cnn1_log_psi(int L, int Kb, int C, const double *w, int marshall,
                         const int8_t *spins, int64_t B, double *log_abs, int8_t *sign,
                         int nthreads);
/* J1-J2 local energy with the CNN1 amplitude (sign ratio of the network
 * and, if marshall, of the Marshall sign), full recomputation.          */
void oracle_cnn1_local_energy(int L, double J1, double J2, int Kb, int C, const double *w,
                              int marshall, const int8_t *spins, int64_t B, double *e_loc,
                              int nthreads);
/* O[s][p] = d log|psi(s)| / d theta_p by reverse mode; a max passes its
 * gradient to the larger input, the first one on a tie.                 */
void oracle_cnn1_log_deriv(int L, int Kb, int C, const double *w, const int8_t *spins,
                           int64_t B, double *O, int nthreads);

/* t-J local energy [Sec. 6.1] with the CNN1 amplitude (its sign included). */
void oracle_tj_cnn1_local_energy(int L, double t, double J, int Kb, int C, const double *w,
                                 int marshall, const int8_t *spins, int64_t B, double *e_loc,
                                 int nthreads);

/* CNN2 [Sec. 5.2], read as: site states {hole, up, down} pick embedding rows
 * E[3][C]; Kb blocks C -> C of a 3x3 circular convolution (W, a), a max over
 * channels c and (c+1) mod C (window 2, stride 1, the first channel copied
 * after the last) and a 3x3 circular transposed convolution (V, v); a final
 * 3x3 circular convolution C -> 1 (F, b); psi = M(s)^marshall prod_p y[p].
 * Canonical order: E, per block W, a, V, v, then F, b:
 * 3C + Kb (18 C^2 + 2C) + 9C + 1 parameters.                               */
int64_t oracle_cnn2_num_params(int Kb, int C);
void oracle_cnn2_log_psi(int L, int Kb, int C, const double *w, int marshall,
                         const int8_t *spins, int64_t B, double *log_abs, int8_t *sign,
                         int nthreads);
/* t-J local energy [Sec. 6.1] with the CNN2 amplitude (its sign included). */
void oracle_tj_cnn2_local_energy(int L, double t, double J, int Kb, int C, const double *w,
                                 int marshall, const int8_t *spins, int64_t B, double *e_loc,
                                 int nthreads);
/* O[s][p] = d log|psi(s)| / d theta_p by reverse mode; the max passes its
 * gradient to channel c unless channel c+1 is strictly larger.          */
void oracle_cnn2_log_deriv(int L, int Kb, int C, const double *w, const int8_t *spins,
                           int64_t B, double *O, int nthreads);

/* Per-sample log-derivatives O[s][p] = d f(s) / d theta_p, FP64, by the
 * reverse-mode chain rule through the network.                          */
void oracle_log_deriv(int L, int K, int C, const double *w, const int8_t *spins,
                      int64_t B, double *O, int nthreads);

/* Rounding-error sensitivities of the network (test support: the bound a
 * reduced-precision evaluation is checked against).  A value v that is
 * rounded with relative error e (|e| <= u) moves f by (d f / d v) v e to
 * first order, so the first-order error of an evaluation is bounded by u
 * times the sum of |(d f / d v) v| over the values it rounds.
 *
 * oracle_sens_layers: every layer of one configuration, channel-major
 * [k][c][p] (k = 0..K-1 for layers 1..K): z, h = ln cosh z,
 * a = |b| + sum |W| |h_in| (magnitude of the accumulation of z),
 * g = d f / d h_k (g = 1 on layer K), d = d f / d z_k = g tanh z_k.
 *
 * oracle_dlog_sens: for M items (sample, bond), out[m][0..5]:
 *   [0] f(S') - f(S) (bond < 0: f(S) of the sample itself, below with only
 *       the sample's own terms);
 *   [1] S1_act = sum over layers 1..K-1 of the activation coefficients,
 *   [2] sqrt(sum of their squares);
 *   [3] S1_acc = same for the accumulations of z over layers 1..K with
 *       coefficient |d| a, [5] sqrt(sum of their squares);
 *   [4] S1_lc = same as [1] over layers 1..K (errors of ln cosh itself).
 * Coefficients: where S' and S differ (v' != v) the two evaluations round
 * independently, |g' v'| + |g v|; elsewhere they share the rounded value,
 * |(g' - g) v|.                                                           */
void oracle_sens_layers(int L, int K, int C, const double *w, const int8_t *spins,
                        double *z, double *h, double *a, double *g, double *d);
void oracle_dlog_sens(int L, int K, int C, const double *w, const int8_t *spins, int64_t B,
                      const int32_t *item_sample, const int32_t *item_bond, int64_t M,
                      double *out, int nthreads);

/* Energy statistics: stats[0] = mean, stats[1] = variance (1/Ns).      */
void oracle_energy_stats(const double *e_loc, int64_t B, double *stats);

/* Stochastic reconfiguration, matrix-free conjugate gradient on
 * (S + lambda I) x = F,  S = Obar^T Obar / Ns,  F = Obar^T (E - Ebar) / Ns,
 * Obar = O - mean(O).  x0 = 0; exactly n_iter iterations (stops early only
 * when r.r <= 1e-60 F.F, i.e. converged far beyond FP64 resolution).
 * stats[0] = recursive ||r|| / ||F|| at exit, stats[1] = iterations run.  */
void oracle_sr_cg(const double *O, const double *e_loc, int64_t B, int64_t P,
                  double lambda, int n_iter, double *x, double *stats);

/* Same system solved densely: build S + lambda I and factor it by Cholesky.
 * Returns 0 on success, -1 when the matrix is not positive definite.     */
int oracle_sr_dense(const double *O, const double *e_loc, int64_t B, int64_t P,
                    double lambda, double *x);

/* Apply the SR matrix once: y = (S + lambda I) v (for operator tests).     */
void oracle_sr_apply(const double *O, int64_t B, int64_t P, double lambda,
                     const double *v, double *y);

#ifdef __cplusplus
}
#endif
#endif
