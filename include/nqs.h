/*
 * nqs.h -- C ABI of libnqs: the MI355X (gfx950) hot path of convolutional
 * neural-network variational Monte Carlo for the spin-1/2 J1-J2 Heisenberg
 * model on an L x L periodic square lattice (arxiv 2204.07816).
 *
 * What the library computes (paper passages in brackets):
 *   H = J1 sum_<ij> S_i.S_j + J2 sum_<<ij>> S_i.S_j, S = sigma/2         [Sec. 6.1, Eq. J1J2]
 *   psi(s) = M(s) exp f(s): M = Marshall sign (-1)^{#up spins on the
 *     sublattice (x+y) even}, f = CNN log-amplitude                      [Sec. 3.2 Eq. psi; Table 1 sign rule]
 *   f: K layers of 3x3 periodic (circular) cross-correlation + bias +
 *     ln cosh, summed over sites and channels (log of a product of
 *     neurons)                                                            [Sec. 5.2]
 *   E_loc(s) = sum_S' psi(S')/psi(s) <S'|H|s>: diagonal part plus one
 *     exchanged configuration per antiparallel J1/J2 pair                 [Sec. 5.4.1, hotspot energy]
 *   O_k(s) = d log|psi(s)| / d theta_k per sample                          [Sec. 3.2, O_loc by backward]
 *   SR: (S + lambda I) dtheta = F, S = Obar^T Obar / Ns,
 *       F = Obar^T (E - Ebar) / Ns                                        [Sec. 3.2; Sec. 5.4.1 distributed SR]
 *   CNN1 contexts (nqs_create_cnn1): blocks of convolution, max-pooling and
 *     transposed convolution, psi the product of the output neurons       [Sec. 5.2]
 *   t-J contexts (nqs_create_tj): H = -t sum_<ij>,sigma (c+_i c_j + h.c.)
 *     + J sum_<ij> (S_i.S_j - n_i n_j / 4), fermions encoded by the
 *     Jordan-Wigner transformation along the site order                   [Sec. 6.1, Eq. tJ]
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer unless marked "host".  The
 *     caller owns every buffer it passes; the context owns its weights and
 *     its workspace.
 *   - spins: int8 +1/-1, layout [B][L][L] (row y, column x), site i = y*L+x.
 *     t-J contexts: +1 up electron, -1 down electron, 0 hole.
 *   - weights: FP64, canonical order, layer by layer: W_k[co][ci][ky][kx]
 *     then b_k[co]; layer 1 has one input channel, layers 2..K have C.
 *     The convolution is a cross-correlation:
 *       z[co][y][x] = b[co] + sum W[co][ci][ky][kx] h[ci][(y+ky-1) mod L][(x+kx-1) mod L].
 *   - Canonical bond id b = 4*i + t, t = 0: (x+1,y) J1, 1: (x,y+1) J1,
 *     2: (x+1,y+1) J2, 3: (x+1,y-1) J2 (all mod L).
 *   - stream: a hipStream_t (NULL = default stream).  All work is enqueued
 *     asynchronously on it; no call synchronises unless documented.
 *   - Limits: even L with 4 <= L <= 64; 1 <= K <= 16; 1 <= C <= 32 for the
 *     FP64/FP32 paths; C in {16, 32}, K >= 2 and L <= 36 for BF16 (its base
 *     pass keeps a whole layer of a configuration in one workgroup's
 *     accumulators, at most 1408 sites); C = 32 and K >= 2 for BF16X3;
 *     B <= 131072 per call.
 *
 * Errors
 *   - Argument problems found on the host are returned at once and nothing
 *     is enqueued.
 *   - Problems found on the device (a spin that is not +1/-1, or not
 *     -1/0/+1 in a t-J context, a non-finite
 *     log-amplitude difference or local energy) set a sticky error word in
 *     the context; nqs_get_error() reads (and clears) it.
 *   - A call that needs more workspace than nqs_reserve() provided allocates
 *     it, unless the stream is being captured into a graph: then it returns
 *     NQS_E_WORKSPACE.
 *   - Thread safety: calls on one context must be serialised by the caller;
 *     distinct contexts are independent.
 */
#ifndef NQS_H
#define NQS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nqs_ctx nqs_ctx;

typedef enum {
    NQS_OK = 0,
    NQS_E_ARG = 1,          /* null pointer, negative size, bad enum          */
    NQS_E_LATTICE = 2,      /* L odd, < 4 or > 64                             */
    NQS_E_SPEC = 3,         /* network spec not supported                      */
    NQS_E_NPARAMS = 4,      /* weight count does not match the spec            */
    NQS_E_SPIN = 5,         /* device: a spin value other than +1 / -1         */
    NQS_E_NONFINITE = 6,    /* device: non-finite log-ratio or local energy    */
    NQS_E_NOMEM = 7,        /* device allocation failed                        */
    NQS_E_WORKSPACE = 8,    /* workspace too small while a capture is active   */
    NQS_E_HIP = 9,          /* a HIP runtime call failed                       */
    NQS_E_UNSUPPORTED = 10  /* valid request this build does not implement     */
} nqs_status;

/* Arithmetic of the convolutions of layers 2..K:
 *   FP64      plain double precision (the paper's);
 *   FP32      single precision on the vector ALU;
 *   BF16      matrix cores, BF16 operands (weights and activations rounded to
 *             nearest even), FP32 accumulation;
 *   BF16X3    matrix cores, split BF16: every operand x is carried as a pair
 *             hi = bf16(x), lo = bf16(x - hi) (|x - hi - lo| <= 2^-16 |x|)
 *             and each product as hi*hi + hi*lo + lo*hi, three BF16 products
 *             with FP32 accumulation (the bf16x3 scheme of Henry, Tang and
 *             Heinecke, 2019).  32 channels only.
 * Layer 1 (one input channel) runs in FP32 in the BF16 forms, FP64
 * otherwise; ratios, sums and reductions are FP64 in every form.           */
typedef enum { NQS_FP64 = 0, NQS_FP32 = 1, NQS_BF16 = 2, NQS_BF16X3 = 3 } nqs_dtype;

/* How psi(S') is evaluated for the exchanged configurations [Sec. 5.4.1]:
 * FULL recomputes the whole network for every S'; INCREMENTAL recomputes only
 * the receptive-field cone of the exchanged pair and reads the rest from the
 * cached activations of S; AUTO lets the library choose.  INCREMENTAL serves
 * the BF16 form, the BF16X3 form where no window of the cone wraps around the
 * torus (L >= 2K + 4), and the FP64 form with 16 or 32 channels, 2 <= K <= 8
 * and L >= 2K + 4 (elsewhere NQS_E_UNSUPPORTED).  The FP64 cone forms every
 * neuron with the full pass's arithmetic, in the same order, so the two
 * differ only in the order of the final sum over sites; its cache holds
 * layers 1 .. K-1 of the samples, (K-1) B N C doubles (at most 16 GiB per
 * fill: larger batches are taken in chunks of samples). */
typedef enum { NQS_AUTO = 0, NQS_FULL = 1, NQS_INCREMENTAL = 2 } nqs_mode;

typedef struct {
    int32_t n_layers;       /* K                                              */
    int32_t channels;       /* C                                              */
    int32_t marshall_sign;  /* 1: psi carries the Marshall sign; 0: psi > 0   */
    nqs_dtype conv_dtype;   /* arithmetic of the convolutions: FP64 (plain),
                               FP32 (vector), BF16 (MFMA, FP32 accumulate)   */
} nqs_cnn_spec;

/* Create a context for one lattice and network on the current HIP device.
 * weights: host, n_weights FP64 values in canonical order (copied).       */
nqs_status nqs_create(int32_t L, double J1, double J2, const nqs_cnn_spec *spec,
                      const double *weights, int64_t n_weights, nqs_ctx **out);

/* A context for the t-J model [Sec. 6.1, Eq. tJ] on an L x L torus, with the
 * same network, limits and entry points as nqs_create.  Site values: +1 up
 * electron, -1 down electron, 0 hole (no double occupancy).  Only nearest-
 * neighbour bonds (t = 0, 1) carry terms:
 *   - diagonal: J (s_i s_j - |s_i||s_j|) / 4 per bond (-J/2 per
 *     antiparallel pair);
 *   - spin exchange of an antiparallel pair (J != 0): <S'|H|S> = +J/2;
 *   - hop of an electron onto a neighbouring hole (t != 0): <S'|H|S> =
 *     -t (-1)^n, n = electrons on the sites strictly between the two in the
 *     order i = y*L + x (the Jordan-Wigner string; the fermion modes are
 *     ordered site by site).
 * Every S' is the pair's values exchanged, so nqs_connected lists them as
 * bond ids like the spin model (mu = M(S')/M(s): -1 when an up spin or
 * electron changes sublattice), nqs_log_ratios gives their f(S') - f(s),
 * and nqs_mcmc proposes nearest-neighbour pairs (n = 2) and exchanges pairs
 * of different values, conserving the numbers of up and down electrons.
 * The Marshall sign counts up electrons on sublattice A.  t-J contexts
 * share the autotuner key of a J2 = 0 spin context of the same shape.
 * Errors as nqs_create (t, J must be finite).                             */
nqs_status nqs_create_tj(int32_t L, double t, double J, const nqs_cnn_spec *spec,
                         const double *weights, int64_t n_weights, nqs_ctx **out);

/* A context whose network is CNN1 [Sec. 5.2: blocks of a 2D convolution, a
 * 1D max-pooling and a transposed convolution, padded by the periodic
 * boundary; the coefficient is the product of the output neurons], for the
 * J1-J2 model, in FP64.  The block figure is missing; the block read here,
 * for k = 1..blocks, c_in = 1 (spins) then channels = C:
 *   z = a + W (*) h       3x3 circular convolution c_in -> 2C, W[2C][c_in][3][3]
 *   m[c] = max(z[2c], z[2c+1])            max-pool of window 2 over channels
 *   u[co][p] = v[co] + sum V[ci][co][ky][kx] m[ci][p - (ky-1, kx-1)]
 *                         3x3 circular transposed convolution C -> C, stride 1
 *   psi = M(s)^marshall_sign * prod_{c,p} u_blocks[c][p]
 * Weights (host FP64, copied), canonical order per block: W, a, V, v;
 * n_weights = sum_k (2C c_in 9 + 2C + 9 C^2 + C).
 * Entry points serving CNN1 contexts: nqs_log_psi (sign = M^marshall times
 * the sign of the neuron product), nqs_local_energy, nqs_log_ratios and
 * nqs_mcmc (the per-item sign ratio of the network enters E_loc),
 * nqs_log_deriv (d log|psi| / d theta by a backward pass: 1/u at the
 * output, a max passes its gradient to the larger input, the first on a
 * tie), nqs_sr_solve, nqs_sr_solve_recompute, nqs_energy_stats,
 * nqs_connected, nqs_set_weights, nqs_update_weights, nqs_get_weights,
 * nqs_reserve, nqs_local_energy_multi (lattice after lattice) and
 * nqs_autotune.  Modes: FULL recomputes every exchanged configuration;
 * INCREMENTAL (channels = 16, blocks <= 6, L >= 4 blocks + 4; otherwise
 * NQS_E_UNSUPPORTED) recomputes only the receptive cone -- stencil l of the
 * network (block b's convolution is stencil 2b - 1, its transposed
 * convolution 2b) changes only within l sites of the exchanged pair -- from
 * every layer's activations of the base pass, kept in the workspace
 * ((2 blocks - 1) B N 16 doubles, and per site of the last layer the sum of
 * log|u| and the count of negative neurons), with the full pass's
 * arithmetic for every neuron; AUTO takes the autotuner's choice, else INCREMENTAL where the
 * cone's positions are below 70% of the full pass's.  nqs_autotune times
 * both forms where the cone serves (FULL is the only form elsewhere) and
 * stores nothing in the tune cache.  An output neuron of
 * exactly 0 makes log|psi| infinite: NQS_E_NONFINITE.
 * Errors: NQS_E_LATTICE, NQS_E_SPEC (blocks or channels outside 1..16 /
 * 1..32, marshall_sign not 0/1), NQS_E_NPARAMS, NQS_E_ARG as nqs_create.  */
nqs_status nqs_create_cnn1(int32_t L, double J1, double J2, int32_t blocks, int32_t channels,
                           int32_t marshall_sign, const double *weights, int64_t n_weights,
                           nqs_ctx **out);

/* The t-J model [Sec. 6.1, Eq. tJ; the terms and site values of
 * nqs_create_tj] with the CNN1 amplitude of nqs_create_cnn1, whose own sign
 * (the sign of the neuron product) multiplies every term of E_loc with the
 * Jordan-Wigner and Marshall signs.  Same entry points and errors as
 * nqs_create_cnn1.                                                          */
nqs_status nqs_create_cnn1_tj(int32_t L, double t, double J, int32_t blocks, int32_t channels,
                              int32_t marshall_sign, const double *weights, int64_t n_weights,
                              nqs_ctx **out);

/* The t-J model [Sec. 6.1, Eq. tJ; the terms and site values of
 * nqs_create_tj] with the CNN2 amplitude [Sec. 5.2], computed in FP64.
 * The block figure is not available; the network is read as: the state of
 * site p (0 hole, +1 up, -1 down) selects the embedding row e = 0, 1, 2 of
 * E[3][C]; each of `blocks` blocks maps C channels to C by
 *   z = a + W (*) h   (3x3 circular convolution),
 *   m[c] = max(z[c], z[(c+1) mod C])   (window 2 over the channels, stride
 *           one, the first channel copied after the last),
 *   u[co][p] = v[co] + sum V[ci][co][t] m[ci][p - off t]   (transposed);
 * then y[p] = b + sum F[c][t] u[c][p + off t] and
 * psi = M(s)^marshall_sign * prod_p y[p].
 * weights: host FP64 [n_weights] in canonical order E[3][C]; per block
 * W[C][C][3][3], a[C], V[C][C][3][3] (input channel first), v[C]; then
 * F[C][3][3], b; n_weights = 3C + blocks (18 C^2 + 2C) + 9C + 1.
 * channels must be 16 or 32 (every block convolution runs on the FP64
 * matrix cores).  Entry points as nqs_create_cnn1_tj, in FULL and AUTO
 * modes (INCREMENTAL: NQS_E_UNSUPPORTED; nqs_autotune answers FULL and
 * stores nothing); a max passes its gradient to channel c unless channel
 * c+1 is strictly larger.
 * Errors: NQS_E_SPEC (blocks outside 1..16, channels not 16 or 32,
 * marshall_sign not 0/1), otherwise as nqs_create_cnn1.                   */
nqs_status nqs_create_cnn2_tj(int32_t L, double t, double J, int32_t blocks, int32_t channels,
                              int32_t marshall_sign, const double *weights, int64_t n_weights,
                              nqs_ctx **out);

/* Matrix-core calibration (no context): `workgroups` workgroups of 4 waves
 * each run `iters` x 8 independent MFMA instructions from registers only
 * (kind 0: v_mfma_f32_16x16x32_bf16; kind 1: v_mfma_f64_16x16x4f64), timed
 * with HIP events on `stream` after one warm-up launch.  *ms (host) is the
 * timed launch and *tflops (host) the sustained rate.  It measures what the
 * matrix cores deliver under full load, beside the published dense peaks the
 * roofline fractions are quoted against.  Allocates and frees a small device
 * buffer and synchronises the stream.  Errors: NQS_E_ARG (kind not 0/1,
 * workgroups outside 1..2^20, iters < 1, null outputs), NQS_E_WORKSPACE
 * (stream under capture), NQS_E_NOMEM, NQS_E_HIP.                          */
nqs_status nqs_mfma_rate(int32_t kind, int64_t workgroups, int32_t iters, double *ms,
                         double *tflops, void *stream);

/* Release the context and its device memory (synchronises the device).  */
nqs_status nqs_destroy(nqs_ctx *ctx);

/* Number of network parameters P (host out).                              */
nqs_status nqs_num_params(const nqs_ctx *ctx, int64_t *P);

/* Replace the weights (host, canonical order, n == P); synchronous.       */
nqs_status nqs_set_weights(nqs_ctx *ctx, const double *weights, int64_t n);

/* The VMC parameter update on the device [Sec. 3.2]: theta <- theta + scale
 * * dtheta (dtheta device FP64 [P], canonical order; product rounded, then
 * the sum), and every kernel family's packing rebuilt from the result on the
 * stream.  Allocates nothing and never synchronises, so it can be captured
 * with the rest of a VMC iteration.  The kernels then see exactly what
 * nqs_set_weights of the updated vector would give them.                  */
nqs_status nqs_update_weights(nqs_ctx *ctx, const double *dtheta, double scale,
                              void *stream);

/* Set the weights from a device vector theta (FP64 [P], canonical order)
 * on the stream [Sec. 3.2: the parameters the amplitude is evaluated at]:
 * copied into the context by a kernel, then every kernel family's packing
 * rebuilt from it, as nqs_update_weights does.  Allocates nothing and never
 * synchronises (capturable); the kernels then see exactly what
 * nqs_set_weights of the same values gives them.  The caller keeps theta
 * alive until the stream has run the copy.                                 */
nqs_status nqs_set_weights_device(nqs_ctx *ctx, const double *theta, void *stream);

/* The current weights (host FP64 [n], canonical order, n == P); waits for
 * the device.                                                               */
nqs_status nqs_get_weights(nqs_ctx *ctx, double *weights, int64_t n);

/* Pre-allocate workspace for batches up to B_max in the given mode (AUTO:
 * the mode AUTO resolves to now; the incremental forms' activation caches
 * are reserved when the mode is INCREMENTAL), so that later calls allocate
 * nothing (and may be captured into a hipGraph).                          */
nqs_status nqs_reserve(nqs_ctx *ctx, int64_t B_max, nqs_mode mode);

/* log|psi(s)| (FP64 [B]) and the sign of psi (int8 [B], may be NULL)
 * [Sec. 3.2 Eq. psi].                                                      */
nqs_status nqs_log_psi(nqs_ctx *ctx, const int8_t *spins, int64_t B,
                       double *log_abs, int8_t *sign, void *stream);

/* Local energies E_loc(s), FP64 [B] [Sec. 5.4.1].  Ratios exp(f(S')-f(s)),
 * their per-sample sums and the diagonal part are FP64 in every mode.     */
nqs_status nqs_local_energy(nqs_ctx *ctx, const int8_t *spins, int64_t B,
                            double *e_loc, nqs_mode mode, void *stream);

/* Batch mean and variance (1/Ns) of e_loc [Sec. 3.2: the energy estimate
 * over the samples and its variance]: stats FP64 [2], device.  Two-stage
 * fixed-order FP64 sums.                                                    */
nqs_status nqs_energy_stats(nqs_ctx *ctx, const double *e_loc, int64_t B,
                            double *stats, void *stream);

/* Per-sample log-derivatives O [B][P] row-major, FP32 or FP64 (O_dtype),
 * computed by a hand-written backward pass in FP64 [Sec. 3.2].  The
 * Marshall sign does not depend on the weights, so O = d f / d theta.     */
nqs_status nqs_log_deriv(nqs_ctx *ctx, const int8_t *spins, int64_t B,
                         void *O, nqs_dtype O_dtype, void *stream);

/* Stochastic reconfiguration [Sec. 3.2; Sec. 5.4.1]: conjugate gradient on
 * (S + diag_shift I) dtheta = F with S applied matrix-free as
 * Obar^T (Obar v) / B + diag_shift v (S is never formed), x0 = 0, exactly
 * n_iter iterations unless the recursive residual falls below 1e-30 ||F||.
 * O: [B][P] in O_dtype (FP32 or FP64); e_loc FP64 [B]; dtheta FP64 [P].
 * stats (device, FP64 [4], may be NULL): mean energy, variance,
 * recursive ||r||/||F|| at exit, iterations run.                          */
nqs_status nqs_sr_solve(nqs_ctx *ctx, const void *O, nqs_dtype O_dtype,
                        const double *e_loc, int64_t B, double diag_shift,
                        int32_t n_iter, double *dtheta, double *stats,
                        void *stream);

/* The same SR solve for batches whose O does not fit in device memory
 * [Sec. 3.2; Sec. 5.4.1]: O is never stored whole.  Its rows are recomputed
 * from the spins (device int8 [B][L][L], as nqs_log_deriv computes them, in
 * O_dtype) in chunks of chunk_rows samples (0: as many as fit in 2 GiB),
 * rounded up to whole reduction blocks of the solve.  Every pass over O
 * recomputes the chunks it does not hold, 2 (ceil(B / chunk) - 1) chunks per
 * CG iteration.  dtheta and stats equal nqs_sr_solve's on the stored O of the
 * same samples bit for bit.  Workspace: one chunk of O plus the backward's
 * buffers for it, owned by the context.  Errors as nqs_sr_solve, plus
 * NQS_E_ARG for chunk_rows < 0 and the spin checks of nqs_log_deriv.        */
nqs_status nqs_sr_solve_recompute(nqs_ctx *ctx, const int8_t *spins,
                                  nqs_dtype O_dtype, const double *e_loc,
                                  int64_t B, double diag_shift, int32_t n_iter,
                                  int64_t chunk_rows, double *dtheta,
                                  double *stats, void *stream);

/* nqs_sr_solve for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, kernels and results (bit for bit) as nqs_sr_solve, with its
 * workspace in a fixed 48 MiB array of device memory that the library holds
 * on every device it runs on until the process ends, instead of the
 * context's workspace.  Allocates nothing and never synchronises.
 * Limit: the workspace of B samples and P parameters, 8 (5 P + 2 B + c P)
 * bytes plus alignment with c = min(64, ceil(B / 64)) partial sums per
 * column, must fit in 48 MiB (P = 65,056 with B = 4096 takes 36 MB);
 * larger problems return NQS_E_WORKSPACE and enqueue nothing.  Every call on
 * a device shares that device's array: calls that overlap on one device
 * (other streams, other threads, other contexts) race and must be
 * serialised by the caller.  Other errors as nqs_sr_solve.                */
nqs_status nqs_sr_solve_noalloc(nqs_ctx *ctx, const void *O, nqs_dtype O_dtype,
                                const double *e_loc, int64_t B, double diag_shift,
                                int32_t n_iter, double *dtheta, double *stats,
                                void *stream);

/* Inspection of the integer stage [Sec. 5.4.1]: for every sample the count
 * of antiparallel bonds with J != 0 (t-J: of the pairs with an off-diagonal
 * term, see nqs_create_tj) (int32 [B]), exclusive offsets
 * (int64 [B+1]), the bond ids in canonical order and the Marshall ratio
 * mu = M(S')/M(s) of each (int32 / int8 [capacity]), and the diagonal energy
 * (FP64 [B]).  capacity must be >= the number of bonds with J != 0 times B
 * (4*L*L*B when J2 != 0; t-J contexts: 2*L*L*B when t or J != 0).  Lists
 * are bit-exact and deterministic.                                          */
nqs_status nqs_connected(nqs_ctx *ctx, const int8_t *spins, int64_t B,
                         int32_t *counts, int64_t *offsets, int32_t *bond_ids,
                         int8_t *mu, int64_t capacity, double *e_diag,
                         void *stream);

/* The log-amplitude differences f(S') - f(s) of every exchanged
 * configuration [Sec. 5.4.1: the network forwards of the exchanged
 * configurations, which take over 95% of the time], FP64 [capacity], in the
 * order of nqs_connected.                                                   */
nqs_status nqs_log_ratios(nqs_ctx *ctx, const int8_t *spins, int64_t B,
                          nqs_mode mode, double *dlog, int64_t capacity,
                          void *stream);

/* Metropolis sampling of |psi|^2 by pair exchanges [Sec. 3.2; Sec. 5.4.1],
 * n_steps steps of every chain; chain b is sample b of spins (device int8
 * [B][L][L], updated in place).  Step t of chain b: the proposal is bond
 * q = rand_bond[t B + b] mod (N * n), n = 2 (J1 or J2 bonds only) or 4 (both),
 * site q / n, type the (q mod n)-th of those of the non-zero couplings
 * (canonical bond id 4 site + type); an antiparallel pair is exchanged when
 * rand_u[t B + b] < exp(2 (f(S') - f(S))).  The proposal is symmetric, so the
 * chains sample |psi|^2.  rand_bond: device uint32 [n_steps][B]; rand_u:
 * device FP64 [n_steps][B] in [0, 1); accepted (device int32 [B], may be
 * NULL) is increased by each chain's accepted exchanges.  f(S') - f(S) is
 * computed as nqs_local_energy computes it, in `mode`.  No coupling: no
 * move.  Errors as nqs_local_energy.                                       */
nqs_status nqs_mcmc(nqs_ctx *ctx, int8_t *spins, int64_t B, int32_t n_steps,
                    const uint32_t *rand_bond, const double *rand_u,
                    int32_t *accepted, nqs_mode mode, void *stream);

/* Several lattices at once: every job has its own context (same network
 * shape and conv dtype, any L, J2 and weights; no context twice).  With BF16
 * contexts each lattice runs its bond stage and base pass, then the
 * exchanged configurations of all lattices of one mode (as `mode` resolves
 * per context) and one kernel family share one persistent launch over their
 * concatenated queues (up to 8 lattices per launch; in incremental mode the
 * lattices with unwrapped cones share the cone kernel and the others the
 * general incremental kernel), then each lattice's FP64 ratio sums are
 * taken, so every lattice's energies equal its single-lattice call's.
 * FP64 / FP32 contexts and CNN1 / CNN2 contexts (every job of one network
 * family) run lattice after lattice.  Errors as nqs_local_energy, checked
 * for every job before any work is queued; NQS_E_SPEC for jobs of different
 * shape, dtype or network family.                                          */
typedef struct {
    nqs_ctx *ctx;
    const int8_t *spins;
    int64_t B;
    double *e_loc;
} nqs_eloc_job;
nqs_status nqs_local_energy_multi(const nqs_eloc_job *jobs, int32_t n_jobs,
                                  nqs_mode mode, void *stream);

/* Which mode AUTO picks for this context (host out): the autotuner's choice
 * once one exists for the configuration, else a work estimate (incremental
 * when its cones are below 70% of the full recomputation's positions).     */
nqs_status nqs_auto_mode(const nqs_ctx *ctx, nqs_mode *mode);

/* Autotuner (serves the batching of [Sec. 5.4.1]: which form of the
 * exchanged-configuration pass is fastest here).  Runs the bond stage and
 * base pass of the B samples (device spins), then times the exchanged-
 * configuration pass in every available form -- full recompute with each
 * fitting tile variant, and the incremental receptive cone with each shape
 * of its kernel (configurations per workgroup, waves) -- and makes AUTO
 * (and the full pass and the cone kernel) use the fastest from then on.  The choice is stored in
 * the tune cache, a JSON file (NQS_TUNE_CACHE, else
 * $HOME/.cache/nqs/tune.json), under the key nqs_tune_key gives; contexts of
 * the same key created later read it.  FP64 contexts where the FP64 cone
 * serves have both forms, timed over the whole log-ratio pass (base pass
 * included: the incremental one also keeps the activations); other FP64 and
 * all FP32 contexts have only the full form.  CNN1 contexts where the receptive cone serves have both
 * forms, timed over the whole log-ratio pass; other CNN1 and CNN2 contexts
 * have the full form only; for block networks nothing is stored in the
 * cache.  Synchronises the stream; NQS_E_WORKSPACE while the stream is
 * capturing; NQS_E_ARG for B = 0.  mode_out (host) may be null.  A cache
 * file that cannot be written is not an error.                             */
nqs_status nqs_autotune(nqs_ctx *ctx, const int8_t *spins, int64_t B,
                        nqs_mode *mode_out, void *stream);

/* Tune-cache key of a configuration (host only, writes a NUL-terminated
 * string of at most len bytes into buf).                                   */
nqs_status nqs_tune_key(int32_t L, int32_t K, int32_t C, nqs_dtype dtype,
                        double J2, char *buf, int64_t len);

/* One entry of a tune-cache file (host only): NQS_OK with the entry when the
 * file parses and holds the key; NQS_E_ARG (outputs untouched) when it is
 * missing, malformed or lacks the key.  cone_items / cone_waves (may be
 * NULL): the tuned shape of the incremental cone kernel, configurations per
 * workgroup and waves per workgroup (1 / 0: the one-configuration kernel;
 * -1 / -1 when the entry has none).                                        */
nqs_status nqs_tune_lookup(const char *path, const char *key, nqs_mode *mode,
                           int32_t *full_nw, int32_t *full_maxt, int32_t *cone_items,
                           int32_t *cone_waves);

/* Sticky device error word: synchronises the context's last stream, returns
 * the first device-detected status since the last call (host out), clears. */
nqs_status nqs_get_error(nqs_ctx *ctx, nqs_status *sticky);

/* Kernel timing: when enabled, the library records HIP events around the
 * exchanged-configuration kernel on the caller's stream.  nqs_kernel_time
 * synchronises and returns the summed milliseconds and launch count since
 * enabling, then resets.                                                  */
nqs_status nqs_enable_timing(nqs_ctx *ctx, int32_t enable);
nqs_status nqs_kernel_time(nqs_ctx *ctx, double *ms, int64_t *launches);

/* Static description of a status code.                                    */
const char *nqs_status_str(nqs_status s);

#ifdef __cplusplus
}
#endif
#endif /* NQS_H */
