// nqs_internal.h -- context, workspace and kernel-launch interfaces shared by
// the translation units of libnqs (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/nqs.h"

namespace nqs {

// Bond type t of canonical bond b = 4*i + t and its displacement.
//   t = 0: (x+1, y)  J1      t = 1: (x, y+1)  J1
//   t = 2: (x+1, y+1) J2     t = 3: (x+1, y-1) J2
__host__ __device__ inline int bond_dx(int t) { return (t == 1) ? 0 : 1; }
__host__ __device__ inline int bond_dy(int t) { return t == 0 ? 0 : (t == 1 ? 1 : (t == 2 ? 1 : -1)); }

// Queue entry: sample index and bond id packed in 32 bits (bond < 2^14).
constexpr int kBondBits = 14;
__host__ __device__ inline uint32_t pack_item(int sample, int bond) {
    return ((uint32_t)sample << kBondBits) | (uint32_t)bond;
}
__host__ __device__ inline int item_sample(uint32_t e) { return (int)(e >> kBondBits); }
__host__ __device__ inline int item_bond(uint32_t e) { return (int)(e & ((1u << kBondBits) - 1)); }

// log(1 + v) for -1/2 <= v <= 0, the range the FP64 ln cosh needs (v =
// expm1(-2|z|) / 2), to about 2 ulp.  With m = 1 + v (its rounding c = v -
// (m - 1) kept exactly) and m2 = m or 2m in [1/sqrt 2, sqrt 2):
// log m2 = 2 atanh s = 2s (1 + s^2/3 + s^4/5 + ...), s = (m2 - 1)/(m2 + 1),
// |s| <= 0.1716, where the first term left out, s^22 / 23, is below 1e-18
// relative; then log(1 + v) = log m2 - [m < 1/sqrt 2] ln 2 + c / m.  The
// general log1p carries extended-precision steps this range does not need
// (113 FP64 instructions against about 25).
__device__ inline double log1p_neg(double v)
{
    const double m = 1.0 + v;
    const double c = v - (m - 1.0);
    const bool lo = m < 0.70710678118654752440;
    const double m2 = lo ? 2.0 * m : m;
    const double num = m2 - 1.0, den = m2 + 1.0;
    double y = __builtin_amdgcn_rcp(den);
    y = fma(fma(-den, y, 1.0), y, y);
    double s = num * y;
    s = fma(fma(-den, s, num), y, s);
    const double w = s * s;
    double p = 1.0 / 21;
    p = fma(p, w, 1.0 / 19);
    p = fma(p, w, 1.0 / 17);
    p = fma(p, w, 1.0 / 15);
    p = fma(p, w, 1.0 / 13);
    p = fma(p, w, 1.0 / 11);
    p = fma(p, w, 1.0 / 9);
    p = fma(p, w, 1.0 / 7);
    p = fma(p, w, 1.0 / 5);
    p = fma(p, w, 1.0 / 3);
    const double s2 = 2.0 * s;
    const double lg = fma(s2 * w, p, s2);
    return (lo ? lg - 0.69314718055994530942 : lg) + c * __builtin_amdgcn_rcp(m);
}

// ln cosh z and tanh z from one expm1, for the forward pass of the backward
// (which keeps tanh z, the derivative of ln cosh, for the data gradient):
// with m = expm1(-2|z|), tanh|z| = -m / (2 + m) at full relative precision,
// and ln cosh z = |z| + log(1 + m / 2) to a few ulp of |z| in absolute terms
// (the pass needs ln cosh only as the next layer's input, where an absolute
// error at FP64 rounding level is what any order of the sums gives).
__device__ inline double ln_cosh_tanh(double z, double *th)
{
    const double a = fabs(z);
    const double m = expm1(-2.0 * a);
    *th = copysign(-m / (2.0 + m), z);
    return a + log1p_neg(0.5 * m);
}

// ln cosh z in FP64 for the forward passes: the same |z| + log(1 + m / 2),
// m = expm1(-2|z|), so a forward and the backward's forward give equal
// activations.  No branch: the lanes of a wave never run two forms (a
// two-branch form with relative precision at small |z| costs twice the FP64
// instructions where a wave's lanes take both).
__device__ inline double ln_cosh_fwd(double z)
{
    const double a = fabs(z);
    return a + log1p_neg(0.5 * expm1(-2.0 * a));
}

// Hamiltonian of a context: the J1-J2 spin model [Sec. 6.1, Eq. J1J2] or
// the t-J model [Sec. 6.1, Eq. tJ] (site values +1 / -1 / 0, nearest-
// neighbour bonds only, J held in J1).
constexpr int kModelSpin = 0;
constexpr int kModelTJ = 1;

// Network family of a context: the ln cosh CNN (K layers of 3x3 circular
// convolutions with ln cosh, summed), CNN1 (K blocks of convolution,
// max-pool over channel pairs and transposed convolution; product of the
// output neurons) or CNN2 (an embedding of the site states, K blocks with a
// stride-one channel max, a final convolution to one channel; product of its
// neurons) [Sec. 5.2].
constexpr int kNetLnCosh = 0;
constexpr int kNetCnn1 = 1;
constexpr int kNetCnn2 = 2;

// Device-side sticky error codes (ORed bits, mapped to nqs_status on read).
constexpr int kErrSpin = 1;
constexpr int kErrNonFinite = 2;

// Superseded workspace allocations of a context.  Once any call on the
// context has run under stream capture, a graph may hold the addresses of its
// buffers, so a buffer that has to grow later keeps its old allocation here
// (freed with the context) instead of freeing it.
struct Graveyard {
    bool captured = false;
    std::vector<void *> bufs;
};

// Growable device buffer.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    Graveyard *gy = nullptr;    // the owning context's graveyard
};

struct Workspace {
    DevBuf counts;      // int32 [B]
    DevBuf ediag;       // f64 [B]
    DevBuf offsets;     // int64 [B+1]
    DevBuf qlen;        // int64 [1] total queue length (device)
    DevBuf queue;       // uint32 [capacity]
    DevBuf dlog;        // f64 [capacity]
    DevBuf fbase;       // f64 [B] log-amplitude of the samples
    DevBuf hsum;        // f64 [B][N] channel sums of the last layer (base pass)
    DevBuf cache;       // activations of the base pass (dtype-dependent)
    DevBuf plane_a;     // scratch planes for the vector path
    DevBuf plane_b;
    DevBuf zsave;       // f64 saved values of the backward pass (tanh z; z for CNN1/CNN2)
    DevBuf hsave;       // f64 activations for the backward pass
    DevBuf delta;       // f64 backward deltas
    DevBuf sr;          // SR vectors
    DevBuf orows;       // O rows of the recompute SR variant
    DevBuf counter;     // work counters for persistent kernels
    DevBuf flags;       // int32 per chain: accepted proposals of a Metropolis step
    DevBuf sgn;         // int8 [B] network sign of the samples (CNN1)
    DevBuf isign;       // int8 [capacity] network sign ratio per queue item (CNN1)
    DevBuf hstmp;       // f64 per-site sums of full-recompute chunks (BF16X3)
    Graveyard gy;

    std::vector<DevBuf *> all()
    {
        return {&counts, &ediag, &offsets, &qlen,  &queue, &dlog,  &fbase,   &hsum,
                &cache,  &plane_a, &plane_b, &zsave, &hsave, &delta, &sr,    &orows,
                &counter, &flags, &sgn,    &isign, &hstmp};
    }
    // every buffer files its superseded allocations with this workspace
    void bind()
    {
        for (DevBuf *b : all()) b->gy = &gy;
    }
};

}  // namespace nqs

struct nqs_ctx {
    int L = 0, N = 0, K = 0, C = 0;
    double J1 = 1.0, J2 = 0.0;
    int model = nqs::kModelSpin;
    int net = nqs::kNetLnCosh;
    double t_hop = 0.0;           // t-J hopping amplitude t
    int marshall = 1;
    nqs_dtype dtype = NQS_FP64;
    int64_t P = 0;
    int device = 0;
    // weights
    std::vector<double> w_host;   // canonical
    double *w_canon = nullptr;    // device canonical FP64 [P]
    double *w_vec64 = nullptr;    // vector-path packing, FP64
    float *w_vec32 = nullptr;     // vector-path packing, FP32
    double *w_bwd64 = nullptr;    // transposed packing for the backward data pass
    uint16_t *w_mfma = nullptr;   // BF16 MFMA A-operand packing, layers 2..K
    uint16_t *w_mfma_lo = nullptr;  // BF16X3: the lo parts of the same packing
    float *w_l1 = nullptr;        // layer-1 weights + all biases, FP32, MFMA path
    int32_t *ring_tab = nullptr;  // incremental mode: ring lists per bond type and layer
    int32_t *ring_off = nullptr;
    int32_t *cone_tab = nullptr;  // same, for the unwrapped-window kernel
    std::vector<int> cone_off;    // [4][16] entry offsets of cone_tab
    int32_t *ls_tab = nullptr;    // frame ring tables of the lockstep cone kernel
    std::vector<int> ls_off;      // [4][16] entry offsets of ls_tab
    int32_t *fr_tab = nullptr;    // cone_tab's rings in frame coordinates (in-place frame form)
    std::vector<int> fr_off;      // [4][16] entry offsets of fr_tab
    int cone_variant = -1;        // lockstep shape (items, waves); -1: one-configuration kernel
    // autotuner choice (from nqs_autotune or the tune cache)
    int tuned = 0;
    nqs_mode tuned_mode = NQS_FULL;
    int full_nw = 0, full_maxt = 0;   // tile variant of the full-recompute pass (0: default)
    // workspace
    nqs::Workspace ws;
    int32_t *err = nullptr;       // device sticky error word
    hipStream_t last_stream = nullptr;
    // timing
    int timing = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    int n_cu = 256;
};

namespace nqs {

// --- launch-error capture: HIP's last-error state is overwritten by the next
// successful call, so every launch is checked right away and the first
// failure of a call is kept (thread-local) until the API entry point returns.
void note_launch(const char *what);
hipError_t take_launch_error(const char **what);

#define NQS_LAUNCH(kernel, ...)                     \
    do {                                            \
        hipLaunchKernelGGL(kernel, __VA_ARGS__);    \
        ::nqs::note_launch(#kernel);                \
    } while (0)

// --- workspace helpers (nqs_abi.hip) ---
nqs_status ensure(DevBuf &b, size_t bytes, hipStream_t stream);
bool stream_capturing(hipStream_t s);

// --- lattice kernels (k_lattice.hip) ---
// a1: antiparallel-bond counts, diagonal energy, spin validation.
void launch_bond_count(const nqs_ctx *c, const int8_t *spins, int B, int32_t *counts,
                       double *ediag, hipStream_t s);
// a2: exclusive scan of counts -> offsets[B+1], qlen[0] = offsets[B].
void launch_scan(const int32_t *counts, int B, int64_t *offsets, int64_t *qlen, hipStream_t s);
// a2: queue entries in canonical bond order.
void launch_queue_fill(const nqs_ctx *c, const int8_t *spins, int B, const int64_t *offsets,
                       uint32_t *queue, hipStream_t s);
// Marshall sign per sample (+ spin validation); sign may be null.
void launch_marshall(const nqs_ctx *c, const int8_t *spins, int B, int8_t *sign, hipStream_t s);
// inspection: bond ids + Marshall ratios from the queue.
void launch_queue_expand(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                         const int64_t *qlen, int64_t capacity, int32_t *bond_ids, int8_t *mu,
                         hipStream_t s);
// whether nearest-neighbour (t = 0, 1) and next-nearest (t = 2, 3) bonds
// carry off-diagonal terms in this context
inline bool nn_moves(const nqs_ctx *c);
inline bool nnn_moves(const nqs_ctx *c);

// --- vector (FP64 / FP32) network kernels (k_conv_vec.hip) ---
// Base pass over B samples: f[B], hsum[B][N]; planes are scratch [B*N*C].
void vec_base_forward(const nqs_ctx *c, const int8_t *spins, int B, double *f, double *hsum,
                      void *plane_a, void *plane_b, hipStream_t s);
// Full recompute of every queue item in chunks: dlog[item] = f(S') - f(s).
// Items q_begin + [0, q_count) of the queue; items at or past qlen[0] are skipped
// on the device, so the host never needs the queue length.
void vec_conn_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                      const int64_t *qlen, int64_t q_begin, int64_t q_count, const double *hsum,
                      double *dlog, void *plane_a, void *plane_b, hipStream_t s);
size_t vec_plane_bytes(const nqs_ctx *c, int64_t items);
// FP64 receptive cone of the ln cosh CNN (k_net_cone64.hip): 16 or 32
// channels, 2 <= K <= 8, L >= 2K + 4.  The base pass of nb samples also keeps
// h_1 .. h_{K-1} in the cache, [K-1][cB][N][C] (the nb samples at the start
// of each slot; plane: one plane of nb samples); then one launch gives dlog
// of the queue items of samples b0 .. b0 + nb - 1 among items 0 .. cap - 1
// (those samples' activations in the cache, hsum of all samples).
bool cone64_ok(const nqs_ctx *c);
size_t cone64_cache_bytes(const nqs_ctx *c, int64_t cB);
int64_t cone64_chunk(const nqs_ctx *c, int64_t B);
void vec_base_forward_cached(const nqs_ctx *c, const int8_t *spins, int nb, double *f,
                             double *hsum, void *plane, double *cache, int64_t cB, hipStream_t s);
void cone64_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                    const int64_t *qlen, int64_t cap, const double *cache, int64_t cB, int64_t b0,
                    int64_t nb, const double *hsum, double *dlog, hipStream_t s);
// Backward: O[B][P] from the saved activations and tanh of the pre-activations.
// forward of B samples for the backward: tanh z and h = ln cosh z of layers
// 1..K-1 into zsave / hsave ([layer][B][N][C] FP64 each), and the last
// layer's delta tanh z_K into delta_last
void vec_deriv_forward(const nqs_ctx *c, const int8_t *spins, int B, double *zsave,
                       double *hsave, double *delta_last, hipStream_t s);
// backward from delta_a = delta_K (overwritten, with delta_b) to the rows of O
void vec_backward(const nqs_ctx *c, const int8_t *spins, int B, const double *zsave,
                  const double *hsave, double *delta_a, double *delta_b, void *O, nqs_dtype odt,
                  hipStream_t s);

// --- FP64 matrix-core layer and weight-gradient kernels (k_conv_f64mma.hip) ---
bool f64mma_conv_ok(int Cin, int Cout);
// epi 0: ln cosh; 1: ln cosh + save tanh z to zk; 2: z * zk (zk the saved
// tanh); 3: tanh z.  qlen (may be null) bounds the live planes to qlen[0] -
// q_begin.
void f64mma_conv(const nqs_ctx *c, const double *in, int64_t M, int Cin, int Cout,
                 const double *w, const double *bias, double *out, int epi, double *zk,
                 const int64_t *qlen, int64_t q_begin, hipStream_t s);
bool f64mma_wgrad_ok(int C);
// Rows O[s][woff ...] of a C -> C layer: weights [co][ci][t] then bias [co].
// trans: a transposed convolution's weights, [ci][co][t] then bias [co].
void f64mma_wgrad(const nqs_ctx *c, const double *hin, const double *delta, int B, int64_t woff,
                  void *O, nqs_dtype odt, hipStream_t s, bool trans = false);
// convolution Cin -> Cout (16 or 32), optional bias, no activation
void f64mma_linear(const nqs_ctx *c, const double *in, int64_t M, int Cin, int Cout,
                   const double *w, const double *bias, double *out, const int64_t *qlen,
                   int64_t q_begin, hipStream_t s);
// CNN2 convolution C -> C (16 or 32) with the stride-one channel max: m into
// out, z into zsave (may be null)
void f64mma_cnn2_conv(const nqs_ctx *c, const double *in, int64_t M, const double *w,
                      const double *bias, double *out, double *zsave, const int64_t *qlen,
                      int64_t q_begin, hipStream_t s);

// --- one lattice's share of a multi-lattice exchanged-configuration launch ---
constexpr int kMaxConnJobs = 8;
struct ConnJob {
    const nqs_ctx *c;
    const int8_t *spins;
    const uint32_t *queue;
    const int64_t *qlen;       // device: number of queue items
    int64_t capacity;
    const double *hsum;        // base-pass site sums
    const void *cache;         // base-pass activation cache
    double *dlog;              // out: f(S') - f(s) per item
};

// --- MFMA (BF16) network kernels (k_conv_mfma.hip) ---
bool mfma_supported(const nqs_ctx *c);
size_t mfma_cache_bytes(const nqs_ctx *c, int64_t B);
void mfma_base_forward(const nqs_ctx *c, const int8_t *spins, int B, double *f, double *hsum,
                       void *cache, hipStream_t s);
// mode: NQS_FULL or NQS_INCREMENTAL.  Items [0, qlen[0]) of the queue.
void mfma_conn_forward(const nqs_ctx *c, nqs_mode mode, const int8_t *spins,
                       const uint32_t *queue, const int64_t *qlen, int64_t capacity,
                       const double *hsum, const void *cache, double *dlog, int *counter,
                       hipStream_t s);
int mfma_lds_full_ok(const nqs_ctx *c);
// One launch over the exchanged configurations of 1..kMaxConnJobs contexts of
// one network shape (mode NQS_FULL or NQS_INCREMENTAL, supported by all).
void mfma_conn_forward_jobs(nqs_mode mode, const ConnJob *jobs, int n, hipStream_t s);
// incremental-mode kernel (k_net_inc.hip)
nqs_status mfma_build_ring_tables(nqs_ctx *c);
size_t mfma_inc_lds_bytes(const nqs_ctx *c);
void mfma_inc_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                      const int64_t *qlen, int64_t capacity, const double *hsum,
                      const void *cache, double *dlog, hipStream_t s);
bool mfma_inc_supported(const nqs_ctx *c);
// jobs: 1..kMaxConnJobs contexts of one network shape, all mfma_inc_supported
void mfma_inc_forward_jobs(const ConnJob *jobs, int n, hipStream_t s);
// incremental mode, unwrapped windows (k_net_cone.hip): C = 32, L >= 2K + 4
bool cone_supported(const nqs_ctx *c);
// jobs: 1..kMaxConnJobs contexts of one network shape, all cone-supported
void cone_forward_jobs(const ConnJob *jobs, int n, hipStream_t s);
// write-back pass of the cone kernel: for every queue item whose chain has
// commit[chain] != 0, the cache and hsum of the chain become those of S'
void cone_commit(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue, const int64_t *qlen,
                 int64_t capacity, double *hsum, void *cache, double *dlog, const int32_t *commit,
                 hipStream_t s);
size_t cone_lds_bytes(const nqs_ctx *c);
// number of lockstep shapes of the cone kernel for this context (0: K > 8);
// shape v's items per workgroup and waves, and the variant of a shape (-1:
// the one-configuration kernel, which is also variant -1)
int cone_variants(const nqs_ctx *c);
void cone_variant_shape(const nqs_ctx *c, int v, int *items, int *waves);
int cone_variant_of(const nqs_ctx *c, int items, int waves);
nqs_status cone_build_ring_tables(nqs_ctx *c);
void cone_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue, const int64_t *qlen,
                  int64_t capacity, const double *hsum, const void *cache, double *dlog,
                  hipStream_t s);

// --- split-BF16 (BF16X3) network kernels (k_x3.hip) ---
bool x3_supported(const nqs_ctx *c);
size_t x3_cache_bytes(const nqs_ctx *c, int64_t B);
// base pass: f[B], hsum[B][N], cache [B][K-1][N][2C] (hi then lo of each site)
void x3_base_forward(const nqs_ctx *c, const int8_t *spins, int B, double *f, double *hsum,
                     void *cache, void *hs_tmp, hipStream_t s);
// full recompute of queue items q0 .. q0+M-1 (items at or past qlen[0] skipped)
void x3_conn_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                     const int64_t *qlen, int64_t q0, int64_t M, const double *hsum,
                     double *dlog, void *plane_a, void *plane_b, void *hs_tmp, hipStream_t s);
// bytes of the full-recompute buffers of M configurations: two planes and the
// per-site sums
size_t x3_plane_bytes(const nqs_ctx *c, int64_t M);
size_t x3_sums_bytes(const nqs_ctx *c, int64_t M);
int64_t x3_chunk(const nqs_ctx *c, int64_t work);
// incremental cone of the split form (k_net_cone.hip)
bool cone_x3_supported(const nqs_ctx *c);

// --- autotuner (tune.hip) ---
std::string tune_cache_path();
std::string tune_key(const nqs_ctx *c);
bool tune_lookup(const std::string &path, const std::string &key, nqs_mode *mode, int *nw,
                 int *maxt, int *cone_items, int *cone_waves);
bool tune_store(const std::string &path, const std::string &key, nqs_mode mode, int nw, int maxt,
                int cone_items, int cone_waves, double ms_full, double ms_inc);
// tile variants (waves, tiles per wave) the full-recompute pass can use here
int mfma_full_variants(const nqs_ctx *c, int *nw, int *maxt, int cap);

// --- energy / SR kernels (k_energy.hip, k_sr.hip) ---
// isign (may be null): per-item sign ratio of the network (CNN1)
void launch_energy_reduce(const nqs_ctx *c, const int8_t *spins, int B, const int64_t *offsets,
                          const uint32_t *queue, const double *dlog, const int8_t *isign,
                          const double *ediag, double *e_loc, int32_t *err, hipStream_t s);

// --- CNN1 network family (k_cnn1.hip), FP64 ---
int64_t cnn1_params(int Kb, int C);
size_t cnn1_plane_bytes(const nqs_ctx *c, int64_t planes);
int64_t cnn1_chunk(const nqs_ctx *c, int64_t work);
// samples: f[B] = log|psi_net|, sgn[B] = its sign; sign_pub (may be null)
// is multiplied by the network sign.  pa, pb: cnn1_plane_bytes(c, B) each.
void cnn1_base_forward(const nqs_ctx *c, const int8_t *spins, int B, double *f, int8_t *sgn,
                       int8_t *sign_pub, void *pa, void *pb, hipStream_t s);
// queue items q0 .. q0+M-1: dlog[q] = f(S') - f(s), isign[q] = sign ratio
void cnn1_conn_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                       const int64_t *qlen, int64_t q0, int64_t M, const double *fbase,
                       const int8_t *sbase, double *dlog, int8_t *isign, void *pa, void *pb,
                       hipStream_t s);
// exchanged configurations by the receptive cone (16 channels, K <= 6,
// L >= 4K + 4): the base pass also keeps the activations (cache: stencils
// 1 .. 2K-1 [2K-1][B][N][16], then per site of the last layer the sum of
// log|u| [B][N] and the negative count [B][N] int32; samples b0 .. b0+nb-1
// of B; f and sgn of those samples), then one launch gives dlog and isign of
// queue items 0 .. cap - 1
bool cnn1_cone_ok(const nqs_ctx *c);
size_t cnn1_cache_bytes(const nqs_ctx *c, int64_t B);
void cnn1_base_forward_cached(const nqs_ctx *c, const int8_t *spins, int nb, double *f,
                              int8_t *sgn, void *pa, void *pb, double *cache, int64_t B,
                              int64_t b0, hipStream_t s);
void cnn1_cone_forward(const nqs_ctx *c, const int8_t *spins, int64_t B, const uint32_t *queue,
                       const int64_t *qlen, int64_t cap, const double *cache, double *dlog,
                       int8_t *isign, hipStream_t s);
// matrix-core packing of blocks 2.. (16 channels): its size in doubles (0
// when the vector kernels serve) and its rebuild from w_canon into w_vec64
size_t cnn1_packed_doubles(const nqs_ctx *c);
void cnn1_pack_device(const nqs_ctx *c, hipStream_t s);
void f64mma_cnn1_conv(const nqs_ctx *c, const double *in, int64_t M, const double *w,
                      const double *bias, double *out, double *zsave, const int64_t *qlen,
                      int64_t q_begin, hipStream_t s);
void f64mma_cnn1_convt(const nqs_ctx *c, const double *in, int64_t M, const double *w,
                       const double *bias, double *out, const int64_t *qlen, int64_t q_begin,
                       hipStream_t s);
void f64mma_cnn1_plain(const nqs_ctx *c, const double *in, int64_t M, int Cin, const double *w,
                       double *out, hipStream_t s);
size_t cnn1_deriv_bytes_per_sample(const nqs_ctx *c);
// O rows of nb samples; zsave: K*2*nb*N*C, usave: K*nb*N*C, work: 5*nb*N*C doubles
void cnn1_deriv_rows(const nqs_ctx *c, const int8_t *spins, int nb, double *zsave,
                     double *usave, double *work, void *O, nqs_dtype odt, hipStream_t s);

// --- CNN2 network family (k_cnn2.hip), FP64, C = 16 or 32 ---
bool cnn2_supported(int Kb, int C);
int64_t cnn2_params(int Kb, int C);
size_t cnn2_plane_bytes(const nqs_ctx *c, int64_t planes);
int64_t cnn2_chunk(const nqs_ctx *c, int64_t work);
void cnn2_base_forward(const nqs_ctx *c, const int8_t *spins, int B, double *f, int8_t *sgn,
                       int8_t *sign_pub, void *pa, void *pb, hipStream_t s);
void cnn2_conn_forward(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                       const int64_t *qlen, int64_t q0, int64_t M, const double *fbase,
                       const int8_t *sbase, double *dlog, int8_t *isign, void *pa, void *pb,
                       hipStream_t s);
size_t cnn2_packed_doubles(const nqs_ctx *c);
void cnn2_pack_device(const nqs_ctx *c, hipStream_t s);
void cnn2_deriv_planes(const nqs_ctx *c, int *zp, int *hp, int *wp);
void cnn2_deriv_rows(const nqs_ctx *c, const int8_t *spins, int nb, double *zsave,
                     double *hsave, double *work, void *O, nqs_dtype odt, hipStream_t s);

// A block network (CNN1, CNN2): an FP64 forward over planes [M][N][C] of
// samples or queue items, every exchanged configuration recomputed in full,
// a sign carried by the network, and a per-sample backward whose buffers
// hold zp, hp and wp planes of N*C doubles per sample.
struct BlockNet {
    int64_t (*params)(int Kb, int C);
    size_t (*plane_bytes)(const nqs_ctx *c, int64_t planes);
    int64_t (*chunk)(const nqs_ctx *c, int64_t work);
    void (*base_forward)(const nqs_ctx *c, const int8_t *spins, int B, double *f, int8_t *sgn,
                         int8_t *sign_pub, void *pa, void *pb, hipStream_t s);
    void (*conn_forward)(const nqs_ctx *c, const int8_t *spins, const uint32_t *queue,
                         const int64_t *qlen, int64_t q0, int64_t M, const double *fbase,
                         const int8_t *sbase, double *dlog, int8_t *isign, void *pa, void *pb,
                         hipStream_t s);
    size_t (*packed_doubles)(const nqs_ctx *c);
    void (*pack_device)(const nqs_ctx *c, hipStream_t s);
    void (*deriv_planes)(const nqs_ctx *c, int *zp, int *hp, int *wp);
    void (*deriv_rows)(const nqs_ctx *c, const int8_t *spins, int nb, double *zsave,
                       double *hsave, double *work, void *O, nqs_dtype odt, hipStream_t s);
    // the incremental form (null: none): whether it serves c, the size of its
    // activation cache, the base pass that fills it, the exchanged pass
    bool (*cone_ok)(const nqs_ctx *c);
    size_t (*cache_bytes)(const nqs_ctx *c, int64_t B);
    void (*base_forward_cached)(const nqs_ctx *c, const int8_t *spins, int nb, double *f,
                                int8_t *sgn, void *pa, void *pb, double *cache, int64_t B,
                                int64_t b0, hipStream_t s);
    void (*cone_forward)(const nqs_ctx *c, const int8_t *spins, int64_t B, const uint32_t *queue,
                         const int64_t *qlen, int64_t cap, const double *cache, double *dlog,
                         int8_t *isign, hipStream_t s);
};
// the context's block network, null for the ln cosh CNN
const BlockNet *block_net(const nqs_ctx *c);
void cnn1_deriv_planes(const nqs_ctx *c, int *zp, int *hp, int *wp);

void launch_energy_stats(const double *e_loc, int B, double *stats, hipStream_t s);

// --- device-side parameter update (k_pack.hip) ---
// theta += scale * dtheta (device FP64 [P]) and every packing rebuilt on the device
void device_update_weights(nqs_ctx *c, const double *dtheta, double scale, hipStream_t s);
// theta (device FP64 [P]) becomes the weights, every packing rebuilt on the device
void device_set_weights(nqs_ctx *c, const double *theta, hipStream_t s);

// --- Metropolis sampling (k_mcmc.hip) ---
// queue[s] = (s, bond of proposal rnd[s]), qlen[0] = B
void launch_mcmc_propose(const nqs_ctx *c, int B, const uint32_t *rnd, uint32_t *queue,
                         int64_t *qlen, hipStream_t s);
// flag[s] (may be null) = chain s accepts (antiparallel pair, u[s] < exp(2 dlog[s]));
// accepted[s] (may be null) counts them; apply: exchange the pair at once
void launch_mcmc_decide(const nqs_ctx *c, int8_t *spins, int B, const uint32_t *queue,
                        const double *dlog, const double *u, int32_t *flag, int32_t *accepted,
                        bool apply, hipStream_t s);
// exchange the pairs of the chains with flag[s] != 0
void launch_mcmc_apply(const nqs_ctx *c, int8_t *spins, int B, const uint32_t *queue,
                       const int32_t *flag, hipStream_t s);
size_t sr_workspace_bytes(int64_t B, int64_t P);
void launch_sr_solve(const void *O, nqs_dtype odt, const double *e_loc, int64_t B, int64_t P,
                     double lambda, int n_iter, double *x, double *stats, void *work,
                     hipStream_t s);
// rows of O recomputed on demand: fills rows [r0, r0 + nb) of O into buf
// (row-major, nb rows) on the stream
using SrRows = std::function<void(int64_t r0, int nb, void *buf, hipStream_t s)>;
// rows per reduction block of the SR solve for a batch of B (chunks of the
// recompute variant are multiples of it)
int64_t sr_row_block(int64_t B);
void launch_sr_solve_rows(const SrRows &rows, void *obuf, int64_t chunk, nqs_dtype odt,
                          const double *e_loc, int64_t B, int64_t P, double lambda, int n_iter,
                          double *x, double *stats, void *work, hipStream_t s);

inline bool nn_moves(const nqs_ctx *c)
{
    return c->J1 != 0.0 || (c->model == kModelTJ && c->t_hop != 0.0);
}
inline bool nnn_moves(const nqs_ctx *c) { return c->J2 != 0.0; }

}  // namespace nqs
