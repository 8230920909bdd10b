// nqs_abi.hip -- host side of the C ABI declared in include/nqs.h: argument
// validation, weight packing for each kernel family, workspace management and
// the order in which the kernels of each call are enqueued.  Nothing here does
// arithmetic of the method; every step runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>

#include "nqs_internal.h"

using namespace nqs;

namespace nqs {

const BlockNet kCnn1Net{cnn1_params,       cnn1_plane_bytes,  cnn1_chunk,
                        cnn1_base_forward, cnn1_conn_forward, cnn1_packed_doubles,
                        cnn1_pack_device,  cnn1_deriv_planes, cnn1_deriv_rows,
                        cnn1_cone_ok,      cnn1_cache_bytes,  cnn1_base_forward_cached,
                        cnn1_cone_forward};
const BlockNet kCnn2Net{cnn2_params,       cnn2_plane_bytes,  cnn2_chunk,
                        cnn2_base_forward, cnn2_conn_forward, cnn2_packed_doubles,
                        cnn2_pack_device,  cnn2_deriv_planes, cnn2_deriv_rows,
                        nullptr,           nullptr,           nullptr,
                        nullptr};

const BlockNet *block_net(const nqs_ctx *c)
{
    return c->net == kNetCnn1 ? &kCnn1Net : (c->net == kNetCnn2 ? &kCnn2Net : nullptr);
}

}  // namespace nqs

namespace {

#define HIP_OK(x)                                   \
    do {                                            \
        if ((x) != hipSuccess) return NQS_E_HIP;    \
    } while (0)

int64_t params_of(int K, int C) { return (int64_t)(C * 9 + C) + (int64_t)(K - 1) * (C * C * 9 + C); }


// FP64 -> BF16, round to nearest even (via FP32, with the double-rounding
// case resolved against the exact midpoint).
uint16_t bf16_rne(double d)
{
    float f = (float)d;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN
    const uint32_t low = u & 0xffffu;
    uint32_t hi = u >> 16;
    if (low == 0x8000u) {
        // f sits on a BF16 midpoint: decide from the exact double
        uint32_t lo_b = u & 0xffff0000u, up_b = lo_b + 0x10000u;
        float flo, fup;
        std::memcpy(&flo, &lo_b, 4);
        std::memcpy(&fup, &up_b, 4);
        const double mid = 0.5 * ((double)flo + (double)fup);
        const double ad = std::fabs(d), am = std::fabs(mid);
        if (ad > am) hi += 1;
        else if (ad == am) hi += (hi & 1);
        return (uint16_t)hi;
    }
    if (low > 0x8000u) hi += 1;
    return (uint16_t)hi;
}

template <int C>
int chan_of_slot_h(int q)
{
    if (C == 32) {
        const int g = q >> 3, r = q & 7;
        return r < 4 ? 4 * g + r : 16 + 4 * g + (r - 4);
    }
    return q;
}

struct Canon {
    const double *w;
    int K, C;
    int64_t off(int l) const
    {
        int64_t o = 0;
        for (int i = 0; i < l; ++i) o += (int64_t)C * (i == 0 ? 1 : C) * 9 + C;
        return o;
    }
    int cin(int l) const { return l == 0 ? 1 : C; }
    double W(int l, int co, int ci, int t) const { return w[off(l) + ((int64_t)co * cin(l) + ci) * 9 + t]; }
    double b(int l, int co) const { return w[off(l) + (int64_t)C * cin(l) * 9 + co]; }
};

template <typename T>
void free_dev(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

// A packing's size depends only on the network shape, which a context never
// changes, so a buffer that exists is refilled in place: its address stays
// valid for kernels captured in a graph before the weights were set again.
template <typename T>
nqs_status upload(T *&dst, const std::vector<T> &src)
{
    if (src.empty()) return NQS_OK;
    if (!dst && hipMalloc((void **)&dst, src.size() * sizeof(T)) != hipSuccess) {
        dst = nullptr;
        return NQS_E_NOMEM;
    }
    HIP_OK(hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return NQS_OK;
}

nqs_status pack_weights(nqs_ctx *c)
{
    if (const BlockNet *bn = block_net(c)) {
        // canonical vector, plus the matrix-core packing built from it on the device
        nqs_status st = upload(c->w_canon, c->w_host);
        const size_t np = bn->packed_doubles(c);
        if (st != NQS_OK || np == 0) return st;
        if (!c->w_vec64 && hipMalloc((void **)&c->w_vec64, np * sizeof(double)) != hipSuccess) {
            c->w_vec64 = nullptr;
            return NQS_E_NOMEM;
        }
        bn->pack_device(c, nullptr);
        HIP_OK(hipDeviceSynchronize());
        return NQS_OK;
    }
    const int K = c->K, C = c->C;
    Canon cn{c->w_host.data(), K, C};
    // vector path: layer 1 [9][C] + b; layer k [9][Cin][C] + b
    std::vector<double> v64;
    for (int l = 0; l < K; ++l) {
        const int ci_n = cn.cin(l);
        for (int t = 0; t < 9; ++t)
            for (int ci = 0; ci < ci_n; ++ci)
                for (int co = 0; co < C; ++co) v64.push_back(cn.W(l, co, ci, t));
        for (int co = 0; co < C; ++co) v64.push_back(cn.b(l, co));
    }
    std::vector<float> v32(v64.begin(), v64.end());
    // backward data pass, layers 2..K: [t'][co][ci] = W[co][ci][8 - t']
    std::vector<double> bw;
    for (int l = 1; l < K; ++l)
        for (int t = 0; t < 9; ++t)
            for (int co = 0; co < C; ++co)
                for (int ci = 0; ci < C; ++ci) bw.push_back(cn.W(l, co, ci, 8 - t));
    nqs_status st;
    if ((st = upload(c->w_vec64, v64)) != NQS_OK) return st;
    if ((st = upload(c->w_vec32, v32)) != NQS_OK) return st;
    if ((st = upload(c->w_bwd64, bw)) != NQS_OK) return st;
    if ((st = upload(c->w_canon, c->w_host)) != NQS_OK) return st;
    if (c->dtype == NQS_BF16 || c->dtype == NQS_BF16X3) {
        // A operands of v_mfma_f32_16x16x32_bf16: lane l holds row m = l % 16
        // (output channel 16 h + m) and the 8 reduction elements (g = l/16, i)
        // that pair with the B operand's 8 elements of lane group g.  BF16X3
        // also packs the lo parts: lo = bf16(W - hi), W - hi exact in FP64.
        std::vector<uint16_t> wm, wlo;
        const int KS = (C == 32) ? 9 : 5, NH = C / 16;
        for (int l = 1; l < K; ++l)
            for (int j = 0; j < KS; ++j)
                for (int h = 0; h < NH; ++h)
                    for (int lane = 0; lane < 64; ++lane)
                        for (int i = 0; i < 8; ++i) {
                            const int g = lane >> 4, co = 16 * h + (lane & 15);
                            int tap, ci;
                            if (C == 32) {
                                tap = j;
                                ci = chan_of_slot_h<32>(g * 8 + i);
                            } else {
                                tap = 2 * j + (g >> 1);
                                ci = chan_of_slot_h<16>((g & 1) * 8 + i);
                            }
                            const double wv = tap <= 8 ? cn.W(l, co, ci, tap) : 0.0;
                            const uint16_t hi = bf16_rne(wv);
                            wm.push_back(hi);
                            if (c->dtype == NQS_BF16X3) {
                                uint32_t hb = (uint32_t)hi << 16;
                                float hf;
                                std::memcpy(&hf, &hb, 4);
                                wlo.push_back(bf16_rne(wv - (double)hf));
                            }
                        }
        std::vector<float> l1;
        for (int t = 0; t < 9; ++t)
            for (int co = 0; co < C; ++co) l1.push_back((float)cn.W(0, co, 0, t));
        for (int l = 0; l < K; ++l)
            for (int co = 0; co < C; ++co) l1.push_back((float)cn.b(l, co));
        if ((st = upload(c->w_mfma, wm)) != NQS_OK) return st;
        if ((st = upload(c->w_l1, l1)) != NQS_OK) return st;
        if (c->dtype == NQS_BF16X3) {
            if ((st = upload(c->w_mfma_lo, wlo)) != NQS_OK) return st;
            if (cone_x3_supported(c) && !c->cone_tab &&
                (st = cone_build_ring_tables(c)) != NQS_OK)
                return st;
            return NQS_OK;
        }
        if (!c->ring_tab && (st = mfma_build_ring_tables(c)) != NQS_OK) return st;
        if (cone_supported(c) && !c->cone_tab && (st = cone_build_ring_tables(c)) != NQS_OK)
            return st;
    }
    return NQS_OK;
}

int64_t bonds_per_sample(const nqs_ctx *c)
{
    return (int64_t)2 * c->N * ((nn_moves(c) ? 1 : 0) + (nnn_moves(c) ? 1 : 0));
}

// whether the incremental cone form serves this context
bool incremental_ok(const nqs_ctx *c)
{
    if (const BlockNet *bn = block_net(c)) return bn->cone_ok && bn->cone_ok(c);
    if (c->net != kNetLnCosh) return false;
    if (c->dtype == NQS_BF16) return mfma_inc_supported(c);
    if (c->dtype == NQS_BF16X3) return cone_x3_supported(c);
    if (c->dtype == NQS_FP64) return cone64_ok(c);
    return false;
}

nqs_mode resolve_mode(const nqs_ctx *c, nqs_mode m)
{
    if (m != NQS_AUTO) return m;
    if (block_net(c) || c->dtype == NQS_FP64) {
        if (!incremental_ok(c)) return NQS_FULL;
        if (c->tuned) return c->tuned_mode;
        // positions of the cone (R_1 .. R_S of a 2x2 box, S stencils: 2K for a
        // block network, K for the ln cosh CNN) against S full layers
        const int S = block_net(c) ? 2 * c->K : c->K;
        double inc = 0.0, full = 0.0;
        for (int l = 1; l <= S; ++l) {
            inc += (2.0 + 2 * l) * (2.0 + 2 * l);
            full += (double)c->N;
        }
        return inc < 0.7 * full ? NQS_INCREMENTAL : NQS_FULL;
    }
    if (c->dtype == NQS_BF16X3) {
        if (c->tuned) return (c->tuned_mode == NQS_INCREMENTAL && !incremental_ok(c)) ? NQS_FULL
                                                                                       : c->tuned_mode;
        return incremental_ok(c) ? NQS_INCREMENTAL : NQS_FULL;
    }
    if (c->dtype != NQS_BF16) return NQS_FULL;
    if (c->tuned) return (c->tuned_mode == NQS_INCREMENTAL && !mfma_inc_supported(c)) ? NQS_FULL
                                                                                      : c->tuned_mode;
    // incremental work: sum_k |R_k| over layers 2..K for a 2x2 seed, clamped
    double inc = 0.0, full = 0.0;
    for (int k = 2; k <= c->K; ++k) {
        const int ex = std::min(2 + 2 * k, c->L);
        inc += (double)ex * ex;
        full += (double)c->N;
    }
    return (inc < 0.7 * full && mfma_inc_supported(c)) ? NQS_INCREMENTAL : NQS_FULL;
}

#define NQS_TRY(x)                        \
    do {                                  \
        nqs_status _s = (x);              \
        if (_s != NQS_OK) return _s;      \
    } while (0)

// Integer stage: counts, diagonal energy, offsets, queue.
nqs_status integer_stage(nqs_ctx *c, const int8_t *spins, int B, hipStream_t s)
{
    Workspace &w = c->ws;
    const int64_t cap = bonds_per_sample(c) * B;
    NQS_TRY(ensure(w.counts, sizeof(int32_t) * std::max(B, 1), s));
    NQS_TRY(ensure(w.ediag, sizeof(double) * std::max(B, 1), s));
    NQS_TRY(ensure(w.offsets, sizeof(int64_t) * (B + 1), s));
    NQS_TRY(ensure(w.qlen, sizeof(int64_t) * 4, s));
    NQS_TRY(ensure(w.queue, sizeof(uint32_t) * std::max<int64_t>(cap, 1), s));
    launch_bond_count(c, spins, B, (int32_t *)w.counts.ptr, (double *)w.ediag.ptr, s);
    launch_scan((int32_t *)w.counts.ptr, B, (int64_t *)w.offsets.ptr, (int64_t *)w.qlen.ptr, s);
    launch_queue_fill(c, spins, B, (int64_t *)w.offsets.ptr, (uint32_t *)w.queue.ptr, s);
    return NQS_OK;
}

// Vector-path chunk size (items per layer launch), bounded by plane memory.
int64_t vec_chunk(const nqs_ctx *c, int64_t cap)
{
    const size_t per = vec_plane_bytes(c, 1);
    int64_t m = (int64_t)((size_t)1 << 30) / (int64_t)std::max<size_t>(per, 1);
    m = std::max<int64_t>(1, std::min<int64_t>(m, 65535));
    return std::min(m, std::max<int64_t>(cap, 1));
}

size_t cache_bytes(const nqs_ctx *c, int64_t B)
{
    return std::max<size_t>(c->dtype == NQS_BF16X3 ? x3_cache_bytes(c, B) : mfma_cache_bytes(c, B),
                            16);
}

// BF16 / BF16X3 base pass: log-amplitudes, per-site sums and the activation
// cache of the samples, in the context's workspace.
nqs_status bf16_base_stage(nqs_ctx *c, const int8_t *spins, int B, hipStream_t s)
{
    Workspace &w = c->ws;
    NQS_TRY(ensure(w.fbase, sizeof(double) * std::max(B, 1), s));
    NQS_TRY(ensure(w.hsum, sizeof(double) * (size_t)std::max(B, 1) * c->N, s));
    NQS_TRY(ensure(w.cache, cache_bytes(c, B), s));
    if (c->dtype == NQS_BF16X3)
        x3_base_forward(c, spins, B, (double *)w.fbase.ptr, (double *)w.hsum.ptr, w.cache.ptr,
                        nullptr, s);
    else
        mfma_base_forward(c, spins, B, (double *)w.fbase.ptr, (double *)w.hsum.ptr, w.cache.ptr,
                          s);
    return NQS_OK;
}

// BF16X3 full recomputation: buffers for chunks of `chunk` configurations
nqs_status x3_full_reserve(nqs_ctx *c, int64_t chunk, hipStream_t s)
{
    Workspace &w = c->ws;
    NQS_TRY(ensure(w.plane_a, x3_plane_bytes(c, chunk), s));
    NQS_TRY(ensure(w.plane_b, x3_plane_bytes(c, chunk), s));
    NQS_TRY(ensure(w.hstmp, x3_sums_bytes(c, chunk), s));
    return NQS_OK;
}

// The exchanged-configuration pass of a BF16X3 context on the queue in the
// workspace (base pass already taken): the incremental cone or the full
// recomputation in chunks.
nqs_status x3_conn_stage(nqs_ctx *c, const int8_t *spins, nqs_mode mode, double *dlog,
                         int64_t cap, hipStream_t s)
{
    Workspace &w = c->ws;
    if (mode == NQS_INCREMENTAL) {
        cone_forward(c, spins, (uint32_t *)w.queue.ptr, (int64_t *)w.qlen.ptr, cap,
                     (double *)w.hsum.ptr, w.cache.ptr, dlog, s);
        return NQS_OK;
    }
    const int64_t chunk = x3_chunk(c, cap);
    NQS_TRY(x3_full_reserve(c, chunk, s));
    for (int64_t q0 = 0; q0 < cap; q0 += chunk)
        x3_conn_forward(c, spins, (uint32_t *)w.queue.ptr, (int64_t *)w.qlen.ptr, q0,
                        std::min(chunk, cap - q0), (double *)w.hsum.ptr, dlog, w.plane_a.ptr,
                        w.plane_b.ptr, w.hstmp.ptr, s);
    return NQS_OK;
}

// Block networks (CNN1, CNN2): base pass (log|psi_net| and sign of the
// samples), then every queue item recomputed in full: dlog[item] and the
// sign ratio in ws.isign.
nqs_status block_ratio_stage(nqs_ctx *c, const BlockNet *bn, const int8_t *spins, int B,
                             nqs_mode mode, double *dlog, int64_t cap, hipStream_t s)
{
    Workspace &w = c->ws;
    const bool cone = mode == NQS_INCREMENTAL && incremental_ok(c);
    const int64_t chunk = bn->chunk(c, std::max<int64_t>(cone ? B : cap, B));
    NQS_TRY(ensure(w.sgn, std::max(B, 1), s));
    NQS_TRY(ensure(w.isign, std::max<int64_t>(cap, 1), s));
    NQS_TRY(ensure(w.plane_a, bn->plane_bytes(c, chunk), s));
    NQS_TRY(ensure(w.plane_b, bn->plane_bytes(c, chunk), s));
    if (cone) NQS_TRY(ensure(w.cache, bn->cache_bytes(c, B), s));
    for (int64_t b0 = 0; b0 < B; b0 += chunk) {
        const int nb = (int)std::min<int64_t>(chunk, B - b0);
        if (cone)
            bn->base_forward_cached(c, spins + b0 * c->N, nb, (double *)w.fbase.ptr + b0,
                                    (int8_t *)w.sgn.ptr + b0, w.plane_a.ptr, w.plane_b.ptr,
                                    (double *)w.cache.ptr, B, b0, s);
        else
            bn->base_forward(c, spins + b0 * c->N, nb, (double *)w.fbase.ptr + b0,
                              (int8_t *)w.sgn.ptr + b0, nullptr, w.plane_a.ptr, w.plane_b.ptr,
                              s);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        (void)hipEventRecord(e0, s);
    }
    if (cone)
        bn->cone_forward(c, spins, B, (const uint32_t *)w.queue.ptr, (const int64_t *)w.qlen.ptr,
                         cap, (const double *)w.cache.ptr, dlog, (int8_t *)w.isign.ptr, s);
    else
        for (int64_t q0 = 0; q0 < cap; q0 += chunk)
            bn->conn_forward(c, spins, (uint32_t *)w.queue.ptr, (int64_t *)w.qlen.ptr, q0,
                              std::min(chunk, cap - q0), (const double *)w.fbase.ptr,
                              (const int8_t *)w.sgn.ptr, dlog, (int8_t *)w.isign.ptr,
                              w.plane_a.ptr, w.plane_b.ptr, s);
    if (c->timing) {
        (void)hipEventRecord(e1, s);
        c->events.push_back({e0, e1});
    }
    return NQS_OK;
}

// Base pass + exchanged-configuration pass: dlog[item].
nqs_status log_ratio_stage(nqs_ctx *c, const int8_t *spins, int B, nqs_mode mode, double *dlog,
                           int64_t cap, hipStream_t s)
{
    Workspace &w = c->ws;
    NQS_TRY(ensure(w.fbase, sizeof(double) * std::max(B, 1), s));
    if (const BlockNet *bn = block_net(c))
        return block_ratio_stage(c, bn, spins, B, mode, dlog, cap, s);
    NQS_TRY(ensure(w.hsum, sizeof(double) * (size_t)std::max(B, 1) * c->N, s));
    if (c->dtype == NQS_BF16X3) {
        NQS_TRY(bf16_base_stage(c, spins, B, s));
        if (mode == NQS_FULL) NQS_TRY(x3_full_reserve(c, x3_chunk(c, cap), s));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) {
            (void)hipEventCreate(&e0);
            (void)hipEventCreate(&e1);
            (void)hipEventRecord(e0, s);
        }
        NQS_TRY(x3_conn_stage(c, spins, mode, dlog, cap, s));
        if (c->timing) {
            (void)hipEventRecord(e1, s);
            c->events.push_back({e0, e1});
        }
        return NQS_OK;
    }
    if (c->dtype == NQS_BF16) {
        NQS_TRY(bf16_base_stage(c, spins, B, s));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) {
            (void)hipEventCreate(&e0);
            (void)hipEventCreate(&e1);
            (void)hipEventRecord(e0, s);
        }
        mfma_conn_forward(c, mode, spins, (uint32_t *)w.queue.ptr, (int64_t *)w.qlen.ptr, cap,
                          (double *)w.hsum.ptr, w.cache.ptr, dlog, nullptr, s);
        if (c->timing) {
            (void)hipEventRecord(e1, s);
            c->events.push_back({e0, e1});
        }
        return NQS_OK;
    }
    if (mode == NQS_INCREMENTAL && incremental_ok(c)) {
        // FP64 receptive cone: per chunk of samples the base pass, which also
        // keeps the activations, then the cone over that chunk's queue items
        const int64_t chunk = std::min(vec_chunk(c, B), cone64_chunk(c, B));
        NQS_TRY(ensure(w.plane_a, vec_plane_bytes(c, chunk), s));
        NQS_TRY(ensure(w.cache, cone64_cache_bytes(c, chunk), s));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) {
            (void)hipEventCreate(&e0);
            (void)hipEventCreate(&e1);
        }
        for (int64_t b0 = 0; b0 < B; b0 += chunk) {
            const int nb = (int)std::min<int64_t>(chunk, B - b0);
            vec_base_forward_cached(c, spins + b0 * c->N, nb, (double *)w.fbase.ptr + b0,
                                    (double *)w.hsum.ptr + b0 * c->N, w.plane_a.ptr,
                                    (double *)w.cache.ptr, chunk, s);
            if (c->timing && b0 == 0) (void)hipEventRecord(e0, s);
            cone64_forward(c, spins, (const uint32_t *)w.queue.ptr, (const int64_t *)w.qlen.ptr,
                           cap, (const double *)w.cache.ptr, chunk, b0, nb,
                           (const double *)w.hsum.ptr, dlog, s);
        }
        if (c->timing) {
            (void)hipEventRecord(e1, s);
            c->events.push_back({e0, e1});
        }
        return NQS_OK;
    }
    const int64_t chunk = vec_chunk(c, std::max<int64_t>(cap, B));
    NQS_TRY(ensure(w.plane_a, vec_plane_bytes(c, chunk), s));
    NQS_TRY(ensure(w.plane_b, vec_plane_bytes(c, chunk), s));
    for (int64_t b0 = 0; b0 < B; b0 += chunk) {
        const int nb = (int)std::min<int64_t>(chunk, B - b0);
        vec_base_forward(c, spins + b0 * c->N, nb, (double *)w.fbase.ptr + b0,
                         (double *)w.hsum.ptr + b0 * c->N, w.plane_a.ptr, w.plane_b.ptr, s);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        (void)hipEventRecord(e0, s);
    }
    for (int64_t q0 = 0; q0 < cap; q0 += chunk)
        vec_conn_forward(c, spins, (uint32_t *)w.queue.ptr, (int64_t *)w.qlen.ptr, q0,
                         std::min(chunk, cap - q0), (double *)w.hsum.ptr, dlog, w.plane_a.ptr,
                         w.plane_b.ptr, s);
    if (c->timing) {
        (void)hipEventRecord(e1, s);
        c->events.push_back({e0, e1});
    }
    return NQS_OK;
}

// Status of the kernels enqueued by one API call (launch errors only; device
// faults surface at the next synchronisation).
nqs_status finish_call()
{
    const char *what = nullptr;
    const hipError_t e = take_launch_error(&what);
    (void)hipGetLastError();
    return e == hipSuccess ? NQS_OK : NQS_E_HIP;
}

nqs_status check_common(nqs_ctx *c, const void *spins, int64_t B)
{
    if (!c) return NQS_E_ARG;
    if (B < 0 || B > 131072) return NQS_E_ARG;
    if (B > 0 && !spins) return NQS_E_ARG;
    return NQS_OK;
}

}  // namespace

namespace nqs {

namespace {
thread_local hipError_t g_launch_err = hipSuccess;
thread_local const char *g_launch_what = nullptr;
}  // namespace

void note_launch(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess && g_launch_err == hipSuccess) {
        g_launch_err = e;
        g_launch_what = what;
        if (std::getenv("NQS_DEBUG"))
            std::fprintf(stderr, "libnqs: launch of %s failed: %s\n", what, hipGetErrorString(e));
    }
}

hipError_t take_launch_error(const char **what)
{
    const hipError_t e = g_launch_err;
    if (what) *what = g_launch_what;
    g_launch_err = hipSuccess;
    g_launch_what = nullptr;
    return e;
}

bool stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st == hipStreamCaptureStatusActive;
}

nqs_status ensure(DevBuf &b, size_t bytes, hipStream_t stream)
{
    const bool capturing = stream_capturing(stream);
    if (capturing && b.gy) b.gy->captured = true;
    if (bytes <= b.bytes) return NQS_OK;
    if (capturing) return NQS_E_WORKSPACE;
    if (b.ptr) {
        if (b.gy && b.gy->captured) {
            // a captured graph may still name this allocation: keep it
            b.gy->bufs.push_back(b.ptr);
        } else {
            HIP_OK(hipDeviceSynchronize());
            (void)hipFree(b.ptr);
        }
        b.ptr = nullptr;
        b.bytes = 0;
    }
    const size_t want = bytes + bytes / 8;
    if (hipMalloc(&b.ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        b.ptr = nullptr;
        return NQS_E_NOMEM;
    }
    b.bytes = want;
    return NQS_OK;
}

}  // namespace nqs

namespace {

// samples per pass of the backward: z and h of layers 1..K-1 plus two
// deltas per sample, at most 8 GB
int64_t deriv_chunk(const nqs_ctx *c, int64_t B)
{
    if (const BlockNet *bn = block_net(c)) {
        int zp, hp, wp;
        bn->deriv_planes(c, &zp, &hp, &wp);
        const size_t per = sizeof(double) * (size_t)c->N * c->C * (zp + hp + wp);
        const int64_t n = (int64_t)(((size_t)8 << 30) / per);
        return std::max<int64_t>(1, std::min<int64_t>(n, B));
    }
    const size_t plane = sizeof(double) * (size_t)c->N * c->C;   // one FP64 plane
    const size_t per = plane * (2 * (size_t)std::max(c->K - 1, 1) + 2);
    const int64_t chunk = (int64_t)(((size_t)8 << 30) / per);
    return std::max<int64_t>(1, std::min<int64_t>(chunk, B));
}

nqs_status deriv_reserve(nqs_ctx *c, int64_t chunk, hipStream_t s)
{
    Workspace &w = c->ws;
    const size_t plane = sizeof(double) * (size_t)c->N * c->C;
    if (const BlockNet *bn = block_net(c)) {
        int zp, hp, wp;
        bn->deriv_planes(c, &zp, &hp, &wp);
        NQS_TRY(ensure(w.zsave, plane * zp * chunk, s));
        NQS_TRY(ensure(w.hsave, plane * hp * chunk, s));
        NQS_TRY(ensure(w.delta, plane * wp * chunk, s));
        return NQS_OK;
    }
    const size_t saved = plane * std::max(c->K - 1, 1) * chunk;
    NQS_TRY(ensure(w.zsave, saved, s));
    NQS_TRY(ensure(w.hsave, saved, s));
    NQS_TRY(ensure(w.delta, plane * 2 * chunk, s));
    return NQS_OK;
}

// O rows of B samples (workspace reserved for `chunk` samples per pass).  The
// backward runs in FP64 whatever the context's conv dtype.
void deriv_rows(const nqs_ctx *c, const int8_t *spins, int64_t B, int64_t chunk, void *O,
                nqs_dtype odt, hipStream_t s)
{
    const Workspace &w = c->ws;
    const size_t esz = odt == NQS_FP32 ? sizeof(float) : sizeof(double);
    for (int64_t b0 = 0; b0 < B; b0 += chunk) {
        const int nb = (int)std::min<int64_t>(chunk, B - b0);
        if (const BlockNet *bn = block_net(c)) {
            bn->deriv_rows(c, spins + b0 * c->N, nb, (double *)w.zsave.ptr,
                            (double *)w.hsave.ptr, (double *)w.delta.ptr,
                            (unsigned char *)O + (size_t)b0 * c->P * esz, odt, s);
            continue;
        }
        double *da = (double *)w.delta.ptr;
        double *db = da + (size_t)nb * c->N * c->C;
        vec_deriv_forward(c, spins + b0 * c->N, nb, (double *)w.zsave.ptr,
                          (double *)w.hsave.ptr, da, s);
        vec_backward(c, spins + b0 * c->N, nb, (const double *)w.zsave.ptr,
                     (const double *)w.hsave.ptr, da, db,
                     (unsigned char *)O + (size_t)b0 * c->P * esz, odt, s);
    }
}

// rows of O held at once by the recompute SR variant: chunk_rows (0: as many
// as fit in 2 GiB) rounded up to whole reduction blocks, at most the batch
int64_t recompute_chunk(const nqs_ctx *c, int64_t B, int64_t chunk_rows, nqs_dtype odt)
{
    const size_t esz = odt == NQS_FP32 ? sizeof(float) : sizeof(double);
    const int64_t blk = sr_row_block(B);
    int64_t want = chunk_rows > 0
                       ? chunk_rows
                       : std::max<int64_t>(1, (int64_t)(((size_t)2 << 30) / (esz * (size_t)c->P)));
    want = (want + blk - 1) / blk * blk;                      // whole reduction blocks
    return std::min<int64_t>(want, (B + blk - 1) / blk * blk);
}

}  // namespace

namespace {

nqs_status create_ctx(int32_t L, int model, int net, double J1, double J2, double t_hop,
                      const nqs_cnn_spec *spec, const double *weights, int64_t n_weights,
                      nqs_ctx **out)
{
    if (!spec || !weights || !out) return NQS_E_ARG;
    *out = nullptr;
    if (L < 4 || L > 64 || (L % 2) != 0) return NQS_E_LATTICE;
    if (!std::isfinite(J1) || !std::isfinite(J2) || !std::isfinite(t_hop)) return NQS_E_ARG;
    const int K = spec->n_layers, C = spec->channels;
    if (K < 1 || K > 16 || C < 1 || C > 32) return NQS_E_SPEC;
    if (spec->conv_dtype != NQS_FP64 && spec->conv_dtype != NQS_FP32 &&
        spec->conv_dtype != NQS_BF16 && spec->conv_dtype != NQS_BF16X3)
        return NQS_E_SPEC;
    if (spec->marshall_sign != 0 && spec->marshall_sign != 1) return NQS_E_SPEC;
    if (net != kNetLnCosh && spec->conv_dtype != NQS_FP64) return NQS_E_SPEC;
    if (net == kNetCnn2 && !cnn2_supported(K, C)) return NQS_E_SPEC;
    const int64_t want = net == kNetCnn1   ? cnn1_params(K, C)
                         : net == kNetCnn2 ? cnn2_params(K, C)
                                           : params_of(K, C);
    if (n_weights != want) return NQS_E_NPARAMS;
    nqs_ctx *c = new nqs_ctx();
    c->ws.bind();
    c->L = L;
    c->N = L * L;
    c->K = K;
    c->C = C;
    c->J1 = J1;
    c->J2 = J2;
    c->model = model;
    c->net = net;
    c->t_hop = t_hop;
    c->marshall = spec->marshall_sign;
    c->dtype = spec->conv_dtype;
    c->P = n_weights;
    if ((c->dtype == NQS_BF16 && !mfma_supported(c)) || (c->dtype == NQS_BF16X3 && !x3_supported(c))) {
        delete c;
        return NQS_E_SPEC;
    }
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return NQS_E_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
    c->w_host.assign(weights, weights + n_weights);
    if (hipMalloc((void **)&c->err, sizeof(int32_t)) != hipSuccess ||
        hipMemset(c->err, 0, sizeof(int32_t)) != hipSuccess) {
        delete c;
        return NQS_E_NOMEM;
    }
    nqs_status st = pack_weights(c);
    if (st != NQS_OK) {
        nqs_destroy(c);
        return st;
    }
    // an earlier autotuner choice for this configuration, if the cache has one
    {
        nqs_mode m;
        int nw = 0, mt = 0, ci = -1, cw = -1;
        // (block networks store no choices; their keys would match the ln
        // cosh CNN's of the same shape)
        if (!block_net(c) && tune_lookup(tune_cache_path(), tune_key(c), &m, &nw, &mt, &ci, &cw)) {
            c->tuned = 1;
            c->tuned_mode = m;
            c->full_nw = nw;
            c->full_maxt = mt;
            if (ci > 0) c->cone_variant = cone_variant_of(c, ci, cw);
        }
    }
    *out = c;
    return NQS_OK;
}

}  // namespace

extern "C" {

const char *nqs_status_str(nqs_status s)
{
    switch (s) {
    case NQS_OK: return "ok";
    case NQS_E_ARG: return "invalid argument";
    case NQS_E_LATTICE: return "unsupported lattice (L must be even, 4 <= L <= 64)";
    case NQS_E_SPEC: return "unsupported network specification";
    case NQS_E_NPARAMS: return "weight count does not match the network";
    case NQS_E_SPIN: return "spin value other than +1/-1";
    case NQS_E_NONFINITE: return "non-finite log-amplitude ratio or local energy";
    case NQS_E_NOMEM: return "device allocation failed";
    case NQS_E_WORKSPACE: return "workspace too small during stream capture";
    case NQS_E_HIP: return "HIP runtime error";
    case NQS_E_UNSUPPORTED: return "not supported by this build";
    }
    return "unknown status";
}

nqs_status nqs_create(int32_t L, double J1, double J2, const nqs_cnn_spec *spec,
                      const double *weights, int64_t n_weights, nqs_ctx **out)
{
    return create_ctx(L, kModelSpin, kNetLnCosh, J1, J2, 0.0, spec, weights, n_weights, out);
}

nqs_status nqs_create_cnn1(int32_t L, double J1, double J2, int32_t blocks, int32_t channels,
                           int32_t marshall_sign, const double *weights, int64_t n_weights,
                           nqs_ctx **out)
{
    const nqs_cnn_spec spec{blocks, channels, marshall_sign, NQS_FP64};
    return create_ctx(L, kModelSpin, kNetCnn1, J1, J2, 0.0, &spec, weights, n_weights, out);
}

nqs_status nqs_create_cnn1_tj(int32_t L, double t, double J, int32_t blocks, int32_t channels,
                              int32_t marshall_sign, const double *weights, int64_t n_weights,
                              nqs_ctx **out)
{
    const nqs_cnn_spec spec{blocks, channels, marshall_sign, NQS_FP64};
    return create_ctx(L, kModelTJ, kNetCnn1, J, 0.0, t, &spec, weights, n_weights, out);
}

nqs_status nqs_create_cnn2_tj(int32_t L, double t, double J, int32_t blocks, int32_t channels,
                              int32_t marshall_sign, const double *weights, int64_t n_weights,
                              nqs_ctx **out)
{
    const nqs_cnn_spec spec{blocks, channels, marshall_sign, NQS_FP64};
    return create_ctx(L, kModelTJ, kNetCnn2, J, 0.0, t, &spec, weights, n_weights, out);
}

nqs_status nqs_create_tj(int32_t L, double t, double J, const nqs_cnn_spec *spec,
                         const double *weights, int64_t n_weights, nqs_ctx **out)
{
    return create_ctx(L, kModelTJ, kNetLnCosh, J, 0.0, t, spec, weights, n_weights, out);
}

nqs_status nqs_destroy(nqs_ctx *c)
{
    if (!c) return NQS_E_ARG;
    (void)hipDeviceSynchronize();
    free_dev(c->w_canon);
    free_dev(c->w_vec64);
    free_dev(c->w_vec32);
    free_dev(c->w_bwd64);
    free_dev(c->w_mfma);
    free_dev(c->w_mfma_lo);
    free_dev(c->w_l1);
    free_dev(c->ring_tab);
    free_dev(c->ring_off);
    free_dev(c->cone_tab);
    free_dev(c->ls_tab);
    free_dev(c->fr_tab);
    free_dev(c->err);
    for (DevBuf *b : c->ws.all())
        if (b->ptr) (void)hipFree(b->ptr);
    for (void *p : c->ws.gy.bufs) (void)hipFree(p);
    for (auto &e : c->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    delete c;
    return NQS_OK;
}

nqs_status nqs_num_params(const nqs_ctx *c, int64_t *P)
{
    if (!c || !P) return NQS_E_ARG;
    *P = c->P;
    return NQS_OK;
}

nqs_status nqs_set_weights(nqs_ctx *c, const double *weights, int64_t n)
{
    if (!c || !weights) return NQS_E_ARG;
    if (n != c->P) return NQS_E_NPARAMS;
    HIP_OK(hipDeviceSynchronize());
    c->w_host.assign(weights, weights + n);
    return pack_weights(c);
}

nqs_status nqs_update_weights(nqs_ctx *c, const double *dtheta, double scale, void *stream)
{
    if (!c || !dtheta || !std::isfinite(scale)) return NQS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    device_update_weights(c, dtheta, scale, s);
    return finish_call();
}

nqs_status nqs_set_weights_device(nqs_ctx *c, const double *theta, void *stream)
{
    if (!c || !theta) return NQS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    device_set_weights(c, theta, s);
    return finish_call();
}

nqs_status nqs_get_weights(nqs_ctx *c, double *weights, int64_t n)
{
    if (!c || !weights) return NQS_E_ARG;
    if (n != c->P) return NQS_E_NPARAMS;
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(weights, c->w_canon, sizeof(double) * n, hipMemcpyDeviceToHost));
    c->w_host.assign(weights, weights + n);
    return NQS_OK;
}

nqs_status nqs_auto_mode(const nqs_ctx *c, nqs_mode *mode)
{
    if (!c || !mode) return NQS_E_ARG;
    *mode = resolve_mode(c, NQS_AUTO);
    return NQS_OK;
}

nqs_status nqs_reserve(nqs_ctx *c, int64_t B_max, nqs_mode mode)
{
    if (!c || B_max < 0 || B_max > 131072) return NQS_E_ARG;
    const int B = (int)B_max;
    hipStream_t s = nullptr;
    Workspace &w = c->ws;
    const int64_t cap = bonds_per_sample(c) * B;
    NQS_TRY(ensure(w.counts, sizeof(int32_t) * std::max(B, 1), s));
    NQS_TRY(ensure(w.ediag, sizeof(double) * std::max(B, 1), s));
    NQS_TRY(ensure(w.offsets, sizeof(int64_t) * (B + 1), s));
    NQS_TRY(ensure(w.qlen, sizeof(int64_t) * 4, s));
    NQS_TRY(ensure(w.queue, sizeof(uint32_t) * std::max<int64_t>(cap, 1), s));
    NQS_TRY(ensure(w.dlog, sizeof(double) * std::max<int64_t>(cap, 1), s));
    NQS_TRY(ensure(w.fbase, sizeof(double) * std::max(B, 1), s));
    NQS_TRY(ensure(w.hsum, sizeof(double) * (size_t)std::max(B, 1) * c->N, s));
    if (const BlockNet *bn = block_net(c)) {
        const int64_t chunk = bn->chunk(c, std::max<int64_t>(cap, B));
        NQS_TRY(ensure(w.sgn, std::max(B, 1), s));
        NQS_TRY(ensure(w.isign, std::max<int64_t>(cap, 1), s));
        NQS_TRY(ensure(w.plane_a, bn->plane_bytes(c, chunk), s));
        NQS_TRY(ensure(w.plane_b, bn->plane_bytes(c, chunk), s));
        if (resolve_mode(c, mode) == NQS_INCREMENTAL && incremental_ok(c))
            NQS_TRY(ensure(w.cache, bn->cache_bytes(c, B), s));
    } else if (c->dtype == NQS_BF16) {
        NQS_TRY(ensure(w.cache, cache_bytes(c, B), s));
    } else if (c->dtype == NQS_BF16X3) {
        NQS_TRY(ensure(w.cache, cache_bytes(c, B), s));
        if (resolve_mode(c, mode) == NQS_FULL) NQS_TRY(x3_full_reserve(c, x3_chunk(c, cap), s));
    } else {
        const int64_t chunk = vec_chunk(c, std::max<int64_t>(cap, B));
        NQS_TRY(ensure(w.plane_a, vec_plane_bytes(c, chunk), s));
        NQS_TRY(ensure(w.plane_b, vec_plane_bytes(c, chunk), s));
        if (resolve_mode(c, mode) == NQS_INCREMENTAL && incremental_ok(c))
            NQS_TRY(ensure(w.cache, cone64_cache_bytes(
                                        c, std::min(vec_chunk(c, B), cone64_chunk(c, B))), s));
    }
    return NQS_OK;
}

nqs_status nqs_log_psi(nqs_ctx *c, const int8_t *spins, int64_t B, double *log_abs, int8_t *sign,
                       void *stream)
{
    NQS_TRY(check_common(c, spins, B));
    if (B > 0 && !log_abs) return NQS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (B == 0) return NQS_OK;
    Workspace &w = c->ws;
    NQS_TRY(ensure(w.hsum, sizeof(double) * (size_t)B * c->N, s));
    launch_marshall(c, spins, (int)B, sign, s);
    if (const BlockNet *bn = block_net(c)) {
        const int64_t chunk = bn->chunk(c, B);
        NQS_TRY(ensure(w.sgn, (size_t)B, s));
        NQS_TRY(ensure(w.plane_a, bn->plane_bytes(c, chunk), s));
        NQS_TRY(ensure(w.plane_b, bn->plane_bytes(c, chunk), s));
        for (int64_t b0 = 0; b0 < B; b0 += chunk) {
            const int nb = (int)std::min<int64_t>(chunk, B - b0);
            bn->base_forward(c, spins + b0 * c->N, nb, log_abs + b0, (int8_t *)w.sgn.ptr + b0,
                              sign ? sign + b0 : nullptr, w.plane_a.ptr, w.plane_b.ptr, s);
        }
    } else if (c->dtype == NQS_BF16) {
        NQS_TRY(ensure(w.cache, cache_bytes(c, B), s));
        mfma_base_forward(c, spins, (int)B, log_abs, (double *)w.hsum.ptr, w.cache.ptr, s);
    } else if (c->dtype == NQS_BF16X3) {
        NQS_TRY(ensure(w.cache, cache_bytes(c, B), s));
        x3_base_forward(c, spins, (int)B, log_abs, (double *)w.hsum.ptr, w.cache.ptr, nullptr, s);
    } else {
        const int64_t chunk = vec_chunk(c, B);
        NQS_TRY(ensure(w.plane_a, vec_plane_bytes(c, chunk), s));
        NQS_TRY(ensure(w.plane_b, vec_plane_bytes(c, chunk), s));
        for (int64_t b0 = 0; b0 < B; b0 += chunk) {
            const int nb = (int)std::min<int64_t>(chunk, B - b0);
            vec_base_forward(c, spins + b0 * c->N, nb, log_abs + b0,
                             (double *)w.hsum.ptr + b0 * c->N, w.plane_a.ptr, w.plane_b.ptr, s);
        }
    }
    return finish_call();
}

nqs_status nqs_local_energy(nqs_ctx *c, const int8_t *spins, int64_t B, double *e_loc,
                            nqs_mode mode, void *stream)
{
    NQS_TRY(check_common(c, spins, B));
    if (B > 0 && !e_loc) return NQS_E_ARG;
    if (mode != NQS_AUTO && mode != NQS_FULL && mode != NQS_INCREMENTAL) return NQS_E_ARG;
    const nqs_mode m = resolve_mode(c, mode);
    if (m == NQS_INCREMENTAL && !incremental_ok(c))
        return NQS_E_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (B == 0) return NQS_OK;
    const int64_t cap = bonds_per_sample(c) * B;
    NQS_TRY(integer_stage(c, spins, (int)B, s));
    NQS_TRY(ensure(c->ws.dlog, sizeof(double) * std::max<int64_t>(cap, 1), s));
    NQS_TRY(log_ratio_stage(c, spins, (int)B, m, (double *)c->ws.dlog.ptr, cap, s));
    launch_energy_reduce(c, spins, (int)B, (int64_t *)c->ws.offsets.ptr,
                         (uint32_t *)c->ws.queue.ptr, (double *)c->ws.dlog.ptr,
                         block_net(c) ? (const int8_t *)c->ws.isign.ptr : nullptr,
                         (double *)c->ws.ediag.ptr, e_loc, c->err, s);
    return finish_call();
}

nqs_status nqs_log_ratios(nqs_ctx *c, const int8_t *spins, int64_t B, nqs_mode mode, double *dlog,
                          int64_t capacity, void *stream)
{
    NQS_TRY(check_common(c, spins, B));
    if (B > 0 && !dlog) return NQS_E_ARG;
    const int64_t cap = bonds_per_sample(c) * B;
    if (capacity < cap) return NQS_E_ARG;
    const nqs_mode m = resolve_mode(c, mode);
    if (m == NQS_INCREMENTAL && !incremental_ok(c))
        return NQS_E_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (B == 0) return NQS_OK;
    NQS_TRY(integer_stage(c, spins, (int)B, s));
    NQS_TRY(log_ratio_stage(c, spins, (int)B, m, dlog, cap, s));
    return finish_call();
}

nqs_status nqs_connected(nqs_ctx *c, const int8_t *spins, int64_t B, int32_t *counts,
                         int64_t *offsets, int32_t *bond_ids, int8_t *mu, int64_t capacity,
                         double *e_diag, void *stream)
{
    NQS_TRY(check_common(c, spins, B));
    if (!counts || !offsets || !bond_ids || !mu || !e_diag) return NQS_E_ARG;
    const int64_t cap = bonds_per_sample(c) * B;
    if (capacity < cap) return NQS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (B == 0) {
        HIP_OK(hipMemsetAsync(offsets, 0, sizeof(int64_t), s));
        return NQS_OK;
    }
    NQS_TRY(integer_stage(c, spins, (int)B, s));
    HIP_OK(hipMemcpyAsync(counts, c->ws.counts.ptr, sizeof(int32_t) * B, hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(offsets, c->ws.offsets.ptr, sizeof(int64_t) * (B + 1),
                          hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(e_diag, c->ws.ediag.ptr, sizeof(double) * B, hipMemcpyDeviceToDevice, s));
    launch_queue_expand(c, spins, (uint32_t *)c->ws.queue.ptr, (int64_t *)c->ws.qlen.ptr,
                        capacity, bond_ids, mu, s);
    return finish_call();
}

nqs_status nqs_energy_stats(nqs_ctx *c, const double *e_loc, int64_t B, double *stats, void *stream)
{
    if (!c || !stats || B <= 0 || !e_loc) return NQS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    launch_energy_stats(e_loc, (int)B, stats, s);
    return finish_call();
}

nqs_status nqs_log_deriv(nqs_ctx *c, const int8_t *spins, int64_t B, void *O, nqs_dtype odt,
                         void *stream)
{
    NQS_TRY(check_common(c, spins, B));
    if (B > 0 && !O) return NQS_E_ARG;
    if (odt != NQS_FP32 && odt != NQS_FP64) return NQS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (B == 0) return NQS_OK;
    const int64_t chunk = deriv_chunk(c, B);
    NQS_TRY(deriv_reserve(c, chunk, s));
    deriv_rows(c, spins, B, chunk, O, odt, s);
    return finish_call();
}

nqs_status nqs_sr_solve(nqs_ctx *c, const void *O, nqs_dtype odt, const double *e_loc, int64_t B,
                        double diag_shift, int32_t n_iter, double *dtheta, double *stats,
                        void *stream)
{
    if (!c || !O || !e_loc || !dtheta || B <= 0 || n_iter < 0) return NQS_E_ARG;
    if (odt != NQS_FP32 && odt != NQS_FP64) return NQS_E_ARG;
    if (!(diag_shift >= 0.0) || !std::isfinite(diag_shift)) return NQS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    NQS_TRY(ensure(c->ws.sr, sr_workspace_bytes(B, c->P), s));
    launch_sr_solve(O, odt, e_loc, B, c->P, diag_shift, n_iter, dtheta, stats, c->ws.sr.ptr, s);
    return finish_call();
}

nqs_status nqs_sr_solve_recompute(nqs_ctx *c, const int8_t *spins, nqs_dtype odt,
                                  const double *e_loc, int64_t B, double diag_shift,
                                  int32_t n_iter, int64_t chunk_rows, double *dtheta,
                                  double *stats, void *stream)
{
    NQS_TRY(check_common(c, spins, B));
    if (!e_loc || !dtheta || B <= 0 || n_iter < 0 || chunk_rows < 0) return NQS_E_ARG;
    if (odt != NQS_FP32 && odt != NQS_FP64) return NQS_E_ARG;
    if (!(diag_shift >= 0.0) || !std::isfinite(diag_shift)) return NQS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    const size_t esz = odt == NQS_FP32 ? sizeof(float) : sizeof(double);
    const int64_t chunk = recompute_chunk(c, B, chunk_rows, odt);
    const int64_t dchunk = deriv_chunk(c, chunk);
    NQS_TRY(ensure(c->ws.sr, sr_workspace_bytes(B, c->P), s));
    NQS_TRY(ensure(c->ws.orows, esz * (size_t)chunk * c->P, s));
    NQS_TRY(deriv_reserve(c, dchunk, s));
    const nqs_ctx *cc = c;
    const SrRows rows = [cc, spins, dchunk, odt](int64_t r0, int nb, void *buf, hipStream_t st) {
        deriv_rows(cc, spins + r0 * cc->N, nb, dchunk, buf, odt, st);
    };
    launch_sr_solve_rows(rows, c->ws.orows.ptr, chunk, odt, e_loc, B, c->P, diag_shift, n_iter,
                         dtheta, stats, c->ws.sr.ptr, s);
    return finish_call();
}

nqs_status nqs_mcmc(nqs_ctx *c, int8_t *spins, int64_t B, int32_t n_steps,
                    const uint32_t *rand_bond, const double *rand_u, int32_t *accepted,
                    nqs_mode mode, void *stream)
{
    NQS_TRY(check_common(c, spins, B));
    if (n_steps < 0) return NQS_E_ARG;
    if (mode != NQS_AUTO && mode != NQS_FULL && mode != NQS_INCREMENTAL) return NQS_E_ARG;
    if (B > 0 && n_steps > 0 && (!rand_bond || !rand_u)) return NQS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (B == 0 || n_steps == 0 || bonds_per_sample(c) == 0) return NQS_OK;
    const nqs_mode m = resolve_mode(c, mode);
    if (m == NQS_INCREMENTAL && c->dtype == NQS_BF16X3 && !incremental_ok(c))
        return NQS_E_UNSUPPORTED;
    Workspace &w = c->ws;
    NQS_TRY(ensure(w.queue, sizeof(uint32_t) * B, s));
    NQS_TRY(ensure(w.qlen, sizeof(int64_t) * 4, s));
    NQS_TRY(ensure(w.dlog, sizeof(double) * B, s));
    uint32_t *queue = (uint32_t *)w.queue.ptr;
    int64_t *qlen = (int64_t *)w.qlen.ptr;
    double *dlog = (double *)w.dlog.ptr;
    if (m == NQS_INCREMENTAL && (cone_supported(c) || cone_x3_supported(c))) {
        // base pass once, kept current by write-back passes of the accepted chains
        NQS_TRY(ensure(w.flags, sizeof(int32_t) * B, s));
        int32_t *flag = (int32_t *)w.flags.ptr;
        NQS_TRY(bf16_base_stage(c, spins, (int)B, s));
        for (int32_t t = 0; t < n_steps; ++t) {
            launch_mcmc_propose(c, (int)B, rand_bond + (int64_t)t * B, queue, qlen, s);
            cone_forward(c, spins, queue, qlen, B, (double *)w.hsum.ptr, w.cache.ptr, dlog, s);
            launch_mcmc_decide(c, spins, (int)B, queue, dlog, rand_u + (int64_t)t * B, flag,
                               accepted, false, s);
            cone_commit(c, spins, queue, qlen, B, (double *)w.hsum.ptr, w.cache.ptr, dlog, flag,
                        s);
            launch_mcmc_apply(c, spins, (int)B, queue, flag, s);
        }
        return finish_call();
    }
    for (int32_t t = 0; t < n_steps; ++t) {
        launch_mcmc_propose(c, (int)B, rand_bond + (int64_t)t * B, queue, qlen, s);
        NQS_TRY(log_ratio_stage(c, spins, (int)B, m, dlog, B, s));
        launch_mcmc_decide(c, spins, (int)B, queue, dlog, rand_u + (int64_t)t * B, nullptr,
                           accepted, true, s);
    }
    return finish_call();
}

nqs_status nqs_local_energy_multi(const nqs_eloc_job *jobs, int32_t n, nqs_mode mode, void *stream)
{
    if (!jobs || n < 0) return NQS_E_ARG;
    if (mode != NQS_AUTO && mode != NQS_FULL && mode != NQS_INCREMENTAL) return NQS_E_ARG;
    for (int i = 0; i < n; ++i) {
        nqs_ctx *c = jobs[i].ctx;
        if (!c) return NQS_E_ARG;
        if (c->K != jobs[0].ctx->K || c->C != jobs[0].ctx->C || c->dtype != jobs[0].ctx->dtype ||
            c->net != jobs[0].ctx->net)
            return NQS_E_SPEC;
        for (int j = 0; j < i; ++j)
            if (jobs[j].ctx == c) return NQS_E_ARG;   // one workspace per job
        NQS_TRY(check_common(c, jobs[i].spins, jobs[i].B));
        if (jobs[i].B > 0 && !jobs[i].e_loc) return NQS_E_ARG;
        const nqs_mode m = resolve_mode(c, mode);
        if (m == NQS_INCREMENTAL && !incremental_ok(c))
            return NQS_E_UNSUPPORTED;
    }
    if (n == 0) return NQS_OK;
    hipStream_t s = (hipStream_t)stream;
    if (jobs[0].ctx->dtype != NQS_BF16) {
        // the FP64 / FP32 forms and the block networks run lattice after lattice
        for (int i = 0; i < n; ++i)
            NQS_TRY(nqs_local_energy(jobs[i].ctx, jobs[i].spins, jobs[i].B, jobs[i].e_loc, mode,
                                     stream));
        return NQS_OK;
    }
    // BF16: per lattice the integer stage and the base pass; then the
    // exchanged configurations of every lattice of one mode and kernel
    // family in one persistent launch (kMaxConnJobs lattices at a time);
    // then per lattice the FP64 ratio sums.
    for (int i = 0; i < n; ++i) {
        nqs_ctx *c = jobs[i].ctx;
        c->last_stream = s;
        if (jobs[i].B == 0) continue;
        const int64_t cap = bonds_per_sample(c) * jobs[i].B;
        NQS_TRY(integer_stage(c, jobs[i].spins, (int)jobs[i].B, s));
        NQS_TRY(ensure(c->ws.dlog, sizeof(double) * std::max<int64_t>(cap, 1), s));
        NQS_TRY(bf16_base_stage(c, jobs[i].spins, (int)jobs[i].B, s));
    }
    nqs_ctx *c0 = jobs[0].ctx;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c0->timing) {
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        (void)hipEventRecord(e0, s);
    }
    for (nqs_mode m : {NQS_FULL, NQS_INCREMENTAL}) {
        ConnJob cj[kMaxConnJobs];
        int k = 0;
        for (int i = 0; i <= n; ++i) {
            if (i < n && jobs[i].B > 0 && resolve_mode(jobs[i].ctx, mode) == m) {
                nqs_ctx *c = jobs[i].ctx;
                cj[k++] = ConnJob{c, jobs[i].spins, (const uint32_t *)c->ws.queue.ptr,
                                  (const int64_t *)c->ws.qlen.ptr, bonds_per_sample(c) * jobs[i].B,
                                  (const double *)c->ws.hsum.ptr, c->ws.cache.ptr,
                                  (double *)c->ws.dlog.ptr};
            }
            if (k == kMaxConnJobs || (i == n && k > 0)) {
                mfma_conn_forward_jobs(m, cj, k, s);
                k = 0;
            }
        }
    }
    if (c0->timing) {
        (void)hipEventRecord(e1, s);
        c0->events.push_back({e0, e1});
    }
    for (int i = 0; i < n; ++i) {
        nqs_ctx *c = jobs[i].ctx;
        if (jobs[i].B == 0) continue;
        launch_energy_reduce(c, jobs[i].spins, (int)jobs[i].B, (int64_t *)c->ws.offsets.ptr,
                             (uint32_t *)c->ws.queue.ptr, (double *)c->ws.dlog.ptr, nullptr,
                             (double *)c->ws.ediag.ptr, jobs[i].e_loc, c->err, s);
    }
    return finish_call();
}

namespace {
// ms[0], ms[1]: one whole log-ratio pass (bond stage excluded, base pass
// included) in the FULL and INCREMENTAL forms, each after a warm run
nqs_status time_ratio_forms(nqs_ctx *c, const int8_t *spins, int64_t B, hipStream_t s,
                            double ms[2])
{
    const int64_t cap = bonds_per_sample(c) * B;
    NQS_TRY(integer_stage(c, spins, (int)B, s));
    NQS_TRY(ensure(c->ws.dlog, sizeof(double) * std::max<int64_t>(cap, 1), s));
    double *dl = (double *)c->ws.dlog.ptr;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    ms[0] = ms[1] = 0.0;
    const nqs_mode form[2] = {NQS_FULL, NQS_INCREMENTAL};
    nqs_status st = NQS_OK;
    for (int i = 0; i < 2 && st == NQS_OK; ++i) {
        st = log_ratio_stage(c, spins, (int)B, form[i], dl, cap, s);
        if (st != NQS_OK) break;
        (void)hipEventRecord(e0, s);
        st = log_ratio_stage(c, spins, (int)B, form[i], dl, cap, s);
        (void)hipEventRecord(e1, s);
        if (st != NQS_OK) break;
        (void)hipEventSynchronize(e1);
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e0, e1);
        ms[i] = t;
        st = finish_call();
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}
}  // namespace

nqs_status nqs_autotune(nqs_ctx *c, const int8_t *spins, int64_t B, nqs_mode *mode_out,
                        void *stream)
{
    NQS_TRY(check_common(c, spins, B));
    if (B == 0) return NQS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (stream_capturing(s)) return NQS_E_WORKSPACE;
    c->last_stream = s;
    if (block_net(c)) {
        // CNN1 / CNN2: where the receptive cone serves, the whole log-ratio pass
        // (base pass included: the incremental one also keeps the activations)
        // is timed in both forms; otherwise full recomputation is the only
        // form.  Nothing goes to the tune cache, whose keys do not name the
        // network family.
        nqs_mode best = NQS_FULL;
        if (incremental_ok(c)) {
            double ms[2];
            NQS_TRY(time_ratio_forms(c, spins, B, s, ms));
            best = ms[1] < ms[0] ? NQS_INCREMENTAL : NQS_FULL;
        }
        c->tuned = 1;
        c->tuned_mode = best;
        if (mode_out) *mode_out = best;
        return finish_call();
    }
    if (c->dtype == NQS_FP64 && incremental_ok(c)) {
        // the FP64 ln cosh CNN where its receptive cone serves: the whole
        // log-ratio pass timed in both forms, the choice stored in the cache
        double ms[2];
        NQS_TRY(time_ratio_forms(c, spins, B, s, ms));
        const nqs_mode best = ms[1] < ms[0] ? NQS_INCREMENTAL : NQS_FULL;
        c->tuned = 1;
        c->tuned_mode = best;
        (void)tune_store(tune_cache_path(), tune_key(c), best, 0, 0, -1, -1, ms[0], ms[1]);
        if (mode_out) *mode_out = best;
        return NQS_OK;
    }
    double ms_full = -1.0, ms_inc = -1.0;
    int best_nw = 0, best_mt = 0;
    nqs_mode best = NQS_FULL;
    if (c->dtype == NQS_BF16 || c->dtype == NQS_BF16X3) {
        const int64_t cap = bonds_per_sample(c) * B;
        NQS_TRY(integer_stage(c, spins, (int)B, s));
        NQS_TRY(ensure(c->ws.dlog, sizeof(double) * std::max<int64_t>(cap, 1), s));
        NQS_TRY(bf16_base_stage(c, spins, (int)B, s));
        if (c->dtype == NQS_BF16X3) NQS_TRY(x3_full_reserve(c, x3_chunk(c, cap), s));
        hipEvent_t e0, e1;
        HIP_OK(hipEventCreate(&e0));
        HIP_OK(hipEventCreate(&e1));
        // one exchanged-configuration pass in form m
        auto run = [&](nqs_mode m) {
            if (c->dtype == NQS_BF16X3) {
                (void)x3_conn_stage(c, spins, m, (double *)c->ws.dlog.ptr, cap, s);
                return;
            }
            const ConnJob j{c, spins, (const uint32_t *)c->ws.queue.ptr,
                            (const int64_t *)c->ws.qlen.ptr, cap, (const double *)c->ws.hsum.ptr,
                            c->ws.cache.ptr, (double *)c->ws.dlog.ptr};
            mfma_conn_forward_jobs(m, &j, 1, s);
        };
        // per candidate a warm run, then two timed ones (ms per pass)
        auto time_pass = [&](nqs_mode m, double *ms) -> nqs_status {
            run(m);
            HIP_OK(hipEventRecord(e0, s));
            run(m);
            run(m);
            HIP_OK(hipEventRecord(e1, s));
            HIP_OK(hipEventSynchronize(e1));
            float t = 0.f;
            HIP_OK(hipEventElapsedTime(&t, e0, e1));
            *ms = t / 2.0;
            return finish_call();
        };
        int nw[8] = {0}, mt[8] = {0};
        // the split form's full pass has a single shape
        const int nv = c->dtype == NQS_BF16X3 ? 1 : mfma_full_variants(c, nw, mt, 8);
        const int keep_nw = c->full_nw, keep_mt = c->full_maxt;
        for (int i = 0; i < nv; ++i) {
            c->full_nw = nw[i];
            c->full_maxt = mt[i];
            double ms;
            const nqs_status st = time_pass(NQS_FULL, &ms);
            if (st != NQS_OK) {
                c->full_nw = keep_nw;
                c->full_maxt = keep_mt;
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return st;
            }
            if (ms_full < 0.0 || ms < ms_full) {
                ms_full = ms;
                best_nw = nw[i];
                best_mt = mt[i];
            }
        }
        c->full_nw = best_nw;
        c->full_maxt = best_mt;
        best = NQS_FULL;
        if (incremental_ok(c)) {
            // every shape of the cone kernel where it serves (the lockstep
            // shapes and the one-configuration kernel), else the one form
            const bool cone = cone_supported(c) || cone_x3_supported(c);
            const int nv_cone = cone ? cone_variants(c) : 0;
            const int keep_v = c->cone_variant;
            int best_v = keep_v;
            for (int v = (nv_cone > 0 ? -1 : keep_v); v < std::max(nv_cone, keep_v + 1); ++v) {
                c->cone_variant = v;
                double ms;
                const nqs_status st = time_pass(NQS_INCREMENTAL, &ms);
                if (st != NQS_OK) {
                    c->cone_variant = keep_v;
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    return st;
                }
                if (ms_inc < 0.0 || ms < ms_inc) {
                    ms_inc = ms;
                    best_v = v;
                }
            }
            c->cone_variant = best_v;
            if (ms_inc < ms_full) best = NQS_INCREMENTAL;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    c->tuned = 1;
    c->tuned_mode = best;
    // a cache that cannot be written leaves the choice with this context only
    int ci = -1, cw = -1;
    if (cone_supported(c) || cone_x3_supported(c)) cone_variant_shape(c, c->cone_variant, &ci, &cw);
    (void)tune_store(tune_cache_path(), tune_key(c), best, best_nw, best_mt, ci, cw, ms_full,
                     ms_inc);
    if (mode_out) *mode_out = best;
    return NQS_OK;
}

nqs_status nqs_get_error(nqs_ctx *c, nqs_status *sticky)
{
    if (!c || !sticky) return NQS_E_ARG;
    HIP_OK(hipStreamSynchronize(c->last_stream));
    int32_t v = 0;
    HIP_OK(hipMemcpy(&v, c->err, sizeof(int32_t), hipMemcpyDeviceToHost));
    HIP_OK(hipMemset(c->err, 0, sizeof(int32_t)));
    *sticky = (v & kErrSpin) ? NQS_E_SPIN : ((v & kErrNonFinite) ? NQS_E_NONFINITE : NQS_OK);
    return NQS_OK;
}

nqs_status nqs_enable_timing(nqs_ctx *c, int32_t enable)
{
    if (!c) return NQS_E_ARG;
    c->timing = enable ? 1 : 0;
    return NQS_OK;
}

nqs_status nqs_kernel_time(nqs_ctx *c, double *ms, int64_t *launches)
{
    if (!c || !ms || !launches) return NQS_E_ARG;
    double total = 0.0;
    for (auto &e : c->events) {
        HIP_OK(hipEventSynchronize(e.second));
        float t = 0.f;
        HIP_OK(hipEventElapsedTime(&t, e.first, e.second));
        total += t;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    *ms = total;
    *launches = (int64_t)c->events.size();
    c->events.clear();
    return NQS_OK;
}

}  // extern "C"
