// sr_noalloc.hip -- the stochastic-reconfiguration solve for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid hipMalloc): the same kernels as nqs_sr_solve,
// with their workspace in a fixed array of device memory instead of the
// context's growable buffer.
//
// The array lives for the life of the process on every device the library
// runs on (each device has its own copy at its own address).  Host code never
// passes the array's name to a kernel: it looks up the device address once per
// device and passes that.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "nqs_internal.h"

// 48 MiB: the SR workspace of P = 65,056 parameters with B = 4096 samples
// (five FP64 P-vectors, 64 partial column sums and the per-sample vectors)
// takes 36 MB.
constexpr size_t kScratchBytes = (size_t)48 << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up on the first
// call on the device, with that device current).
nqs_status scratch_ptr(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return NQS_E_HIP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return NQS_E_HIP;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return NQS_OK;
}

}  // namespace

extern "C" {

nqs_status nqs_sr_solve_noalloc(nqs_ctx *c, const void *O, nqs_dtype odt, const double *e_loc,
                                int64_t B, double diag_shift, int32_t n_iter, double *dtheta,
                                double *stats, void *stream)
{
    if (!c || !O || !e_loc || !dtheta || B <= 0 || n_iter < 0) return NQS_E_ARG;
    if (odt != NQS_FP32 && odt != NQS_FP64) return NQS_E_ARG;
    if (!(diag_shift >= 0.0) || !std::isfinite(diag_shift)) return NQS_E_ARG;
    if (nqs::sr_workspace_bytes(B, c->P) > kScratchBytes) return NQS_E_WORKSPACE;
    void *w = nullptr;
    const nqs_status st = scratch_ptr(&w);
    if (st != NQS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    nqs::launch_sr_solve(O, odt, e_loc, B, c->P, diag_shift, n_iter, dtheta, stats, w, s);
    const char *what = nullptr;
    const hipError_t e = nqs::take_launch_error(&what);
    (void)hipGetLastError();
    return e == hipSuccess ? NQS_OK : NQS_E_HIP;
}

}  // extern "C"
