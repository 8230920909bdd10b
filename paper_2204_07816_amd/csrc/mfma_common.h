// mfma_common.h -- pieces shared by the BF16 matrix-core network kernels.
// The base pass (a sample's own network, whose activations are cached) and
// the exchanged-configuration passes must run bit-identical arithmetic on
// identical inputs, so that a site the exchange does not reach contributes
// exactly zero to f(S') - f(s).  Everything that produces a value — ln cosh,
// the layer-1 FMA order, the MFMA K-step order, the channel permutation — is
// defined once, here.
#pragma once

#include "nqs_internal.h"

namespace nqs {
namespace mf {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

// ln cosh z in FP32.  |z| < 0.5: ln cosh z = s P(s), s = z^2, with P the
// degree-2 minimax fit (relative error) of ln cosh(sqrt s)/s on [0, 0.25]:
// 5.9e-6 relative, 3e-3 of a BF16 rounding step, with no cancellation near 0.
// |z| >= 0.5: ln cosh z = |z| - ln 2 + ln 2 * log2(1 + 2^(-2|z| log2 e)) on the
// hardware exp2 / log2 units (the result is >= 0.12 there, so the absolute
// error of the logarithm stays ~1e-6 relative).
__device__ __forceinline__ float ln_cosh_small(float a)
{
    const float s = a * a;
    float p = __builtin_fmaf(0.019911346957087517f, s, -0.08312316238880157f);
    p = __builtin_fmaf(p, s, 0.4999971091747284f);
    return s * p;
}

__device__ __forceinline__ float ln_cosh_large(float a)
{
    const float t = __builtin_amdgcn_exp2f(-2.8853900817779268f * a);
    return __builtin_fmaf(0.69314718055994531f, __builtin_amdgcn_logf(1.0f + t),
                          a - 0.69314718055994531f);
}

__device__ __forceinline__ float ln_cosh(float z)
{
    const float a = fabsf(z);
    float h = ln_cosh_small(a);
    if (a >= 0.5f) h = ln_cosh_large(a);
    return h;
}

// ln cosh of n values with a single wave-uniform test for the large branch;
// every element gets exactly the value ln_cosh() gives it.
template <int n>
__device__ __forceinline__ void ln_cosh_n(const float *z, float *h)
{
    float amax = 0.0f;
#pragma unroll
    for (int i = 0; i < n; ++i) {
        const float a = fabsf(z[i]);
        h[i] = ln_cosh_small(a);
        amax = fmaxf(amax, a);
    }
    if (__any(amax >= 0.5f)) {
        // keeps the compiler from if-converting (always executing) this branch
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < n; ++i) {
            const float a = fabsf(z[i]);
            const float big = ln_cosh_large(a);
            h[i] = (a >= 0.5f) ? big : h[i];
        }
    }
}

// ln cosh z in FP32 for the split (BF16X3) form, whose operands carry 16
// significant bits: |z| < 0.5: s P(s), s = z^2, with P the degree-4 fit of
// ln cosh(sqrt s)/s on [0, 0.25] (relative error 2.2e-9, 9e-8 once evaluated
// in FP32); |z| >= 0.5: |z| - ln 2 + log1p(t), t = e^{-2|z|}, from the
// hardware base-2 exponential and logarithm (no cancellation: the result is
// >= 0.12 there).  The exponent -2|z| log2 e is carried as hi + lo (hi
// rounded; lo its FMA residual plus the constant's tail) and lo enters as
// t = 2^hi (1 + lo ln 2); log1p(t) = ln u + (t - (u - 1)) with u = 1 + t
// rounded (the bracket is u's rounding error, exact; dropping its 1/u factor
// costs < 2e-8); ln 2 is subtracted as hi + lo.  With both hardware functions
// within 1 ulp the relative error stays below 6.4e-7 (3.6e-7 when they round
// correctly), against 7e-7 for the library's FP32 exp and log1p, at about a
// third of their instructions.
// Contraction is off in these helpers: the base pass and the cone kernel must
// round every intermediate identically, whatever code the inlined result
// lands next to (a fused s * p - hi would change the lo part).
__device__ __forceinline__ float ln_cosh_x3_small(float a)
{
#pragma clang fp contract(off)
    const float s = a * a;
    float p = __builtin_fmaf(0.0017842349592950431f, s, -0.006661991475716793f);
    p = __builtin_fmaf(p, s, 0.02221489379770223f);
    p = __builtin_fmaf(p, s, -0.08333310755059982f);
    p = __builtin_fmaf(p, s, 0.49999999888185015f);
    return s * p;
}

__device__ __forceinline__ float ln_cosh_x3_large(float a)
{
#pragma clang fp contract(off)
    constexpr float kE1 = -2.8853900817779268f;       // -2 log2 e, rounded
    constexpr float kE2 = -3.8519260670e-08f;         // its tail
    constexpr float kLn2Hi = 0.69314718055994531f;
    constexpr float kLn2Lo = -1.9046542121e-09f;
    const float xh = a * kE1;
    const float xl = __builtin_fmaf(a, kE1, -xh) + a * kE2;
    const float e = __builtin_amdgcn_exp2f(xh);
    const float t = __builtin_fmaf(e, xl * kLn2Hi, e);
    const float u = 1.0f + t;
    const float lg = __builtin_fmaf(__builtin_amdgcn_logf(u), kLn2Hi, t - (u - 1.0f));
    return ((a - kLn2Hi) - kLn2Lo) + lg;
}

// ln cosh of n values (split form) with a single wave-uniform test for the
// large branch; every element gets the value ln_cosh_x3_small / _large gives.
template <int n>
__device__ __forceinline__ void ln_cosh_x3_n(const float *z, float *h)
{
    float amax = 0.0f;
#pragma unroll
    for (int i = 0; i < n; ++i) {
        const float a = fabsf(z[i]);
        h[i] = ln_cosh_x3_small(a);
        amax = fmaxf(amax, a);
    }
    if (__any(amax >= 0.5f)) {
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < n; ++i) {
            const float a = fabsf(z[i]);
            const float big = ln_cosh_x3_large(a);
            h[i] = (a >= 0.5f) ? big : h[i];
        }
    }
}

__device__ __forceinline__ float ln_cosh_x3(float z)
{
    const float a = fabsf(z);
    return a < 0.5f ? ln_cosh_x3_small(a) : ln_cosh_x3_large(a);
}

// Split of an FP32 value into BF16 hi + lo (both rounded to nearest even):
// x - hi is exact in FP32, so |x - hi - lo| <= 2^-8 |x - hi| <= 2^-16 |x|.
__device__ __forceinline__ void split_bf16(float x, uint16_t *hi, uint16_t *lo)
{
#pragma clang fp contract(off)
    const __bf16 h = (__bf16)x;
    *hi = __builtin_bit_cast(uint16_t, h);
    *lo = __builtin_bit_cast(uint16_t, (__bf16)(x - (float)h));
}

// Channel permutation: physical slot q of a site holds logical channel
// chan_of_slot(q).  MFMA lane group g (lanes 16g..16g+15) owns the slots of
// chunk g, so its outputs are contiguous.
template <int C>
__device__ __host__ __forceinline__ int chan_of_slot(int q)
{
    if (C == 32) {
        const int g = q >> 3, r = q & 7;
        return r < 4 ? 4 * g + r : 16 + 4 * g + (r - 4);
    }
    return q;
}

template <int C>
struct Shape {
    static constexpr int NH = C / 16;              // 16-channel output halves
    static constexpr int KS = (C == 32) ? 9 : 5;   // K-steps of 32 reduction elements
    static constexpr int CG = C / 4;               // channels per lane group
    static constexpr int PSB = C * 2;              // bytes per site (BF16)
    static constexpr int CHUNKS = PSB / 16;        // 16-byte chunks per site
};

// Tap and 16-byte chunk read by lane group g at K-step j.
template <int C>
__device__ __forceinline__ void kstep_tap(int j, int g, int *tap, int *chunk)
{
    if (C == 32) {
        *tap = j;
        *chunk = g;
    } else {
        int t = 2 * j + (g >> 1);
        *tap = t > 8 ? 8 : t;      // padding step: its weights are zero
        *chunk = g & 1;
    }
}

// Layer-1 pre-activation of logical channel co from the 9 spins of a site's
// 3x3 neighbourhood, in a fixed FMA order.
__device__ __forceinline__ float layer1_z(const float *w1, const float *b1, int C, int co,
                                          const float sv[9])
{
    float z = b1[co];
#pragma unroll
    for (int t = 0; t < 9; ++t) z = __builtin_fmaf(w1[t * C + co], sv[t], z);
    return z;
}

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

}  // namespace mf
}  // namespace nqs
