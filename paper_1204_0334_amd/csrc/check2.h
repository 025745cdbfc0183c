// Check-node update (Algorithm 1, Eq. 3) with messages in base-2 units, for
// the decoders whose time goes into this arithmetic rather than into memory
// traffic: the on-chip block decoder (onchip.hip) and the convolutional-code
// decoders (decode.hip).  A message x here is the LLR times log2(e), so
// tanh(|L|/2) = (1 - 2^-|x|) / (1 + 2^-|x|) and the output magnitude
// 2 atanh(P) = ln((1 + P) / (1 - P)) becomes log2((1 + P) / (1 - P)): the
// hardware's 2^x and log2 apply without a scaling multiply on either side.
// The decoders scale the channel LLRs once when they read them and the
// posteriors back when they write them; the clip at 30 becomes a clip at
// 30 log2(e).  The arithmetic is that of sp_check (device.h) otherwise:
// inputs as (t, q) = (tanh(|x|/2), 1 - tanh(|x|/2)) pairs, exclusive products
// from a forward-backward sweep over pairs combined as
// (t_a t_b, q_a + t_a q_b), |alpha| = log2((1 + P) / Q).
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

namespace ldpc {

constexpr float kClip2 = 43.2808512266689f;   // 30 * log2(e)
constexpr float kLog2eF = 1.4426950408889634f;
constexpr float kLn2F = 0.6931471805599453f;

__device__ __forceinline__ float clip2(float x) { return __builtin_amdgcn_fmed3f(x, -kClip2, kClip2); }

// (t, q) of an input with |x| <= 30 log2 e: e = 2^-|x|, q = 2e / (1 + e),
// t = 1 - q (t + q = 1 exactly in real arithmetic; computing t from q costs
// no more accuracy than (1 - e) / (1 + e), whose 1 - e cancels the same way)
__device__ __forceinline__ void tq2_of(float x, float& t, float& q) {
    const float e = __builtin_amdgcn_exp2f(-fabsf(x));
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    q = 2.0f * (e * r);
    t = 1.0f - q;
}

// |alpha_k| for every slot from the pairs (identity pairs (1, 0) in unused
// slots); the first and last steps of each sweep are written out, so no
// product with the identity pair is formed.
template <int DC>
__device__ __forceinline__ void boxplus2_fb(const float (&t)[DC], const float (&q)[DC], float (&mag)[DC]) {
    static_assert(DC >= 2, "rows carry at least two slots");
    // suffix pairs over slots k+1 .. DC-1 (slot DC-1: the identity)
    float sP[DC], sQ[DC];
    sP[DC - 1] = 1.0f;
    sQ[DC - 1] = 0.0f;
    sP[DC - 2] = t[DC - 1];
    sQ[DC - 2] = q[DC - 1];
#pragma unroll
    for (int k = DC - 3; k >= 0; --k) {
        sP[k] = sP[k + 1] * t[k + 1];
        sQ[k] = fmaf(sQ[k + 1], t[k + 1], q[k + 1]);
    }
    // prefix pair over slots 0 .. k-1, combined with the suffix
    float P = t[0], Q = q[0];
    float eP[DC], eQ[DC];
    eP[0] = sP[0];
    eQ[0] = sQ[0];
#pragma unroll
    for (int k = 1; k < DC; ++k) {
        if (k == DC - 1) {
            eP[k] = P;
            eQ[k] = Q;
        } else {
            eP[k] = P * sP[k];
            eQ[k] = fmaf(sQ[k], P, Q);
            Q = fmaf(q[k], P, Q);
            P = P * t[k];
        }
    }
#pragma unroll
    for (int k = 0; k < DC; ++k) mag[k] = __builtin_amdgcn_logf((1.0f + eP[k]) * __builtin_amdgcn_rcpf(eQ[k]));
}

// One row: in[k] = beta of slot k for k < d (|beta| <= 30 log2 e; slots k >= d
// are ignored); out[k] = alpha of slot k for k < d.
template <int DC>
__device__ __forceinline__ void check2_row(const float (&in)[DC], int d, float (&out)[DC]) {
    float t[DC], q[DC];
    uint32_t sgn = 0;
#pragma unroll
    for (int k = 0; k < DC; ++k) {
        if (k < d) {
            tq2_of(in[k], t[k], q[k]);
            sgn ^= __float_as_uint(in[k]);
        } else {
            t[k] = 1.0f;
            q[k] = 0.0f;
        }
    }
    float mag[DC];
    boxplus2_fb<DC>(t, q, mag);
#pragma unroll
    for (int k = 0; k < DC; ++k)
        out[k] = __uint_as_float(__float_as_uint(mag[k]) | ((sgn ^ __float_as_uint(in[k])) & 0x80000000u));
}

}  // namespace ldpc
