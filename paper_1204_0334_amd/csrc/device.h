// Device helpers shared by the single-code decoders (decode.hip) and the
// multi-code plan (plan.hip): frame loads and stores, the FP32 check-node
// arithmetic, and the QC indexers that turn circulant shifts into package
// addresses.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace ldpc {

constexpr float kClip = 30.0f;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = 64 * kWavesPerBlock;

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

template <int FPL>
__device__ __forceinline__ void load_frames(const float* __restrict__ p, float (&v)[FPL]) {
    if constexpr (FPL == 4) {
        float4 x = *reinterpret_cast<const float4*>(p);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else if constexpr (FPL == 2) {
        float2 x = *reinterpret_cast<const float2*>(p);
        v[0] = x.x; v[1] = x.y;
    } else {
        v[0] = *p;
    }
}

template <int FPL>
__device__ __forceinline__ void store_frames(float* __restrict__ p, const float (&v)[FPL]) {
    if constexpr (FPL == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    } else if constexpr (FPL == 2) {
        *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
    } else {
        *p = v[0];
    }
}

__device__ __forceinline__ int wave_in_block() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

__device__ __forceinline__ float clip30(float x) { return __builtin_amdgcn_fmed3f(x, -kClip, kClip); }

// valid-frame mask of word f (bit b <-> frame FPL*b + f of the tile)
template <int FPL>
__device__ __forceinline__ uint64_t valid_word(int nvalid, int f) {
    int cnt = nvalid - f;
    if (cnt <= 0) return 0;
    cnt = (cnt + FPL - 1) / FPL;
    return cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull);
}

// Horizontal step for one frame over DC inputs given as (t, q) pairs with
// identity pairs (1, 0) in unused slots.  Writes |alpha_k| for every slot.
template <int DC>
__device__ __forceinline__ void boxplus_fb(const float (&t)[DC], const float (&q)[DC], float (&mag)[DC]) {
    float sP[DC], sQ[DC];
    float P = 1.0f, Q = 0.0f;
#pragma unroll
    for (int k = DC - 1; k >= 0; --k) {
        sP[k] = P;
        sQ[k] = Q;
        Q = fmaf(Q, t[k], q[k]);
        P = P * t[k];
    }
    P = 1.0f;
    Q = 0.0f;
#pragma unroll
    for (int k = 0; k < DC; ++k) {
        const float eP = P * sP[k];
        const float eQ = fmaf(sQ[k], P, Q);
        mag[k] = kLn2 * __builtin_amdgcn_logf((1.0f + eP) * __builtin_amdgcn_rcpf(eQ));
        Q = fmaf(q[k], P, Q);
        P = P * t[k];
    }
}

// (t, q) = (tanh(x/2), 1 - tanh(x/2)) for x = min(|b|, 30)
__device__ __forceinline__ void tq_of(float b, float& t, float& q) {
    const float x = fminf(fabsf(b), kClip);
    const float e = __builtin_amdgcn_exp2f(-x * kLog2e);
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    t = (1.0f - e) * r;
    q = (e + e) * r;
}

// Horizontal step (Eq. 3) for the FPL frames of a lane: in[k] holds beta of
// edge k for k < d (other slots are ignored); out[k] = alpha_k for k < d.
template <int DCMAX, int FPL>
__device__ __forceinline__ void sp_check(const float (&in)[DCMAX][FPL], int d, float (&out)[DCMAX][FPL]) {
    float t[FPL][DCMAX], q[FPL][DCMAX];
    uint32_t sgn[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) sgn[f] = 0;
#pragma unroll
    for (int k = 0; k < DCMAX; ++k) {
        const bool ok = k < d;
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            if (ok) {
                tq_of(in[k][f], t[f][k], q[f][k]);
                sgn[f] ^= __float_as_uint(in[k][f]) & 0x80000000u;
            } else {
                t[f][k] = 1.0f;
                q[f][k] = 0.0f;
            }
        }
    }
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        float mag[DCMAX];
        boxplus_fb<DCMAX>(t[f], q[f], mag);
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            const uint32_t sg = sgn[f] ^ (__float_as_uint(in[k][f]) & 0x80000000u);
            out[k][f] = __uint_as_float(__float_as_uint(mag[k]) | sg);
        }
    }
}

// Vertical step (Eq. 4, 5) for the FPL frames of a lane: a[k] = alpha of
// edge k (0 in unused slots); b[k] = clip(mu + sum of the other alphas) by
// prefix and suffix sums; L = mu + sum of all alphas.
template <int DVMAX, int FPL>
__device__ __forceinline__ void sp_variable(const float (&mu)[FPL], const float (&a)[DVMAX][FPL],
                                            float (&b)[DVMAX][FPL], float (&L)[FPL]) {
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        float suf[DVMAX];
        float S = 0.0f;
#pragma unroll
        for (int k = DVMAX - 1; k >= 0; --k) {
            suf[k] = S;
            S += a[k][f];
        }
        float pre = 0.0f;
#pragma unroll
        for (int k = 0; k < DVMAX; ++k) {
            b[k][f] = clip30(mu[f] + (pre + suf[k]));
            pre += a[k][f];
        }
        L[f] = mu[f] + pre;
    }
}

// ---------------------------------------------------------------------------
// indexers: which packages a check row / a variable touches
// ---------------------------------------------------------------------------

// Block code.  Row (j, s) = row j*p + s; edge k of the row is edge block
// b = rstart[j] + k (base columns ascending), package b*p + s, variable
// ecol[b]*p + (s + a) mod p.
struct QCRow {
    int b0, d, s, j;
    __device__ __forceinline__ QCRow(const QCDesc& D, int row) {
        j = row / D.p;
        s = row - j * D.p;
        b0 = D.rstart[j];
        d = D.rstart[j + 1] - b0;
    }
    __device__ __forceinline__ bool valid(const QCDesc&, int k) const { return k < d; }
    __device__ __forceinline__ int64_t pkg(const QCDesc& D, int k) const { return (int64_t)(b0 + k) * D.p + s; }
    __device__ __forceinline__ int var(const QCDesc& D, int k) const {
        const int b = b0 + k;
        int t = s + D.eshift[b];
        if (t >= D.p) t -= D.p;
        return D.ecol[b] * D.p + t;
    }
    __device__ __forceinline__ bool writable(int) const { return true; }
};

// Variable (l, t) = column l*p + t; edge k is edge block b = cedge[cstart[l] + k]
// (base rows ascending), package b*p + (t - a) mod p.
struct QCCol {
    int c0, d, t, v;
    __device__ __forceinline__ QCCol(const QCDesc& D, int col) {
        const int l = col / D.p;
        t = col - l * D.p;
        c0 = D.cstart[l];
        d = D.cstart[l + 1] - c0;
        v = col;
    }
    __device__ __forceinline__ bool valid(const QCDesc&, int k) const { return k < d; }
    __device__ __forceinline__ bool contributes(const QCDesc&, int) const { return true; }
    __device__ __forceinline__ int64_t pkg(const QCDesc& D, int k) const {
        const int b = D.cedge[c0 + k];
        int s = t - D.eshift[b];
        if (s < 0) s += D.p;
        return (int64_t)b * D.p + s;
    }
};

}  // namespace ldpc
