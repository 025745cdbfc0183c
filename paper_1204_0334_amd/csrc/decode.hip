// Batched flooding sum-product decoder for gfx950 (MI355X).
//
// Data layout.  Gamma frames are split into tiles of Gt = 64 * FPL frames
// (FPL = frames per lane: 1, 2 or 4).  Every edge of the Tanner graph owns a
// message package of Gt FP32 values, one per frame of the tile, and the
// packages of a tile are stored contiguously: msg[tile][package][Gt].  A
// wavefront processes one check row (or one variable) for the 64 * FPL frames
// of a tile, lane i holding frames FPL*i .. FPL*i+FPL-1, so every package
// access is one contiguous 256*FPL-byte segment (dwordx4 per lane at FPL=4).
// This is the paper's "message package" idea (Sec. IV-A) sized for 64-wide
// wavefronts.  As in the paper, one array holds alpha after the check-node
// pass and beta after the variable-node pass (each package is written by the
// one row and the one column it belongs to, so the in-place update is race
// free).  Package numbering follows the circulant blocks rather than the rows
// of H, and per-edge addresses are computed from the circulant shifts
// (Eq. 2) instead of being read from LUT_c / LUT_v tables.
//
// Check-node update (Algorithm 1, Eq. 3).  alpha_k = 2 atanh(prod_{k' != k}
// tanh(beta_k' / 2)).  Each input is carried as the pair (t, q) with
// t = tanh(|beta|/2) and q = 1 - t, both computed without cancellation from
// e = exp(-|beta|): t = (1 - e)/(1 + e), q = 2e/(1 + e).  Two pairs combine
// as (t_a t_b, q_a + q_b t_a), which is the product of the t's and, exactly,
// one minus it, again without cancellation.  The products over "all inputs
// but k" are formed by a forward-backward sweep (prefix and suffix, no
// division), as the paper does, and |alpha_k| = ln((1 + P)/Q).  Signs are
// handled separately (XOR of sign bits).  This keeps FP32 accurate where the
// literal tanh product saturates at 1.
//
// Variable-node update (Eq. 4, 5).  beta_k = clip(mu + sum_{k' != k} alpha_k')
// by prefix/suffix sums (never L - alpha_k), L = mu + sum alpha; hard decision
// c = (L < 0) (Eq. 6) packed by wave ballots into 64-bit words.
//
// Early stopping (an addition to the paper, which always runs I_max
// iterations): the check-node pass of iteration i+1 also computes the
// syndrome of iteration i's packed decisions; unsatisfied frames are OR-ed
// into a per-iteration flag word; the variable-node pass of iteration i+1
// freezes frames whose syndrome became zero (their posterior and decisions
// are no longer written) and tiles whose frames are all frozen are skipped.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <vector>

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

// ---------------------------------------------------------------------------
// indexers: which packages a check row / a variable touches
// ---------------------------------------------------------------------------

// Block code.  Row (j, s) = row j*p + s; edge k of the row is edge block
// b = rstart[j] + k (base columns ascending), package b*p + s, variable
// ecol[b]*p + (s + a) mod p.
struct QCRow {
    int b0, d, s;
    __device__ __forceinline__ QCRow(const QCDesc& D, int row) {
        const int j = row / D.p;
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

// Window state of the convolutional decoder for one launch.
struct WinState {
    int s;        // target position
    int lay_lo;   // first window layer (== s)
    int lay_hi;   // last window layer
    int R;        // ring slots
    int eps;      // edge packages per ring slot = (ms+1)*Jb*Lb*p
};

__device__ __forceinline__ int sf_at(const ConvDesc& D, int cls, int dd, int rr, int q) {
    return D.sf[((cls * (D.ms + 1) + dd) * D.Jb + rr) * D.Lb + q];
}

// Window check row r: layer tau = lay_lo + r / (Jb p), circulant row rr,
// offset s.  Edge k <-> (lag dd = ms - k / Lb, circulant column q = k % Lb):
// position tau - dd, oldest position first.  Only edges of active positions
// (>= s) receive alpha; edges of frozen positions keep their beta.
struct ConvRow {
    int tau, rr, s, cls;
    __device__ __forceinline__ ConvRow(const ConvDesc& D, const WinState& W, int r) {
        const int per = D.Jb * D.p;
        const int l = r / per;
        const int rem = r - l * per;
        tau = W.lay_lo + l;
        rr = rem / D.p;
        s = rem - rr * D.p;
        cls = tau % D.T;
    }
    __device__ __forceinline__ bool valid(const ConvDesc& D, int k) const {
        if (k >= (D.ms + 1) * D.Lb) return false;
        const int dd = D.ms - k / D.Lb, q = k % D.Lb;
        const int t = tau - dd;
        if (t < 0 || t >= D.positions) return false;
        return sf_at(D, cls, dd, rr, q) >= 0;
    }
    __device__ __forceinline__ int64_t pkg(const ConvDesc& D, const WinState& W, int k) const {
        const int dd = D.ms - k / D.Lb, q = k % D.Lb;
        const int slot = (tau - dd) % W.R;
        return (int64_t)slot * W.eps + ((int64_t)((dd * D.Jb + rr) * D.Lb + q)) * D.p + s;
    }
    __device__ __forceinline__ bool writable(const ConvDesc& D, const WinState& W, int k) const {
        return tau - (D.ms - k / D.Lb) >= W.s;
    }
};

// Window variable r: position t = s + r / c, circulant column q, offset u.
// Edge k <-> (lag dd = k / Jb, circulant row rr = k % Jb): layer t + dd.
struct ConvCol {
    int t, q, u, jc;
    __device__ __forceinline__ ConvCol(const ConvDesc& D, const WinState& W, int r) {
        const int pos = r / D.c;
        const int rem = r - pos * D.c;
        t = W.s + pos;
        q = rem / D.p;
        u = rem - q * D.p;
        jc = t % D.T;
    }
    __device__ __forceinline__ int shift(const ConvDesc& D, int k) const {
        const int dd = k / D.Jb, rr = k % D.Jb;
        return sf_at(D, (jc + dd) % D.T, dd, rr, q);
    }
    __device__ __forceinline__ bool valid(const ConvDesc& D, int k) const {
        if (k >= (D.ms + 1) * D.Jb) return false;
        if (t + k / D.Jb >= D.layers) return false;
        return shift(D, k) >= 0;
    }
    __device__ __forceinline__ bool contributes(const WinState& W, const ConvDesc& D, int k) const {
        return t + k / D.Jb <= W.lay_hi;
    }
    __device__ __forceinline__ int64_t pkg(const ConvDesc& D, const WinState& W, int k) const {
        const int dd = k / D.Jb, rr = k % D.Jb;
        int s = u - shift(D, k);
        if (s < 0) s += D.p;
        const int slot = t % W.R;
        return (int64_t)slot * W.eps + ((int64_t)((dd * D.Jb + rr) * D.Lb + q)) * D.p + s;
    }
    __device__ __forceinline__ int64_t mu_index(const ConvDesc& D, const WinState& W) const {
        return (int64_t)(t % W.R) * D.c + q * D.p + u;
    }
};

// ---------------------------------------------------------------------------
// kernels: block code
// ---------------------------------------------------------------------------

struct BlockParams {
    float* msg;              // [tiles][E][Gt]
    const float* mu;         // [tiles][n][Gt]
    uint64_t* bits;          // [tiles][n][FPL] packed decisions
    uint64_t* unsat;         // [max_iters+1][tiles][FPL]
    uint64_t* frozen;        // [max_iters+1][tiles][FPL]
    int gamma, tiles, iter, last, early;
};

// Check-node pass of iteration P.iter.  With early stopping, also ORs the
// syndrome of iteration iter-1's decisions into unsat[iter-1] and skips tiles
// whose frames were all frozen by iteration iter-2.
template <int DCMAX, int FPL>
__global__ void __launch_bounds__(kBlock) cn_block_kernel(const QCDesc D, const BlockParams P) {
    constexpr int Gt = 64 * FPL;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / D.m;
    const int row = wave - tile * D.m;
    if (tile >= P.tiles) return;
    const int nvalid = min(P.gamma - tile * Gt, Gt);

    if (P.early && P.iter >= 3) {
        const uint64_t* fz = P.frozen + ((size_t)(P.iter - 2) * P.tiles + tile) * FPL;
        bool all = true;
#pragma unroll
        for (int f = 0; f < FPL; ++f) all = all && (fz[f] == ~0ull);
        if (all) return;
    }
    const QCRow R(D, row);

    if (P.early && P.iter >= 2) {
        // syndrome of the previous iteration's decisions for this row
        uint64_t par[FPL];
#pragma unroll
        for (int f = 0; f < FPL; ++f) par[f] = 0;
        const uint64_t* bt = P.bits + (size_t)tile * D.n * FPL;
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            if (!R.valid(D, k)) continue;
            const uint64_t* w = bt + (size_t)R.var(D, k) * FPL;
#pragma unroll
            for (int f = 0; f < FPL; ++f) par[f] ^= w[f];
        }
        uint64_t* un = P.unsat + ((size_t)(P.iter - 1) * P.tiles + tile) * FPL;
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            const uint64_t bad = par[f] & valid_word<FPL>(nvalid, f);
            if (bad && lane == f) {
                // a stale read can only miss bits (the word only gains bits
                // during this pass), which costs a redundant atomic, never a
                // missed one
                if ((__atomic_load_n(un + f, __ATOMIC_RELAXED) & bad) != bad)
                    atomicOr((unsigned long long*)(un + f), (unsigned long long)bad);
            }
        }
    }

    // gather the row's messages (iteration 1 reads the channel LLRs)
    const size_t lane_off = (size_t)lane * FPL;
    float t[FPL][DCMAX], q[FPL][DCMAX];
    uint32_t sgn[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) sgn[f] = 0;
    float* mt = P.msg + (size_t)tile * D.E * Gt + lane_off;
    const float* ut = P.mu + (size_t)tile * D.n * Gt + lane_off;
    float in[DCMAX][FPL];
#pragma unroll
    for (int k = 0; k < DCMAX; ++k) {
        if (R.valid(D, k)) {
            const float* src = (P.iter == 1) ? ut + (size_t)R.var(D, k) * Gt : mt + (size_t)R.pkg(D, k) * Gt;
            load_frames<FPL>(src, in[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) in[k][f] = 0.0f;
        }
    }
#pragma unroll
    for (int k = 0; k < DCMAX; ++k) {
        const bool ok = R.valid(D, k);
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
    float outv[DCMAX][FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        float mag[DCMAX];
        boxplus_fb<DCMAX>(t[f], q[f], mag);
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            const uint32_t s = sgn[f] ^ (__float_as_uint(in[k][f]) & 0x80000000u);
            outv[k][f] = __uint_as_float(__float_as_uint(mag[k]) | s);
        }
    }
#pragma unroll
    for (int k = 0; k < DCMAX; ++k)
        if (R.valid(D, k)) store_frames<FPL>(mt + (size_t)R.pkg(D, k) * Gt, outv[k]);
}

// Frames of a tile frozen before iteration P.iter (bit set = frozen; padding
// frames count as frozen).  Frozen as of iteration i-1 = frozen as of i-2, or
// the syndrome of iteration i-1 was zero.
template <int FPL>
__device__ __forceinline__ void frozen_words(const BlockParams& P, int tile, int nvalid, uint64_t (&frz)[FPL],
                                             bool& any, bool& all) {
    any = false;
    all = true;
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        uint64_t z = ~valid_word<FPL>(nvalid, f);
        if (P.early && P.iter >= 2) {
            const size_t prev = ((size_t)(P.iter - 2) * P.tiles + tile) * FPL + f;
            const size_t un = ((size_t)(P.iter - 1) * P.tiles + tile) * FPL + f;
            z |= P.frozen[prev] | ~P.unsat[un];
        }
        frz[f] = z;
        any = any || (z & valid_word<FPL>(nvalid, f)) != 0;
        all = all && (z == ~0ull);
    }
}

// One variable (column col of tile) for the 64*FPL frames of the wave: reads
// mu and the d_v incoming alphas, writes the outgoing betas (not after the
// last iteration: nobody reads them), returns the posterior L, and with early
// stopping or at the last iteration stores the packed decisions (frozen frames
// keep their bits).
template <int DVMAX, int FPL>
__device__ __forceinline__ void vn_column(const QCDesc& D, const BlockParams& P, int tile, int col, int lane,
                                          bool any, const uint64_t (&frz)[FPL], float (&L)[FPL]) {
    constexpr int Gt = 64 * FPL;
    const QCCol C(D, col);
    const size_t lane_off = (size_t)lane * FPL;
    float* mt = P.msg + (size_t)tile * D.E * Gt + lane_off;
    float mu[FPL];
    load_frames<FPL>(P.mu + ((size_t)tile * D.n + C.v) * Gt + lane_off, mu);
    float a[DVMAX][FPL];
#pragma unroll
    for (int k = 0; k < DVMAX; ++k) {
        if (C.valid(D, k)) {
            load_frames<FPL>(mt + (size_t)C.pkg(D, k) * Gt, a[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) a[k][f] = 0.0f;
        }
    }
    float b[DVMAX][FPL];
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
    if (!P.last) {
#pragma unroll
        for (int k = 0; k < DVMAX; ++k)
            if (C.valid(D, k)) store_frames<FPL>(mt + (size_t)C.pkg(D, k) * Gt, b[k]);
    }
    if (P.early || P.last) {
        // decisions, packed: word f, bit i <-> frame FPL*i + f
        uint64_t* bw = P.bits + ((size_t)tile * D.n + C.v) * FPL;
        uint64_t mine = 0;
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            uint64_t w = __ballot(L[f] < 0.0f);
            if (any) w = (w & ~frz[f]) | (bw[f] & frz[f]);
            if (lane == f) mine = w;
        }
        if (lane < FPL) bw[lane] = mine;
    }
}

template <int FPL>
__device__ __forceinline__ uint64_t pick_word(const uint64_t (&a)[FPL], int i);

template <int FPL>
__device__ __forceinline__ void publish_frozen(const BlockParams& P, int tile, int lane, const uint64_t (&frz)[FPL]) {
    if (lane < FPL) P.frozen[((size_t)(P.iter - 1) * P.tiles + tile) * FPL + lane] = pick_word<FPL>(frz, lane);
}

// a[i] for a register array, blended with masks: a select chain or a
// dynamic index gets turned into a private-memory array by the compiler
template <int FPL>
__device__ __forceinline__ uint64_t pick_word(const uint64_t (&a)[FPL], int i) {
    uint64_t r = a[0];
#pragma unroll
    for (int f = 1; f < FPL; ++f) {
        const uint64_t m = 0ull - (uint64_t)(i == f);
        r = (a[f] & m) | (r & ~m);
    }
    return r;
}

// Variable-node pass of an iteration whose posterior is not returned
// (no early stopping, not the last iteration): betas only.
template <int DVMAX, int FPL>
__global__ void __launch_bounds__(kBlock) vn_block_kernel(const QCDesc D, const BlockParams P) {
    constexpr int Gt = 64 * FPL;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / D.n;
    const int col = wave - tile * D.n;
    if (tile >= P.tiles) return;
    const int nvalid = min(P.gamma - tile * Gt, Gt);
    uint64_t frz[FPL];
    bool any, all;
    frozen_words<FPL>(P, tile, nvalid, frz, any, all);
    float L[FPL];
    vn_column<DVMAX, FPL>(D, P, tile, col, lane, any, frz, L);
}

// Variable-node pass that also returns the posterior and decisions in the
// caller's frame-major layout (every iteration with early stopping, else the
// last one).  A block of 16 waves covers 64 consecutive variables of one tile
// (4 per wave); the posteriors go through LDS so that each store instruction
// writes 64 consecutive values of one frame.  Frozen frames are not written.
constexpr int kOutVars = 64;
constexpr int kOutBlock = 1024;

template <int DVMAX, int FPL>
__global__ void __launch_bounds__(kOutBlock) vn_block_out_kernel(const QCDesc D, const BlockParams P, float* post,
                                                                 uint8_t* bits_out) {
    constexpr int Gt = 64 * FPL;
    __shared__ float Ls[kOutVars][Gt + 1];
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_block();
    const int nchunks = (D.n + kOutVars - 1) / kOutVars;
    const int tile = blockIdx.x / nchunks;
    const int v0 = (blockIdx.x - tile * nchunks) * kOutVars;
    const int nvalid = min(P.gamma - tile * Gt, Gt);
    uint64_t frz[FPL];
    bool any, all;
    frozen_words<FPL>(P, tile, nvalid, frz, any, all);
    if (P.early && v0 == 0 && wv == 0) publish_frozen<FPL>(P, tile, lane, frz);
    if (P.early && all) return;   // the same for every wave of the block
    constexpr int per_wave = kOutVars / (kOutBlock / 64);
#pragma unroll 1
    for (int i = 0; i < per_wave; ++i) {
        const int vs = wv * per_wave + i;
        const int col = v0 + vs;
        if (col >= D.n) break;
        float L[FPL];
        vn_column<DVMAX, FPL>(D, P, tile, col, lane, any, frz, L);
#pragma unroll
        for (int f = 0; f < FPL; ++f) Ls[vs][lane * FPL + f] = L[f];
    }
    __syncthreads();
    const int var = threadIdx.x & (kOutVars - 1);
    const int col = v0 + var;
    if (col >= D.n) return;
    // this thread's frames fr = fr0, fr0 + 16, ... all lie in word fr0 % FPL
    constexpr int fstep = kOutBlock / kOutVars;
    static_assert(fstep % FPL == 0, "frame stride must keep the flag word fixed");
    const int fr0 = threadIdx.x / kOutVars;
    const uint64_t fw = pick_word<FPL>(frz, fr0 % FPL);
    for (int fr = fr0; fr < nvalid; fr += fstep) {
        if (any && ((fw >> (fr / FPL)) & 1ull)) continue;
        const float L = Ls[var][fr];
        const size_t o = (size_t)(tile * Gt + fr) * D.n + col;
        post[o] = clip30(L);
        bits_out[o] = (uint8_t)(L < 0.0f);
    }
}

// Syndrome of the decisions in P.bits for iteration P.iter (one thread per
// check row and tile; the wave ORs its rows before one atomic per word).
template <int FPL>
__global__ void __launch_bounds__(kBlock) syndrome_kernel(const QCDesc D, const BlockParams P) {
    constexpr int Gt = 64 * FPL;
    const int gid = blockIdx.x * kBlock + threadIdx.x;
    const int tile = gid / D.m;
    const int row = gid - tile * D.m;
    uint64_t par[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) par[f] = 0;
    const bool live = tile < P.tiles;
    if (live) {
        const QCRow R(D, row);
        const uint64_t* bt = P.bits + (size_t)tile * D.n * FPL;
        const int nvalid = min(P.gamma - tile * Gt, Gt);
        for (int k = 0; k < R.d; ++k) {
            const uint64_t* w = bt + (size_t)R.var(D, k) * FPL;
#pragma unroll
            for (int f = 0; f < FPL; ++f) par[f] ^= w[f];
        }
#pragma unroll
        for (int f = 0; f < FPL; ++f) par[f] &= valid_word<FPL>(nvalid, f);
    }
    // rows of one wave may straddle two tiles: reduce per tile of lane 0 and
    // let lanes of another tile issue their own atomics
    const int tile0 = __shfl(tile, 0);
    const bool same = (tile == tile0);
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        uint64_t v = same ? par[f] : 0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off);
        if (live) {
            uint64_t* un = P.unsat + ((size_t)P.iter * P.tiles + tile) * FPL + f;
            if (same) {
                if ((threadIdx.x & 63) == 0 && v) atomicOr((unsigned long long*)un, (unsigned long long)v);
            } else if (par[f]) {
                atomicOr((unsigned long long*)un, (unsigned long long)par[f]);
            }
        }
    }
}

// Per-frame iteration count and convergence flag from the flag words.
template <int FPL>
__global__ void frame_status_kernel(const BlockParams P, int max_iters, int32_t* iters, uint8_t* converged) {
    constexpr int Gt = 64 * FPL;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= P.gamma) return;
    const int tile = g / Gt, fl = g - tile * Gt;
    const int f = fl % FPL, bit = fl / FPL;
    int it = max_iters, ok = 0;
    if (P.early) {
        for (int i = 1; i <= max_iters; ++i) {
            if (!((P.unsat[((size_t)i * P.tiles + tile) * FPL + f] >> bit) & 1ull)) {
                it = i;
                ok = 1;
                break;
            }
        }
    } else {
        ok = !((P.unsat[((size_t)max_iters * P.tiles + tile) * FPL + f] >> bit) & 1ull);
    }
    if (iters) iters[g] = it;
    if (converged) converged[g] = (uint8_t)ok;
}

// ---------------------------------------------------------------------------
// kernels: layout changes (frame-major <-> packages), through LDS
// ---------------------------------------------------------------------------

// src [gamma][ld], columns col0 .. col0+ncols-1  ->  dst[tile*dstride + col*Gt + frame]
// (frames >= gamma are written as 0).  64 columns x 64 frames per block.
// Block (0, 0) also clears `zero_count` words at `zero` (flag words of a decode).
__global__ void __launch_bounds__(256) to_packages_kernel(const float* __restrict__ src, int64_t ld, int64_t col0,
                                                          int ncols, int gamma, int gpad, int Gt,
                                                          float* __restrict__ dst, int64_t dstride,
                                                          uint64_t* __restrict__ zero, int64_t zero_count) {
    __shared__ float tileS[64][65];
    const int c0 = blockIdx.x * 64, f0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    if (zero && blockIdx.x == 0 && blockIdx.y == 0)
        for (int64_t i = threadIdx.x; i < zero_count; i += 256) zero[i] = 0ull;
#pragma unroll 4
    for (int r = ty; r < 64; r += 4) {
        const int g = f0 + r, c = c0 + tx;
        float v = 0.0f;
        if (g < gamma && c < ncols) v = src[(size_t)g * ld + col0 + c];
        tileS[r][tx] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int r = ty; r < 64; r += 4) {
        const int c = c0 + r, g = f0 + tx;
        if (c < ncols && g < gpad) {
            const int tile = g / Gt, fl = g - tile * Gt;
            dst[(size_t)tile * dstride + (size_t)c * Gt + fl] = tileS[tx][r];
        }
    }
}

// src[tile*sstride + col*Gt + frame]  ->  post [gamma][ld] = clip(L), bits = (L < 0)
__global__ void __launch_bounds__(256) from_packages_kernel(const float* __restrict__ src, int64_t sstride, int ncols,
                                                            int gamma, int Gt, float* __restrict__ post,
                                                            uint8_t* __restrict__ bits, int64_t ld, int64_t col0) {
    __shared__ float tileS[64][65];
    const int c0 = blockIdx.x * 64, f0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll 4
    for (int r = ty; r < 64; r += 4) {
        const int c = c0 + r, g = f0 + tx;
        float v = 0.0f;
        if (c < ncols && g < gamma) {
            const int tile = g / Gt, fl = g - tile * Gt;
            v = src[(size_t)tile * sstride + (size_t)c * Gt + fl];
        }
        tileS[tx][r] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int r = ty; r < 64; r += 4) {
        const int g = f0 + r, c = c0 + tx;
        if (g < gamma && c < ncols) {
            const float L = tileS[r][tx];
            post[(size_t)g * ld + col0 + c] = clip30(L);
            bits[(size_t)g * ld + col0 + c] = (uint8_t)(L < 0.0f);
        }
    }
}

// ---------------------------------------------------------------------------
// kernels: convolutional code, sliding window
// ---------------------------------------------------------------------------

struct WinParams {
    float* msg;       // [tiles][R*eps][Gt]
    const float* mu;  // [tiles][R*c][Gt]
    float* stage;     // [tiles][c][Gt] posterior of the decided position
    int tiles, rows, decide;
};

template <int DCMAX, int FPL>
__global__ void __launch_bounds__(kBlock) cn_window_kernel(const ConvDesc D, const WinState W, const WinParams P) {
    constexpr int Gt = 64 * FPL;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / P.rows;
    const int row = wave - tile * P.rows;
    if (tile >= P.tiles) return;
    const ConvRow R(D, W, row);
    float* mt = P.msg + (size_t)tile * W.R * W.eps * Gt + (size_t)lane * FPL;
    float in[DCMAX][FPL];
    float t[FPL][DCMAX], q[FPL][DCMAX];
    uint32_t sgn[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) sgn[f] = 0;
#pragma unroll
    for (int k = 0; k < DCMAX; ++k) {
        if (R.valid(D, k)) {
            load_frames<FPL>(mt + (size_t)R.pkg(D, W, k) * Gt, in[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) in[k][f] = 0.0f;
        }
    }
#pragma unroll
    for (int k = 0; k < DCMAX; ++k) {
        const bool ok = R.valid(D, k);
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
    float outv[DCMAX][FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        float mag[DCMAX];
        boxplus_fb<DCMAX>(t[f], q[f], mag);
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            const uint32_t s = sgn[f] ^ (__float_as_uint(in[k][f]) & 0x80000000u);
            outv[k][f] = __uint_as_float(__float_as_uint(mag[k]) | s);
        }
    }
#pragma unroll
    for (int k = 0; k < DCMAX; ++k)
        if (R.valid(D, k) && R.writable(D, W, k)) store_frames<FPL>(mt + (size_t)R.pkg(D, W, k) * Gt, outv[k]);
}

template <int DVMAX, int FPL>
__global__ void __launch_bounds__(kBlock) vn_window_kernel(const ConvDesc D, const WinState W, const WinParams P) {
    constexpr int Gt = 64 * FPL;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / P.rows;
    const int col = wave - tile * P.rows;
    if (tile >= P.tiles) return;
    const ConvCol C(D, W, col);
    const size_t lane_off = (size_t)lane * FPL;
    float* mt = P.msg + (size_t)tile * W.R * W.eps * Gt + lane_off;
    float mu[FPL];
    load_frames<FPL>(P.mu + ((size_t)tile * W.R * D.c + C.mu_index(D, W)) * Gt + lane_off, mu);
    float a[DVMAX][FPL];
#pragma unroll
    for (int k = 0; k < DVMAX; ++k) {
        if (C.valid(D, k) && C.contributes(W, D, k)) {
            load_frames<FPL>(mt + (size_t)C.pkg(D, W, k) * Gt, a[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) a[k][f] = 0.0f;
        }
    }
    float L[FPL];
    float b[DVMAX][FPL];
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
#pragma unroll
    for (int k = 0; k < DVMAX; ++k)
        if (C.valid(D, k)) store_frames<FPL>(mt + (size_t)C.pkg(D, W, k) * Gt, b[k]);
    if (P.decide && C.t == W.s)
        store_frames<FPL>(P.stage + ((size_t)tile * D.c + C.q * D.p + C.u) * Gt + lane_off, L);
}

// Positions entering the window: beta = clip(mu) on all their edges.
template <int DVMAX, int FPL>
__global__ void __launch_bounds__(kBlock) init_window_kernel(const ConvDesc D, const WinState W, const WinParams P) {
    constexpr int Gt = 64 * FPL;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / P.rows;
    const int col = wave - tile * P.rows;
    if (tile >= P.tiles) return;
    const ConvCol C(D, W, col);
    const size_t lane_off = (size_t)lane * FPL;
    float* mt = P.msg + (size_t)tile * W.R * W.eps * Gt + lane_off;
    float mu[FPL];
    load_frames<FPL>(P.mu + ((size_t)tile * W.R * D.c + C.mu_index(D, W)) * Gt + lane_off, mu);
#pragma unroll
    for (int f = 0; f < FPL; ++f) mu[f] = clip30(mu[f]);
#pragma unroll
    for (int k = 0; k < DVMAX; ++k)
        if (C.valid(D, k)) store_frames<FPL>(mt + (size_t)C.pkg(D, W, k) * Gt, mu);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace timing {
struct Rec { int cls; hipEvent_t a, b; };
std::mutex mtx;
bool enabled = false;
std::vector<Rec> recs;
std::vector<hipEvent_t> pool;
int64_t launches[LDPC_TIMING_CLASSES];
double total_ms[LDPC_TIMING_CLASSES];

hipEvent_t get_event() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct Scope {
    int idx = -1;
    hipStream_t st;
    Scope(int cls, hipStream_t s) : st(s) {
        std::lock_guard<std::mutex> g(mtx);
        if (!enabled) return;
        Rec r{cls, get_event(), get_event()};
        if (!r.a || !r.b) return;
        (void)hipEventRecord(r.a, st);
        recs.push_back(r);
        idx = (int)recs.size() - 1;
    }
    ~Scope() {
        if (idx < 0) return;
        std::lock_guard<std::mutex> g(mtx);
        if (idx < (int)recs.size()) (void)hipEventRecord(recs[idx].b, st);
    }
};
}  // namespace timing

struct Tiling {
    int fpl, gt, tiles, gpad;
};

// Frames per lane: as many as padding allows (at most 1/8 extra frames),
// capped by the row weight so the check-node kernel stays in registers.
static int row_slots(const ldpc_graph* g) {
    return g->kind == LDPC_GRAPH_CONV ? (g->ms + 1) * g->Lb : g->dc_max;
}

static Tiling choose_tiling(int gamma, const ldpc_graph* g) {
    const int base = (gamma + 63) / 64 * 64;
    const int rs = row_slots(g);
    const int fmax = rs <= 8 ? 4 : (rs <= 16 ? 2 : 1);
    int fpl = 1;
    // LDPC_FRAMES_PER_LANE (1, 2 or 4) overrides the choice, within the row-weight cap
    const char* env = getenv("LDPC_FRAMES_PER_LANE");
    const int forced = env ? atoi(env) : 0;
    if (forced == 1 || forced == 2 || forced == 4) {
        fpl = std::min(forced, fmax);
    } else {
        for (int f : {4, 2}) {
            if (f > fmax) continue;
            const int gt = 64 * f;
            const int pad = (gamma + gt - 1) / gt * gt;
            if (pad * 8 <= base * 9) { fpl = f; break; }
        }
    }
    Tiling t;
    t.fpl = fpl;
    t.gt = 64 * fpl;
    t.tiles = (gamma + t.gt - 1) / t.gt;
    t.gpad = t.tiles * t.gt;
    return t;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BlockLayout {
    size_t mu, msg, bits, flags, flag_words, total;   // flags: unsat words, then frozen words
};

static BlockLayout block_layout(const ldpc_graph* g, const Tiling& t, int max_iters) {
    BlockLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.mu = take((size_t)t.gpad * g->n * sizeof(float));
    L.msg = take((size_t)t.gpad * g->E * sizeof(float));
    L.bits = take((size_t)t.tiles * g->n * t.fpl * sizeof(uint64_t));
    L.flag_words = (size_t)(max_iters + 1) * t.tiles * t.fpl;
    L.flags = take(2 * L.flag_words * sizeof(uint64_t));
    L.total = off;
    return L;
}

struct WinLayout {
    int R, eps;
    size_t mu, msg, stage, total;
};

static WinLayout win_layout(const ldpc_graph* g, const Tiling& t, int W) {
    WinLayout L{};
    L.R = std::min(W, g->positions) + g->ms;
    L.eps = (g->ms + 1) * g->Jb * g->Lb * g->p;
    const int c = g->Lb * g->p;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.mu = take((size_t)t.gpad * L.R * c * sizeof(float));
    L.msg = take((size_t)t.gpad * L.R * L.eps * sizeof(float));
    L.stage = take((size_t)t.gpad * c * sizeof(float));
    L.total = off;
    return L;
}

template <int FPL>
struct MaxDC {
    static constexpr int value = FPL == 4 ? 8 : (FPL == 2 ? 16 : 32);
};

static int dc_class(int d) {
    for (int c : {4, 6, 8, 12, 16, 24, 32})
        if (d <= c) return c;
    return -1;
}
static int dv_class(int d) {
    for (int c : {2, 3, 4, 6, 8, 16})
        if (d <= c) return c;
    return -1;
}

static unsigned grid_for_waves(int64_t waves) {
    return (unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
}

#define LDPC_DC_SWITCH(DCV, ...)                                    \
    switch (DCV) {                                                  \
        case 4: { constexpr int DC = 4; __VA_ARGS__; } break;       \
        case 6: { constexpr int DC = 6; __VA_ARGS__; } break;       \
        case 8: { constexpr int DC = 8; __VA_ARGS__; } break;       \
        case 12: { constexpr int DC = 12; __VA_ARGS__; } break;     \
        case 16: { constexpr int DC = 16; __VA_ARGS__; } break;     \
        case 24: { constexpr int DC = 24; __VA_ARGS__; } break;     \
        default: { constexpr int DC = 32; __VA_ARGS__; } break;     \
    }
#define LDPC_DV_SWITCH(DVV, ...)                                    \
    switch (DVV) {                                                  \
        case 2: { constexpr int DV = 2; __VA_ARGS__; } break;       \
        case 3: { constexpr int DV = 3; __VA_ARGS__; } break;       \
        case 4: { constexpr int DV = 4; __VA_ARGS__; } break;       \
        case 6: { constexpr int DV = 6; __VA_ARGS__; } break;       \
        case 8: { constexpr int DV = 8; __VA_ARGS__; } break;       \
        default: { constexpr int DV = 16; __VA_ARGS__; } break;     \
    }

template <int FPL>
static void run_block(const ldpc_graph* g, const float* llr, int gamma, int max_iters, int early, float* post,
                      uint8_t* bits, int32_t* iters, uint8_t* converged, char* ws, const BlockLayout& lay,
                      const Tiling& tl, hipStream_t st) {
    const QCDesc& D = g->qc;
    BlockParams P{};
    P.msg = reinterpret_cast<float*>(ws + lay.msg);
    P.mu = reinterpret_cast<const float*>(ws + lay.mu);
    P.bits = reinterpret_cast<uint64_t*>(ws + lay.bits);
    P.unsat = reinterpret_cast<uint64_t*>(ws + lay.flags);
    P.frozen = P.unsat + lay.flag_words;
    P.gamma = gamma;
    P.tiles = tl.tiles;
    P.early = early;

    {
        timing::Scope ts(0, st);
        dim3 grid((g->n + 63) / 64, tl.gpad / 64);
        to_packages_kernel<<<grid, 256, 0, st>>>(llr, g->n, 0, g->n, gamma, tl.gpad, tl.gt,
                                                 reinterpret_cast<float*>(ws + lay.mu), (int64_t)g->n * tl.gt,
                                                 P.unsat, (int64_t)(2 * lay.flag_words));
    }
    const int dcc = dc_class(D.dc_max), dvc = dv_class(D.dv_max);
    const unsigned cn_grid = grid_for_waves((int64_t)D.m * tl.tiles);
    const unsigned vn_grid = grid_for_waves((int64_t)D.n * tl.tiles);
    const unsigned out_grid = (unsigned)(((D.n + kOutVars - 1) / kOutVars) * tl.tiles);
    for (int it = 1; it <= max_iters; ++it) {
        P.iter = it;
        P.last = (it == max_iters);
        {
            timing::Scope ts(1, st);
            LDPC_DC_SWITCH(dcc, if constexpr (DC <= MaxDC<FPL>::value) {
                cn_block_kernel<DC, FPL><<<cn_grid, kBlock, 0, st>>>(D, P);
            });
        }
        {
            timing::Scope ts(2, st);
            if (early || P.last) {
                LDPC_DV_SWITCH(dvc, (vn_block_out_kernel<DV, FPL><<<out_grid, kOutBlock, 0, st>>>(D, P, post, bits)));
            } else {
                LDPC_DV_SWITCH(dvc, (vn_block_kernel<DV, FPL><<<vn_grid, kBlock, 0, st>>>(D, P)));
            }
        }
    }
    P.iter = max_iters;
    {
        timing::Scope ts(3, st);
        const int64_t threads = (int64_t)D.m * tl.tiles;
        syndrome_kernel<FPL><<<(unsigned)((threads + kBlock - 1) / kBlock), kBlock, 0, st>>>(D, P);
    }
    if (iters || converged) {
        timing::Scope ts(5, st);
        frame_status_kernel<FPL><<<(gamma + 255) / 256, 256, 0, st>>>(P, max_iters, iters, converged);
    }
}

template <int FPL>
static void run_window(const ldpc_graph* g, const float* llr, int gamma, int Wlen, int K, float* post,
                       uint8_t* bits, char* ws, const WinLayout& lay, const Tiling& tl, hipStream_t st) {
    const ConvDesc& D = g->cv;
    WinParams P{};
    P.msg = reinterpret_cast<float*>(ws + lay.msg);
    P.mu = reinterpret_cast<const float*>(ws + lay.mu);
    P.stage = reinterpret_cast<float*>(ws + lay.stage);
    P.tiles = tl.tiles;
    const int c = D.c;
    const int64_t ld = (int64_t)D.positions * c;
    // edges are enumerated by syndrome-former slot, zero blocks included
    const int dcc = dc_class((D.ms + 1) * D.Lb), dvc = dv_class((D.ms + 1) * D.Jb);
    WinState W{};
    W.R = lay.R;
    W.eps = lay.eps;
    for (int s = 0; s < D.positions; ++s) {
        W.s = s;
        W.lay_lo = s;
        W.lay_hi = std::min(s + Wlen - 1, D.layers - 1);
        const int pos_hi = std::min(s + Wlen - 1, D.positions - 1);
        const int in_lo = (s == 0) ? 0 : s + Wlen - 1;
        if (in_lo <= pos_hi) {
            const int npos = pos_hi - in_lo + 1;
            {
                timing::Scope ts(6, st);
                dim3 grid((npos * c + 63) / 64, tl.gpad / 64);
                float* dst = reinterpret_cast<float*>(ws + lay.mu) + (size_t)(in_lo % lay.R) * c * tl.gt;
                to_packages_kernel<<<grid, 256, 0, st>>>(llr, ld, (int64_t)in_lo * c, npos * c, gamma, tl.gpad,
                                                         tl.gt, dst, (int64_t)lay.R * c * tl.gt, nullptr, 0);
            }
            {
                timing::Scope ts(7, st);
                WinState Wi = W;
                Wi.s = in_lo;
                WinParams Pi = P;
                Pi.rows = npos * c;
                LDPC_DV_SWITCH(dvc, (init_window_kernel<DV, FPL>
                                     <<<grid_for_waves((int64_t)Pi.rows * tl.tiles), kBlock, 0, st>>>(D, Wi, Pi)));
            }
        }
        const int nlay = W.lay_hi - W.lay_lo + 1;
        const int ncol = (pos_hi - s + 1) * c;
        for (int k = 1; k <= K; ++k) {
            {
                timing::Scope ts(8, st);
                WinParams Pc = P;
                Pc.rows = nlay * D.Jb * D.p;
                LDPC_DC_SWITCH(dcc, if constexpr (DC <= MaxDC<FPL>::value) {
                    cn_window_kernel<DC, FPL><<<grid_for_waves((int64_t)Pc.rows * tl.tiles), kBlock, 0, st>>>(D, W, Pc);
                });
            }
            {
                timing::Scope ts(9, st);
                WinParams Pv = P;
                Pv.rows = ncol;
                Pv.decide = (k == K);
                LDPC_DV_SWITCH(dvc, (vn_window_kernel<DV, FPL>
                                     <<<grid_for_waves((int64_t)Pv.rows * tl.tiles), kBlock, 0, st>>>(D, W, Pv)));
            }
        }
        {
            timing::Scope ts(10, st);
            dim3 grid((c + 63) / 64, (gamma + 63) / 64);
            from_packages_kernel<<<grid, 256, 0, st>>>(P.stage, (int64_t)c * tl.gt, c, gamma, tl.gt, post, bits, ld,
                                                       (int64_t)s * c);
        }
    }
}

}  // namespace ldpc

using namespace ldpc;

extern "C" {

ldpc_status ldpc_workspace_size(const ldpc_graph* g, int32_t gamma, int32_t max_iters, int32_t window,
                                size_t* bytes) {
    if (!g || !bytes || gamma < 1 || max_iters < 1 || max_iters > LDPC_MAX_ITERS || window < 0)
        return LDPC_EINVAL;
    const Tiling tl = choose_tiling(gamma, g);
    if (window == 0) {
        if (g->kind != LDPC_GRAPH_QC) return LDPC_EUNSUPPORTED;
        *bytes = block_layout(g, tl, max_iters).total;
    } else {
        if (g->kind != LDPC_GRAPH_CONV) return LDPC_EUNSUPPORTED;
        if (window < g->ms + 1) return LDPC_EINVAL;
        *bytes = win_layout(g, tl, window).total;
    }
    return LDPC_OK;
}

ldpc_status ldpc_decode(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t max_iters, int32_t early_stop,
                        float* post, uint8_t* bits, int32_t* iters, uint8_t* converged, void* workspace,
                        size_t workspace_bytes, void* stream) {
    if (!g || !llr || !post || !bits) return LDPC_EINVAL;
    if (g->kind != LDPC_GRAPH_QC) return LDPC_EINVAL;
    if (gamma < 1 || max_iters < 1 || max_iters > LDPC_MAX_ITERS) return LDPC_EINVAL;
    if ((int64_t)gamma * g->n > ((int64_t)1 << 40)) return LDPC_EUNSUPPORTED;
    const Tiling tl = choose_tiling(gamma, g);
    const BlockLayout lay = block_layout(g, tl, max_iters);
    if (!workspace || workspace_bytes < lay.total) return LDPC_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return LDPC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(llr) | reinterpret_cast<uintptr_t>(post)) & 3) return LDPC_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(workspace);
    (void)hipGetLastError();
    switch (tl.fpl) {
        case 4: run_block<4>(g, llr, gamma, max_iters, early_stop ? 1 : 0, post, bits, iters, converged, ws, lay, tl, st); break;
        case 2: run_block<2>(g, llr, gamma, max_iters, early_stop ? 1 : 0, post, bits, iters, converged, ws, lay, tl, st); break;
        default: run_block<1>(g, llr, gamma, max_iters, early_stop ? 1 : 0, post, bits, iters, converged, ws, lay, tl, st); break;
    }
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

ldpc_status ldpc_decode_window(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t W,
                               int32_t iters_per_window, float* post, uint8_t* bits, void* workspace,
                               size_t workspace_bytes, void* stream) {
    if (!g || !llr || !post || !bits) return LDPC_EINVAL;
    if (g->kind != LDPC_GRAPH_CONV) return LDPC_EINVAL;
    if (gamma < 1 || iters_per_window < 1 || iters_per_window > LDPC_MAX_ITERS || W < g->ms + 1) return LDPC_EINVAL;
    if ((int64_t)gamma * g->n > ((int64_t)1 << 40)) return LDPC_EUNSUPPORTED;
    const Tiling tl = choose_tiling(gamma, g);
    const WinLayout lay = win_layout(g, tl, W);
    if (!workspace || workspace_bytes < lay.total) return LDPC_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return LDPC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(llr) | reinterpret_cast<uintptr_t>(post)) & 3) return LDPC_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(workspace);
    (void)hipGetLastError();
    switch (tl.fpl) {
        case 4: run_window<4>(g, llr, gamma, W, iters_per_window, post, bits, ws, lay, tl, st); break;
        case 2: run_window<2>(g, llr, gamma, W, iters_per_window, post, bits, ws, lay, tl, st); break;
        default: run_window<1>(g, llr, gamma, W, iters_per_window, post, bits, ws, lay, tl, st); break;
    }
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

ldpc_status ldpc_timing_enable(int32_t enable) {
    std::lock_guard<std::mutex> g(timing::mtx);
    timing::enabled = enable != 0;
    return LDPC_OK;
}

ldpc_status ldpc_timing_read(int64_t* launches, double* total_ms, int32_t capacity) {
    if (!launches || !total_ms || capacity < LDPC_TIMING_CLASSES) return LDPC_EINVAL;
    std::lock_guard<std::mutex> g(timing::mtx);
    ldpc_status st = LDPC_OK;
    for (auto& r : timing::recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            st = LDPC_EHIP;
        } else {
            timing::launches[r.cls] += 1;
            timing::total_ms[r.cls] += ms;
        }
        timing::pool.push_back(r.a);
        timing::pool.push_back(r.b);
    }
    timing::recs.clear();
    for (int c = 0; c < LDPC_TIMING_CLASSES; ++c) {
        launches[c] = timing::launches[c];
        total_ms[c] = timing::total_ms[c];
        timing::launches[c] = 0;
        timing::total_ms[c] = 0.0;
    }
    return st;
}

const char* ldpc_kernel_class_name(int32_t cls) {
    static const char* names[LDPC_TIMING_CLASSES] = {"ingest",     "check_node",  "variable_node", "syndrome",
                                                     "output",     "frame_status", "window_ingest", "window_init",
                                                     "window_check_node", "window_variable_node", "window_output"};
    if (cls < 0 || cls >= LDPC_TIMING_CLASSES) return "unknown";
    return names[cls];
}

}  // extern "C"
