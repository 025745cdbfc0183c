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
#include <cstring>
#include <mutex>
#include <vector>

#include "check2.h"
#include "device.h"
#include "internal.h"
#include "onchip.h"

namespace ldpc {

// Convolutional code.  Its decoders (window and pipeline, ring kernels and
// the window kernel with the ring in LDS) carry messages in base-2 units
// (check2.h): channel LLRs are scaled by log2(e) at ingest and posteriors
// unscaled at output.  A launch works on a list of "units": check layers
// (check-node launches) or code positions (variable-node launches), with
// everything that depends on the unit precomputed on the host: its ring slot,
// its class (index mod T) and the range of positions / layers it exchanges
// messages with.  The edges of position t live in ring slot t mod R, grouped
// in blocks (d, rr, q) of p packages: package s of block (d, rr, q) is the
// edge of check row s of circulant row rr of layer t + d and circulant column
// q of position t.  The edge slots k of a check row (d = ms - k / Lb,
// q = k % Lb, oldest position first) and of a variable (d = k / Jb,
// rr = k % Jb) come from small tables, so no per-edge integer division is
// done on the GPU.
constexpr int kMaxUnits = 64;

struct ConvUnits {
    int n;                        // units in this launch
    int ring;                     // R
    int eps;                      // edge packages per ring slot: (ms+1) * Jb * Lb * p
    int out_unit;                 // variable-node launch: unit whose posterior is returned, or -1
    int32_t pos[kMaxUnits];       // check-node launch: layer tau; variable-node launch: position t
    int32_t slot[kMaxUnits];      // ring slot of position pos[u]
    int32_t cls[kMaxUnits];       // pos[u] mod T
    int32_t lo[kMaxUnits];        // CN: alpha is written only on edges of positions >= lo
                                  // VN: alphas of layers lo..hi are summed (others count as 0)
    int32_t hi[kMaxUnits];
};

struct ConvSlots {
    int8_t cn_dd[LDPC_MAX_ROW_WEIGHT], cn_q[LDPC_MAX_ROW_WEIGHT];
    int8_t vn_dd[LDPC_MAX_COL_WEIGHT], vn_rr[LDPC_MAX_COL_WEIGHT];
};

__device__ __forceinline__ int sf_at(const ConvDesc& D, int cls, int dd, int rr, int q) {
    return D.sf[((cls * (D.ms + 1) + dd) * D.Jb + rr) * D.Lb + q];
}

// check row r of a launch: unit u, circulant row rr, offset s
struct ConvRow {
    int tau, rr, s, cls, slot0, lo;
    __device__ __forceinline__ ConvRow(const ConvDesc& D, const ConvUnits& U, int r) {
        const int per = D.Jb * D.p;
        const int u = r / per;
        const int rem = r - u * per;
        rr = rem / D.p;
        s = rem - rr * D.p;
        tau = U.pos[u];
        cls = U.cls[u];
        slot0 = U.slot[u];
        lo = U.lo[u];
    }
    __device__ __forceinline__ bool valid(const ConvDesc& D, const ConvSlots& S, int k) const {
        if (k >= (D.ms + 1) * D.Lb) return false;
        const int dd = S.cn_dd[k];
        const int t = tau - dd;
        if (t < 0 || t >= D.positions) return false;
        return sf_at(D, cls, dd, rr, S.cn_q[k]) >= 0;
    }
    __device__ __forceinline__ int64_t pkg(const ConvDesc& D, const ConvSlots& S, const ConvUnits& U, int k) const {
        const int dd = S.cn_dd[k];
        int sl = slot0 - dd;
        if (sl < 0) sl += U.ring;
        return (int64_t)sl * U.eps + ((int64_t)((dd * D.Jb + rr) * D.Lb + S.cn_q[k])) * D.p + s;
    }
    __device__ __forceinline__ bool writable(const ConvSlots& S, int k) const { return tau - S.cn_dd[k] >= lo; }
};

// variable column r of a launch: unit u, circulant column q, offset uu
struct ConvCol {
    int t, q, uu, jc, slot, lo, hi, unit;
    __device__ __forceinline__ ConvCol(const ConvDesc& D, const ConvUnits& U, int r) {
        unit = r / D.c;
        const int rem = r - unit * D.c;
        q = rem / D.p;
        uu = rem - q * D.p;
        t = U.pos[unit];
        jc = U.cls[unit];
        slot = U.slot[unit];
        lo = U.lo[unit];
        hi = U.hi[unit];
    }
    __device__ __forceinline__ int shift(const ConvDesc& D, const ConvSlots& S, int k) const {
        const int dd = S.vn_dd[k];
        int ic = jc + dd;
        while (ic >= D.T) ic -= D.T;
        return sf_at(D, ic, dd, S.vn_rr[k], q);
    }
    __device__ __forceinline__ bool valid(const ConvDesc& D, const ConvSlots& S, int k) const {
        if (k >= (D.ms + 1) * D.Jb) return false;
        if (t + S.vn_dd[k] >= D.layers) return false;
        return shift(D, S, k) >= 0;
    }
    __device__ __forceinline__ bool contributes(const ConvSlots& S, int k) const {
        const int tau = t + S.vn_dd[k];
        return tau >= lo && tau <= hi;
    }
    __device__ __forceinline__ int64_t pkg(const ConvDesc& D, const ConvSlots& S, const ConvUnits& U, int k) const {
        int s = uu - shift(D, S, k);
        if (s < 0) s += D.p;
        return (int64_t)slot * U.eps + ((int64_t)((S.vn_dd[k] * D.Jb + S.vn_rr[k]) * D.Lb + q)) * D.p + s;
    }
    __device__ __forceinline__ int64_t mu_index(const ConvDesc& D) const { return (int64_t)slot * D.c + q * D.p + uu; }
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
    const float* nms_w;      // learned min-sum: device [iters][J][2] (scale, offset); NULL = sum-product
    uint64_t* badw;          // early stopping: [tiles * m][FPL] frames violating each row (per pass)
};

// Learned min-sum check rule for one frame (neural normalized-offset
// min-sum): alpha_k = w * s_k * max(m_k - b, 0), m_k the smallest |beta| of
// the other edges, s_k the product of their signs (negative iff beta < 0).
// Unused slots carry |beta| = +inf.  Also returns the first index of the
// minimum and the second minimum (for the backward pass).
struct MinInfo {
    float min1, min2;
    int idx1, idx2;
    uint32_t parity;
};

template <int DC>
__device__ __forceinline__ MinInfo row_minima(const float (&mag)[DC], const uint32_t (&neg)[DC]) {
    MinInfo r{__builtin_inff(), __builtin_inff(), -1, -1, 0u};
#pragma unroll
    for (int k = 0; k < DC; ++k) {
        const float m = mag[k];
        if (m < r.min1) {
            r.min2 = r.min1;
            r.idx2 = r.idx1;
            r.min1 = m;
            r.idx1 = k;
        } else if (m < r.min2) {
            r.min2 = m;
            r.idx2 = k;
        }
        r.parity ^= neg[k];
    }
    return r;
}

template <int FPL>
__device__ __forceinline__ uint64_t pick_word(const uint64_t (&a)[FPL], int i);

// Check-node pass with early stopping: false when every frame of the tile was
// frozen by iteration iter-2 (the wave has nothing to do).
// lane_live: false when every frame of the lane (frames FPL*lane .. +FPL-1:
// bit `lane` of each word) is frozen; such lanes skip their loads, arithmetic
// and stores (a frozen frame's messages are never used again).
template <int FPL>
__device__ __forceinline__ bool cn_tile_live(const BlockParams& P, int tile, int lane, bool& lane_live) {
    lane_live = true;
    if (!(P.early && P.iter >= 3)) return true;
    const uint64_t* fz = P.frozen + ((size_t)(P.iter - 2) * P.tiles + tile) * FPL;
    bool all = true, mine = true;
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        const uint64_t w = fz[f];
        all = all && (w == ~0ull);
        mine = mine && ((w >> lane) & 1ull);
    }
    lane_live = !mine;
    return !all;
}

// Horizontal step of iteration P.iter for the check row R and the 64*FPL
// frames of the wave, reading beta from `src` (iteration 1: the channel LLRs
// gathered from `mu`) and writing alpha to `dst` (which may be `src`: each
// package belongs to one row).  RULE 0: sum-product (Eq. 3); RULE 1: learned
// min-sum with the weights of P.nms_w.  SYN: with early stopping from
// iteration 2 on, also test the row against iteration iter-1's packed
// decisions and store the violated (valid) frames in the row's own words of
// badw (lane f writes word f); unsat_reduce_kernel then ORs a tile's rows
// into unsat[iter-1].  Plain stores: every row of every tile would otherwise
// update the same few flag words, and those updates serialise.
template <int DCMAX, int FPL, int RULE, bool SYN = false>
__device__ __forceinline__ void cn_row(const QCDesc& D, const BlockParams& P, const QCRow& R, int tile, int lane,
                                       const float* src, const float* mu, float* dst, bool from_mu,
                                       int nvalid = 0, int64_t wave = 0, bool lane_live = true) {
    constexpr int Gt = 64 * FPL;
    const size_t lane_off = (size_t)lane * FPL;
    const float* st = src + (size_t)tile * D.E * Gt + lane_off;
    const float* ut = mu + (size_t)tile * D.n * Gt + lane_off;
    float* dt = dst + (size_t)tile * D.E * Gt + lane_off;
    float in[DCMAX][FPL];
#pragma unroll
    for (int k = 0; k < DCMAX; ++k) {
        if (R.valid(D, k) && lane_live) {
            const float* s = from_mu ? ut + (size_t)R.var(D, k) * Gt : st + (size_t)R.pkg(D, k) * Gt;
            load_frames<FPL>(s, in[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) in[k][f] = 0.0f;
        }
    }
    // syndrome: lane k*FPL + f loads decision word f of the row's variable k
    // (one load instruction for the wave instead of d*FPL uniform ones), and
    // an XOR butterfly over the lanes of equal f leaves parity word f in
    // lane f
    const bool syn = SYN && P.early && P.iter >= 2;
    uint64_t par = 0;
    if (syn) {
        const int kk = lane / FPL, ff = lane - kk * FPL;
        if (kk < R.d) par = P.bits[((size_t)tile * D.n + R.var(D, kk)) * FPL + ff];
#pragma unroll
        for (int off = 32; off >= FPL; off >>= 1) par ^= __shfl_xor(par, off);
    }
    float outv[DCMAX][FPL];
    if constexpr (RULE == 0) {
        sp_check<DCMAX, FPL>(in, R.d, outv);
    } else {
        // (scale, offset) of each edge's class: its circulant block b0 + k
        const float* wp = P.nms_w + ((size_t)(P.iter - 1) * D.nb + R.b0) * 2;
        float w[DCMAX], b[DCMAX];
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            w[k] = R.valid(D, k) ? wp[2 * k] : 0.0f;
            b[k] = R.valid(D, k) ? wp[2 * k + 1] : 0.0f;
        }
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            float mag[DCMAX];
            uint32_t neg[DCMAX];
#pragma unroll
            for (int k = 0; k < DCMAX; ++k) {
                const bool ok = R.valid(D, k);
                mag[k] = ok ? fminf(fabsf(in[k][f]), kClip) : __builtin_inff();
                neg[k] = ok ? (uint32_t)(in[k][f] < 0.0f) : 0u;
            }
            const MinInfo mi = row_minima<DCMAX>(mag, neg);
#pragma unroll
            for (int k = 0; k < DCMAX; ++k) {
                const float m = (k == mi.idx1) ? mi.min2 : mi.min1;
                const float a = w[k] * fmaxf(m - b[k], 0.0f);
                outv[k][f] = (mi.parity ^ neg[k]) ? -a : a;
            }
        }
    }
    if (lane_live) {
#pragma unroll
        for (int k = 0; k < DCMAX; ++k)
            if (R.valid(D, k)) store_frames<FPL>(dt + (size_t)R.pkg(D, k) * Gt, outv[k]);
    }
    if (syn && lane < FPL) P.badw[(size_t)wave * FPL + lane] = par & valid_word<FPL>(nvalid, lane);
}

// Check-node pass of iteration P.iter (in place in P.msg; iteration 1 reads
// the channel LLRs).
template <int DCMAX, int FPL, int RULE>
__global__ void __launch_bounds__(kBlock) cn_block_kernel(const QCDesc D, const BlockParams P) {
    constexpr int Gt = 64 * FPL;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / D.m;
    const int row = wave - tile * D.m;
    if (tile >= P.tiles) return;
    const int nvalid = min(P.gamma - tile * Gt, Gt);
    const QCRow R(D, row);
    bool lane_live;
    if (!cn_tile_live<FPL>(P, tile, lane, lane_live)) return;
    cn_row<DCMAX, FPL, RULE, true>(D, P, R, tile, lane, P.msg, P.mu, P.msg, P.iter == 1, nvalid, wave, lane_live);
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
    // a lane whose frames are all frozen (or padding) skips its loads and stores
    bool lane_live = false;
#pragma unroll
    for (int f = 0; f < FPL; ++f) lane_live = lane_live || !((frz[f] >> lane) & 1ull);
    // the edges' packages first, outside the per-lane branch: the column is
    // the wave's, so its edge-block table reads are uniform (scalar); inside
    // the branch each became a vector load whose wait also drained the
    // previous message load, one round trip per edge
    int64_t pk[DVMAX];
#pragma unroll
    for (int k = 0; k < DVMAX; ++k) pk[k] = C.valid(D, k) ? C.pkg(D, k) : 0;
    float mu[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) mu[f] = 0.0f;
    if (lane_live) load_frames<FPL>(P.mu + ((size_t)tile * D.n + C.v) * Gt + lane_off, mu);
    float a[DVMAX][FPL];
#pragma unroll
    for (int k = 0; k < DVMAX; ++k) {
        if (C.valid(D, k) && lane_live) {
            load_frames<FPL>(mt + (size_t)pk[k] * Gt, a[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) a[k][f] = 0.0f;
        }
    }
    float b[DVMAX][FPL];
    sp_variable<DVMAX, FPL>(mu, a, b, L);
    if (!P.last && lane_live) {
#pragma unroll
        for (int k = 0; k < DVMAX; ++k)
            if (C.valid(D, k)) store_frames<FPL>(mt + (size_t)pk[k] * Gt, b[k]);
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

// Variable-node pass with early stopping: one variable per wave as in
// vn_block_kernel, plus the packed decisions and the posterior of the frames
// still running, the latter into the package-layout array postw
// [tile][n][Gt] (coalesced like the betas; frozen frames keep the value of
// their stopping iteration).  block_output_kernel turns postw and the
// decision words into the caller's layout once, after the last iteration.
template <int DVMAX, int FPL>
__global__ void __launch_bounds__(kBlock) vn_block_early_kernel(const QCDesc D, const BlockParams P, float* postw) {
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
    if (col == 0) publish_frozen<FPL>(P, tile, lane, frz);
    if (all) return;
    float L[FPL];
    vn_column<DVMAX, FPL>(D, P, tile, col, lane, any, frz, L);
    float pv[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) pv[f] = clip30(L[f]);
    float* pw = postw + ((size_t)tile * D.n + col) * Gt + (size_t)lane * FPL;
    if (!any) {
        store_frames<FPL>(pw, pv);
    } else {
        // frame lane*FPL + f: word f, bit lane
#pragma unroll
        for (int f = 0; f < FPL; ++f)
            if (!((frz[f] >> lane) & 1ull)) pw[f] = pv[f];
    }
}

// Posterior and decisions of every frame from the package layout (postw,
// packed decision words) to the caller's [gamma][n] buffers, through LDS:
// 64 variables x 64 frames per block.
template <int FPL>
__global__ void __launch_bounds__(256) block_output_kernel(const float* __restrict__ postw,
                                                           const uint64_t* __restrict__ bitw, int n, int gamma,
                                                           float* __restrict__ post, uint8_t* __restrict__ bits_out) {
    constexpr int Gt = 64 * FPL;
    __shared__ float Ps[64][65];
    __shared__ uint8_t Bs[64][65];
    const int c0 = blockIdx.x * 64, f0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {           // r: variable, tx: frame
        const int c = c0 + r, g = f0 + tx;
        if (c < n && g < gamma) {
            const int tile = g / Gt, fl = g - tile * Gt;
            Ps[r][tx] = postw[((size_t)tile * n + c) * Gt + fl];
            const uint64_t w = bitw[((size_t)tile * n + c) * FPL + fl % FPL];
            Bs[r][tx] = (uint8_t)((w >> (fl / FPL)) & 1ull);
        }
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {           // r: frame, tx: variable
        const int c = c0 + tx, g = f0 + r;
        if (c < n && g < gamma) {
            const size_t o = (size_t)g * n + c;
            post[o] = Ps[tx][r];
            bits_out[o] = Bs[tx][r];
        }
    }
}

// unsat[iter-1][tile][f] |= OR over the tile's rows of badw.  Block (tile,
// chunk) reads kRedWords consecutive words of the tile (row r, word f at
// r*FPL + f), each thread kRedPerThread independent ones, so the loads of a
// block are in flight together instead of one round trip per row group.
// 256 and kRedWords are multiples of FPL: a thread only meets words of
// f = threadIdx.x % FPL.  The flag words are cleared at ingest and each
// block adds its nonzero words with one atomicOr per f; a tile whose frames
// were all frozen by iteration iter-2 skipped its check-node pass and keeps
// a zero word.
constexpr int kRedPerThread = 8;
constexpr int kRedWords = 256 * kRedPerThread;

template <int FPL>
__global__ void __launch_bounds__(256) unsat_reduce_kernel(const QCDesc D, const BlockParams P, int chunks) {
    __shared__ uint64_t part[4][FPL];
    const int tile = blockIdx.x / chunks;
    const int chunk = blockIdx.x - tile * chunks;
    if (P.iter >= 3) {
        const uint64_t* fz = P.frozen + ((size_t)(P.iter - 2) * P.tiles + tile) * FPL;
        bool all = true;
#pragma unroll
        for (int f = 0; f < FPL; ++f) all = all && (fz[f] == ~0ull);
        if (all) return;
    }
    const int64_t nw = (int64_t)D.m * FPL;
    const uint64_t* bw = P.badw + (size_t)tile * nw;
    const int64_t w0 = (int64_t)chunk * kRedWords + threadIdx.x;
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kRedPerThread; ++k) {
        const int64_t w = w0 + (int64_t)k * 256;
        if (w < nw) acc |= bw[w];
    }
#pragma unroll
    for (int off = 32; off >= FPL; off >>= 1) acc |= __shfl_xor(acc, off);
    const int lane = threadIdx.x & 63;
    if (lane < FPL) part[threadIdx.x >> 6][lane] = acc;
    __syncthreads();
    if (threadIdx.x < FPL) {
        const int f = threadIdx.x;
        const uint64_t v = part[0][f] | part[1][f] | part[2][f] | part[3][f];
        if (v) atomicOr((unsigned long long*)(P.unsat + ((size_t)(P.iter - 1) * P.tiles + tile) * FPL + f),
                        (unsigned long long)v);
    }
}

// Syndrome of the decisions in P.bits for iteration P.iter: block b covers
// rows (b % bpt)*256 .. +255 of tile b / bpt (bpt blocks per tile, so a block
// never straddles two tiles); the block ORs its rows' violated frames through
// LDS and adds them with one atomicOr per word (the flag words are cleared at
// ingest).
template <int FPL>
__global__ void __launch_bounds__(kBlock) syndrome_kernel(const QCDesc D, const BlockParams P, int bpt) {
    constexpr int Gt = 64 * FPL;
    __shared__ uint64_t part[kWavesPerBlock][FPL];
    const int tile = blockIdx.x / bpt;
    const int row = (blockIdx.x - tile * bpt) * kBlock + threadIdx.x;
    uint64_t par[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) par[f] = 0;
    if (row < D.m) {
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
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        uint64_t v = par[f];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off);
        if (lane == 0) part[threadIdx.x >> 6][f] = v;
    }
    __syncthreads();
    if (threadIdx.x < FPL) {
        const int f = threadIdx.x;
        uint64_t v = 0;
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) v |= part[w][f];
        if (v) atomicOr((unsigned long long*)(P.unsat + ((size_t)P.iter * P.tiles + tile) * FPL + f),
                        (unsigned long long)v);
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
// kernels: training the learned min-sum decoder (forward with checkpoints,
// backward through the unrolled iterations).  The transmitted codeword is
// all-zero, so the loss of a posterior L is softplus(-L).
// ---------------------------------------------------------------------------

// Forward check-node pass of a training step: beta from `src` (NULL: the
// channel LLRs), alpha to `dst`, learned rule.
template <int DCMAX, int FPL>
__global__ void __launch_bounds__(kBlock) nms_train_cn_kernel(const QCDesc D, const BlockParams P, const float* src,
                                                              float* dst) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / D.m;
    const int row = wave - tile * D.m;
    if (tile >= P.tiles) return;
    const QCRow R(D, row);
    cn_row<DCMAX, FPL, 1>(D, P, R, tile, lane, src ? src : P.mu, P.mu, dst, src == nullptr);
}

__device__ __forceinline__ float softplus_neg(float L) {   // log(1 + exp(-L))
    return fmaxf(-L, 0.0f) + log1pf(__expf(-fabsf(L)));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Forward variable-node pass of a training step: alpha from A, beta to dst
// (NULL: not needed), and, when `lpart` is not NULL, the wave's share of the
// iteration's mean loss (sum of softplus(-L) over its valid frames, times
// inv_count = 1 / (gamma n)) written to lpart[wave].
template <int DVMAX, int FPL>
__global__ void __launch_bounds__(kBlock) nms_train_vn_kernel(const QCDesc D, const BlockParams P, const float* A,
                                                              float* dst, float* lpart, float inv_count) {
    constexpr int Gt = 64 * FPL;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / D.n;
    const int col = wave - tile * D.n;
    if (tile >= P.tiles) return;
    const int nvalid = min(P.gamma - tile * Gt, Gt);
    const QCCol C(D, col);
    const size_t lane_off = (size_t)lane * FPL;
    const size_t base = (size_t)tile * D.E * Gt + lane_off;
    // the edges' packages before any message load (see vn_column)
    int64_t pk[DVMAX];
#pragma unroll
    for (int k = 0; k < DVMAX; ++k) pk[k] = C.valid(D, k) ? C.pkg(D, k) : 0;
    float mu[FPL];
    load_frames<FPL>(P.mu + ((size_t)tile * D.n + C.v) * Gt + lane_off, mu);
    float a[DVMAX][FPL];
#pragma unroll
    for (int k = 0; k < DVMAX; ++k) {
        if (C.valid(D, k)) {
            load_frames<FPL>(A + base + (size_t)pk[k] * Gt, a[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) a[k][f] = 0.0f;
        }
    }
    float b[DVMAX][FPL];
    float lsum = 0.0f;
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
        const float L = mu[f] + pre;
        if (lane * FPL + f < nvalid) lsum += softplus_neg(L);
    }
#pragma unroll
    for (int k = 0; k < DVMAX; ++k) {
        if (!C.valid(D, k)) continue;
        if (dst) store_frames<FPL>(dst + base + (size_t)pk[k] * Gt, b[k]);
    }
    if (lpart) {
        lsum = wave_sum(lsum);
        if (lane == 0) lpart[wave] = lsum * inv_count;
    }
}

// Backward of the variable-node pass of iteration P.iter.  Inputs: alpha of
// the iteration (A), the gradient with respect to its betas (dB; NULL at the
// last iteration, whose betas are not used).  The iteration's mean loss, with
// upstream gradient dloss[iter-1], contributes dloss/dL = -dloss[iter-1] *
// inv_count / (1 + exp(L)) on valid frames.  Output: the gradient with
// respect to the iteration's alphas, dA_k = dL + sum_{k' != k} dB_k' [beta_k'
// not clipped].
template <int DVMAX, int FPL>
__global__ void __launch_bounds__(kBlock) nms_vn_backward_kernel(const QCDesc D, const BlockParams P, const float* A,
                                                                 const float* dB, float* dA, const float* dloss,
                                                                 float inv_count) {
    constexpr int Gt = 64 * FPL;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / D.n;
    const int col = wave - tile * D.n;
    if (tile >= P.tiles) return;
    const int nvalid = min(P.gamma - tile * Gt, Gt);
    const QCCol C(D, col);
    const size_t lane_off = (size_t)lane * FPL;
    const size_t base = (size_t)tile * D.E * Gt + lane_off;
    const float scale = dloss[P.iter - 1] * inv_count;
    // the edges' packages before any message load (see vn_column)
    int64_t pk[DVMAX];
#pragma unroll
    for (int k = 0; k < DVMAX; ++k) pk[k] = C.valid(D, k) ? C.pkg(D, k) : 0;
    float mu[FPL];
    load_frames<FPL>(P.mu + ((size_t)tile * D.n + C.v) * Gt + lane_off, mu);
    float a[DVMAX][FPL], gb[DVMAX][FPL];
#pragma unroll
    for (int k = 0; k < DVMAX; ++k) {
        const bool ok = C.valid(D, k);
        if (ok) {
            load_frames<FPL>(A + base + (size_t)pk[k] * Gt, a[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) a[k][f] = 0.0f;
        }
        if (ok && dB) {
            load_frames<FPL>(dB + base + (size_t)pk[k] * Gt, gb[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) gb[k][f] = 0.0f;
        }
    }
    float out[DVMAX][FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        float suf[DVMAX];
        float S = 0.0f;
#pragma unroll
        for (int k = DVMAX - 1; k >= 0; --k) {
            suf[k] = S;
            S += a[k][f];
        }
        float pre = 0.0f, g[DVMAX];
#pragma unroll
        for (int k = 0; k < DVMAX; ++k) {
            const float beta = mu[f] + (pre + suf[k]);          // before the clip
            g[k] = (fabsf(beta) <= kClip) ? gb[k][f] : 0.0f;
            pre += a[k][f];
        }
        const float L = mu[f] + pre;
        const float dL = (lane * FPL + f < nvalid) ? -scale / (1.0f + __expf(L)) : 0.0f;
        float gs[DVMAX];
        float G = 0.0f;
#pragma unroll
        for (int k = DVMAX - 1; k >= 0; --k) {
            gs[k] = G;
            G += g[k];
        }
        float gp = 0.0f;
#pragma unroll
        for (int k = 0; k < DVMAX; ++k) {
            out[k][f] = dL + (gp + gs[k]);
            gp += g[k];
        }
    }
#pragma unroll
    for (int k = 0; k < DVMAX; ++k)
        if (C.valid(D, k)) store_frames<FPL>(dA + base + (size_t)pk[k] * Gt, out[k]);
}

__device__ __forceinline__ float abs_grad(float x) { return x > 0.0f ? 1.0f : (x < 0.0f ? -1.0f : 0.0f); }

// Backward of the check-node pass of iteration P.iter.  Inputs: the betas the
// pass read (src; NULL at iteration 1: the channel LLRs, whose gradient is not
// needed) and the gradient with respect to its alphas (dA).  With
// m_k = min over the other edges, s_k their sign product, a_k = m_k - b:
//   dw += dA_k s_k max(a_k, 0),  db -= dA_k w s_k [a_k > 0],
//   the gradient w s_k [a_k > 0] dA_k reaches |beta| of the edge holding m_k
// (the row minimum for k != argmin, the second minimum for k = argmin).
// Weights per edge class (the edge's circulant block).  Writes dB (gradient
// with respect to the betas read; NULL at iteration 1) and the wave's (dw, db)
// partial sums, one pair per edge slot of the row.
template <int DCMAX, int FPL>
__global__ void __launch_bounds__(kBlock) nms_cn_backward_kernel(const QCDesc D, const BlockParams P,
                                                                 const float* src, const float* dA, float* dB,
                                                                 float2* partial) {
    constexpr int Gt = 64 * FPL;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / D.m;
    const int row = wave - tile * D.m;
    if (tile >= P.tiles) return;
    const QCRow R(D, row);
    const size_t lane_off = (size_t)lane * FPL;
    const size_t base = (size_t)tile * D.E * Gt + lane_off;
    const float* ut = P.mu + (size_t)tile * D.n * Gt + lane_off;
    float in[DCMAX][FPL], da[DCMAX][FPL];
#pragma unroll
    for (int k = 0; k < DCMAX; ++k) {
        if (R.valid(D, k)) {
            load_frames<FPL>(src ? src + base + (size_t)R.pkg(D, k) * Gt : ut + (size_t)R.var(D, k) * Gt, in[k]);
            load_frames<FPL>(dA + base + (size_t)R.pkg(D, k) * Gt, da[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) {
                in[k][f] = 0.0f;
                da[k][f] = 0.0f;
            }
        }
    }
    const float* wp = P.nms_w + ((size_t)(P.iter - 1) * D.nb + R.b0) * 2;
    float w[DCMAX], b[DCMAX], dw[DCMAX], db[DCMAX];
#pragma unroll
    for (int k = 0; k < DCMAX; ++k) {
        w[k] = R.valid(D, k) ? wp[2 * k] : 0.0f;
        b[k] = R.valid(D, k) ? wp[2 * k + 1] : 0.0f;
        dw[k] = 0.0f;
        db[k] = 0.0f;
    }
    float out[DCMAX][FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        float mag[DCMAX];
        uint32_t neg[DCMAX];
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            const bool ok = R.valid(D, k);
            mag[k] = ok ? fminf(fabsf(in[k][f]), kClip) : __builtin_inff();
            neg[k] = ok ? (uint32_t)(in[k][f] < 0.0f) : 0u;
        }
        const MinInfo mi = row_minima<DCMAX>(mag, neg);
        float G1 = 0.0f, G2 = 0.0f;
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            if (!R.valid(D, k)) continue;
            const float m = (k == mi.idx1) ? mi.min2 : mi.min1;
            const float sg = (mi.parity ^ neg[k]) ? -1.0f : 1.0f;
            const float a = m - b[k];
            const float act = a >= 0.0f ? 1.0f : 0.0f;
            dw[k] += da[k][f] * sg * fmaxf(a, 0.0f);
            db[k] -= da[k][f] * w[k] * sg * act;
            const float gk = da[k][f] * w[k] * sg * act;
            if (k == mi.idx1) G2 = gk;
            else G1 += gk;
        }
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            float v = 0.0f;
            if (k == mi.idx1) v = G1 * abs_grad(in[k][f]);
            if (k == mi.idx2) v = G2 * abs_grad(in[k][f]);
            out[k][f] = v;
        }
    }
    if (dB) {
#pragma unroll
        for (int k = 0; k < DCMAX; ++k)
            if (R.valid(D, k)) store_frames<FPL>(dB + base + (size_t)R.pkg(D, k) * Gt, out[k]);
    }
    // one (dw, db) pair per edge slot of the row: slot k feeds block b0 + k
#pragma unroll
    for (int k = 0; k < DCMAX; ++k) {
        if (!R.valid(D, k)) continue;
        const float sw = wave_sum(dw[k]);
        const float sb = wave_sum(db[k]);
        if (lane == 0) partial[(size_t)wave * D.dc_max + k] = make_float2(sw, sb);
    }
}

// grad[t][b] = sum of the check-node backward partials of iteration t + 1
// over the rows of block b's base row j, slot b - rstart[j], in a fixed
// order; grid (nb, T), partial [T][tiles * m][dc_max].
__global__ void __launch_bounds__(256) nms_grad_reduce_kernel(const QCDesc D, const float2* partial, int tiles,
                                                              float* grad) {
    __shared__ float sw[256], sb[256];
    const int blk = blockIdx.x, t = blockIdx.y;
    int j = 0;
    while (j + 1 < D.J && D.rstart[j + 1] <= blk) ++j;
    const int k = blk - D.rstart[j];
    const float2* pt = partial + (size_t)t * tiles * D.m * D.dc_max;
    float aw = 0.0f, ab = 0.0f;
    for (int i = threadIdx.x; i < tiles * D.p; i += 256) {
        const int tile = i / D.p, s = i - tile * D.p;
        const float2 v = pt[((size_t)tile * D.m + (size_t)j * D.p + s) * D.dc_max + k];
        aw += v.x;
        ab += v.y;
    }
    sw[threadIdx.x] = aw;
    sb[threadIdx.x] = ab;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sw[threadIdx.x] += sw[threadIdx.x + h];
            sb[threadIdx.x] += sb[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        grad[((size_t)t * D.nb + blk) * 2 + 0] = sw[0];
        grad[((size_t)t * D.nb + blk) * 2 + 1] = sb[0];
    }
}

// loss[t] = sum of the count wave partials of iteration t + 1, in a fixed
// order; one block per iteration.
__global__ void __launch_bounds__(256) nms_loss_reduce_kernel(const float* lpart, int64_t count, float* loss) {
    __shared__ float sl[256];
    const float* pt = lpart + (size_t)blockIdx.x * count;
    float a = 0.0f;
    for (int64_t i = threadIdx.x; i < count; i += 256) a += pt[i];
    sl[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) sl[threadIdx.x] += sl[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[blockIdx.x] = sl[0];
}


// ---------------------------------------------------------------------------
// kernels: layout changes (frame-major <-> packages), through LDS
// ---------------------------------------------------------------------------

// src [gamma][ld], columns col0 .. col0+ncols-1  ->  dst[tile*dstride + col*Gt + frame]
// (frames >= gamma are written as 0).  A block of 512 threads covers 256
// columns x 32 frames (one-dimensional grid, frame chunks fastest): each frame
// row is read as one 1-KB run (a frame row of n floats is in general not
// aligned to the 128-byte lines, so short runs fetch the lines they share
// with the neighbouring block twice), and each column's 32 frames are written
// as one 128-byte run.  Gt must be a
// multiple of 32.  Block 0 also clears `zero_count` words at `zero` (flag
// words of a decode).
constexpr int kIngCols = 256;
constexpr int kIngFrames = 32;
constexpr int kIngBlock = 512;

__global__ void __launch_bounds__(kIngBlock) to_packages_kernel(const float* __restrict__ src, int64_t ld,
                                                                int64_t col0, int ncols, int gamma, int gpad, int Gt,
                                                                float* __restrict__ dst, int64_t dstride,
                                                                uint64_t* __restrict__ zero, int64_t zero_count) {
    __shared__ float tileS[kIngFrames][kIngCols + 1];
    constexpr int kWaves = kIngBlock / 64;
    const int fchunks = (gpad + kIngFrames - 1) / kIngFrames;
    const int cb = (int)(blockIdx.x / fchunks);
    const int f0 = (int)(blockIdx.x - (unsigned)cb * fchunks) * kIngFrames, c0 = cb * kIngCols;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (zero && blockIdx.x == 0)
        for (int64_t i = threadIdx.x; i < zero_count; i += kIngBlock) zero[i] = 0ull;
    // wave wv reads frame rows wv, wv + 8, ...: 256 consecutive columns each
#pragma unroll
    for (int i = 0; i < kIngFrames / kWaves; ++i) {
        const int r = wv + i * kWaves;
        const int g = f0 + r;
#pragma unroll
        for (int k = 0; k < kIngCols / 64; ++k) {
            const int c = c0 + lane + 64 * k;
            float v = 0.0f;
            if (g < gamma && c < ncols) v = src[(size_t)g * ld + col0 + c];
            tileS[r][lane + 64 * k] = v;
        }
    }
    __syncthreads();
    // lanes 0-31 and 32-63 of a wave write the 32 frames of one column each
    const int fr = threadIdx.x & (kIngFrames - 1);
    const int g = f0 + fr;
    if (g >= gpad) return;
    const int tile = g / Gt, fl = g - tile * Gt;
    float* d = dst + (size_t)tile * dstride + fl;
#pragma unroll
    for (int j = 0; j < kIngCols * kIngFrames / kIngBlock; ++j) {
        const int cc = (int)threadIdx.x / kIngFrames + j * (kIngBlock / kIngFrames);
        const int c = c0 + cc;
        if (c < ncols) d[(size_t)c * Gt] = tileS[fr][cc];
    }
}

// grid of to_packages_kernel for ncols columns and gpad frames: one block per
// (column chunk, frame chunk), frame chunks fastest
static dim3 packages_grid(int ncols, int gpad) {
    const int64_t blocks = (int64_t)((gpad + kIngFrames - 1) / kIngFrames) * ((ncols + kIngCols - 1) / kIngCols);
    return dim3((unsigned)blocks);
}

// ---------------------------------------------------------------------------
// kernels: convolutional code (window and pipelined schedules)
// ---------------------------------------------------------------------------

struct ConvParams {
    float* msg;       // [tiles][R * eps][Gt]
    float* mu;        // [tiles][R * c][Gt]
    int tiles, rows, gamma;
};

template <int DCMAX, int FPL>
__global__ void __launch_bounds__(kBlock) conv_cn_kernel(const ConvDesc D, const ConvSlots S, const ConvUnits U,
                                                         const ConvParams P) {
    constexpr int Gt = 64 * FPL;
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / P.rows;
    const int row = wave - tile * P.rows;
    if (tile >= P.tiles) return;
    const ConvRow R(D, U, row);
    float* mt = P.msg + (size_t)tile * U.ring * U.eps * Gt + (size_t)lane * FPL;
    float in[DCMAX][FPL];
    float t[FPL][DCMAX], q[FPL][DCMAX];
    uint32_t sgn[FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) sgn[f] = 0;
#pragma unroll
    for (int k = 0; k < DCMAX; ++k) {
        if (R.valid(D, S, k)) {
            load_frames<FPL>(mt + (size_t)R.pkg(D, S, U, k) * Gt, in[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) in[k][f] = 0.0f;
        }
    }
#pragma unroll
    for (int k = 0; k < DCMAX; ++k) {
        const bool ok = R.valid(D, S, k);
#pragma unroll
        for (int f = 0; f < FPL; ++f) {
            if (ok) {
                tq2_of(in[k][f], t[f][k], q[f][k]);
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
        boxplus2_fb<DCMAX>(t[f], q[f], mag);
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            const uint32_t sg = sgn[f] ^ (__float_as_uint(in[k][f]) & 0x80000000u);
            outv[k][f] = __uint_as_float(__float_as_uint(mag[k]) | sg);
        }
    }
#pragma unroll
    for (int k = 0; k < DCMAX; ++k)
        if (R.valid(D, S, k) && R.writable(S, k)) store_frames<FPL>(mt + (size_t)R.pkg(D, S, U, k) * Gt, outv[k]);
}

// One variable column: betas on every existing edge, posterior from the
// alphas of layers lo..hi.
template <int DVMAX, int FPL>
__device__ __forceinline__ void conv_vn_column(const ConvDesc& D, const ConvSlots& S, const ConvUnits& U,
                                               const ConvParams& P, const ConvCol& C, int tile, int lane,
                                               float (&L)[FPL]) {
    constexpr int Gt = 64 * FPL;
    const size_t lane_off = (size_t)lane * FPL;
    float* mt = P.msg + (size_t)tile * U.ring * U.eps * Gt + lane_off;
    float mu[FPL];
    load_frames<FPL>(P.mu + ((size_t)tile * U.ring * D.c + C.mu_index(D)) * Gt + lane_off, mu);
    float a[DVMAX][FPL];
#pragma unroll
    for (int k = 0; k < DVMAX; ++k) {
        if (C.valid(D, S, k) && C.contributes(S, k)) {
            load_frames<FPL>(mt + (size_t)C.pkg(D, S, U, k) * Gt, a[k]);
        } else {
#pragma unroll
            for (int f = 0; f < FPL; ++f) a[k][f] = 0.0f;
        }
    }
    float b[DVMAX][FPL];
#pragma unroll
    for (int f = 0; f < FPL; ++f) {
        float suf[DVMAX];
        float Ssum = 0.0f;
#pragma unroll
        for (int k = DVMAX - 1; k >= 0; --k) {
            suf[k] = Ssum;
            Ssum += a[k][f];
        }
        float pre = 0.0f;
#pragma unroll
        for (int k = 0; k < DVMAX; ++k) {
            b[k][f] = clip2(mu[f] + (pre + suf[k]));
            pre += a[k][f];
        }
        L[f] = mu[f] + pre;
    }
#pragma unroll
    for (int k = 0; k < DVMAX; ++k)
        if (C.valid(D, S, k)) store_frames<FPL>(mt + (size_t)C.pkg(D, S, U, k) * Gt, b[k]);
}

template <int DVMAX, int FPL>
__global__ void __launch_bounds__(kBlock) conv_vn_kernel(const ConvDesc D, const ConvSlots S, const ConvUnits U,
                                                         const ConvParams P) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * kWavesPerBlock + wave_in_block();
    const int tile = wave / P.rows;
    const int col = wave - tile * P.rows;
    if (tile >= P.tiles) return;
    const ConvCol C(D, U, col);
    float L[FPL];
    conv_vn_column<DVMAX, FPL>(D, S, U, P, C, tile, lane, L);
}

// Variable-node launch that also returns the posterior and decisions of unit
// U.out_unit in the caller's frame-major layout [gamma][positions * c].  The
// first out_blocks blocks take the output unit's columns through LDS as in
// the block decoder (16 waves cover 64 consecutive columns); the blocks after
// them update the other units' columns, one column per wave, as
// conv_vn_kernel does.
template <int DVMAX, int FPL>
__global__ void __launch_bounds__(kOutBlock) conv_vn_out_kernel(const ConvDesc D, const ConvSlots S,
                                                                const ConvUnits U, const ConvParams P, float* post,
                                                                uint8_t* bits_out, int out_blocks) {
    constexpr int Gt = 64 * FPL;
    __shared__ float Ls[kOutVars][Gt + 1];
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_block();
    if ((int)blockIdx.x >= out_blocks) {
        // plain columns: every unit but the output one
        const int plain = P.rows - D.c;
        const int64_t w = (int64_t)(blockIdx.x - out_blocks) * (kOutBlock / 64) + wv;
        const int tile = (int)(w / plain);
        if (tile >= P.tiles) return;
        const int idx = (int)(w - (int64_t)tile * plain);
        const int col = idx < U.out_unit * D.c ? idx : idx + D.c;
        const ConvCol C(D, U, col);
        float L[FPL];
        conv_vn_column<DVMAX, FPL>(D, S, U, P, C, tile, lane, L);
        return;
    }
    const int nchunks = (D.c + kOutVars - 1) / kOutVars;
    const int tile = blockIdx.x / nchunks;
    const int u0 = U.out_unit * D.c;
    const int c0 = (blockIdx.x - tile * nchunks) * kOutVars;      // column within the output unit
    constexpr int per_wave = kOutVars / (kOutBlock / 64);
#pragma unroll 1
    for (int i = 0; i < per_wave; ++i) {
        const int vs = wv * per_wave + i;
        if (c0 + vs >= D.c) break;
        const ConvCol C(D, U, u0 + c0 + vs);
        float L[FPL];
        conv_vn_column<DVMAX, FPL>(D, S, U, P, C, tile, lane, L);
#pragma unroll
        for (int f = 0; f < FPL; ++f) Ls[vs][lane * FPL + f] = L[f];
    }
    __syncthreads();
    const int var = threadIdx.x & (kOutVars - 1);
    if (c0 + var >= D.c) return;
    const int64_t ld = (int64_t)D.positions * D.c;
    const int64_t oc = (int64_t)U.pos[U.out_unit] * D.c + c0 + var;
    const int nvalid = min(P.gamma - tile * Gt, Gt);
    for (int fr = threadIdx.x / kOutVars; fr < nvalid; fr += kOutBlock / kOutVars) {
        const float L = Ls[var][fr] * kLn2F;   // base-2 units to an LLR
        const size_t o = (size_t)(tile * Gt + fr) * ld + oc;
        post[o] = clip30(L);
        bits_out[o] = (uint8_t)(L < 0.0f);
    }
}

// Positions t0 .. t0+npos-1 enter the ring: channel LLRs go from the caller's
// layout into the mu ring (through LDS), and every edge of the entering
// positions starts with beta = clip(mu).  64 columns x 64 frames per block of
// 16 waves (one position is only 16 x Gt/64 blocks, so the block is wide).
constexpr int kIngestBlock = 1024;

__global__ void __launch_bounds__(kIngestBlock) conv_ingest_kernel(const ConvDesc D, const ConvSlots S, const ConvUnits U,
                                                          const ConvParams P, const float* __restrict__ llr, int t0,
                                                          int npos, int gpad, int Gt) {
    __shared__ float tileS[64][65];
    const int ncols = npos * D.c;
    const int64_t ld = (int64_t)D.positions * D.c;
    const int c0 = blockIdx.x * 64, f0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll 4
    for (int r = ty; r < 64; r += kIngestBlock / 64) {
        const int g = f0 + r, cc = c0 + tx;
        float v = 0.0f;
        if (g < P.gamma && cc < ncols) v = llr[(size_t)g * ld + (int64_t)t0 * D.c + cc];
        tileS[r][tx] = v;
    }
    __syncthreads();
    const int nslots = (D.ms + 1) * D.Jb;
#pragma unroll 1
    for (int r = ty; r < 64; r += kIngestBlock / 64) {
        const int cc = c0 + r, g = f0 + tx;
        if (cc >= ncols || g >= gpad) continue;
        const int tile = g / Gt, fl = g - tile * Gt;
        const int pu = cc / D.c;
        const int rem = cc - pu * D.c;
        const int t = t0 + pu;
        const int q = rem / D.p, uu = rem - q * D.p;
        const int slot = t % U.ring;
        const float mu = tileS[tx][r] * kLog2eF;   // base-2 units
        P.mu[((size_t)tile * U.ring * D.c + (size_t)slot * D.c + rem) * Gt + fl] = mu;
        const float b = clip2(mu);
        const int jc = t % D.T;
        for (int k = 0; k < nslots; ++k) {
            const int dd = S.vn_dd[k], rr = S.vn_rr[k];
            if (t + dd >= D.layers) continue;
            int ic = jc + dd;
            while (ic >= D.T) ic -= D.T;
            const int a = sf_at(D, ic, dd, rr, q);
            if (a < 0) continue;
            int sidx = uu - a;
            if (sidx < 0) sidx += D.p;
            const int64_t pk = (int64_t)slot * U.eps + ((int64_t)((dd * D.Jb + rr) * D.Lb + q)) * D.p + sidx;
            P.msg[((size_t)tile * U.ring * U.eps + pk) * Gt + fl] = b;
        }
    }
}

// Sliding-window decoding with one workgroup per frame and the frame's ring
// in LDS: msg [R][eps] (the edge messages of the R = W + ms positions the
// window holds, in the ring layout of the launch-per-phase kernels with one
// frame per package) and mu [R][c].  A workgroup runs every slide of its
// frame: the entering positions are read from the caller's LLRs (mu, and
// beta = clip(mu) on their edges), then K flooding iterations (check rows of
// layers s..s+W-1, barrier, variable columns of positions s..s+W-1,
// barrier), and the last one writes position s to the caller's buffers.
// Everything about an edge except the row's (column's) offset within its
// circulant is shared by the p rows (columns) of that circulant, so it is
// worked out once per slide into small LDS tables: for check unit u and
// circulant row rr, the ring offset of edge slot e (or -1 where the edge
// does not exist); for variable unit u and circulant column q, the ring
// offset and shift of slot e.  The per-row and per-column arithmetic is that
// of conv_cn_kernel and conv_vn_column, in the same order, so the results
// are the same bit for bit.  Frames never interact and no workgroup waits
// for another.
constexpr int kWinBlock = 1024;
constexpr int kNoEdge = -(1 << 30);     // variable-edge table: no such edge
constexpr int kWinPre = 6;              // columns per thread whose packages are kept per slide

template <int DCMAX, int DVMAX>
__host__ __device__ constexpr size_t window_lds_tables(int W, int Jb, int Lb) {
    return (size_t)W * Jb * DCMAX + 2 * (size_t)W * Lb * DVMAX;
}

// a / b for 0 <= a < 2^22 and 0 < b: the float quotient is within one of
// the exact one, and one integer step corrects it
__device__ __forceinline__ int div_small(int a, int b, float inv_b) {
    int q = (int)((float)a * inv_b);
    const int r = a - q * b;
    q = r < 0 ? q - 1 : (r >= b ? q + 1 : q);
    return q;
}

// FIX: the host has checked that the block size is a multiple of the rows
// per layer and of the columns per position, so only the paths that split a
// thread's rows and columns once are compiled (fewer live registers).
template <int DCMAX, int DVMAX, bool FIX>
__global__ void __launch_bounds__(kWinBlock) window_lds_kernel(const ConvDesc D, const ConvSlots S, int R, int W,
                                                               int K, const float* __restrict__ llr,
                                                               float* __restrict__ post, uint8_t* __restrict__ bits_out) {
    extern __shared__ float lds[];
    // the shift table, indexed per lane below: from LDS, not from the
    // kernel arguments (a per-lane index into those becomes a memory load)
    __shared__ int sfl[LDPC_MAX_BLOCKS];
    const int nsf = D.T * (D.ms + 1) * D.Jb * D.Lb;
    for (int i = threadIdx.x; i < nsf; i += kWinBlock) sfl[i] = D.sf[i];
    auto sf = [&](int cls, int dd, int rr, int q) { return sfl[((cls * (D.ms + 1) + dd) * D.Jb + rr) * D.Lb + q]; };
    const int eps = (D.ms + 1) * D.Jb * D.Lb * D.p;
    float* msg = lds;
    float* mu = msg + (size_t)R * eps;
    int* ctab = reinterpret_cast<int*>(mu + (size_t)R * D.c);    // [W][Jb][DCMAX]
    int* vtab = ctab + (size_t)W * D.Jb * DCMAX;                  // [W][Lb][DVMAX]
    int* vsh = vtab + (size_t)W * D.Lb * DVMAX;                   // [W][Lb][DVMAX]
    const int64_t ld = (int64_t)D.positions * D.c;
    const size_t frame_off = (size_t)blockIdx.x * ld;
    const float* x = llr + frame_off;
    const int ncs = (D.ms + 1) * D.Lb;      // edge slots of a check row
    const int nvs = (D.ms + 1) * D.Jb;      // edge slots of a variable column
    const int per = D.Jb * D.p;             // check rows per layer
    int cdd[DCMAX], vdd[DVMAX];
#pragma unroll
    for (int e = 0; e < DCMAX; ++e) cdd[e] = S.cn_dd[e < ncs ? e : 0];
#pragma unroll
    for (int e = 0; e < DVMAX; ++e) vdd[e] = S.vn_dd[e < nvs ? e : 0];
    const float inv_per = 1.0f / (float)per, inv_p = 1.0f / (float)D.p, inv_c = 1.0f / (float)D.c;
    // When the block size is a multiple of the rows per layer (columns per
    // position), a thread's rows (columns) r = threadIdx.x + j * kWinBlock
    // all have the same offset within their layer (position) and consecutive
    // units kWinBlock / per apart: split once here.
    const bool rows_fixed = FIX || kWinBlock % per == 0, cols_fixed = FIX || kWinBlock % D.c == 0;
    const int rstep = rows_fixed ? kWinBlock / per : 1, cstep = cols_fixed ? kWinBlock / D.c : 1;
    const int ru0 = threadIdx.x / per, rrem0 = threadIdx.x - ru0 * per;
    const int rr0 = rrem0 / D.p, so0 = rrem0 - rr0 * D.p;
    const int cu0 = threadIdx.x / D.c, crem0 = threadIdx.x - cu0 * D.c;
    const int cq0 = crem0 / D.p, cuu0 = crem0 - cq0 * D.p;
    __syncthreads();
    for (int s = 0; s < D.positions; ++s) {
        const int lay_hi = min(s + W - 1, D.layers - 1);
        const int pos_hi = min(s + W - 1, D.positions - 1);
        const int in_lo = (s == 0) ? 0 : s + W - 1;
        const int ncu = lay_hi - s + 1, nvu = pos_hi - s + 1;
        if (in_lo <= pos_hi) {
            const int ncols = (pos_hi - in_lo + 1) * D.c;
            for (int i = threadIdx.x; i < ncols; i += kWinBlock) {
                const int pu = i / D.c;
                const int rem = i - pu * D.c;
                const int t = in_lo + pu;
                const int q = rem / D.p, uu = rem - q * D.p;
                const int slot = t % R;
                const float m = x[(int64_t)t * D.c + rem] * kLog2eF;   // base-2 units
                mu[slot * D.c + rem] = m;
                const float b = clip2(m);
                const int jc = t % D.T;
                for (int k = 0; k < nvs; ++k) {
                    const int dd = S.vn_dd[k], rr = S.vn_rr[k];
                    if (t + dd >= D.layers) continue;
                    int ic = jc + dd;
                    while (ic >= D.T) ic -= D.T;
                    const int a = sf(ic, dd, rr, q);
                    if (a < 0) continue;
                    int sidx = uu - a;
                    if (sidx < 0) sidx += D.p;
                    msg[slot * eps + ((dd * D.Jb + rr) * D.Lb + q) * D.p + sidx] = b;
                }
            }
        }
        // this slide's edge tables
        for (int i = threadIdx.x; i < ncu * D.Jb * DCMAX; i += kWinBlock) {
            const int e = i % DCMAX, ur = i / DCMAX;
            const int u = ur / D.Jb, rr = ur - u * D.Jb;
            int v = -1;
            if (e < ncs) {
                const int tau = s + u, dd = S.cn_dd[e], q = S.cn_q[e];
                const int tp = tau - dd;
                if (tp >= 0 && tp < D.positions && sf(tau % D.T, dd, rr, q) >= 0) {
                    int sl = tau % R - dd;
                    if (sl < 0) sl += R;
                    v = sl * eps + ((dd * D.Jb + rr) * D.Lb + q) * D.p;
                }
            }
            ctab[i] = v;
        }
        for (int i = threadIdx.x; i < nvu * D.Lb * DVMAX; i += kWinBlock) {
            const int e = i % DVMAX, uq = i / DVMAX;
            const int u = uq / D.Lb, q = uq - u * D.Lb;
            int v = kNoEdge, sh = 0;
            if (e < nvs) {
                const int tpos = s + u, dd = S.vn_dd[e], rr = S.vn_rr[e];
                int ic = tpos % D.T + dd;
                while (ic >= D.T) ic -= D.T;
                const int a = sf(ic, dd, rr, q);
                if (tpos + dd < D.layers && a >= 0) {
                    v = (tpos % R) * eps + ((dd * D.Jb + rr) * D.Lb + q) * D.p - a;
                    sh = a;
                }
            }
            vtab[i] = v;
            vsh[i] = sh;
        }
        __syncthreads();
        const int sR = s % R, span = lay_hi - s;
        // check row (unit u = layer s + u, circulant row rr, offset so)
        auto check_row = [&](int u, int rr, int so) {
            const int* tb = ctab + (u * D.Jb + rr) * DCMAX;
            if (DCMAX == ncs && u >= D.ms) {
                // every slot is an edge and none leads to a frozen position
                // (the row's circulants all exist): no per-edge tests
                int o[DCMAX];
#pragma unroll
                for (int e = 0; e < DCMAX; ++e) o[e] = tb[e];
                int any_missing = 0;      // all table reads first, then one test
#pragma unroll
                for (int e = 0; e < DCMAX; ++e) any_missing |= o[e];
                const bool full = any_missing >= 0;
                if (full) {
                    float in[DCMAX], t[DCMAX], q[DCMAX], mag[DCMAX];
                    uint32_t sgn = 0;
#pragma unroll
                    for (int e = 0; e < DCMAX; ++e) in[e] = msg[o[e] + so];
#pragma unroll
                    for (int e = 0; e < DCMAX; ++e) {
                        tq2_of(in[e], t[e], q[e]);
                        sgn ^= __float_as_uint(in[e]) & 0x80000000u;
                    }
                    boxplus2_fb<DCMAX>(t, q, mag);
#pragma unroll
                    for (int e = 0; e < DCMAX; ++e) {
                        const uint32_t sg = sgn ^ (__float_as_uint(in[e]) & 0x80000000u);
                        msg[o[e] + so] = __uint_as_float(__float_as_uint(mag[e]) | sg);
                    }
                    return;
                }
            }
            float in[DCMAX], t[DCMAX], q[DCMAX];
            int idx[DCMAX];
            uint32_t sgn = 0;
#pragma unroll
            for (int e = 0; e < DCMAX; ++e) {
                const int o = tb[e];
                idx[e] = o < 0 ? -1 : o + so;
                in[e] = o < 0 ? 0.0f : msg[o + so];
            }
#pragma unroll
            for (int e = 0; e < DCMAX; ++e) {
                if (idx[e] >= 0) {
                    tq2_of(in[e], t[e], q[e]);
                    sgn ^= __float_as_uint(in[e]) & 0x80000000u;
                } else {
                    t[e] = 1.0f;
                    q[e] = 0.0f;
                }
            }
            float mag[DCMAX];
            boxplus2_fb<DCMAX>(t, q, mag);
#pragma unroll
            for (int e = 0; e < DCMAX; ++e) {
                if (idx[e] >= 0 && u >= cdd[e]) {     // position s + u - dd is not frozen
                    const uint32_t sg = sgn ^ (__float_as_uint(in[e]) & 0x80000000u);
                    msg[idx[e]] = __uint_as_float(__float_as_uint(mag[e]) | sg);
                }
            }
        };
        // variable column (unit u = position s + u, circulant column q,
        // offset uu; rem = q * p + uu); the table holds the edge's ring
        // offset minus its shift, so the package is base + uu (+ p on wrap)
        auto variable_col = [&](int u, int q, int uu, int rem, bool out) {
            int slot = sR + u;
            if (slot >= R) slot -= R;
            const float m = mu[slot * D.c + rem];
            const int* tb = vtab + (u * D.Lb + q) * DVMAX;
            const int* shb = vsh + (u * D.Lb + q) * DVMAX;
            float a[DVMAX];
            int idx[DVMAX];
            if (DVMAX == nvs && u + D.ms <= span) {
                // every slot is an edge to a window layer: no per-edge tests
                int o[DVMAX], sh[DVMAX];
#pragma unroll
                for (int e = 0; e < DVMAX; ++e) {
                    o[e] = tb[e];
                    sh[e] = shb[e];
                }
                bool full = true;         // all table reads first, then one test
#pragma unroll
                for (int e = 0; e < DVMAX; ++e) {
                    idx[e] = o[e] + uu + (uu < sh[e] ? D.p : 0);
                    full = full & (o[e] != kNoEdge);
                }
                if (full) {
#pragma unroll
                    for (int e = 0; e < DVMAX; ++e) a[e] = msg[idx[e]];
                    float suf[DVMAX];
                    float Ssum = 0.0f;
#pragma unroll
                    for (int e = DVMAX - 1; e >= 0; --e) {
                        suf[e] = Ssum;
                        Ssum += a[e];
                    }
                    float pre = 0.0f;
#pragma unroll
                    for (int e = 0; e < DVMAX; ++e) {
                        const float b = clip2(m + (pre + suf[e]));
                        pre += a[e];
                        msg[idx[e]] = b;
                    }
                    if (out && u == 0) {
                        const float L = (m + pre) * kLn2F;
                        const size_t o = frame_off + (size_t)s * D.c + rem;
                        post[o] = clip30(L);
                        bits_out[o] = (uint8_t)(L < 0.0f);
                    }
                    return;
                }
            }
#pragma unroll
            for (int e = 0; e < DVMAX; ++e) {
                const int o = tb[e];
                const int i = o + uu + (uu < shb[e] ? D.p : 0);
                idx[e] = o == kNoEdge ? -1 : i;
                // only messages from window layers (s + u + dd <= lay_hi) are summed
                a[e] = (o != kNoEdge && u + vdd[e] <= span) ? msg[i] : 0.0f;
            }
            float suf[DVMAX];
            float Ssum = 0.0f;
#pragma unroll
            for (int e = DVMAX - 1; e >= 0; --e) {
                suf[e] = Ssum;
                Ssum += a[e];
            }
            float pre = 0.0f;
#pragma unroll
            for (int e = 0; e < DVMAX; ++e) {
                const float b = clip2(m + (pre + suf[e]));
                pre += a[e];
                if (idx[e] >= 0) msg[idx[e]] = b;
            }
            if (out && u == 0) {
                const float L = (m + pre) * kLn2F;
                const size_t o = frame_off + (size_t)s * D.c + rem;
                post[o] = clip30(L);
                bits_out[o] = (uint8_t)(L < 0.0f);
            }
        };
        // fixed columns (at most kWinPre per thread): each edge's package for
        // this slide, worked out once for the K iterations: >= 0 summed
        // (window layer), <= -2 written only (package -2 - v), -1 no edge
        // (compiled only for light rows and columns: the kept packages live
        // in registers through the check half too)
        constexpr bool kKeep = DVMAX <= 3 && DCMAX <= 6;
        const int ncol = cols_fixed ? (nvu - cu0 + cstep - 1) / cstep : 0;
        const bool pre = kKeep && cols_fixed && ncol <= kWinPre;
        int vix[kWinPre][DVMAX], mix[kWinPre];
        if constexpr (kKeep) {
            if (pre) {
#pragma unroll
                for (int j = 0; j < kWinPre; ++j) {
                    const int u = cu0 + j * cstep;
                    int slot = sR + u;
                    if (slot >= R) slot -= R;
                    mix[j] = slot * D.c + crem0;
                    const int* tb = vtab + (u * D.Lb + cq0) * DVMAX;
                    const int* shb = vsh + (u * D.Lb + cq0) * DVMAX;
#pragma unroll
                    for (int e = 0; e < DVMAX; ++e) {
                        int v = -1;
                        if (j < ncol) {
                            const int o = tb[e];
                            const int i = o + cuu0 + (cuu0 < shb[e] ? D.p : 0);
                            v = o == kNoEdge ? -1 : (u + vdd[e] <= span ? i : -2 - i);
                        }
                        vix[j][e] = v;
                    }
                }
            }
        }
        for (int k = 1; k <= K; ++k) {
            if (rows_fixed) {
                for (int u = ru0; u < ncu; u += rstep) check_row(u, rr0, so0);
            } else {
                for (int r = threadIdx.x; r < ncu * per; r += kWinBlock) {
                    const int u = div_small(r, per, inv_per);
                    const int rem = r - u * per;
                    const int rr = div_small(rem, D.p, inv_p);
                    check_row(u, rr, rem - rr * D.p);
                }
            }
            __syncthreads();
            bool kept = false;
            if constexpr (kKeep) {
                if (pre) {
                    kept = true;
#pragma unroll
                    for (int j = 0; j < kWinPre; ++j) {
                        if (j >= ncol) break;
                        const float m = mu[mix[j]];
                        float a[DVMAX];
#pragma unroll
                        for (int e = 0; e < DVMAX; ++e) a[e] = vix[j][e] >= 0 ? msg[vix[j][e]] : 0.0f;
                        float suf[DVMAX];
                        float Ssum = 0.0f;
#pragma unroll
                        for (int e = DVMAX - 1; e >= 0; --e) {
                            suf[e] = Ssum;
                            Ssum += a[e];
                        }
                        float pre_sum = 0.0f;
#pragma unroll
                        for (int e = 0; e < DVMAX; ++e) {
                            const float b = clip2(m + (pre_sum + suf[e]));
                            pre_sum += a[e];
                            const int v = vix[j][e];
                            if (v != -1) msg[v >= 0 ? v : -2 - v] = b;
                        }
                        if (k == K && cu0 + j * cstep == 0) {
                            const float L = (m + pre_sum) * kLn2F;
                            const size_t o = frame_off + (size_t)s * D.c + crem0;
                            post[o] = clip30(L);
                            bits_out[o] = (uint8_t)(L < 0.0f);
                        }
                    }
                }
            }
            if (!kept && cols_fixed) {
                for (int u = cu0; u < nvu; u += cstep) variable_col(u, cq0, cuu0, crem0, k == K);
            } else if (!kept) {
                for (int cidx = threadIdx.x; cidx < nvu * D.c; cidx += kWinBlock) {
                    const int u = div_small(cidx, D.c, inv_c);
                    const int rem = cidx - u * D.c;
                    const int q = div_small(rem, D.p, inv_p);
                    variable_col(u, q, rem - q * D.p, rem, k == K);
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// kernels: simulation (channel LLRs and error counts on the GPU, Sec. V-B)
// ---------------------------------------------------------------------------

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two
// 32x32->64-bit products with the multipliers 0xD2511F53 / 0xCD9E8D57; the
// key is bumped by 0x9E3779B9 / 0xBB67AE85 between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
    }
}

// Channel LLRs of the all-zero codeword over BPSK/AWGN (Sec. II-B):
// y = 1 + sigma z, mu = 2 y / sigma^2, for frames frame0 .. frame0+gamma-1.
// Thread = (frame f, block b of 4 bits): the counter (b, f mod 2^32, tag,
// f >> 32) gives four uniforms u = (w + 0.5) 2^-32 and two Box-Muller pairs
// r0 (cos, sin)(2 pi u1), r1 (cos, sin)(2 pi u3), r = sqrt(-2 ln u), in FP64.
__global__ void awgn_llr_kernel(float* __restrict__ llr, int64_t n, int gamma, uint64_t seed, int64_t frame0,
                                uint32_t tag, double sigma2) {
    const int64_t nblk = (n + 3) / 4;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nblk * gamma) return;
    const int64_t g = id / nblk, b = id - g * nblk;
    const uint64_t f = (uint64_t)(frame0 + g);
    uint32_t c[4] = {(uint32_t)b, (uint32_t)f, tag, (uint32_t)(f >> 32)};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double inv = 1.0 / 4294967296.0;
    const double two_pi = 6.283185307179586476925286766559;
    const double u0 = ((double)c[0] + 0.5) * inv, u1 = ((double)c[1] + 0.5) * inv;
    const double u2 = ((double)c[2] + 0.5) * inv, u3 = ((double)c[3] + 0.5) * inv;
    const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
    const double v[4] = {r0 * cos(two_pi * u1), r0 * sin(two_pi * u1), r1 * cos(two_pi * u3), r1 * sin(two_pi * u3)};
    const double sigma = sqrt(sigma2);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t i = 4 * b + q;
        if (i < n) llr[g * n + i] = (float)(2.0 * (1.0 + sigma * v[q]) / sigma2);
    }
}

// Bit errors against the all-zero codeword: per frame (one block per frame)
// and accumulated into totals[0] (bit errors) and totals[1] (frame errors).
__global__ void __launch_bounds__(256) count_errors_kernel(const uint8_t* __restrict__ bits, int64_t n,
                                                           int32_t* frame_errors, unsigned long long* totals) {
    __shared__ unsigned int part[4];
    const int g = blockIdx.x;
    const uint8_t* row = bits + (size_t)g * n;
    unsigned int cnt = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) cnt += row[i] != 0;
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int tot = part[0] + part[1] + part[2] + part[3];
        if (frame_errors) frame_errors[g] = (int32_t)tot;
        if (totals) {
            atomicAdd(totals, (unsigned long long)tot);
            if (tot) atomicAdd(totals + 1, 1ull);
        }
    }
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
thread_local bool suppressed = false;   // set while an entry point that must not create events runs
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

Scope::Scope(int cls, hipStream_t s) : st(s) {
    if (suppressed) return;
    std::lock_guard<std::mutex> g(mtx);
    if (!enabled) return;
    Rec r{cls, get_event(), get_event()};
    if (!r.a || !r.b) return;
    (void)hipEventRecord(r.a, st);
    recs.push_back(r);
    idx = (int)recs.size() - 1;
}

Scope::~Scope() {
    if (idx < 0) return;
    std::lock_guard<std::mutex> g(mtx);
    if (idx < (int)recs.size()) (void)hipEventRecord(recs[idx].b, st);
}

bool set_enabled(bool on) {
    std::lock_guard<std::mutex> g(mtx);
    const bool old = enabled;
    enabled = on;
    return old;
}
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
    size_t mu, msg, bits, postw, badw, flags, flag_words, total;   // flags: unsat words, then frozen words
};

static BlockLayout block_layout(const ldpc_graph* g, const Tiling& t, int max_iters) {
    BlockLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.mu = take((size_t)t.gpad * g->n * sizeof(float));
    L.msg = take((size_t)t.gpad * g->E * sizeof(float));
    L.bits = take((size_t)t.tiles * g->n * t.fpl * sizeof(uint64_t));
    L.postw = take((size_t)t.gpad * g->n * sizeof(float));   // early stopping: posteriors [tile][n][Gt]
    L.badw = take((size_t)t.tiles * g->m * t.fpl * sizeof(uint64_t));
    L.flag_words = (size_t)(max_iters + 1) * t.tiles * t.fpl;
    L.flags = take(2 * L.flag_words * sizeof(uint64_t));
    L.total = off;
    return L;
}

// Ring of code positions for the convolutional decoders (window: the W
// active positions plus the ms frozen ones; pipeline: the I (ms+1) frames held
// by the I processors).
struct ConvLayout {
    int R, eps;
    size_t mu, msg, total;
};

static ConvLayout conv_layout(const ldpc_graph* g, const Tiling& t, int ring) {
    ConvLayout L{};
    L.R = ring;
    L.eps = (g->ms + 1) * g->Jb * g->Lb * g->p;
    const int c = g->Lb * g->p;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.mu = take((size_t)t.gpad * L.R * c * sizeof(float));
    L.msg = take((size_t)t.gpad * L.R * L.eps * sizeof(float));
    L.total = off;
    return L;
}

// The pipelined decoder ingests kPipeAhead positions per ingest launch (one
// launch every kPipeAhead slots instead of one per slot).  Position x is
// decided at slot x + I(ms+1) - 1 and its ring slot is free from the next
// one, so a position ingested up to kPipeAhead - 1 slots early needs
// kPipeAhead - 1 extra ring slots.
constexpr int kPipeAhead = 8;

static int window_ring(const ldpc_graph* g, int W) { return std::min(W, g->positions) + g->ms; }
static int pipeline_ring(const ldpc_graph* g, int I) { return I * (g->ms + 1) + kPipeAhead - 1; }

static ConvSlots conv_slots(const ldpc_graph* g) {
    ConvSlots S{};
    for (int k = 0; k < (g->ms + 1) * g->Lb && k < LDPC_MAX_ROW_WEIGHT; ++k) {
        S.cn_dd[k] = (int8_t)(g->ms - k / g->Lb);
        S.cn_q[k] = (int8_t)(k % g->Lb);
    }
    for (int k = 0; k < (g->ms + 1) * g->Jb && k < LDPC_MAX_COL_WEIGHT; ++k) {
        S.vn_dd[k] = (int8_t)(k / g->Jb);
        S.vn_rr[k] = (int8_t)(k % g->Jb);
    }
    return S;
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
                      const Tiling& tl, hipStream_t st, const float* nms_w) {
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
    P.nms_w = nms_w;
    float* postw = reinterpret_cast<float*>(ws + lay.postw);
    P.badw = reinterpret_cast<uint64_t*>(ws + lay.badw);

    {
        timing::Scope ts(0, st);
        const dim3 grid = packages_grid(g->n, tl.gpad);
        to_packages_kernel<<<grid, kIngBlock, 0, st>>>(llr, g->n, 0, g->n, gamma, tl.gpad, tl.gt,
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
                if (nms_w)
                    cn_block_kernel<DC, FPL, 1><<<cn_grid, kBlock, 0, st>>>(D, P);
                else
                    cn_block_kernel<DC, FPL, 0><<<cn_grid, kBlock, 0, st>>>(D, P);
            });
        }
        if (early && it >= 2) {
            timing::Scope ts(3, st);
            const int chunks = (int)(((int64_t)D.m * FPL + kRedWords - 1) / kRedWords);
            unsat_reduce_kernel<FPL><<<(unsigned)(tl.tiles * chunks), 256, 0, st>>>(D, P, chunks);
        }
        {
            // the last pass of a fixed-iteration decode writes the outputs: timed as class 4
            timing::Scope ts(!early && P.last ? 4 : 2, st);
            if (early) {
                LDPC_DV_SWITCH(dvc, (vn_block_early_kernel<DV, FPL><<<vn_grid, kBlock, 0, st>>>(D, P, postw)));
            } else if (P.last) {
                LDPC_DV_SWITCH(dvc, (vn_block_out_kernel<DV, FPL><<<out_grid, kOutBlock, 0, st>>>(D, P, post, bits)));
            } else {
                LDPC_DV_SWITCH(dvc, (vn_block_kernel<DV, FPL><<<vn_grid, kBlock, 0, st>>>(D, P)));
            }
        }
    }
    if (early) {
        timing::Scope ts(4, st);
        dim3 grid((D.n + 63) / 64, (gamma + 63) / 64);
        block_output_kernel<FPL><<<grid, 256, 0, st>>>(postw, P.bits, D.n, gamma, post, bits);
    }
    P.iter = max_iters;
    {
        timing::Scope ts(3, st);
        const int bpt = (D.m + kBlock - 1) / kBlock;
        syndrome_kernel<FPL><<<(unsigned)((int64_t)bpt * tl.tiles), kBlock, 0, st>>>(D, P, bpt);
    }
    if (iters || converged) {
        timing::Scope ts(5, st);
        frame_status_kernel<FPL><<<(gamma + 255) / 256, 256, 0, st>>>(P, max_iters, iters, converged);
    }
}

// Learned min-sum training.  The T iterations form segments of k
// (ckpt_every); the last one may be shorter.  The workspace holds the
// packaged channel LLRs, the betas at the checkpoints k, 2k, ... (< T), the
// alphas and betas of the last segment (written by the forward pass, so the
// backward pass starts without recomputing), buffers for recomputing one
// other segment (k alphas, k - 1 betas), the gradient buffers, and the
// per-wave partial sums of the loss ([T][tiles n]) and of the gradient
// ([T][tiles m][dc_max] pairs: one per edge slot of a row).
struct TrainLayout {
    int k, nseg, nck, last;
    size_t arr, mu, ckpt, A, B, Al, Bl, dA, dB, lpart, gpart, total;
};

static TrainLayout train_layout(const ldpc_graph* g, const Tiling& t, int T, int k) {
    TrainLayout L{};
    L.k = k;
    L.nseg = (T + k - 1) / k;
    L.nck = L.nseg - 1;
    L.last = T - L.nck * k;
    L.arr = align256((size_t)t.gpad * g->E * sizeof(float));
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.mu = take((size_t)t.gpad * g->n * sizeof(float));
    L.ckpt = take(L.arr * L.nck);
    L.A = take(L.nseg > 1 ? L.arr * k : 0);
    L.B = take(L.nseg > 1 ? L.arr * (k - 1) : 0);
    L.Al = take(L.arr * L.last);
    L.Bl = take(L.arr * (L.last - 1));
    L.dA = take(L.arr);
    L.dB = take(L.arr);
    L.lpart = take((size_t)T * t.tiles * g->n * sizeof(float));
    L.gpart = take((size_t)T * t.tiles * g->m * g->dc_max * sizeof(float2));
    L.total = off;
    return L;
}

struct TrainRun {
    const ldpc_graph* g;
    QCDesc D;
    BlockParams P;
    TrainLayout L;
    Tiling tl;
    char* ws;
    hipStream_t st;
    int T;
    float inv_count;
    float* arr(size_t base, int i) const { return reinterpret_cast<float*>(ws + base + L.arr * (size_t)i); }
    // beta at checkpoint iteration c (c = 0: the channel LLRs, read from mu)
    float* ckpt(int c) const { return c == 0 ? nullptr : arr(L.ckpt, c / L.k - 1); }
};

static TrainRun make_train_run(const ldpc_graph* g, int gamma, int T, int k, const float* w, char* ws,
                               const Tiling& tl, hipStream_t st) {
    TrainRun r{};
    r.g = g;
    r.D = g->qc;
    r.L = train_layout(g, tl, T, k);
    r.tl = tl;
    r.ws = ws;
    r.st = st;
    r.T = T;
    r.inv_count = (float)(1.0 / ((double)gamma * g->n));
    r.P.mu = reinterpret_cast<const float*>(ws + r.L.mu);
    r.P.gamma = gamma;
    r.P.tiles = tl.tiles;
    r.P.nms_w = w;
    return r;
}

template <int FPL>
static void train_cn(TrainRun& r, int t, const float* src, float* dst) {
    r.P.iter = t;
    const unsigned grid = grid_for_waves((int64_t)r.D.m * r.tl.tiles);
    timing::Scope ts(12, r.st);
    LDPC_DC_SWITCH(dc_class(r.D.dc_max), if constexpr (DC <= MaxDC<FPL>::value) {
        nms_train_cn_kernel<DC, FPL><<<grid, kBlock, 0, r.st>>>(r.D, r.P, src, dst);
    });
}

template <int FPL>
static void train_vn(TrainRun& r, int t, const float* A, float* dst, bool with_loss) {
    r.P.iter = t;
    const int64_t waves = (int64_t)r.D.n * r.tl.tiles;
    float* lpart = with_loss ? reinterpret_cast<float*>(r.ws + r.L.lpart) + (size_t)(t - 1) * waves : nullptr;
    timing::Scope ts(13, r.st);
    LDPC_DV_SWITCH(dv_class(r.D.dv_max), (nms_train_vn_kernel<DV, FPL><<<grid_for_waves(waves), kBlock, 0, r.st>>>(
                                             r.D, r.P, A, dst, lpart, r.inv_count)));
}

template <int FPL>
static void train_forward(TrainRun& r, const float* llr, float* loss) {
    {
        timing::Scope ts(0, r.st);
        const dim3 grid = packages_grid(r.g->n, r.tl.gpad);
        to_packages_kernel<<<grid, kIngBlock, 0, r.st>>>(llr, r.g->n, 0, r.g->n, r.P.gamma, r.tl.gpad, r.tl.gt,
                                                   reinterpret_cast<float*>(r.ws + r.L.mu),
                                                   (int64_t)r.g->n * r.tl.gt, nullptr, 0);
    }
    const int cl = r.L.nck * r.L.k;     // the last segment holds iterations cl+1 .. T
    const float* src = nullptr;
    for (int t = 1; t <= r.T; ++t) {
        float* A;
        float* dst = nullptr;
        if (t > cl) {
            A = r.arr(r.L.Al, t - cl - 1);
            if (t < r.T) dst = r.arr(r.L.Bl, t - cl - 1);
        } else {
            A = r.arr(r.L.A, 0);
            dst = (t % r.L.k == 0) ? r.ckpt(t) : r.arr(r.L.B, 0);
        }
        train_cn<FPL>(r, t, src, A);
        train_vn<FPL>(r, t, A, dst, true);
        src = dst;
    }
    timing::Scope ts(16, r.st);
    nms_loss_reduce_kernel<<<r.T, 256, 0, r.st>>>(reinterpret_cast<const float*>(r.ws + r.L.lpart),
                                                  (int64_t)r.D.n * r.tl.tiles, loss);
}

template <int FPL>
static void train_backward(TrainRun& r, const float* dloss, float* grad) {
    const QCDesc& D = r.D;
    const int k = r.L.k;
    float* dA = r.arr(r.L.dA, 0);
    float* dB = r.arr(r.L.dB, 0);
    float2* gpart = reinterpret_cast<float2*>(r.ws + r.L.gpart);
    const unsigned cn_grid = grid_for_waves((int64_t)D.m * r.tl.tiles);
    const unsigned vn_grid = grid_for_waves((int64_t)D.n * r.tl.tiles);
    const int dcc = dc_class(D.dc_max), dvc = dv_class(D.dv_max);
    const int cl = r.L.nck * k;
    for (int c = cl; c >= 0; c -= k) {
        const int e = std::min(c + k, r.T);
        // the last segment's alphas and betas are the forward pass's; any other
        // segment's are recomputed from its checkpoint (alphas c+1..e, betas
        // c+1..e-1)
        const size_t Abuf = c == cl ? r.L.Al : r.L.A, Bbuf = c == cl ? r.L.Bl : r.L.B;
        if (c != cl) {
            const float* src = r.ckpt(c);
            for (int t = c + 1; t <= e; ++t) {
                float* A = r.arr(Abuf, t - c - 1);
                train_cn<FPL>(r, t, src, A);
                float* dst = t < e ? r.arr(Bbuf, t - c - 1) : nullptr;
                train_vn<FPL>(r, t, A, dst, false);
                src = dst;
            }
        }
        for (int t = e; t > c; --t) {
            r.P.iter = t;
            {
                timing::Scope ts(14, r.st);
                const float* A = r.arr(Abuf, t - c - 1);
                const float* dBin = t == r.T ? nullptr : dB;
                LDPC_DV_SWITCH(dvc, (nms_vn_backward_kernel<DV, FPL><<<vn_grid, kBlock, 0, r.st>>>(
                                        D, r.P, A, dBin, dA, dloss, r.inv_count)));
            }
            {
                timing::Scope ts(15, r.st);
                const float* bsrc = t == c + 1 ? r.ckpt(c) : r.arr(Bbuf, t - c - 2);
                float* dBout = t == 1 ? nullptr : dB;
                float2* part = gpart + (size_t)(t - 1) * r.tl.tiles * D.m * D.dc_max;
                LDPC_DC_SWITCH(dcc, if constexpr (DC <= MaxDC<FPL>::value) {
                    nms_cn_backward_kernel<DC, FPL><<<cn_grid, kBlock, 0, r.st>>>(D, r.P, bsrc, dA, dBout, part);
                });
            }
        }
    }
    timing::Scope ts(16, r.st);
    nms_grad_reduce_kernel<<<dim3(D.nb, r.T), 256, 0, r.st>>>(D, gpart, r.tl.tiles, grad);
}

// host-side helpers for the convolutional schedules
struct ConvRun {
    const ldpc_graph* g;
    ConvDesc D;
    ConvSlots S;
    ConvParams P;
    ConvLayout lay;
    Tiling tl;
    int dcc, dvc;
    hipStream_t st;
    const float* llr;
    float* post;
    uint8_t* bits;
    int cls_ingest, cls_cn, cls_vn;

    void unit(ConvUnits& U, int pos, int lo, int hi) const {
        const int u = U.n++;
        U.pos[u] = pos;
        U.slot[u] = pos % lay.R;
        U.cls[u] = pos % D.T;
        U.lo[u] = lo;
        U.hi[u] = hi;
    }
    ConvUnits units() const {
        ConvUnits U{};
        U.ring = lay.R;
        U.eps = lay.eps;
        U.out_unit = -1;
        return U;
    }

    template <int FPL>
    void ingest(int t0, int npos) const {
        timing::Scope ts(cls_ingest, st);
        ConvUnits U = units();
        dim3 grid((npos * D.c + 63) / 64, tl.gpad / 64);
        conv_ingest_kernel<<<grid, kIngestBlock, 0, st>>>(D, S, U, P, llr, t0, npos, tl.gpad, tl.gt);
    }

    template <int FPL>
    void check(const ConvUnits& U) const {
        if (U.n == 0) return;
        timing::Scope ts(cls_cn, st);
        ConvParams Pc = P;
        Pc.rows = U.n * D.Jb * D.p;
        LDPC_DC_SWITCH(dcc, if constexpr (DC <= MaxDC<FPL>::value) {
            conv_cn_kernel<DC, FPL><<<grid_for_waves((int64_t)Pc.rows * tl.tiles), kBlock, 0, st>>>(D, S, U, Pc);
        });
    }

    template <int FPL>
    void variable(const ConvUnits& U) const {
        if (U.n == 0) return;
        timing::Scope ts(cls_vn, st);
        ConvParams Pv = P;
        Pv.rows = U.n * D.c;
        if (U.out_unit >= 0) {
            const int out_blocks = ((D.c + kOutVars - 1) / kOutVars) * tl.tiles;
            const int64_t plain_waves = (int64_t)(Pv.rows - D.c) * tl.tiles;
            const unsigned grid = (unsigned)(out_blocks + (plain_waves + kOutBlock / 64 - 1) / (kOutBlock / 64));
            LDPC_DV_SWITCH(dvc, (conv_vn_out_kernel<DV, FPL>
                                 <<<grid, kOutBlock, 0, st>>>(D, S, U, Pv, post, bits, out_blocks)));
        } else {
            LDPC_DV_SWITCH(dvc, (conv_vn_kernel<DV, FPL>
                                 <<<grid_for_waves((int64_t)Pv.rows * tl.tiles), kBlock, 0, st>>>(D, S, U, Pv)));
        }
    }
};

static ConvRun make_conv_run(const ldpc_graph* g, const float* llr, int gamma, float* post, uint8_t* bits, char* ws,
                             const ConvLayout& lay, const Tiling& tl, hipStream_t st) {
    ConvRun r{};
    r.g = g;
    r.D = g->cv;
    r.S = conv_slots(g);
    r.P.msg = reinterpret_cast<float*>(ws + lay.msg);
    r.P.mu = reinterpret_cast<float*>(ws + lay.mu);
    r.P.tiles = tl.tiles;
    r.P.gamma = gamma;
    r.lay = lay;
    r.tl = tl;
    // edges are enumerated by syndrome-former slot, zero blocks included
    r.dcc = dc_class((g->ms + 1) * g->Lb);
    r.dvc = dv_class((g->ms + 1) * g->Jb);
    r.st = st;
    r.llr = llr;
    r.post = post;
    r.bits = bits;
    return r;
}

// Sliding window (target position s = 0 .. positions-1): window layers
// s..s+W-1, active positions s..s+W-1; entering positions start from
// beta = clip(mu); K flooding iterations; position s decided at the end.
template <int FPL>
static void run_window(ConvRun& r, int Wlen, int K) {
    const ConvDesc& D = r.D;
    r.cls_ingest = 6;
    r.cls_cn = 7;
    r.cls_vn = 8;
    for (int s = 0; s < D.positions; ++s) {
        const int lay_hi = std::min(s + Wlen - 1, D.layers - 1);
        const int pos_hi = std::min(s + Wlen - 1, D.positions - 1);
        const int in_lo = (s == 0) ? 0 : s + Wlen - 1;
        if (in_lo <= pos_hi) r.ingest<FPL>(in_lo, pos_hi - in_lo + 1);
        ConvUnits Uc = r.units();
        for (int tau = s; tau <= lay_hi; ++tau) r.unit(Uc, tau, s, 0);
        ConvUnits Uv = r.units();
        for (int t = s; t <= pos_hi; ++t) r.unit(Uv, t, s, lay_hi);
        for (int k = 1; k <= K; ++k) {
            r.check<FPL>(Uc);
            Uv.out_unit = (k == K) ? 0 : -1;
            r.variable<FPL>(Uv);
        }
    }
}

// Pipelined decoder of Algorithm 2 with I processors: at slot t, frame t
// enters (ingested with the next kPipeAhead - 1 at slots that are multiples
// of kPipeAhead); processor i updates check layer t - (i-1)(ms+1), then
// frame t - (i-1)(ms+1) - ms; the frame leaving processor I is decided.
template <int FPL>
static void run_pipeline(ConvRun& r, int I) {
    const ConvDesc& D = r.D;
    r.cls_ingest = 9;
    r.cls_cn = 10;
    r.cls_vn = 11;
    const int last_slot = D.positions - 1 + D.ms + (I - 1) * (D.ms + 1);
    for (int t = 0; t <= last_slot; ++t) {
        if (t < D.positions && t % kPipeAhead == 0) r.ingest<FPL>(t, std::min(kPipeAhead, D.positions - t));
        ConvUnits Uc = r.units();
        ConvUnits Uv = r.units();
        for (int i = 1; i <= I; ++i) {
            const int tau = t - (i - 1) * (D.ms + 1);
            if (tau >= 0 && tau < D.layers) r.unit(Uc, tau, 0, 0);
            const int f = tau - D.ms;
            if (f >= 0 && f < D.positions) {
                if (i == I) Uv.out_unit = Uv.n;
                r.unit(Uv, f, 0, D.layers - 1);
            }
        }
        r.check<FPL>(Uc);
        r.variable<FPL>(Uv);
    }
}

// The window decoder with one workgroup per stream and its ring in LDS
// (window_lds_kernel), when the ring fits the device's LDS per workgroup and
// the row / column weights have an instantiation; false if the caller must
// use the launch-per-phase form (nothing enqueued then).
template <int DC, int DV>
static bool launch_window_lds(const ldpc_graph* g, const float* llr, int gamma, int W, int K, float* post,
                              uint8_t* bits, int R, size_t bytes, hipStream_t st) {
    // bytes: the ring; the edge tables are added here
    bytes += window_lds_tables<DC, DV>(W, g->Jb, g->Lb) * sizeof(int);
    int dev = 0, limit = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (bytes + LDPC_MAX_BLOCKS * sizeof(int) > (size_t)limit) return false;
    // row and column indices of a window stay below 2^22 (div_small)
    const int wl = std::min(W, g->positions + g->ms);
    if ((int64_t)wl * std::max(g->Jb, g->Lb) * g->p >= ((int64_t)1 << 22)) return false;
    const bool fix = kWinBlock % (g->Jb * g->p) == 0 && kWinBlock % (g->Lb * g->p) == 0;
    const void* fn = fix ? reinterpret_cast<const void*>(&window_lds_kernel<DC, DV, true>)
                         : reinterpret_cast<const void*>(&window_lds_kernel<DC, DV, false>);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    timing::Scope ts(21, st);
    if (fix)
        window_lds_kernel<DC, DV, true><<<(unsigned)gamma, kWinBlock, bytes, st>>>(g->cv, conv_slots(g), R, W, K, llr,
                                                                                   post, bits);
    else
        window_lds_kernel<DC, DV, false><<<(unsigned)gamma, kWinBlock, bytes, st>>>(g->cv, conv_slots(g), R, W, K,
                                                                                    llr, post, bits);
    return true;
}

static bool window_lds(const ldpc_graph* g, const float* llr, int gamma, int W, int K, float* post, uint8_t* bits,
                       hipStream_t st) {
    const char* env = std::getenv("LDPC_WINDOW_PATH");
    if (env && std::strcmp(env, "launch") == 0) return false;
    const int R = window_ring(g, W);
    const size_t eps = (size_t)(g->ms + 1) * g->Jb * g->Lb * g->p;
    const size_t c = (size_t)g->Lb * g->p;
    const size_t bytes = (size_t)R * (eps + c) * sizeof(float);
    const int dcc = dc_class((g->ms + 1) * g->Lb), dvc = dv_class((g->ms + 1) * g->Jb);
    if (dcc > 8 || dvc > 4) return false;
    bool done = false;
    switch (dcc) {
        case 4: LDPC_DV_SWITCH(dvc, if constexpr (DV <= 4) {
                    done = launch_window_lds<4, DV>(g, llr, gamma, W, K, post, bits, R, bytes, st);
                }); break;
        case 6: LDPC_DV_SWITCH(dvc, if constexpr (DV <= 4) {
                    done = launch_window_lds<6, DV>(g, llr, gamma, W, K, post, bits, R, bytes, st);
                }); break;
        default: LDPC_DV_SWITCH(dvc, if constexpr (DV <= 4) {
                    done = launch_window_lds<8, DV>(g, llr, gamma, W, K, post, bits, R, bytes, st);
                }); break;
    }
    return done;
}

}  // namespace ldpc

using namespace ldpc;

extern "C" {

ldpc_status ldpc_workspace_size(const ldpc_graph* g, int32_t gamma, int32_t max_iters, int32_t window,
                                size_t* bytes) {
    if (!g || !bytes || gamma < 1 || max_iters < 1 || max_iters > LDPC_MAX_ITERS || window < 0)
        return LDPC_EINVAL;
    const Tiling tl = choose_tiling(gamma, g);
    if (g->kind == LDPC_GRAPH_QC) {
        if (window != 0) return LDPC_EUNSUPPORTED;
        *bytes = block_layout(g, tl, max_iters).total;
    } else if (window == 0) {
        if (max_iters > kMaxUnits) return LDPC_EUNSUPPORTED;
        *bytes = conv_layout(g, tl, pipeline_ring(g, max_iters)).total;
    } else {
        if (window < g->ms + 1) return LDPC_EINVAL;
        if (window > kMaxUnits) return LDPC_EUNSUPPORTED;
        *bytes = conv_layout(g, tl, window_ring(g, window)).total;
    }
    return LDPC_OK;
}

static bool packages_forced() {
    const char* path = std::getenv("LDPC_BLOCK_PATH");
    return path && std::strcmp(path, "packages") == 0;
}

static ldpc_status decode_block(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t max_iters,
                                int32_t early_stop, float* post, uint8_t* bits, int32_t* iters, uint8_t* converged,
                                void* workspace, size_t workspace_bytes, void* stream, const float* nms_w) {
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
    // decodes of codes that fit one compute unit run on chip (onchip.hip),
    // sum-product and learned min-sum alike; LDPC_BLOCK_PATH=packages keeps
    // them on this decoder
    if (!packages_forced()) {
        const int r = onchip_decode(g, llr, gamma, max_iters, early_stop ? 1 : 0, post, bits, iters, converged, st,
                                    nms_w);
        if (r != 0) return r > 0 && hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
    }
    switch (tl.fpl) {
        case 4: run_block<4>(g, llr, gamma, max_iters, early_stop ? 1 : 0, post, bits, iters, converged, ws, lay, tl, st, nms_w); break;
        case 2: run_block<2>(g, llr, gamma, max_iters, early_stop ? 1 : 0, post, bits, iters, converged, ws, lay, tl, st, nms_w); break;
        default: run_block<1>(g, llr, gamma, max_iters, early_stop ? 1 : 0, post, bits, iters, converged, ws, lay, tl, st, nms_w); break;
    }
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

static ldpc_status conv_checks(const ldpc_graph* g, const float* llr, int32_t gamma, const float* post,
                               const uint8_t* bits) {
    if (!g || !llr || !post || !bits) return LDPC_EINVAL;
    if (g->kind != LDPC_GRAPH_CONV || gamma < 1) return LDPC_EINVAL;
    if ((int64_t)gamma * g->n > ((int64_t)1 << 40)) return LDPC_EUNSUPPORTED;
    if ((reinterpret_cast<uintptr_t>(llr) | reinterpret_cast<uintptr_t>(post)) & 3) return LDPC_EINVAL;
    return LDPC_OK;
}

ldpc_status ldpc_decode(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t max_iters, int32_t early_stop,
                        float* post, uint8_t* bits, int32_t* iters, uint8_t* converged, void* workspace,
                        size_t workspace_bytes, void* stream) {
    return decode_block(g, llr, gamma, max_iters, early_stop, post, bits, iters, converged, workspace, workspace_bytes,
                        stream, nullptr);
}

ldpc_status ldpc_decode_path(const ldpc_graph* g, int32_t* onchip) {
    if (!g || !onchip || g->kind != LDPC_GRAPH_QC) return LDPC_EINVAL;
    *onchip = (!packages_forced() && onchip_fits(g)) ? 1 : 0;
    return LDPC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Decoding without allocation.  The workspace of ldpc_decode_noalloc is this
// static device array: every device the library runs on holds one copy of
// it, at its own address, until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol); it looks up each device's address once with hipGetSymbolAddress
// and uses that.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[LDPC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex scratch_mtx;
void* scratch_addr[kScratchDevices];

// address of the current device's copy (looked up at the first call on it)
ldpc_status scratch_for_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return LDPC_EHIP;
    }
    if (dev < 0 || dev >= kScratchDevices) return LDPC_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(scratch_mtx);
    if (!scratch_addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return LDPC_EHIP;
        }
        scratch_addr[dev] = p;
    }
    *out = scratch_addr[dev];
    return LDPC_OK;
}

struct NoTimingEvents {
    bool was = timing::suppressed;
    NoTimingEvents() { timing::suppressed = true; }
    ~NoTimingEvents() { timing::suppressed = was; }
};
}  // namespace

extern "C" {

ldpc_status ldpc_decode_noalloc(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t max_iters,
                                int32_t early_stop, float* post, uint8_t* bits, int32_t* iters, uint8_t* converged,
                                void* stream) {
    if (!g || !llr || !post || !bits) return LDPC_EINVAL;
    if (g->kind != LDPC_GRAPH_QC) return LDPC_EINVAL;
    if (gamma < 1 || max_iters < 1 || max_iters > LDPC_MAX_ITERS) return LDPC_EINVAL;
    if ((int64_t)gamma * g->n > ((int64_t)1 << 40)) return LDPC_EUNSUPPORTED;
    const size_t need = block_layout(g, choose_tiling(gamma, g), max_iters).total;
    if (need > (size_t)LDPC_NOALLOC_SCRATCH_BYTES) return LDPC_EWORKSPACE;
    void* ws = nullptr;
    const ldpc_status got = scratch_for_current_device(&ws);
    if (got != LDPC_OK) return got;
    NoTimingEvents quiet;
    return decode_block(g, llr, gamma, max_iters, early_stop, post, bits, iters, converged, ws,
                        (size_t)LDPC_NOALLOC_SCRATCH_BYTES, stream, nullptr);
}

ldpc_status ldpc_nms_decode(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t iters, const float* weights,
                            int32_t early_stop, float* post, uint8_t* bits, int32_t* iters_out, uint8_t* converged,
                            void* workspace, size_t workspace_bytes, void* stream) {
    if (!weights) return LDPC_EINVAL;
    return decode_block(g, llr, gamma, iters, early_stop, post, bits, iters_out, converged, workspace,
                        workspace_bytes, stream, weights);
}

static ldpc_status train_checks(const ldpc_graph* g, int32_t gamma, int32_t iters, int32_t ckpt_every) {
    if (!g || g->kind != LDPC_GRAPH_QC) return LDPC_EINVAL;
    if (gamma < 1 || iters < 1 || iters > LDPC_MAX_ITERS || ckpt_every < 1 || ckpt_every > iters) return LDPC_EINVAL;
    if ((int64_t)gamma * g->n > ((int64_t)1 << 40)) return LDPC_EUNSUPPORTED;
    return LDPC_OK;
}

ldpc_status ldpc_nms_train_workspace_size(const ldpc_graph* g, int32_t gamma, int32_t iters, int32_t ckpt_every,
                                          size_t* bytes) {
    ldpc_status chk = train_checks(g, gamma, iters, ckpt_every);
    if (chk != LDPC_OK) return chk;
    if (!bytes) return LDPC_EINVAL;
    *bytes = train_layout(g, choose_tiling(gamma, g), iters, ckpt_every).total;
    return LDPC_OK;
}

ldpc_status ldpc_nms_train_forward(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t iters,
                                   int32_t ckpt_every, const float* weights, float* loss, void* workspace,
                                   size_t workspace_bytes, void* stream) {
    ldpc_status chk = train_checks(g, gamma, iters, ckpt_every);
    if (chk != LDPC_OK) return chk;
    if (!llr || !weights || !loss) return LDPC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(llr) | reinterpret_cast<uintptr_t>(weights) |
         reinterpret_cast<uintptr_t>(loss)) & 3)
        return LDPC_EINVAL;
    const Tiling tl = choose_tiling(gamma, g);
    const TrainLayout lay = train_layout(g, tl, iters, ckpt_every);
    if (!workspace || workspace_bytes < lay.total) return LDPC_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return LDPC_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    TrainRun r = make_train_run(g, gamma, iters, ckpt_every, weights, reinterpret_cast<char*>(workspace), tl, st);
    (void)hipGetLastError();
    switch (tl.fpl) {
        case 4: train_forward<4>(r, llr, loss); break;
        case 2: train_forward<2>(r, llr, loss); break;
        default: train_forward<1>(r, llr, loss); break;
    }
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

ldpc_status ldpc_nms_train_backward(const ldpc_graph* g, int32_t gamma, int32_t iters, int32_t ckpt_every,
                                    const float* weights, const float* dloss, float* grad, void* workspace,
                                    size_t workspace_bytes, void* stream) {
    ldpc_status chk = train_checks(g, gamma, iters, ckpt_every);
    if (chk != LDPC_OK) return chk;
    if (!weights || !dloss || !grad) return LDPC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(weights) | reinterpret_cast<uintptr_t>(dloss) |
         reinterpret_cast<uintptr_t>(grad)) & 3)
        return LDPC_EINVAL;
    const Tiling tl = choose_tiling(gamma, g);
    const TrainLayout lay = train_layout(g, tl, iters, ckpt_every);
    if (!workspace || workspace_bytes < lay.total) return LDPC_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return LDPC_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    TrainRun r = make_train_run(g, gamma, iters, ckpt_every, weights, reinterpret_cast<char*>(workspace), tl, st);
    (void)hipGetLastError();
    switch (tl.fpl) {
        case 4: train_backward<4>(r, dloss, grad); break;
        case 2: train_backward<2>(r, dloss, grad); break;
        default: train_backward<1>(r, dloss, grad); break;
    }
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

ldpc_status ldpc_decode_window(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t W,
                               int32_t iters_per_window, float* post, uint8_t* bits, void* workspace,
                               size_t workspace_bytes, void* stream) {
    ldpc_status chk = conv_checks(g, llr, gamma, post, bits);
    if (chk != LDPC_OK) return chk;
    if (iters_per_window < 1 || iters_per_window > LDPC_MAX_ITERS || W < g->ms + 1) return LDPC_EINVAL;
    if (W > kMaxUnits) return LDPC_EUNSUPPORTED;
    const Tiling tl = choose_tiling(gamma, g);
    const ConvLayout lay = conv_layout(g, tl, window_ring(g, W));
    if (!workspace || workspace_bytes < lay.total) return LDPC_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return LDPC_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    if (window_lds(g, llr, gamma, W, iters_per_window, post, bits, st))
        return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
    ConvRun r = make_conv_run(g, llr, gamma, post, bits, reinterpret_cast<char*>(workspace), lay, tl, st);
    switch (tl.fpl) {
        case 4: run_window<4>(r, W, iters_per_window); break;
        case 2: run_window<2>(r, W, iters_per_window); break;
        default: run_window<1>(r, W, iters_per_window); break;
    }
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

ldpc_status ldpc_decode_pipeline(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t iters, float* post,
                                 uint8_t* bits, void* workspace, size_t workspace_bytes, void* stream) {
    ldpc_status chk = conv_checks(g, llr, gamma, post, bits);
    if (chk != LDPC_OK) return chk;
    if (iters < 1 || iters > LDPC_MAX_ITERS) return LDPC_EINVAL;
    if (iters > kMaxUnits) return LDPC_EUNSUPPORTED;
    const Tiling tl = choose_tiling(gamma, g);
    const ConvLayout lay = conv_layout(g, tl, pipeline_ring(g, iters));
    if (!workspace || workspace_bytes < lay.total) return LDPC_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return LDPC_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    ConvRun r = make_conv_run(g, llr, gamma, post, bits, reinterpret_cast<char*>(workspace), lay, tl, st);
    (void)hipGetLastError();
    switch (tl.fpl) {
        case 4: run_pipeline<4>(r, iters); break;
        case 2: run_pipeline<2>(r, iters); break;
        default: run_pipeline<1>(r, iters); break;
    }
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

ldpc_status ldpc_awgn_llr(int64_t n, int32_t gamma, double sigma2, uint64_t seed, int64_t frame0, float* llr,
                          void* stream) {
    if (!llr || n < 1 || gamma < 1 || !(sigma2 > 0.0) || frame0 < 0) return LDPC_EINVAL;
    if (n > ((int64_t)1 << 31) || (int64_t)gamma * n > ((int64_t)1 << 40)) return LDPC_EUNSUPPORTED;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t threads = (n + 3) / 4 * gamma;
    (void)hipGetLastError();
    awgn_llr_kernel<<<(unsigned)((threads + 255) / 256), 256, 0, st>>>(llr, n, gamma, seed, frame0, 0x4E5Au, sigma2);
    return hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

ldpc_status ldpc_count_errors(const uint8_t* bits, int32_t gamma, int64_t n, int32_t* frame_errors,
                              uint64_t* totals, void* stream) {
    if (!bits || gamma < 1 || n < 1 || (!frame_errors && !totals)) return LDPC_EINVAL;
    if (reinterpret_cast<uintptr_t>(totals) & 7) return LDPC_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    count_errors_kernel<<<gamma, 256, 0, st>>>(bits, n, frame_errors, reinterpret_cast<unsigned long long*>(totals));
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
    static const char* names[LDPC_TIMING_CLASSES] = {
        "ingest",          "check_node",        "variable_node",        "syndrome",
        "output",          "frame_status",      "window_ingest",        "window_check_node",
        "window_variable_node", "pipeline_ingest", "pipeline_check_node", "pipeline_variable_node",
        "train_check_node", "train_variable_node", "train_variable_node_backward", "train_check_node_backward",
        "train_reduce", "plan_ingest", "plan_check_node", "plan_variable_node", "plan_finish",
        "window_lds", "plan_persistent", "onchip_decode"};
    if (cls < 0 || cls >= LDPC_TIMING_CLASSES) return "unknown";
    return names[cls];
}

}  // extern "C"
