// Block decoder with a whole frame on one compute unit (gfx950).
//
// The message-package decoder of decode.hip streams every edge message
// through HBM twice per iteration, so it can never run faster than HBM
// bandwidth allows (52 bytes per coded bit per iteration for a (3,6) code).
// One frame of a code of moderate length fits on a single CU: for the
// (3,6) code with p = 3060 its 55,080 check-to-variable messages are 215 KB
// against a 512 KB register file, and its posterior sums are 72 KB against
// 160 KB of LDS.  Here one workgroup decodes one frame from start to end:
//
//   * thread i owns check rows (j, i + q*TB) of every base row j (q < NQ) and
//     keeps the check-to-variable messages alpha of those rows' edges in
//     registers for the whole decode;
//   * LDS holds, for every variable, the posterior sum L = mu + sum alpha
//     (Eq. 5) of two consecutive iterations;
//   * the variable-to-check message of an edge is recovered as
//     beta = clip(L_v - alpha_e) (Eq. 4 written as "all but the own edge")
//     from the previous iteration's sum and the edge's own alpha, so no beta
//     is stored;
//   * the check update (Eq. 3) is the FP32 (t, 1 - t) forward-backward form
//     of the package decoder, in base-2 units (check2.h), with each input's
//     pair left unnormalised (check2u_row: no reciprocal per input).
//
// One iteration, for base rows j = 0 .. J-1 in turn (a workgroup barrier
// after each): every thread updates its rows of base row j from L_old
// (the previous iteration's sums) and adds the new alphas into L_new.  A
// weight-1 circulant block joins each variable of its base column to exactly
// one row of its base row, so within one base row no two threads touch the
// same variable and the additions need no atomics; the base-row order fixes
// the order of every sum, so results are deterministic.  The lowest nonzero
// block of each base column starts its variables' sums from mu (held in
// registers for regular bases, whose columns are stored rotated by base row
// 0's shifts; else read from the caller's LLR array, which stays in L2).
// HBM traffic per frame is the
// channel LLRs in and the outputs out; the decode is bound by the vector
// ALUs (the transcendentals of Eq. 3).
//
// Early stopping: the syndrome of iteration i-1 is computed in iteration i
// from the signs of L_old that the check update reads anyway; each wave ORs
// its verdict into an LDS flag before the last barrier of the iteration, and
// every thread reads the flag after it.  A zero syndrome ends the decode with
// the outputs of iteration i-1, which are still in L_old (iteration i wrote
// only L_new).  The syndrome of the last iteration is tested once after the
// loop.  Flags rotate over three words so that clearing the next one never
// races with a late reader of the previous one.  Decodes with and without
// early stopping run separate instantiations of the kernel.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "check2.h"
#include "device.h"
#include "internal.h"
#include "onchip.h"

namespace ldpc {

constexpr int kOcMaxThreads = 1024;
constexpr int kOcRows = 4;    // base rows (J) an instantiation may have
constexpr int kOcSlots = 9;   // edge slots per row an instantiation may have

struct OnchipArgs {
    const float* llr;       // [gamma][n]
    float* post;            // [gamma][n]
    uint8_t* bits;          // [gamma][n]
    int32_t* iters;         // [gamma] or NULL
    uint8_t* conv;          // [gamma] or NULL
    int max_iters;
    // edge slot k of base row j (index j * kOcSlots + k): row (j, s) meets
    // variable l*p + (s + a) mod p of base column l; held as byte offsets
    // into the LDS posterior pairs (8 bytes per variable): cb8 = 8 l p and
    // sh8 = 8 a
    int32_t cb8[kOcRows * kOcSlots];
    int32_t sh8[kOcRows * kOcSlots];
    // regular bases with rows of weight <= 6 (oc_mu_in_regs) store base
    // column l rotated by base row 0's shift a_0l: variable (l, t) at pair
    // l p + (t - a_0l) mod p, so a row of base row 0 meets its variables at
    // l p + s (no wrap); rot8[l] = 8 a_0l, 0 otherwise, and sh8 holds the
    // shifts relative to it
    int32_t rot8[kOcSlots];
    int32_t deg[kOcRows];   // nonzero blocks of base row j
    uint64_t first;         // bit j * kOcSlots + k: the lowest nonzero block of its base column
    // learned min-sum (RULE 1): weights [iters][blocks][2] (scale, offset in
    // natural units), the number of blocks, the first block of each base row
    const float* nms_w;
    int32_t nb;
    int32_t rb0[kOcRows];
};

// Byte offset of the posterior pair of the variable that edge slot jk of
// row (j, s) meets, from s8 = 8 s: one wrap of s + shift (unsigned min picks
// t - p exactly when t >= p).
__device__ __forceinline__ uint32_t oc_wrap8(uint32_t t, uint32_t p8) { return min(t, t - p8); }

__device__ __forceinline__ uint32_t oc_pair(const OnchipArgs& A, int jk, uint32_t s8, uint32_t p8) {
    const uint32_t t = s8 + (uint32_t)A.sh8[jk];
    return (uint32_t)A.cb8[jk] + min(t, t - p8);
}

// The posterior pairs start at LDS address 0 (the kernel has no static LDS),
// so a pair's byte offset is its address and the component an immediate.
__device__ __forceinline__ float lds_at(const float2* L, uint32_t byte) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(L) + byte);
}

__device__ __forceinline__ float* lds_ptr(float2* L, uint32_t byte) {
    return reinterpret_cast<float*>(reinterpret_cast<char*>(L) + byte);
}

// Messages and sums are carried in base-2 units (check2.h): the channel
// LLRs are scaled by log2(e) once when read and the posteriors unscaled when
// written.

// Learned min-sum rule (the package decoder's RULE 1) in base-2 units:
// alpha_k = w_k s_k max(m_k - b_k, 0), m_k the smallest |beta| of the row's
// other edges (|beta| <= 30 log2 e already), s_k the product of their signs
// (negative iff beta < 0); w[2k], w[2k+1] = (scale, offset) of slot k's
// block, the offset in natural units (scaled here).
template <int DC>
__device__ __forceinline__ void nms2_row(const float (&in)[DC], int d, const float* __restrict__ w,
                                         float (&out)[DC]) {
    float min1 = __builtin_inff(), min2 = __builtin_inff();
    int idx1 = -1;
    uint32_t parity = 0;
#pragma unroll
    for (int k = 0; k < DC; ++k) {
        if (k < d) {
            const float m = fabsf(in[k]);
            if (m < min1) {
                min2 = min1;
                min1 = m;
                idx1 = k;
            } else if (m < min2) {
                min2 = m;
            }
            parity ^= (uint32_t)(in[k] < 0.0f);
        }
    }
#pragma unroll
    for (int k = 0; k < DC; ++k) {
        if (k < d) {
            const float m = k == idx1 ? min2 : min1;
            const float a = w[2 * k] * fmaxf(m - w[2 * k + 1] * kLog2eF, 0.0f);
            out[k] = (parity ^ (uint32_t)(in[k] < 0.0f)) ? -a : a;
        }
    }
}

// Eq. 3 for one row in base-2 units (check2.h's check2_row) with each
// input's pair left unnormalised: (u, w, s) = (1 - e, 2e, 1 + e), e =
// 2^-|x|, is (t, q, 1) times 1 + e, so no reciprocal is taken per input.
// Triples combine as (u_a u_b, w_a s_b + u_a w_b, s_a s_b) (again (t, q, 1)
// of the combined pair times s_a s_b), and for the exclusive triple
// (U, W, S) of slot k, S = U + W, so |alpha_k| = log2((S + U) / W) =
// log2((2U + W) / W); only the suffix sweep needs S.  Magnitudes stay in
// range: s <= 2, u <= 1, w >= 2^-42.3 for |x| <= 30 log2 e.  Per edge 3
// transcendentals instead of 4, per sweep step 2 more operations: 30d - 22
// issue slots per row of weight d instead of 30d - 11.  in[k] = beta of slot
// k for k < d; out[k] = alpha of slot k for k < d.
template <int DC>
__device__ __forceinline__ void check2u_row(const float (&in)[DC], int d, float (&out)[DC]) {
    static_assert(DC >= 2, "rows carry at least two slots");
    float u[DC], w[DC], s[DC];
    uint32_t sgn = 0;
#pragma unroll
    for (int k = 0; k < DC; ++k) {
        if (k < d) {
            const float e = __builtin_amdgcn_exp2f(-fabsf(in[k]));
            u[k] = 1.0f - e;
            w[k] = e + e;
            s[k] = 1.0f + e;
            sgn ^= __float_as_uint(in[k]);
        } else {
            u[k] = 1.0f;
            w[k] = 0.0f;
            s[k] = 1.0f;
        }
    }
    // suffix triples over slots k+1 .. DC-1 (slot DC-1: the identity)
    float sU[DC], sW[DC], sS[DC];
    sU[DC - 1] = 1.0f;
    sW[DC - 1] = 0.0f;
    sS[DC - 1] = 1.0f;
    sU[DC - 2] = u[DC - 1];
    sW[DC - 2] = w[DC - 1];
    sS[DC - 2] = s[DC - 1];
#pragma unroll
    for (int k = DC - 3; k >= 0; --k) {
        sU[k] = u[k + 1] * sU[k + 1];
        sW[k] = fmaf(w[k + 1], sS[k + 1], u[k + 1] * sW[k + 1]);
        sS[k] = s[k + 1] * sS[k + 1];
    }
    // prefix (U, W) over slots 0 .. k-1, combined with the suffix
    float PU = u[0], PW = w[0];
    float eU[DC], eW[DC];
    eU[0] = sU[0];
    eW[0] = sW[0];
#pragma unroll
    for (int k = 1; k < DC; ++k) {
        if (k == DC - 1) {
            eU[k] = PU;
            eW[k] = PW;
        } else {
            eU[k] = PU * sU[k];
            eW[k] = fmaf(PW, sS[k], PU * sW[k]);
            PW = fmaf(PW, s[k], PU * w[k]);
            PU = PU * u[k];
        }
    }
#pragma unroll
    for (int k = 0; k < DC; ++k) {
        const float mag = __builtin_amdgcn_logf(fmaf(2.0f, eU[k], eW[k]) * __builtin_amdgcn_rcpf(eW[k]));
        out[k] = __uint_as_float(__float_as_uint(mag) | ((sgn ^ __float_as_uint(in[k])) & 0x80000000u));
    }
}

// Regular bases with rows of weight <= 6 keep the scaled channel LLRs of the
// thread's base-row-0 edges in registers (the 3 x 9 rows would spill them);
// the others read them from the frame's LLRs in L2 when a sum starts.
constexpr bool oc_mu_in_regs(bool reg, int dc) { return reg && dc <= 6; }

// One iteration: PAR = it & 1.  L of iteration i lives in component i & 1 of
// each variable's pair, so this iteration reads component 1 - PAR (the
// previous iteration's sums) and accumulates into component PAR; both are
// immediate offsets of one address.  The signs read are the previous
// iteration's decisions: with SYN and flag != NULL, a wave with a violated
// row sets *flag (SYN = false compiles the test out, for decodes without
// early stopping).  mu0: with oc_mu_in_regs, the scaled channel LLRs of the thread's
// base-row-0 edges (their variables' sums start there).
template <int NJ, int NQ, int DC, bool REG, int RULE, int PAR, bool SYN>
__device__ __forceinline__ void oc_iteration(const OnchipArgs& A, float2* L, const float* __restrict__ mu,
                                             float (&al)[NJ][NQ][DC], const float (&mu0)[NQ][DC], uint32_t tid8,
                                             uint32_t TB8, uint32_t p8, uint32_t* flag, const float* wit) {
    uint64_t viol = 0;
    constexpr uint32_t kOld = 4u * (1 - PAR), kNew = 4u * PAR;
    constexpr bool kMuInRegs = oc_mu_in_regs(REG, DC);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int d = REG ? DC : A.deg[j];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const uint32_t s8 = tid8 + (uint32_t)q * TB8;
            if (s8 < p8) {
                uint32_t va[DC];
                float in[DC];
                // XOR of the signs read: the row's parity in bit 31 (a sum is
                // never -0: every one starts from mu + 0, and in round-to-nearest
                // a sum is -0 only if both terms are, so the sign bit is x < 0)
                uint32_t sx = 0;
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    if (REG || k < d) {
                        // rotated columns: base row 0 meets pair l p + s
                        va[k] = (kMuInRegs && j == 0) ? (uint32_t)A.cb8[k] + s8
                                                      : oc_pair(A, j * kOcSlots + k, s8, p8);
                        const float x = lds_at(L, va[k] + kOld);
                        if (SYN) sx ^= __float_as_uint(x);
                        in[k] = clip2(x - al[j][q][k]);
                    } else {
                        va[k] = 0;
                        in[k] = 0.0f;
                    }
                }
                if (SYN) viol |= __ballot((int32_t)sx < 0);
                float out[DC];
                if constexpr (RULE == 0)
                    check2u_row<DC>(in, d, out);
                else
                    nms2_row<DC>(in, d, wit + 2 * A.rb0[j], out);
#pragma unroll
                for (int k = 0; k < DC; ++k) {
                    if (REG || k < d) {
                        al[j][q][k] = out[k];
                        float* acc = lds_ptr(L, va[k] + kNew);
                        const bool first = REG ? (j == 0) : ((A.first >> (j * kOcSlots + k)) & 1ull);
                        if (first && kMuInRegs) {
                            *acc = mu0[q][k] + out[k];
                        } else if (first) {
                            // mu of variable v at byte 4 v of the frame (va = 8 v)
                            const float m = *reinterpret_cast<const float*>(
                                reinterpret_cast<const char*>(mu) + (va[k] >> 1));
                            *acc = (m * kLog2eF + 0.0f) + out[k];
                        } else {
                            // the only update of this variable in this base row: no other
                            // thread touches it before the barrier, so a plain read and
                            // write suffice (LDS float atomics ran the decode 4x slower)
                            *acc = *acc + out[k];
                        }
                    }
                }
            }
        }
        // with early stopping (flag != NULL) each wave ORs its verdict on the
        // previous iteration's syndrome in before the last barrier
        if (SYN && j == NJ - 1 && flag && viol != 0ull && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
        __syncthreads();
    }
}

// REG: every base row has DC nonzero blocks and every block of base row 0 is
// nonzero (so every base column starts in base row 0); otherwise the row
// weights and the first blocks of the columns come from the tables.  EARLY:
// with early stopping; a kernel of its own, so that the loop
// without the syndrome test gets the registers to itself.
template <int NJ, int NQ, int DC, bool REG, int RULE, int MAXT, bool EARLY>
__global__ void __launch_bounds__(MAXT) onchip_block_kernel(const int n, const int p, const OnchipArgs A) {
    // dynamic LDS: [n] posterior pairs (L of even iterations, L of odd
    // iterations), then three flag words
    extern __shared__ float2 Lpair[];
    uint32_t* flag = reinterpret_cast<uint32_t*>(Lpair + n);
    const int tid = threadIdx.x;
    const int TB = blockDim.x;
    const size_t f0 = (size_t)blockIdx.x * n;
    const float* __restrict__ mu = A.llr + f0;
    // L of "iteration 0" is mu, so that iteration 1 reads beta = clip(mu - 0)
    if constexpr (oc_mu_in_regs(REG, DC)) {
        // rotated columns (pair l p + u holds variable l p + (u + a_0l) mod p)
        for (int l = 0; l < DC; ++l) {
            const int rot = A.rot8[l] >> 3;
            for (int u = tid; u < p; u += TB) {
                int t = u + rot;
                t = t >= p ? t - p : t;
                Lpair[l * p + u].x = mu[l * p + t] * kLog2eF + 0.0f;
            }
        }
    } else {
        for (int v = tid; v < n; v += TB) Lpair[v].x = mu[v] * kLog2eF + 0.0f;
    }
    if (tid < 3) flag[tid] = 0u;
    const uint32_t p8 = 8u * (uint32_t)p, TB8 = 8u * (uint32_t)TB;
    float al[NJ][NQ][DC];
    float mu0[NQ][DC];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const uint32_t s8 = 8u * (uint32_t)tid + (uint32_t)q * TB8;
#pragma unroll
        for (int k = 0; k < DC; ++k) {
            mu0[q][k] = 0.0f;
            if (oc_mu_in_regs(REG, DC) && s8 < p8)
                mu0[q][k] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(mu) +
                                                            ((A.cb8[k] + oc_wrap8(s8 + A.rot8[k], p8)) >> 1)) *
                            kLog2eF + 0.0f;
        }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int k = 0; k < DC; ++k) al[j][q][k] = 0.0f;
    __syncthreads();

    int stop = 0;
    // each step: iteration it, then the test of the syndrome of it - 1
    auto step = [&](int it, auto parity, auto early) -> bool {
        constexpr int PAR = decltype(parity)::value;
        constexpr bool SYN = decltype(early)::value;
        // the edges' offsets do not change between iterations, but holding
        // them would take as many registers as the alphas: the thread index
        // passes through an opaque copy so that they are recomputed
        uint32_t tid8 = 8u * (uint32_t)tid;
        asm volatile("" : "+v"(tid8));
        const bool syn = SYN && it >= 2;
        if (tid == 0) flag[(it + 1) % 3] = 0u;
        const float* wit = RULE == 1 ? A.nms_w + (size_t)(it - 1) * A.nb * 2 : nullptr;
        oc_iteration<NJ, NQ, DC, REG, RULE, PAR, SYN>(A, Lpair, mu, al, mu0, tid8, TB8, p8,
                                                      syn ? &flag[it % 3] : nullptr, wit);
        if (syn && flag[it % 3] == 0u) {   // the syndrome of iteration it - 1 is zero
            stop = it - 1;
            return true;
        }
        return false;
    };
    using Odd = std::integral_constant<int, 1>;
    using Even = std::integral_constant<int, 0>;
    if constexpr (EARLY) {
        using On = std::true_type;
        for (int it = 1; it <= A.max_iters; it += 2) {
            if (step(it, Odd{}, On{})) break;
            if (it + 1 > A.max_iters) break;
            if (step(it + 1, Even{}, On{})) break;
        }
    } else {
        using Off = std::false_type;
        for (int it = 1; it <= A.max_iters; it += 2) {
            step(it, Odd{}, Off{});
            if (it + 1 > A.max_iters) break;
            step(it + 1, Even{}, Off{});
        }
    }

    int iters_out, conv_out;
    const float* Lf = reinterpret_cast<const float*>(Lpair);
    int comp;
    if (stop) {
        comp = stop & 1;
        iters_out = stop;
        conv_out = 1;
    } else {
        // syndrome of the last iteration (flag word (max + 1) % 3 was cleared in it)
        const int last = A.max_iters;
        comp = last & 1;
        uint64_t viol = 0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int d = REG ? DC : A.deg[j];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const uint32_t s8 = 8u * (uint32_t)tid + (uint32_t)q * TB8;
                if (s8 < p8) {
                    uint64_t par = 0;
#pragma unroll
                    for (int k = 0; k < DC; ++k)
                        if (REG || k < d)
                            par ^= __ballot(lds_at(Lpair, oc_pair(A, j * kOcSlots + k, s8, p8) + 4u * comp) < 0.0f);
                    viol |= par;
                }
            }
        }
        const int fw = (last + 1) % 3;
        if (viol != 0ull && (tid & 63) == 0) atomicOr(&flag[fw], 1u);
        __syncthreads();
        iters_out = last;
        conv_out = flag[fw] == 0u ? 1 : 0;
    }
    // back to natural units; a nonzero x keeps its sign (|x| ln 2 never
    // rounds to zero), so the decision is that of the sums above
    auto put = [&](int v, int pair) {
        const float x = Lf[2 * pair + comp] * kLn2F;
        A.post[f0 + v] = clip30(x);
        A.bits[f0 + v] = (uint8_t)(x < 0.0f);
    };
    if constexpr (oc_mu_in_regs(REG, DC)) {
        for (int l = 0; l < DC; ++l) {
            const int rot = A.rot8[l] >> 3;
            for (int u = tid; u < p; u += TB) {
                int t = u + rot;
                t = t >= p ? t - p : t;
                put(l * p + t, l * p + u);
            }
        }
    } else {
        for (int v = tid; v < n; v += TB) put(v, v);
    }
    if (tid == 0) {
        if (A.iters) A.iters[blockIdx.x] = iters_out;
        if (A.conv) A.conv[blockIdx.x] = (uint8_t)conv_out;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {

struct Variant {
    int nj, nq, dc;
    bool reg;
    int rule, maxt;
    const void* fn;         // without early stopping
    const void* fn_early;   // with early stopping
};

template <int NJ, int NQ, int DC, bool REG, int RULE = 0, int MAXT = kOcMaxThreads>
constexpr Variant variant() {
    return Variant{NJ, NQ, DC, REG, RULE, MAXT,
                   reinterpret_cast<const void*>(&onchip_block_kernel<NJ, NQ, DC, REG, RULE, MAXT, false>),
                   reinterpret_cast<const void*>(&onchip_block_kernel<NJ, NQ, DC, REG, RULE, MAXT, true>)};
}

// (base rows, rows per thread and base row, row-weight capacity, regular
// base); each compiles without spilled vector registers but the general
// 3 x 9 variant with two rows per thread (4 values, 12 with early stopping;
// 54 alphas per thread at most: rows of weight 18 would spill and stay with
// the package decoder)
const Variant kVariants[] = {
    variant<3, 1, 6, true>(),  variant<3, 2, 6, true>(),  variant<3, 3, 6, true>(),
    variant<3, 1, 9, true>(),  variant<3, 2, 9, true>(),
    variant<3, 1, 6, false>(), variant<3, 2, 6, false>(), variant<3, 3, 6, false>(),
    variant<3, 1, 9, false>(), variant<3, 2, 9, false>(),
    variant<4, 1, 8, false>(),
    // learned min-sum
    variant<3, 1, 6, true, 1>(),  variant<3, 2, 6, true, 1>(),  variant<3, 3, 6, true, 1>(),
    variant<3, 1, 9, true, 1>(),  variant<3, 2, 9, true, 1>(),
    variant<3, 1, 6, false, 1>(), variant<3, 2, 6, false, 1>(), variant<3, 3, 6, false, 1>(),
    variant<3, 1, 9, false, 1>(), variant<3, 2, 9, false, 1>(),
    variant<4, 1, 8, false, 1>(),
};

struct Choice {
    const Variant* v;
    int tb;
    size_t lds;
};

bool choose(const ldpc_graph* g, int rule, Choice& c) {
    if (!g || g->kind != LDPC_GRAPH_QC) return false;
    const QCDesc& D = g->qc;
    if (D.J > kOcRows || D.dc_max > kOcSlots) return false;
    for (int l = 0; l < D.L; ++l)
        if (D.cstart[l + 1] == D.cstart[l]) return false;   // a base column without edges
    bool reg = D.rstart[1] - D.rstart[0] == D.L;            // base row 0 full: every column starts there
    for (int j = 0; j < D.J; ++j) reg = reg && (D.rstart[j + 1] - D.rstart[j] == D.dc_max);
    int dev = 0, limit = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const size_t lds = (size_t)D.n * sizeof(float2) + 3 * sizeof(uint32_t);   // pairs, flags
    if (lds > (size_t)limit) return false;
    const Variant* best = nullptr;
    int best_tb = 0;
    for (const Variant& v : kVariants) {
        if (v.rule != rule || v.nj != D.J || v.dc < D.dc_max) continue;
        if (v.reg && !(reg && v.dc == D.dc_max)) continue;
        const int per = (D.p + v.nq - 1) / v.nq;
        const int tb = (per + 63) / 64 * 64;
        if (tb > v.maxt) continue;
        // fewest rows per thread, then a regular variant, then the smallest row-weight capacity
        const bool better = !best || v.nq < best->nq ||
                            (v.nq == best->nq && (v.reg > best->reg || (v.reg == best->reg && v.dc < best->dc)));
        if (better) {
            best = &v;
            best_tb = tb;
        }
    }
    if (!best) return false;
    c.v = best;
    c.tb = best_tb;
    c.lds = lds;
    return true;
}

}  // namespace

bool onchip_fits(const ldpc_graph* g) {
    Choice c;
    return choose(g, 0, c);
}

bool onchip_selected(const ldpc_graph* g) {
    const char* path = std::getenv("LDPC_BLOCK_PATH");
    if (path && std::strcmp(path, "packages") == 0) return false;
    return onchip_fits(g);
}

int onchip_decode(const ldpc_graph* g, const float* llr, int gamma, int max_iters, int early, float* post,
                  uint8_t* bits, int32_t* iters, uint8_t* converged, hipStream_t st, const float* nms_w) {
    Choice c;
    if (!choose(g, nms_w ? 1 : 0, c)) return 0;
    const QCDesc& D = g->qc;
    OnchipArgs A{};
    A.llr = llr;
    A.post = post;
    A.bits = bits;
    A.iters = iters;
    A.conv = converged;
    A.max_iters = max_iters;
    A.nms_w = nms_w;
    A.nb = D.nb;
    // the kernel stores columns rotated by base row 0's shifts when it keeps
    // mu in registers (regular bases, rows of weight <= 6: base row 0 holds
    // one block of every column, in column order)
    int rot[kOcSlots] = {0};
    if (oc_mu_in_regs(c.v->reg, c.v->dc))
        for (int k = 0; k < D.rstart[1]; ++k) rot[D.ecol[k]] = D.eshift[k];
    for (int l = 0; l < kOcSlots; ++l) A.rot8[l] = 8 * rot[l];
    for (int j = 0; j < D.J; ++j) {
        A.deg[j] = D.rstart[j + 1] - D.rstart[j];
        A.rb0[j] = D.rstart[j];
        for (int k = 0; k < A.deg[j]; ++k) {
            const int b = D.rstart[j] + k;
            A.cb8[j * kOcSlots + k] = 8 * D.ecol[b] * D.p;
            A.sh8[j * kOcSlots + k] = 8 * ((D.eshift[b] - rot[D.ecol[b]] + D.p) % D.p);
            if (D.cedge[D.cstart[D.ecol[b]]] == b)   // edge blocks of a column ascend by base row
                A.first |= 1ull << (j * kOcSlots + k);
        }
    }
    const void* fn = early ? c.v->fn_early : c.v->fn;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    timing::Scope ts(23, st);
    int n = D.n, p = D.p;
    void* args[] = {&n, &p, &A};
    return hipLaunchKernel(fn, dim3((unsigned)gamma), dim3((unsigned)c.tb), args, c.lds, st) == hipSuccess ? 1 : -1;
}

}  // namespace ldpc
