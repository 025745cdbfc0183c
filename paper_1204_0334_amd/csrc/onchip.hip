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
//   * the check update (Eq. 3) is the same FP32 (t, 1 - t) forward-backward
//     form as the package decoder (sp_check in device.h).
//
// One iteration, for base rows j = 0 .. J-1 in turn (a workgroup barrier
// after each): every thread updates its rows of base row j from L_old
// (the previous iteration's sums) and adds the new alphas into L_new.  A
// weight-1 circulant block joins each variable of its base column to exactly
// one row of its base row, so within one base row no two threads touch the
// same variable and the additions need no atomics; the base-row order fixes
// the order of every sum, so results are deterministic.  The lowest nonzero
// block of each base column starts its variables' sums from mu (read from
// the caller's LLR array, which stays in L2).  HBM traffic per frame is the
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
// races with a late reader of the previous one.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "device.h"
#include "internal.h"
#include "onchip.h"

namespace ldpc {

constexpr int kOcMaxThreads = 1024;

struct OnchipArgs {
    const float* llr;       // [gamma][n]
    float* post;            // [gamma][n]
    uint8_t* bits;          // [gamma][n]
    int32_t* iters;         // [gamma] or NULL
    uint8_t* conv;          // [gamma] or NULL
    int max_iters, early;
    uint32_t first[LDPC_MAX_BLOCKS / 32];   // bit b: edge block b is the lowest nonzero block of its base column
};

template <int NJ, int NQ, int DC>
__global__ void __launch_bounds__(kOcMaxThreads) onchip_block_kernel(const QCDesc D, const OnchipArgs A) {
    extern __shared__ float Lbuf[];   // [2][n]: L of iteration i in Lbuf + (i & 1) * n
    __shared__ uint32_t flag[3];
    const int tid = threadIdx.x;
    const int TB = blockDim.x;
    const int n = D.n, p = D.p;
    const size_t f0 = (size_t)blockIdx.x * n;
    const float* __restrict__ mu = A.llr + f0;
    // L of "iteration 0" is mu, so that iteration 1 reads beta = clip(mu - 0)
    for (int v = tid; v < n; v += TB) Lbuf[v] = mu[v];
    if (tid < 3) flag[tid] = 0u;
    float al[NJ][NQ][DC];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int k = 0; k < DC; ++k) al[j][q][k] = 0.0f;
    __syncthreads();

    int it = 1, stop = 0;
    for (; it <= A.max_iters; ++it) {
        const float* Lo = Lbuf + ((it - 1) & 1) * n;
        float* Ln = Lbuf + (it & 1) * n;
        const bool syn = A.early && it >= 2;
        if (tid == 0) flag[(it + 1) % 3] = 0u;
        uint32_t viol = 0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int b0 = D.rstart[j];
            const int d = D.rstart[j + 1] - b0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int s = tid + q * TB;
                if (s < p) {
                    int vk[DC];
                    float in[DC][1];
                    uint32_t par = 0;
#pragma unroll
                    for (int k = 0; k < DC; ++k) {
                        if (k < d) {
                            const int b = b0 + k;
                            int t = s + D.eshift[b];
                            t = t >= p ? t - p : t;
                            vk[k] = D.ecol[b] * p + t;
                            const float x = Lo[vk[k]];
                            par ^= (uint32_t)(x < 0.0f);
                            in[k][0] = clip30(x - al[j][q][k]);
                        } else {
                            vk[k] = 0;
                            in[k][0] = 0.0f;
                        }
                    }
                    viol |= par;
                    float out[DC][1];
                    sp_check<DC, 1>(in, d, out);
#pragma unroll
                    for (int k = 0; k < DC; ++k) {
                        if (k < d) {
                            al[j][q][k] = out[k][0];
                            const int b = b0 + k;
                            const bool first = (A.first[b >> 5] >> (b & 31)) & 1u;
                            const float base = first ? mu[vk[k]] : Ln[vk[k]];
                            Ln[vk[k]] = base + out[k][0];
                        }
                    }
                }
            }
            if (j == NJ - 1 && syn && __ballot(viol != 0u) != 0ull && (tid & 63) == 0)
                atomicOr(&flag[it % 3], 1u);
            __syncthreads();
        }
        if (syn && flag[it % 3] == 0u) {   // the syndrome of iteration it - 1 is zero
            stop = it - 1;
            break;
        }
    }

    int iters_out, conv_out;
    const float* Lf;
    if (stop) {
        Lf = Lbuf + (stop & 1) * n;
        iters_out = stop;
        conv_out = 1;
    } else {
        // syndrome of the last iteration (flag word (max + 1) % 3 was cleared in it)
        const int last = A.max_iters;
        Lf = Lbuf + (last & 1) * n;
        uint32_t viol = 0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int b0 = D.rstart[j];
            const int d = D.rstart[j + 1] - b0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int s = tid + q * TB;
                if (s < p) {
                    uint32_t par = 0;
#pragma unroll
                    for (int k = 0; k < DC; ++k) {
                        if (k < d) {
                            const int b = b0 + k;
                            int t = s + D.eshift[b];
                            t = t >= p ? t - p : t;
                            par ^= (uint32_t)(Lf[D.ecol[b] * p + t] < 0.0f);
                        }
                    }
                    viol |= par;
                }
            }
        }
        const int fw = (last + 1) % 3;
        if (__ballot(viol != 0u) != 0ull && (tid & 63) == 0) atomicOr(&flag[fw], 1u);
        __syncthreads();
        iters_out = last;
        conv_out = flag[fw] == 0u ? 1 : 0;
    }
    for (int v = tid; v < n; v += TB) {
        const float x = Lf[v];
        A.post[f0 + v] = clip30(x);
        A.bits[f0 + v] = (uint8_t)(x < 0.0f);
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
    const void* fn;
};

template <int NJ, int NQ, int DC>
constexpr Variant variant() {
    return Variant{NJ, NQ, DC, reinterpret_cast<const void*>(&onchip_block_kernel<NJ, NQ, DC>)};
}

// (base rows, rows per thread and base row, row-weight capacity); each
// compiles without spilled vector registers (54 alphas per thread at most:
// 3 x 1 x 18 would spill, so rows of weight 18 stay with the package decoder)
const Variant kVariants[] = {
    variant<3, 1, 6>(), variant<3, 2, 6>(), variant<3, 3, 6>(),
    variant<3, 1, 9>(), variant<3, 2, 9>(),
    variant<4, 1, 8>(),
};

struct Choice {
    const Variant* v;
    int tb;
    size_t lds;
};

bool choose(const ldpc_graph* g, Choice& c) {
    if (!g || g->kind != LDPC_GRAPH_QC) return false;
    const QCDesc& D = g->qc;
    for (int l = 0; l < D.L; ++l)
        if (D.cstart[l + 1] == D.cstart[l]) return false;   // a base column without edges
    int dev = 0, limit = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    const size_t lds = (size_t)2 * D.n * sizeof(float);
    if (lds + 64 > (size_t)limit) return false;
    const Variant* best = nullptr;
    int best_tb = 0;
    for (const Variant& v : kVariants) {
        if (v.nj != D.J || v.dc < D.dc_max) continue;
        const int per = (D.p + v.nq - 1) / v.nq;
        const int tb = (per + 63) / 64 * 64;
        if (tb > kOcMaxThreads) continue;
        // fewest rows per thread, then the smallest row-weight capacity
        if (!best || v.nq < best->nq || (v.nq == best->nq && v.dc < best->dc)) {
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
    return choose(g, c);
}

int onchip_decode(const ldpc_graph* g, const float* llr, int gamma, int max_iters, int early, float* post,
                  uint8_t* bits, int32_t* iters, uint8_t* converged, hipStream_t st) {
    Choice c;
    if (!choose(g, c)) return 0;
    const QCDesc& D = g->qc;
    OnchipArgs A{};
    A.llr = llr;
    A.post = post;
    A.bits = bits;
    A.iters = iters;
    A.conv = converged;
    A.max_iters = max_iters;
    A.early = early;
    for (int l = 0; l < D.L; ++l) {
        const int b = D.cedge[D.cstart[l]];   // edge blocks of a column ascend by base row
        A.first[b >> 5] |= 1u << (b & 31);
    }
    if (hipFuncSetAttribute(c.v->fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    timing::Scope ts(23, st);
    void* args[] = {const_cast<QCDesc*>(&D), &A};
    return hipLaunchKernel(c.v->fn, dim3((unsigned)gamma), dim3((unsigned)c.tb), args, c.lds, st) == hipSuccess ? 1 : -1;
}

}  // namespace ldpc
