// Multi-code plan: frames of several QC-LDPC codes, each with its own batch
// size, decoded together by flooding sum-product (Algorithm 1, Eq. 3-6).
//
// One launch per phase covers every code of the plan: the check-node launch
// of iteration i runs the rows of all codes, the variable-node launch all
// their variables, so small codes ride along with large ones instead of each
// paying for its own 2 * I_max launches.  The whole sequence (ingest,
// 2 * I_max phase launches, final syndrome, frame status, output) can be
// captured once into a HIP graph and replayed.
//
// Lane layouts.  A code's frames are tiled by Gt = G * FPL frames.  A wave
// holds R = 64 / G rows (or variables) x G frames: lane = r * G + f works on
// row (variable) r of the wave and frame f of the tile (G = 64: one row per
// wave, FPL frames per lane as in the single-code decoder).  Message packages
// stay [tile][package][Gt]; the R rows of a wave are consecutive rows of a
// circulant block, so their packages are consecutive and the wave's access
// to an edge slot is one contiguous 64 * FPL * 4-byte run whatever G is.
// Small batches (Gamma < 64) therefore use G = 8, 16 or 32 instead of
// padding every tile to 64 frames.  The layout of each code is chosen by
// the caller or by ldpc_plan_autotune (which times the candidates).
//
// Per-code descriptors (the QC description, buffer addresses, tiling and the
// code's first wave in each launch) live in a table at the start of the
// caller's workspace; a launch's waves find their code by scanning that
// table (a handful of entries).  The arithmetic per frame is the single-code
// decoder's (shared helpers sp_check / sp_variable, same edge order), so a
// plan returns bit for bit what ldpc_decode returns for each code; the split
// layouts (a check row's edges over several lanes) agree with it to FP32
// rounding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "device.h"
#include "internal.h"
#include "onchip.h"

namespace ldpc {

// Base lane layouts: G lanes per row (variable) group, FPL frames per lane,
// tiles of G * FPL frames.  0-3: G8, G16, G32, G64 with one frame per lane;
// 4, 5: G64 with 4 and 2; 6-11: G8, G16, G32 with 2 and 4 frames per lane
// (small tiles whose lanes still move 8 or 16 bytes per access).
constexpr int kPlanLayouts = 12;

// A code's layout value: base lane layout (bits 0-3), log2 of the number of
// variable groups each variable-node wave handles (bits 4-5) and of row groups
// per check-node wave (bits 6-7); groups only with one frame per lane; log2
// of the number of lanes that share each check row's edges (bits 8-9, split
// layouts: G8, G16 or G32 with one frame per lane and one row group).
constexpr int kLayoutValues = 1024;
__host__ __device__ constexpr int layout_base(int l) { return l & 15; }
__host__ __device__ constexpr int layout_vpw(int l) { return 1 << ((l >> 4) & 3); }
__host__ __device__ constexpr int layout_cpw(int l) { return 1 << ((l >> 6) & 3); }
__host__ __device__ constexpr int layout_split(int l) { return 1 << ((l >> 8) & 3); }
__host__ __device__ constexpr int layout_g(int l) {
    const int b = layout_base(l);
    return b <= 3 ? 8 << b : b <= 5 ? 64 : b <= 7 ? 8 : b <= 9 ? 16 : 32;
}
__host__ __device__ constexpr int layout_fpl(int l) {
    const int b = layout_base(l);
    return b <= 3 ? 1 : b == 4 ? 4 : b == 5 ? 2 : (b & 1) ? 4 : 2;
}

struct PlanCode {
    QCDesc D;
    float* mu;            // [tiles][n][Gt]
    float* msg;           // [tiles][E][Gt]
    float* postw;         // [2][tiles][n][Gt]: posteriors, slot = iteration & 1
    uint64_t* bits;       // [2][tiles][n][FPL] packed decisions, slot = iteration & 1
    uint64_t* unsat;      // [max_iters+1][tiles][FPL]
    uint64_t* frozen;     // [max_iters+1][tiles][FPL]
    const float* llr;     // caller, [gamma][n]
    float* post;          // caller, [gamma][n]
    uint8_t* bits_out;    // caller, [gamma][n]
    int32_t* iters;       // caller, [gamma] or NULL
    uint8_t* converged;   // caller, [gamma] or NULL
    int64_t flag_words;   // (max_iters+1) * tiles * FPL
    int gamma, tiles, layout, Gt, fpl, dcc, dvc;   // layout: the base lane layout
    int cn_wpt, vn_wpt;   // waves per tile in the check / variable launches
    int io_vchunks, io_fchunks;
    int64_t cn0, vn0;     // first wave of the code in the check / variable launches
    int64_t syn0, st0;    // first thread in the syndrome / frame-status launches (multiples of 64)
    int64_t io0;          // first block in the ingest / output launches
    int vpw;              // variable-node launch: groups of R variables per wave (1, 2 or 4)
    int cpw;              // check-node launch: groups of R rows per wave (1, 2 or 4)
    int split;            // check-node launch: lanes sharing each row's edges (1, 2, 4 or 8)
    uint64_t* badw;       // early stopping: [2][tiles * cn_wpt][FPL] frames violating each check wave's
                          // rows, slot = (iteration of the decisions tested) & 1
    uint32_t* slot;       // [gamma]: slot holding each frame's returned iteration
    int64_t bits_slot, postw_slot, badw_slot;   // elements per slot
    int64_t red0;         // first block in the flag-reduction launch (red_chunks blocks per tile)
    int red_chunks;       // blocks per tile in the flag-reduction launch
    char* region;         // start of the code's workspace region (mu .. badw lie inside it)
};

// Memory access policies of the plan bodies.  PlainMem: ordinary loads and
// stores (the phase launches; a kernel boundary separates producer and
// consumer).  CoherentMem: device-coherent buffer accesses (cache policy
// sc1: stores write through the L2 of their XCD, loads do not hit stale
// lines), addressed relative to the code's region, for the persistent launch
// where one ticket's stores are read by tickets on other XCDs within the same
// launch; the region of a code stays below 2^31 bytes there.
struct PlainMem {
    template <int FPL>
    static __device__ __forceinline__ void ld(const PlanCode&, const float* p, float (&v)[FPL]) {
        load_frames<FPL>(p, v);
    }
    template <int FPL>
    static __device__ __forceinline__ void st(const PlanCode&, float* p, const float (&v)[FPL]) {
        store_frames<FPL>(p, v);
    }
    static __device__ __forceinline__ uint64_t ld64(const PlanCode&, const uint64_t* p) { return *p; }
    static __device__ __forceinline__ void st64(const PlanCode&, uint64_t* p, uint64_t v) { *p = v; }
    static __device__ __forceinline__ float ldf(const PlanCode&, const float* p) { return *p; }
    static __device__ __forceinline__ void stf(const PlanCode&, float* p, float v) { *p = v; }
    static __device__ __forceinline__ uint32_t ld32(const PlanCode&, const uint32_t* p) { return *p; }
    static __device__ __forceinline__ void st32(const PlanCode&, uint32_t* p, uint32_t v) { *p = v; }
};

struct CoherentMem {
    static constexpr int kSc1 = 16;   // cache-policy operand: sc1
    static __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const PlanCode& C) {
        return __builtin_amdgcn_make_buffer_rsrc(C.region, 0, 0x7fffffff, 0x00020000);
    }
    static __device__ __forceinline__ int off(const PlanCode& C, const void* p) {
        return (int)(reinterpret_cast<const char*>(p) - C.region);
    }
    template <int FPL>
    static __device__ __forceinline__ void ld(const PlanCode& C, const float* p, float (&v)[FPL]) {
        if constexpr (FPL == 4) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b128(rsrc(C), off(C, p), 0, kSc1);
            v[0] = __uint_as_float(x[0]); v[1] = __uint_as_float(x[1]);
            v[2] = __uint_as_float(x[2]); v[3] = __uint_as_float(x[3]);
        } else if constexpr (FPL == 2) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b64(rsrc(C), off(C, p), 0, kSc1);
            v[0] = __uint_as_float(x[0]); v[1] = __uint_as_float(x[1]);
        } else {
            v[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc(C), off(C, p), 0, kSc1));
        }
    }
    template <int FPL>
    static __device__ __forceinline__ void st(const PlanCode& C, float* p, const float (&v)[FPL]) {
        if constexpr (FPL == 4) {
            __attribute__((ext_vector_type(4))) unsigned x = {__float_as_uint(v[0]), __float_as_uint(v[1]),
                                                              __float_as_uint(v[2]), __float_as_uint(v[3])};
            __builtin_amdgcn_raw_buffer_store_b128(x, rsrc(C), off(C, p), 0, kSc1);
        } else if constexpr (FPL == 2) {
            __attribute__((ext_vector_type(2))) unsigned x = {__float_as_uint(v[0]), __float_as_uint(v[1])};
            __builtin_amdgcn_raw_buffer_store_b64(x, rsrc(C), off(C, p), 0, kSc1);
        } else {
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[0]), rsrc(C), off(C, p), 0, kSc1);
        }
    }
    static __device__ __forceinline__ uint64_t ld64(const PlanCode& C, const uint64_t* p) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b64(rsrc(C), off(C, p), 0, kSc1);
        return (uint64_t)x[0] | ((uint64_t)x[1] << 32);
    }
    static __device__ __forceinline__ void st64(const PlanCode& C, uint64_t* p, uint64_t v) {
        __attribute__((ext_vector_type(2))) unsigned x = {(unsigned)v, (unsigned)(v >> 32)};
        __builtin_amdgcn_raw_buffer_store_b64(x, rsrc(C), off(C, p), 0, kSc1);
    }
    static __device__ __forceinline__ float ldf(const PlanCode& C, const float* p) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rsrc(C), off(C, p), 0, kSc1));
    }
    static __device__ __forceinline__ void stf(const PlanCode& C, float* p, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rsrc(C), off(C, p), 0, kSc1);
    }
    static __device__ __forceinline__ uint32_t ld32(const PlanCode& C, const uint32_t* p) {
        return __builtin_amdgcn_raw_buffer_load_b32(rsrc(C), off(C, p), 0, kSc1);
    }
    static __device__ __forceinline__ void st32(const PlanCode& C, uint32_t* p, uint32_t v) {
        __builtin_amdgcn_raw_buffer_store_b32(v, rsrc(C), off(C, p), 0, kSc1);
    }
};

struct PlanStep {
    int iter, last, early, max_iters;
};

__device__ __forceinline__ int plan_find(const PlanCode* __restrict__ codes, int ncodes, int64_t x,
                                         int64_t PlanCode::*first) {
    int c = 0;
    for (int i = 1; i < ncodes; ++i)
        if (x >= codes[i].*first) c = i;
    return c;
}

// Row (j, s) and variable (l, t) of a QC code with the base row / column
// shared by the whole wave (so the circulant block indices and shifts are
// wave-uniform) and the offset s (t) per lane; same edge order as QCRow /
// QCCol.
struct PlanRow {
    int b0, d, s;
    __device__ __forceinline__ PlanRow(const QCDesc& D, int j, int s_, bool active) : s(s_) {
        b0 = D.rstart[j];
        d = active ? D.rstart[j + 1] - b0 : 0;
    }
    __device__ __forceinline__ int64_t pkg(const QCDesc& D, int k) const { return (int64_t)(b0 + k) * D.p + s; }
    __device__ __forceinline__ int var(const QCDesc& D, int k) const {
        const int b = b0 + k;
        int t = s + D.eshift[b];
        if (t >= D.p) t -= D.p;
        return D.ecol[b] * D.p + t;
    }
};

struct PlanCol {
    int c0, d, t;
    __device__ __forceinline__ PlanCol(const QCDesc& D, int l, int t_, bool active) : t(t_) {
        c0 = D.cstart[l];
        d = active ? D.cstart[l + 1] - c0 : 0;
    }
    __device__ __forceinline__ int64_t pkg(const QCDesc& D, int k) const {
        const int b = D.cedge[c0 + k];
        int s = t - D.eshift[b];
        if (s < 0) s += D.p;
        return (int64_t)b * D.p + s;
    }
};

// a[i] of a register array by mask blending (a dynamic index would move the
// array to private memory)
template <int FPL>
__device__ __forceinline__ uint64_t plan_pick(const uint64_t (&a)[FPL], int i) {
    uint64_t r = a[0];
#pragma unroll
    for (int f = 1; f < FPL; ++f) {
        const uint64_t m = 0ull - (uint64_t)(i == f);
        r = (a[f] & m) | (r & ~m);
    }
    return r;
}

#define PLAN_LAYOUT_SWITCH(LV, ...)                                           \
    switch (LV) {                                                             \
        case 0: { constexpr int G = 8, FPL = 1; __VA_ARGS__; } break;         \
        case 1: { constexpr int G = 16, FPL = 1; __VA_ARGS__; } break;        \
        case 2: { constexpr int G = 32, FPL = 1; __VA_ARGS__; } break;        \
        case 3: { constexpr int G = 64, FPL = 1; __VA_ARGS__; } break;        \
        case 4: { constexpr int G = 64, FPL = 4; __VA_ARGS__; } break;        \
        case 5: { constexpr int G = 64, FPL = 2; __VA_ARGS__; } break;        \
        case 6: { constexpr int G = 8, FPL = 2; __VA_ARGS__; } break;         \
        case 7: { constexpr int G = 8, FPL = 4; __VA_ARGS__; } break;         \
        case 8: { constexpr int G = 16, FPL = 2; __VA_ARGS__; } break;        \
        case 9: { constexpr int G = 16, FPL = 4; __VA_ARGS__; } break;        \
        case 10: { constexpr int G = 32, FPL = 2; __VA_ARGS__; } break;       \
        default: { constexpr int G = 32, FPL = 4; __VA_ARGS__; } break;       \
    }
// row-weight classes of a plan (at most 24: one kernel serves every code, and
// its register budget is that of the heaviest variant it contains)
#define PLAN_DC_SWITCH(DCV, ...)                                    \
    switch (DCV) {                                                  \
        case 4: { constexpr int DC = 4; __VA_ARGS__; } break;       \
        case 6: { constexpr int DC = 6; __VA_ARGS__; } break;       \
        case 8: { constexpr int DC = 8; __VA_ARGS__; } break;       \
        case 12: { constexpr int DC = 12; __VA_ARGS__; } break;     \
        case 16: { constexpr int DC = 16; __VA_ARGS__; } break;     \
        default: { constexpr int DC = 24; __VA_ARGS__; } break;     \
    }
#define PLAN_DV_SWITCH(DVV, ...)                                    \
    switch (DVV) {                                                  \
        case 2: { constexpr int DV = 2; __VA_ARGS__; } break;       \
        case 3: { constexpr int DV = 3; __VA_ARGS__; } break;       \
        case 4: { constexpr int DV = 4; __VA_ARGS__; } break;       \
        case 6: { constexpr int DV = 6; __VA_ARGS__; } break;       \
        case 8: { constexpr int DV = 8; __VA_ARGS__; } break;       \
        default: { constexpr int DV = 16; __VA_ARGS__; } break;     \
    }

// Check-node pass of iteration S.iter for wave lw of code C (in place; the
// first iteration gathers the channel LLRs).  With early stopping it first
// skips tiles whose frames had all stopped by iteration iter-3 (the last
// iteration the variable pass before it knew of), and tests the rows against
// iteration iter-1's decisions (slot (iter-1) & 1), storing the violated
// frames in the wave's words of badw slot (iter-1) & 1; the decision words
// are loaded right after the messages and the flag stores come after the
// message stores.
template <int DCMAX, int G, int FPL, int V, class M>
__device__ __forceinline__ void plan_cn_body(const PlanCode& C, const PlanStep& S, int64_t lw, int lane) {
    constexpr int R = 64 / G;
    constexpr int Gt = G * FPL;
    const QCDesc& D = C.D;
    const int tile = (int)(lw / C.cn_wpt);
    const int rw = (int)(lw - (int64_t)tile * C.cn_wpt);
    const int r = lane / G, f = lane % G;
    const int nvalid = min(C.gamma - tile * Gt, Gt);
    if (S.early && S.iter >= 4) {
        const uint64_t* fz = C.frozen + ((size_t)(S.iter - 3) * C.tiles + tile) * FPL;
        bool all = true;
#pragma unroll
        for (int i = 0; i < FPL; ++i) all = all && (M::ld64(C, fz + i) == ~0ull);
        if (all) return;
    }
    const size_t lane_off = (size_t)f * FPL;   // lane f of its group: frames f*FPL .. f*FPL+FPL-1
    float* mt = C.msg + (size_t)tile * D.E * Gt + lane_off;
    const float* ut = C.mu + (size_t)tile * D.n * Gt + lane_off;
    // the wave's rows: base row j (uniform), offsets sw*V*R .. within it
    const int spw = C.cn_wpt / D.J;
    const int j = rw / spw, sw = rw - j * spw;
    int srow[V], d[V];
    float in[V][DCMAX][FPL];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        srow[v] = (sw * V + v) * R + r;
        const bool active = srow[v] < D.p;
        const PlanRow Rw(D, j, active ? srow[v] : 0, active);
        d[v] = Rw.d;
#pragma unroll
        for (int k = 0; k < DCMAX; ++k) {
            if (k < d[v]) {
                const float* s = S.iter == 1 ? ut + (size_t)Rw.var(D, k) * Gt : mt + (size_t)Rw.pkg(D, k) * Gt;
                M::template ld<FPL>(C, s, in[v][k]);
            } else {
#pragma unroll
                for (int i = 0; i < FPL; ++i) in[v][k][i] = 0.0f;
            }
        }
    }
    // frames violating any of the wave's rows: the decision words are spread
    // over the lanes (one or a few loads per lane rather than d uniform ones)
    // and combined by XOR butterflies (parity of a row) and OR (over rows)
    const bool syn = S.early && S.iter >= 2;
    uint64_t par = 0;
    if (syn) {
        const uint64_t* bt = C.bits + ((S.iter - 1) & 1) * C.bits_slot + (size_t)tile * D.n * FPL;
        if constexpr (G == 64 && FPL > 1) {
            // lane k*FPL + f: word f of variable k; lane f ends with parity word f
            const int kk = lane / FPL, ff = lane - kk * FPL;
            const PlanRow Rw(D, j, d[0] ? srow[0] : 0, d[0] > 0);
            if (kk < d[0]) par = M::ld64(C, bt + (size_t)Rw.var(D, kk) * FPL + ff);
#pragma unroll
            for (int off = 32; off >= FPL; off >>= 1) par ^= __shfl_xor(par, off);
        } else {
            // lane f of a group of G lanes takes the (variable k, word i)
            // pairs q = f, f + G, ... of its row (k = q / FPL, i = q % FPL);
            // XOR butterflies over the group give the row's parity words, an
            // OR over the groups the wave's; lane i < FPL keeps word i
            uint64_t acc[FPL];
#pragma unroll
            for (int i = 0; i < FPL; ++i) acc[i] = 0;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const PlanRow Rw(D, j, d[v] ? srow[v] : 0, d[v] > 0);
                uint64_t x[FPL];
#pragma unroll
                for (int i = 0; i < FPL; ++i) x[i] = 0;
#pragma unroll
                for (int q0 = 0; q0 < (DCMAX * FPL + G - 1) / G; ++q0) {
                    const int q = q0 * G + f;
                    const int k = q / FPL, iq = q - k * FPL;
                    if (k < d[v]) {
                        const uint64_t word = M::ld64(C, bt + (size_t)Rw.var(D, k) * FPL + iq);
#pragma unroll
                        for (int i = 0; i < FPL; ++i)
                            if (i == iq) x[i] ^= word;
                    }
                }
#pragma unroll
                for (int i = 0; i < FPL; ++i) {
#pragma unroll
                    for (int off = G / 2; off >= 1; off >>= 1) x[i] ^= __shfl_xor(x[i], off);
                    acc[i] |= x[i];
                }
            }
#pragma unroll
            for (int i = 0; i < FPL; ++i) {
#pragma unroll
                for (int off = 32; off >= G; off >>= 1) acc[i] |= __shfl_xor(acc[i], off);
            }
            par = plan_pick<FPL>(acc, lane);
        }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const PlanRow Rw(D, j, d[v] ? srow[v] : 0, d[v] > 0);
        float out[DCMAX][FPL];
        sp_check<DCMAX, FPL>(in[v], d[v], out);
#pragma unroll
        for (int k = 0; k < DCMAX; ++k)
            if (k < d[v]) M::template st<FPL>(C, mt + (size_t)Rw.pkg(D, k) * Gt, out[k]);
    }
    // the wave's violated frames go to its own words (plain stores; the flag
    // word of the tile is formed by the flag reduction of the next check launch)
    if (syn && lane < FPL)
        M::st64(C, C.badw + ((S.iter - 1) & 1) * C.badw_slot + lw * FPL + lane, par & valid_word<FPL>(nvalid, lane));
}

// Check-node pass of a split layout: each row's edges are spread over H
// lanes, so that a heavy row with few frames is not one lane's chain of d
// loads and d-step sweeps.  Lane = (r * H + h) * G + f: row r of the wave's
// R = 64 / (G H) rows, part h of its edges (slots h, h + H, h + 2H, ...),
// frame f of the tile (one frame per lane; the message layout is that of
// the base layout, so the variable-node pass is unchanged).  Eq. 3 in the
// (t, q) form of sp_check: each lane combines its slots' pairs into one
// pair, takes the pairs of the row's other parts by shuffles (lanes
// lane + (h' - h) G) and combines those before and after its own into a
// prefix and a suffix, then runs the forward-backward sweep over its own
// slots starting from them; the sign is the XOR over the H lanes.  The
// products are therefore formed in another order than sp_check's sweep
// over the whole row: the results agree with it to FP32 rounding, not bit
// for bit.  Early stopping as in plan_cn_body: the row's decision words
// are spread over its G H lanes and combined by XOR butterflies, the rows
// of the wave by OR.
template <int DCMAX, int G, int H, class M>
__device__ __forceinline__ void plan_cn_split_body(const PlanCode& C, const PlanStep& S, int64_t lw, int lane) {
    constexpr int R = 64 / (G * H);
    constexpr int Gt = G;
    constexpr int KL = (DCMAX + H - 1) / H;
    static_assert(R >= 1 && KL >= 1, "a wave holds at least one row");
    const QCDesc& D = C.D;
    const int tile = (int)(lw / C.cn_wpt);
    const int rw = (int)(lw - (int64_t)tile * C.cn_wpt);
    const int f = lane % G, h = (lane / G) % H, r = lane / (G * H);
    const int nvalid = min(C.gamma - tile * Gt, Gt);
    if (S.early && S.iter >= 4) {
        const uint64_t* fz = C.frozen + ((size_t)(S.iter - 3) * C.tiles + tile);
        if (M::ld64(C, fz) == ~0ull) return;
    }
    float* mt = C.msg + (size_t)tile * D.E * Gt + f;
    const float* ut = C.mu + (size_t)tile * D.n * Gt + f;
    const int spw = C.cn_wpt / D.J;
    const int j = rw / spw, sw = rw - j * spw;
    const int srow = sw * R + r;
    const bool active = srow < D.p;
    const PlanRow Rw(D, j, active ? srow : 0, active);
    const int d = Rw.d;
    float in[KL];
#pragma unroll
    for (int i = 0; i < KL; ++i) {
        const int k = h + H * i;
        in[i] = 0.0f;
        if (k < d) {
            const float* s = S.iter == 1 ? ut + (size_t)Rw.var(D, k) * Gt : mt + (size_t)Rw.pkg(D, k) * Gt;
            float v[1];
            M::template ld<1>(C, s, v);
            in[i] = v[0];
        }
    }
    const bool syn = S.early && S.iter >= 2;
    uint64_t par = 0;
    if (syn) {
        // lane gi of the row's G H lanes takes variables gi, gi + G H, ...
        const uint64_t* bt = C.bits + ((S.iter - 1) & 1) * C.bits_slot + (size_t)tile * D.n;
        const int gi = lane % (G * H);
#pragma unroll
        for (int q0 = 0; q0 < (DCMAX + G * H - 1) / (G * H); ++q0) {
            const int k = q0 * G * H + gi;
            if (k < d) par ^= M::ld64(C, bt + Rw.var(D, k));
        }
#pragma unroll
        for (int off = G * H / 2; off >= 1; off >>= 1) par ^= __shfl_xor(par, off);
#pragma unroll
        for (int off = 32; off >= G * H; off >>= 1) par |= __shfl_xor(par, off);
    }
    float t[KL], q[KL];
    uint32_t sgn = 0;
#pragma unroll
    for (int i = 0; i < KL; ++i) {
        if (h + H * i < d) {
            tq_of(in[i], t[i], q[i]);
            sgn ^= __float_as_uint(in[i]) & 0x80000000u;
        } else {
            t[i] = 1.0f;
            q[i] = 0.0f;
        }
    }
    // this part's pair, slots in ascending order
    float P = t[0], Q = q[0];
#pragma unroll
    for (int i = 1; i < KL; ++i) {
        Q = fmaf(q[i], P, Q);
        P = P * t[i];
    }
#pragma unroll
    for (int off = G; off < G * H; off <<= 1) sgn ^= __shfl_xor(sgn, off);
    // prefix over parts h' < h and suffix over parts h' > h, each ascending
    float aP = 1.0f, aQ = 0.0f, cP = 1.0f, cQ = 0.0f;
    const int part0 = lane - h * G;
#pragma unroll
    for (int hh = 0; hh < H; ++hh) {
        const float Ph = __shfl(P, part0 + hh * G);
        const float Qh = __shfl(Q, part0 + hh * G);
        if (hh < h) {
            aQ = fmaf(Qh, aP, aQ);
            aP = aP * Ph;
        } else if (hh > h) {
            cQ = fmaf(Qh, cP, cQ);
            cP = cP * Ph;
        }
    }
    // suffix pairs of the own slots, each followed by the later parts
    float sP[KL], sQ[KL];
#pragma unroll
    for (int i = KL - 1; i >= 0; --i) {
        sP[i] = cP;
        sQ[i] = cQ;
        cQ = fmaf(cQ, t[i], q[i]);
        cP = cP * t[i];
    }
#pragma unroll
    for (int i = 0; i < KL; ++i) {
        const int k = h + H * i;
        const float eP = aP * sP[i];
        const float eQ = fmaf(sQ[i], aP, aQ);
        const float mag = kLn2 * __builtin_amdgcn_logf((1.0f + eP) * __builtin_amdgcn_rcpf(eQ));
        aQ = fmaf(q[i], aP, aQ);
        aP = aP * t[i];
        if (k < d) {
            const float o[1] = {__uint_as_float(__float_as_uint(mag) | (sgn ^ (__float_as_uint(in[i]) & 0x80000000u)))};
            M::template st<1>(C, mt + (size_t)Rw.pkg(D, k) * Gt, o);
        }
    }
    if (syn && lane == 0)
        M::st64(C, C.badw + ((S.iter - 1) & 1) * C.badw_slot + lw, par & valid_word<1>(nvalid, 0));
}

// Variable-node pass of iteration S.iter for wave lw of code C: betas (not
// after the last iteration), and with early stopping or at the last
// iteration the packed decisions and the posterior, into slot iter & 1, of
// every frame not known to have stopped.  With early stopping the pass knows
// the stops up to iteration iter-2 (unsat[iter-2] is formed by the flag
// reduction inside this iteration's check launch): a frame that stopped at
// iter-1 is updated once more, into the other slot, and its returned slot
// (iter-1) & 1 is left alone from iteration iter+1 on.  A wave handles V
// groups of R variables; all their loads are issued before the first result
// is stored.
template <int DVMAX, int G, int FPL, int V, class M>
__device__ __forceinline__ void plan_vn_body(const PlanCode& C, const PlanStep& S, int64_t lw, int lane) {
    constexpr int R = 64 / G;
    constexpr int Gt = G * FPL;
    const QCDesc& D = C.D;
    const int tile = (int)(lw / C.vn_wpt);
    const int rw = (int)(lw - (int64_t)tile * C.vn_wpt);
    const int r = lane / G, f = lane % G;
    const int nvalid = min(C.gamma - tile * Gt, Gt);
    // frames that stopped by iteration iter-2 (padding frames count as stopped)
    uint64_t frz[FPL];
    bool any = false, all = true;
#pragma unroll
    for (int i = 0; i < FPL; ++i) {
        uint64_t z = ~valid_word<FPL>(nvalid, i);
        if (S.early && S.iter >= 3) {
            z |= M::ld64(C, C.frozen + ((size_t)(S.iter - 3) * C.tiles + tile) * FPL + i) |
                 ~M::ld64(C, C.unsat + ((size_t)(S.iter - 2) * C.tiles + tile) * FPL + i);
        }
        frz[i] = z;
        any = any || (z & valid_word<FPL>(nvalid, i)) != 0;
        all = all && (z == ~0ull);
    }
    if (S.early && S.iter >= 3 && rw == 0 && lane < FPL)
        M::st64(C, C.frozen + ((size_t)(S.iter - 2) * C.tiles + tile) * FPL + lane, plan_pick<FPL>(frz, lane));
    if (S.early && all) return;
    const size_t lane_off = (size_t)f * FPL;   // lane f of its group: frames f*FPL .. f*FPL+FPL-1
    float* mt = C.msg + (size_t)tile * D.E * Gt + lane_off;
    // the wave's variables: base column l (uniform), offsets sw*V*R .. within it
    const int spw = C.vn_wpt / D.L;
    const int l = rw / spw, sw = rw - l * spw;
    int tcol[V], var[V], dv[V];
    bool active[V];
    float mu[V][FPL], a[V][DVMAX][FPL];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        tcol[v] = (sw * V + v) * R + r;
        active[v] = tcol[v] < D.p;
        var[v] = l * D.p + (active[v] ? tcol[v] : 0);
        const PlanCol Cc(D, l, active[v] ? tcol[v] : 0, active[v]);
        dv[v] = Cc.d;
        if (active[v]) {
            M::template ld<FPL>(C, C.mu + ((size_t)tile * D.n + var[v]) * Gt + lane_off, mu[v]);
        } else {
#pragma unroll
            for (int i = 0; i < FPL; ++i) mu[v][i] = 0.0f;
        }
#pragma unroll
        for (int k = 0; k < DVMAX; ++k) {
            if (k < dv[v]) {
                M::template ld<FPL>(C, mt + (size_t)Cc.pkg(D, k) * Gt, a[v][k]);
            } else {
#pragma unroll
                for (int i = 0; i < FPL; ++i) a[v][k][i] = 0.0f;
            }
        }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const PlanCol Cc(D, l, active[v] ? tcol[v] : 0, active[v]);
        float b[DVMAX][FPL], L[FPL];
        sp_variable<DVMAX, FPL>(mu[v], a[v], b, L);
        if (!S.last) {
#pragma unroll
            for (int k = 0; k < DVMAX; ++k)
                if (k < dv[v]) M::template st<FPL>(C, mt + (size_t)Cc.pkg(D, k) * Gt, b[k]);
        }
        if (S.early || S.last) {
            uint64_t* bw = C.bits + (S.iter & 1) * C.bits_slot + ((size_t)tile * D.n + (active[v] ? var[v] : 0)) * FPL;
            if constexpr (G == 64) {
                // word i, bit j <-> frame FPL * j + i
                uint64_t mine = 0;
#pragma unroll
                for (int i = 0; i < FPL; ++i) {
                    uint64_t w = __ballot(L[i] < 0.0f);
                    if (any) w = (w & ~frz[i]) | (M::ld64(C, bw + i) & frz[i]);
                    if (lane == i) mine = w;
                }
                if (active[v] && lane < FPL) M::st64(C, bw + lane, mine);
            } else {
                // bits r*G .. r*G+G-1 of ballot i are the G lanes of variable
                // r, frames f*FPL + i: word i, bit f; lane f < FPL of the
                // group stores word f
                const uint64_t gmask = (1ull << G) - 1ull;
                uint64_t mine = 0;
#pragma unroll
                for (int i = 0; i < FPL; ++i) {
                    const uint64_t w = (__ballot(active[v] && L[i] < 0.0f) >> (r * G)) & gmask;
                    if (f == i) mine = w;
                }
                if (active[v] && f < FPL) {
                    if (any) {
                        const uint64_t z = plan_pick<FPL>(frz, f);
                        mine = (mine & ~z) | (M::ld64(C, bw + f) & z);
                    }
                    M::st64(C, bw + f, mine);
                }
            }
            if (active[v]) {
                float* pw = C.postw + (S.iter & 1) * C.postw_slot + ((size_t)tile * D.n + var[v]) * Gt + lane_off;
#pragma unroll
                for (int i = 0; i < FPL; ++i) {
                    // frame f*FPL + i: word i, bit f
                    if (!((frz[i] >> f) & 1ull)) M::stf(C, pw + i, clip30(L[i]));
                }
            }
        }
    }
}

// unsat[r][tile] |= OR of the tile's check-wave words of iteration r (badw
// slot r & 1, written by the check launch of iteration r + 1).  Block (code,
// tile, chunk) reads kPlanRedWords consecutive words of the tile (wave w,
// word i at w*fpl + i), kPlanRedPerThread independent loads per thread; 256
// and kPlanRedWords are multiples of fpl, so a thread only meets words of
// i = threadIdx.x % fpl.  The flag words are cleared at ingest and each block
// adds its nonzero words with one atomicOr per i; a tile whose frames had
// all stopped by iteration r-2 skipped that check pass and keeps its zero
// word.  The blocks run inside the check launch of iteration r + 2 (and,
// for r = max_iters - 1, before the final syndrome): no launch of their own.
constexpr int kPlanRedPerThread = 8;
constexpr int kPlanRedWords = 256 * kPlanRedPerThread;

// Block b of code C's flag reduction of iteration r (256 threads; every
// early return is uniform over the block).
template <class M>
__device__ __forceinline__ void plan_unsat_block(const PlanCode& C, int r, int64_t b, uint64_t (&part)[4][4]) {
    const int tile = (int)(b / C.red_chunks);
    const int chunk = (int)(b - (int64_t)tile * C.red_chunks);
    if (tile >= C.tiles) return;
    const int fpl = C.fpl;
    if (r >= 3) {
        const uint64_t* fz = C.frozen + ((size_t)(r - 2) * C.tiles + tile) * fpl;
        bool all = true;
        for (int i = 0; i < fpl; ++i) all = all && (M::ld64(C, fz + i) == ~0ull);
        if (all) return;
    }
    const int64_t nw = (int64_t)C.cn_wpt * fpl;
    const uint64_t* bw = C.badw + (r & 1) * C.badw_slot + (size_t)tile * nw;
    const int64_t w0 = (int64_t)chunk * kPlanRedWords + threadIdx.x;
    uint64_t acc = 0;
#pragma unroll
    for (int k = 0; k < kPlanRedPerThread; ++k) {
        const int64_t w = w0 + (int64_t)k * 256;
        if (w < nw) acc |= M::ld64(C, bw + w);
    }
    for (int off = 32; off >= fpl; off >>= 1) acc |= __shfl_xor(acc, off);
    const int lane = threadIdx.x & 63;
    if (lane < fpl) part[threadIdx.x >> 6][lane] = acc;
    __syncthreads();
    if ((int)threadIdx.x < fpl) {
        const int i = threadIdx.x;
        const uint64_t v = part[0][i] | part[1][i] | part[2][i] | part[3][i];
        if (v) atomicOr((unsigned long long*)(C.unsat + ((size_t)r * C.tiles + tile) * fpl + i),
                        (unsigned long long)v);
    }
}

// One wave of the check-node pass (every layout and row-weight class).
template <class M>
__device__ __forceinline__ void plan_cn_wave(const PlanCode& C, const PlanStep& S, int64_t lw, int lane) {
    if (C.split > 1) {
        PLAN_LAYOUT_SWITCH(C.layout, PLAN_DC_SWITCH(C.dcc, if constexpr (FPL == 1 && G <= 32) {
            if (C.split == 2) {
                plan_cn_split_body<DC, G, 2, M>(C, S, lw, lane);
            } else if (C.split == 4) {
                if constexpr (DC >= 8 && G <= 16) plan_cn_split_body<DC, G, 4, M>(C, S, lw, lane);
            } else {
                if constexpr (DC >= 16 && G == 8) plan_cn_split_body<DC, G, 8, M>(C, S, lw, lane);
            }
        }));
    } else if (C.cpw == 1) {
        PLAN_LAYOUT_SWITCH(C.layout, PLAN_DC_SWITCH(C.dcc, if constexpr (FPL == 1 || DC <= (FPL == 4 ? 6 : 12)) {
            plan_cn_body<DC, G, FPL, 1, M>(C, S, lw, lane);
        }));
    } else if (C.cpw == 2) {
        PLAN_LAYOUT_SWITCH(C.layout, PLAN_DC_SWITCH(C.dcc, if constexpr (FPL == 1 && DC <= 8) {
            plan_cn_body<DC, G, FPL, 2, M>(C, S, lw, lane);
        }));
    } else {
        PLAN_LAYOUT_SWITCH(C.layout, PLAN_DC_SWITCH(C.dcc, if constexpr (FPL == 1 && DC <= 6) {
            plan_cn_body<DC, G, FPL, 4, M>(C, S, lw, lane);
        }));
    }
}

// One wave of the variable-node pass.
template <class M>
__device__ __forceinline__ void plan_vn_wave(const PlanCode& C, const PlanStep& S, int64_t lw, int lane) {
    if (C.vpw == 1) {
        PLAN_LAYOUT_SWITCH(C.layout, PLAN_DV_SWITCH(C.dvc, if constexpr (FPL == 1 || DV <= 8) {
            plan_vn_body<DV, G, FPL, 1, M>(C, S, lw, lane);
        }));
    } else if (C.vpw == 2) {
        PLAN_LAYOUT_SWITCH(C.layout, PLAN_DV_SWITCH(C.dvc, if constexpr (FPL == 1 && DV <= 8) {
            plan_vn_body<DV, G, FPL, 2, M>(C, S, lw, lane);
        }));
    } else {
        PLAN_LAYOUT_SWITCH(C.layout, PLAN_DV_SWITCH(C.dvc, if constexpr (FPL == 1 && DV <= 8) {
            plan_vn_body<DV, G, FPL, 4, M>(C, S, lw, lane);
        }));
    }
}

// Check-node launch of iteration S.iter: blocks below cn_blocks run the
// check waves of every code; with early stopping from iteration 3 on, the
// blocks after them reduce the check words of iteration S.iter - 2.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
plan_cn_kernel(const PlanCode* __restrict__ codes, int ncodes, PlanStep S, int64_t cn_blocks) {
    if ((int64_t)blockIdx.x >= cn_blocks) {
        __shared__ uint64_t part[4][4];
        const int64_t b = (int64_t)blockIdx.x - cn_blocks;
        const PlanCode& C = codes[plan_find(codes, ncodes, b, &PlanCode::red0)];
        plan_unsat_block<PlainMem>(C, S.iter - 2, b - C.red0, part);
        return;
    }
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
    const PlanCode& C = codes[plan_find(codes, ncodes, wave, &PlanCode::cn0)];
    const int64_t lw = wave - C.cn0;
    if (lw >= (int64_t)C.tiles * C.cn_wpt) return;
    plan_cn_wave<PlainMem>(C, S, lw, lane);
}

// 8 waves per SIMD (64 VGPRs; a few values the wave keeps for its whole life
// are spilled): the launch is latency-bound, and the extra waves hide more
// of it than the spills cost.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8)))
plan_vn_kernel(const PlanCode* __restrict__ codes, int ncodes, PlanStep S) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + wave_in_block();
    const PlanCode& C = codes[plan_find(codes, ncodes, wave, &PlanCode::vn0)];
    const int64_t lw = wave - C.vn0;
    if (lw >= (int64_t)C.tiles * C.vn_wpt) return;
    plan_vn_wave<PlainMem>(C, S, lw, lane);
}

// The flag reduction of iteration r = S.iter on its own (the last check
// words, those of iteration max_iters - 1, after the last check launch).
__global__ void __launch_bounds__(256) plan_unsat_kernel(const PlanCode* __restrict__ codes, int ncodes,
                                                         PlanStep S) {
    __shared__ uint64_t part[4][4];
    const PlanCode& C = codes[plan_find(codes, ncodes, blockIdx.x, &PlanCode::red0)];
    plan_unsat_block<PlainMem>(C, S.iter, blockIdx.x - C.red0, part);
}

// Syndrome of the final decisions into unsat[max_iters]: one thread per
// (code, tile, row); each code's threads start at a multiple of 64, so a
// wave belongs to one code; its rows may straddle two tiles.
template <int FPL, class M>
__device__ __forceinline__ void plan_syndrome_body(const PlanCode& C, const PlanStep& S, int64_t t, int lane) {
    const QCDesc& D = C.D;
    const int Gt = C.Gt;
    const int tile = (int)(t / D.m);
    const int row = (int)(t - (int64_t)tile * D.m);
    const bool live = tile < C.tiles;
    uint64_t par[FPL];
#pragma unroll
    for (int i = 0; i < FPL; ++i) par[i] = 0;
    if (live) {
        const QCRow Rw(D, row);
        const uint64_t* bt = C.bits + (S.max_iters & 1) * C.bits_slot + (size_t)tile * D.n * FPL;
        for (int k = 0; k < Rw.d; ++k) {
            const uint64_t* w = bt + (size_t)Rw.var(D, k) * FPL;
#pragma unroll
            for (int i = 0; i < FPL; ++i) par[i] ^= M::ld64(C, w + i);
        }
        const int nvalid = min(C.gamma - tile * Gt, Gt);
#pragma unroll
        for (int i = 0; i < FPL; ++i) par[i] &= valid_word<FPL>(nvalid, i);
    }
    const int tile0 = __shfl(tile, 0);
    const bool same = tile == tile0;
#pragma unroll
    for (int i = 0; i < FPL; ++i) {
        uint64_t v = same ? par[i] : 0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off);
        if (live) {
            uint64_t* un = C.unsat + ((size_t)S.max_iters * C.tiles + tile) * FPL + i;
            if (same) {
                if (lane == 0 && v) atomicOr((unsigned long long*)un, (unsigned long long)v);
            } else if (par[i]) {
                atomicOr((unsigned long long*)un, (unsigned long long)par[i]);
            }
        }
    }
}

template <class M>
__device__ __forceinline__ void plan_syndrome_thread(const PlanCode& C, const PlanStep& S, int64_t t, int lane) {
    if (C.fpl == 4) {
        plan_syndrome_body<4, M>(C, S, t, lane);
    } else if (C.fpl == 2) {
        plan_syndrome_body<2, M>(C, S, t, lane);
    } else {
        plan_syndrome_body<1, M>(C, S, t, lane);
    }
}

__global__ void __launch_bounds__(kBlock) plan_syndrome_kernel(const PlanCode* __restrict__ codes, int ncodes,
                                                               PlanStep S) {
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t wave0 = (int64_t)blockIdx.x * kBlock + wave_in_block() * 64;
    const PlanCode& C = codes[plan_find(codes, ncodes, wave0, &PlanCode::syn0)];
    plan_syndrome_thread<PlainMem>(C, S, gid - C.syn0, threadIdx.x & 63);
}

// Per-frame iteration count and convergence flag from the flag words (frame g
// of code C).
template <class M>
__device__ __forceinline__ void plan_status_thread(const PlanCode& C, const PlanStep& S, int64_t g) {
    if (g >= C.gamma) return;
    const int tile = (int)(g / C.Gt), fl = (int)(g - (int64_t)tile * C.Gt);
    const int w = fl % C.fpl, bit = fl / C.fpl;
    int it = S.max_iters, ok = 0;
    if (S.early) {
        for (int i = 1; i <= S.max_iters; ++i) {
            if (!((M::ld64(C, C.unsat + ((size_t)i * C.tiles + tile) * C.fpl + w) >> bit) & 1ull)) {
                it = i;
                ok = 1;
                break;
            }
        }
    } else {
        ok = !((M::ld64(C, C.unsat + ((size_t)S.max_iters * C.tiles + tile) * C.fpl + w) >> bit) & 1ull);
    }
    if (C.iters) C.iters[g] = it;
    if (C.converged) C.converged[g] = (uint8_t)ok;
    M::st32(C, C.slot + g, (uint32_t)(it & 1));   // the slot that holds iteration `it`
}

__global__ void __launch_bounds__(kBlock) plan_status_kernel(const PlanCode* __restrict__ codes, int ncodes,
                                                             PlanStep S) {
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t wave0 = (int64_t)blockIdx.x * kBlock + wave_in_block() * 64;
    const PlanCode& C = codes[plan_find(codes, ncodes, wave0, &PlanCode::st0)];
    plan_status_thread<PlainMem>(C, S, gid - C.st0);
}

// Ingest: llr [gamma][n] -> mu [tile][n][Gt] (padding frames 0), through LDS,
// 64 variables x 64 frames per block; block 0 of a code clears its flags.
template <class M>
__device__ __forceinline__ void plan_ingest_block(const PlanCode& C, int64_t b, float (&tileS)[64][65]) {
    if (b >= (int64_t)C.io_vchunks * C.io_fchunks) return;
    if (b == 0)
        for (int64_t i = threadIdx.x; i < 2 * C.flag_words; i += 256) M::st64(C, C.unsat + i, 0ull);
    const int n = C.D.n, Gt = C.Gt, gpad = C.tiles * C.Gt;
    const int c0 = (int)(b % C.io_vchunks) * 64, f0 = (int)(b / C.io_vchunks) * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int g = f0 + r, c = c0 + tx;
        float v = 0.0f;
        if (g < C.gamma && c < n) v = C.llr[(size_t)g * n + c];
        tileS[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int c = c0 + r, g = f0 + tx;
        if (c < n && g < gpad) {
            const int tile = g / Gt, fl = g - tile * Gt;
            M::stf(C, C.mu + ((size_t)tile * n + c) * Gt + fl, tileS[tx][r]);
        }
    }
}

__global__ void __launch_bounds__(256) plan_ingest_kernel(const PlanCode* __restrict__ codes, int ncodes) {
    __shared__ float tileS[64][65];
    const PlanCode& C = codes[plan_find(codes, ncodes, blockIdx.x, &PlanCode::io0)];
    plan_ingest_block<PlainMem>(C, blockIdx.x - C.io0, tileS);
}

// Output: posterior and decisions of every frame from the package layout to
// the caller's [gamma][n] buffers, through LDS.
template <class M>
__device__ __forceinline__ void plan_output_block(const PlanCode& C, int64_t b, float (&Ps)[64][65],
                                                  uint8_t (&Bs)[64][65]) {
    if (b >= (int64_t)C.io_vchunks * C.io_fchunks) return;
    const int n = C.D.n, Gt = C.Gt, fpl = C.fpl;
    const int c0 = (int)(b % C.io_vchunks) * 64, f0 = (int)(b / C.io_vchunks) * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int gf = f0 + tx;
    const uint32_t sl = gf < C.gamma ? M::ld32(C, C.slot + gf) : 0u;   // this thread's frame's slot
    const float* pw = C.postw + sl * C.postw_slot;
    const uint64_t* bw = C.bits + sl * C.bits_slot;
    for (int r = ty; r < 64; r += 4) {           // r: variable, tx: frame
        const int c = c0 + r, g = f0 + tx;
        if (c < n && g < C.gamma) {
            const int tile = g / Gt, fl = g - tile * Gt;
            Ps[r][tx] = M::ldf(C, pw + ((size_t)tile * n + c) * Gt + fl);
            const uint64_t w = M::ld64(C, bw + ((size_t)tile * n + c) * fpl + fl % fpl);
            Bs[r][tx] = (uint8_t)((w >> (fl / fpl)) & 1ull);
        }
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {           // r: frame, tx: variable
        const int c = c0 + tx, g = f0 + r;
        if (c < n && g < C.gamma) {
            const size_t o = (size_t)g * n + c;
            C.post[o] = Ps[tx][r];
            C.bits_out[o] = Bs[tx][r];
        }
    }
}

__global__ void __launch_bounds__(256) plan_output_kernel(const PlanCode* __restrict__ codes, int ncodes) {
    __shared__ float Ps[64][65];
    __shared__ uint8_t Bs[64][65];
    const PlanCode& C = codes[plan_find(codes, ncodes, blockIdx.x, &PlanCode::io0)];
    plan_output_block<PlainMem>(C, blockIdx.x - C.io0, Ps, Bs);
}

// ---------------------------------------------------------------------------
// Persistent decode: one launch runs a whole decode of the plan.
//
// The work is cut into tickets.  A ticket is a run of up to
// items_per_ticket consecutive items of one step of one code; an item is 4
// waves of a check- or variable-node pass, or one 256-thread block of the
// other steps.  Tickets are numbered step-major: the ingest of every code,
// then per iteration the check passes of every code, their flag reductions
// (early stopping), their variable passes, and last the final syndrome, the
// frame status and the output.  A workgroup takes the next number from a
// counter.  Before working on a ticket it waits until its code's completion
// counter has counted every ticket of that code's earlier steps, so codes
// advance independently of each other.  A ticket only waits for tickets with
// smaller numbers, and those have all been taken by workgroups already
// running: the launch needs no co-residency and cannot deadlock.
//
// Ordering: everything one ticket hands to another goes through
// device-coherent accesses (CoherentMem: stores write through the L2 of
// their XCD, loads never hit a stale line), so no cache is written back or
// invalidated.  Each wave waits until its stores have completed, then the
// workgroup barrier, then one thread counts the ticket done (an atomic).  The
// waiting thread polls the counter before the barrier that releases its
// workgroup's waves.  (Agent-scope fences instead write back the whole L2 of
// the XCD at every ticket: measured 7-15x slower.)
//
// Each wait is bounded in time.  On expiry the workgroup sets the error word
// and stops; the others stop at their next wait or ticket.  The last
// workgroup to leave resets the counters for the next launch and folds the
// error into the word the host reads (ldpc_plan_check).
// ---------------------------------------------------------------------------
enum PersistKind { kKindIngest = 0, kKindCN, kKindUnsat, kKindVN, kKindSyn, kKindStatus, kKindOut, kKinds };

// Each counter has a 128-byte line of its own: every workgroup takes tickets
// from `next`, and the workgroups waiting on one code poll its `done` line.
struct alignas(128) PersistCounter {
    uint32_t v;
    uint32_t pad[31];
};
struct PersistState {
    PersistCounter next;                          // next ticket number
    PersistCounter exited;                        // workgroups that have left
    PersistCounter err;                           // a wait expired during this launch
    PersistCounter err_sticky;                    // OR of err over launches; read and cleared by the host
    PersistCounter done[LDPC_PLAN_MAX_CODES];     // completed tickets per code (cumulative over the launch)
};

struct PersistArgs {
    int ncodes, max_iters, early, items_per_ticket;
    uint32_t total;                       // tickets of one decode
    uint32_t T0, Titer;                   // tickets of the ingest block, of one iteration block
    uint64_t wait_ticks;                  // bound of one wait, wall-clock ticks
    int32_t tk[kKinds][LDPC_PLAN_MAX_CODES];      // tickets per step kind and code
    int32_t items[kKinds][LDPC_PLAN_MAX_CODES];   // items per step kind and code
};

// kind, code, iteration and ticket index within the (kind, code) step of
// ticket t (t < A.total; wave-uniform)
__device__ __forceinline__ void persist_decode(const PersistArgs& A, uint32_t t, int& kind, int& code, int& iter,
                                               uint32_t& idx) {
    iter = 0;
    if (t < A.T0) {
        kind = kKindIngest;
    } else {
        t -= A.T0;
        const uint32_t body = (uint32_t)A.max_iters * A.Titer;
        if (t < body) {
            iter = (int)(t / A.Titer) + 1;
            t -= (uint32_t)(iter - 1) * A.Titer;
            kind = kKindCN;
        } else {
            t -= body;
            iter = A.max_iters;
            kind = kKindSyn;
        }
    }
    const int last_kind = kind == kKindIngest ? kKindIngest : kind == kKindCN ? kKindVN : kKindOut;
    for (;; ++kind) {
        for (int c = 0; c < A.ncodes; ++c) {
            const uint32_t k = (uint32_t)A.tk[kind][c];
            if (t < k) {
                code = c;
                idx = t;
                return;
            }
            t -= k;
        }
        if (kind == last_kind) break;
    }
    code = 0;   // not reached for t < A.total
    idx = 0;
}

// tickets of code c in the steps before (kind, iter)
__device__ __forceinline__ uint32_t persist_before(const PersistArgs& A, int kind, int c, int iter) {
    const uint32_t per_it = (uint32_t)(A.tk[kKindCN][c] + A.tk[kKindUnsat][c] + A.tk[kKindVN][c]);
    const uint32_t ing = (uint32_t)A.tk[kKindIngest][c];
    switch (kind) {
        case kKindIngest: return 0;
        case kKindCN: return ing + (uint32_t)(iter - 1) * per_it;
        case kKindUnsat: return ing + (uint32_t)(iter - 1) * per_it + A.tk[kKindCN][c];
        case kKindVN: return ing + (uint32_t)(iter - 1) * per_it + A.tk[kKindCN][c] + A.tk[kKindUnsat][c];
        case kKindSyn: return ing + (uint32_t)A.max_iters * per_it;
        case kKindStatus: return ing + (uint32_t)A.max_iters * per_it + A.tk[kKindSyn][c];
        default: return ing + (uint32_t)A.max_iters * per_it + A.tk[kKindSyn][c] + A.tk[kKindStatus][c];
    }
}

// one thread waits until code c has completed `need` tickets; 0 if the wait
// expired or another workgroup reported an expired wait
__device__ __forceinline__ int persist_wait(PersistState* st, int c, uint32_t need, uint64_t limit) {
    if (__hip_atomic_load(&st->done[c].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        const uint64_t t0 = wall_clock64();
        int nap = 1;   // polls back off exponentially (s_sleep units of 64 clocks)
        for (;;) {
            for (int i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(1);
            if (nap < 64) nap *= 2;
            if (__hip_atomic_load(&st->done[c].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) break;
            if (__hip_atomic_load(&st->err.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return 0;
            if (wall_clock64() - t0 > limit) {
                __hip_atomic_fetch_or(&st->err.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return 0;
            }
        }
    }
    return 1;
}

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
plan_persistent_kernel(const PlanCode* __restrict__ codes, PersistState* st, PersistArgs A) {
    __shared__ float lf[64][65];
    __shared__ uint8_t lb[64][65];
    __shared__ uint64_t part[4][4];
    __shared__ uint32_t sh_next;
    __shared__ int sh_go;
    const int lane = threadIdx.x & 63;
    const int wv = wave_in_block();
    if (threadIdx.x == 0) sh_next = __hip_atomic_fetch_add(&st->next.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    uint32_t t = sh_next;
    __syncthreads();
    while (t < A.total) {
        int kind, c, iter;
        uint32_t idx;
        persist_decode(A, t, kind, c, iter, idx);
        if (threadIdx.x == 0) {
            // take the following ticket now (it is processed after this one)
            sh_next = __hip_atomic_fetch_add(&st->next.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t need = persist_before(A, kind, c, iter);
            sh_go = need ? persist_wait(st, c, need, A.wait_ticks) : 1;
        }
        __syncthreads();
        const uint32_t t_next = sh_next;
        if (!sh_go) break;
        const PlanCode& C = codes[c];
        PlanStep S{iter, iter == A.max_iters, A.early, A.max_iters};
        const int64_t i0 = (int64_t)idx * A.items_per_ticket;
        const int64_t i1 = min(i0 + A.items_per_ticket, (int64_t)A.items[kind][c]);
        for (int64_t it = i0; it < i1; ++it) {
            switch (kind) {
                case kKindIngest:
                    plan_ingest_block<CoherentMem>(C, it, lf);
                    __syncthreads();
                    break;
                case kKindCN: {
                    const int64_t lw = it * kWavesPerBlock + wv;
                    if (lw < (int64_t)C.tiles * C.cn_wpt) plan_cn_wave<CoherentMem>(C, S, lw, lane);
                    break;
                }
                case kKindUnsat:
                    if (A.early && iter >= 3) {
                        plan_unsat_block<CoherentMem>(C, iter - 2, it, part);
                        __syncthreads();
                    }
                    break;
                case kKindVN: {
                    const int64_t lw = it * kWavesPerBlock + wv;
                    if (lw < (int64_t)C.tiles * C.vn_wpt) plan_vn_wave<CoherentMem>(C, S, lw, lane);
                    break;
                }
                case kKindSyn: {
                    // first the flag reduction of iteration max_iters - 1, then the final syndrome
                    const int64_t nred = (A.early && A.max_iters >= 2) ? (int64_t)C.tiles * C.red_chunks : 0;
                    if (it < nred) {
                        plan_unsat_block<CoherentMem>(C, A.max_iters - 1, it, part);
                        __syncthreads();
                    } else {
                        plan_syndrome_thread<CoherentMem>(C, S, (it - nred) * kBlock + threadIdx.x, lane);
                    }
                    break;
                }
                case kKindStatus:
                    plan_status_thread<CoherentMem>(C, S, it * kBlock + threadIdx.x);
                    break;
                default:
                    plan_output_block<CoherentMem>(C, it, lf, lb);
                    __syncthreads();
                    break;
            }
        }
        // this wave's stores (write-through) have completed: wait for its
        // vector memory counter (it counts stores on this architecture)
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_fetch_add(&st->done[c].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t = t_next;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t left = __hip_atomic_fetch_add(&st->exited.v, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (left == gridDim.x - 1) {
            // every other workgroup has left: reset the counters for the next launch
            const uint32_t e = __hip_atomic_load(&st->err.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (e) __hip_atomic_fetch_or(&st->err_sticky.v, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&st->err.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&st->next.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int i = 0; i < LDPC_PLAN_MAX_CODES; ++i)
                __hip_atomic_store(&st->done[i].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&st->exited.v, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace ldpc

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

using namespace ldpc;

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kPlanMaxRowWeight = 24;

int plan_dc_class(int d) {
    for (int c : {4, 6, 8, 12, 16, 24})
        if (d <= c) return c;
    return -1;
}
int plan_dv_class(int d) {
    for (int c : {2, 3, 4, 6, 8, 16})
        if (d <= c) return c;
    return -1;
}

bool layout_allowed(const ldpc_graph* g, int l) {
    if (l < 0 || l >= kLayoutValues || layout_base(l) >= kPlanLayouts || ((l >> 4) & 3) == 3 || ((l >> 6) & 3) == 3)
        return false;
    if (const int H = layout_split(l); H > 1) {
        // G8, G16, G32 with one frame per lane and one row group per check
        // wave; at least two edges per lane (the kernel's instantiations)
        if (layout_base(l) > 2 || layout_cpw(l) > 1 || layout_g(l) * H > 64 || g->dc_max < 2 * H) return false;
    }
    if (layout_vpw(l) > 1 && (layout_fpl(l) != 1 || g->dv_max > 8)) return false;
    if (layout_cpw(l) > 1 && (layout_fpl(l) != 1 || g->dc_max > (layout_cpw(l) == 2 ? 8 : 6))) return false;
    if (layout_fpl(l) == 4) return g->dc_max <= 6 && g->dv_max <= 8;
    if (layout_fpl(l) == 2) return g->dc_max <= 12 && g->dv_max <= 8;
    return true;
}

struct CodeRegion {
    int tiles, Gt, cn_wpt;
    int64_t flag_words;
    size_t mu, msg, postw, bits, flags, badw, slot, total;
    int64_t bits_slot, postw_slot, badw_slot;   // elements per slot (two slots each)
};

// check-node waves per tile: per base row, enough waves for its p rows
int plan_cn_wpt(const ldpc_graph* g, int l) {
    const int rows = (64 / (layout_g(l) * layout_split(l))) * layout_cpw(l);
    return g->J * ((g->p + rows - 1) / rows);
}

CodeRegion code_region(const ldpc_graph* g, int gamma, int layout, int max_iters) {
    CodeRegion R{};
    R.Gt = layout_g(layout) * layout_fpl(layout);
    R.tiles = (gamma + R.Gt - 1) / R.Gt;
    const size_t gpad = (size_t)R.tiles * R.Gt;
    R.flag_words = (int64_t)(max_iters + 1) * R.tiles * layout_fpl(layout);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    R.postw_slot = (int64_t)gpad * g->n;
    R.bits_slot = (int64_t)R.tiles * g->n * layout_fpl(layout);
    R.cn_wpt = plan_cn_wpt(g, layout);
    R.badw_slot = (int64_t)R.tiles * R.cn_wpt * layout_fpl(layout);
    R.mu = take(gpad * g->n * sizeof(float));
    R.msg = take(gpad * g->E * sizeof(float));
    R.postw = take(2 * (size_t)R.postw_slot * sizeof(float));
    R.bits = take(2 * (size_t)R.bits_slot * sizeof(uint64_t));
    R.flags = take(2 * (size_t)R.flag_words * sizeof(uint64_t));
    R.badw = take(2 * (size_t)R.badw_slot * sizeof(uint64_t));
    R.slot = take(gpad * sizeof(uint32_t));
    R.total = off;
    return R;
}

// default layout: the smallest G >= gamma (at least 8); 64 frames per lane
// group with 4 frames per lane when the row weight allows it and the padding
// stays under 1/8
int default_layout(const ldpc_graph* g, int gamma) {
    if (gamma <= 8) return 0;
    if (gamma <= 16) return 1;
    if (gamma <= 32) return 2;
    const int base = (gamma + 63) / 64 * 64;
    if (layout_allowed(g, 4) && (gamma + 255) / 256 * 256 * 8 <= base * 9) return 4;
    if (layout_allowed(g, 5) && (gamma + 127) / 128 * 128 * 8 <= base * 9) return 5;
    return 3;
}

}  // namespace

struct ldpc_plan {
    int ncodes = 0, max_iters = 0, early = 0;
    std::vector<const ldpc_graph*> graphs;
    std::vector<int> gammas, layouts;
    std::vector<size_t> region_off;       // byte offset of each code's region in the workspace
    size_t table_bytes = 0, ws_bytes = 0;
    std::vector<PlanCode> table;          // host copy of the device table
    // launch geometry
    int64_t cn_waves = 0, vn_waves = 0, syn_threads = 0, st_threads = 0, io_blocks = 0, red_blocks = 0;
    // what the device table currently describes
    bool table_valid = false;
    const void* table_ws = nullptr;
    uint64_t generation = 1;              // bumped whenever layouts or bound buffers change
    // persistent launch (ldpc_plan_set_persistent)
    int persistent = 0;
    int64_t wait_us = 2000000;
    uint64_t wait_ticks = 0;              // wait_us in device wall-clock ticks
    int persist_grid = 0;                 // workgroups: what fits the device at once
    size_t state_off = 0;                 // PersistState in the workspace
    PersistArgs pa{};
    // codes decoded by the on-chip block decoder (onchip.hip) instead of the
    // phase launches: decided when the table is built (phase launches only,
    // as ldpc_decode decides), launched on a stream forked from the caller's
    std::vector<uint8_t> onchip;
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    // graph
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t graph_generation = 0;
};

namespace {

struct PlanBuffers {
    const float* const* llr;
    float* const* post;
    uint8_t* const* bits;
    int32_t* const* iters;
    uint8_t* const* converged;
};

ldpc_status check_buffers(const ldpc_plan* P, const PlanBuffers& B, const void* ws, size_t ws_bytes) {
    if (!B.llr || !B.post || !B.bits) return LDPC_EINVAL;
    for (int c = 0; c < P->ncodes; ++c) {
        if (!B.llr[c] || !B.post[c] || !B.bits[c]) return LDPC_EINVAL;
        if ((reinterpret_cast<uintptr_t>(B.llr[c]) | reinterpret_cast<uintptr_t>(B.post[c])) & 3) return LDPC_EINVAL;
        if (B.iters && B.iters[c] && (reinterpret_cast<uintptr_t>(B.iters[c]) & 3)) return LDPC_EINVAL;
    }
    if (!ws || ws_bytes < P->ws_bytes) return LDPC_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) & 255) return LDPC_EINVAL;
    return LDPC_OK;
}

// items per ticket of the persistent launch; LDPC_PLAN_TICKET_ITEMS (1..64)
// overrides the default
int persist_items_per_ticket() {
    const char* env = std::getenv("LDPC_PLAN_TICKET_ITEMS");
    const int v = env ? std::atoi(env) : 0;
    return v >= 1 && v <= 64 ? v : 2;
}

// fill the host table for the current layouts and buffers
std::vector<uint8_t> onchip_choice(const ldpc_plan* P) {
    std::vector<uint8_t> v(P->ncodes, 0);
    if (!P->persistent)
        for (int c = 0; c < P->ncodes; ++c) v[c] = onchip_selected(P->graphs[c]) ? 1 : 0;
    return v;
}

void build_table(ldpc_plan* P, const PlanBuffers& B, char* ws) {
    P->table.assign(P->ncodes, PlanCode{});
    P->onchip = onchip_choice(P);
    int64_t cn = 0, vn = 0, syn = 0, st = 0, io = 0, red = 0;
    for (int c = 0; c < P->ncodes; ++c) {
        const ldpc_graph* g = P->graphs[c];
        const int l = P->layouts[c];
        const CodeRegion R = code_region(g, P->gammas[c], l, P->max_iters);
        char* base = ws + P->region_off[c];
        PlanCode& T = P->table[c];
        T.D = g->qc;
        T.mu = reinterpret_cast<float*>(base + R.mu);
        T.msg = reinterpret_cast<float*>(base + R.msg);
        T.postw = reinterpret_cast<float*>(base + R.postw);
        T.bits = reinterpret_cast<uint64_t*>(base + R.bits);
        T.unsat = reinterpret_cast<uint64_t*>(base + R.flags);
        T.badw = reinterpret_cast<uint64_t*>(base + R.badw);
        T.slot = reinterpret_cast<uint32_t*>(base + R.slot);
        T.bits_slot = R.bits_slot;
        T.postw_slot = R.postw_slot;
        T.badw_slot = R.badw_slot;
        T.frozen = T.unsat + R.flag_words;
        T.region = base;
        T.llr = B.llr[c];
        T.post = B.post[c];
        T.bits_out = B.bits[c];
        T.iters = B.iters ? B.iters[c] : nullptr;
        T.converged = B.converged ? B.converged[c] : nullptr;
        T.flag_words = R.flag_words;
        T.gamma = P->gammas[c];
        T.tiles = R.tiles;
        T.layout = layout_base(l);
        T.Gt = R.Gt;
        T.fpl = layout_fpl(l);
        T.dcc = plan_dc_class(g->dc_max);
        T.dvc = plan_dv_class(g->dv_max);
        const int rows_per_wave = 64 / layout_g(l);
        T.vpw = layout_vpw(l);
        T.cpw = layout_cpw(l);
        T.split = layout_split(l);
        // waves per tile: per base row (column), enough waves for its p rows (variables)
        T.cn_wpt = plan_cn_wpt(g, l);
        T.vn_wpt = g->L * ((g->p + rows_per_wave * T.vpw - 1) / (rows_per_wave * T.vpw));
        T.io_vchunks = (g->n + 63) / 64;
        T.io_fchunks = (R.tiles * R.Gt + 63) / 64;
        T.cn0 = cn;
        T.vn0 = vn;
        T.syn0 = syn;
        T.st0 = st;
        T.io0 = io;
        T.red0 = red;
        T.red_chunks = (int)(((int64_t)T.cn_wpt * T.fpl + kPlanRedWords - 1) / kPlanRedWords);
        if (P->onchip[c]) continue;   // no work in the phase launches: an empty range in each
        cn += (int64_t)T.tiles * T.cn_wpt;
        vn += (int64_t)T.tiles * T.vn_wpt;
        syn += ((int64_t)T.tiles * g->m + 63) / 64 * 64;
        st += ((int64_t)T.gamma + 63) / 64 * 64;
        io += (int64_t)T.io_vchunks * T.io_fchunks;
        red += (int64_t)T.tiles * T.red_chunks;
    }
    // persistent launch: items and tickets per step kind and code
    PersistArgs& A = P->pa;
    A = PersistArgs{};
    A.ncodes = P->ncodes;
    A.max_iters = P->max_iters;
    A.early = P->early;
    A.items_per_ticket = persist_items_per_ticket();
    uint64_t T0 = 0, Titer = 0, Ttail = 0;
    for (int c = 0; c < P->ncodes; ++c) {
        const PlanCode& T = P->table[c];
        const ldpc_graph* g = P->graphs[c];
        const int64_t io = (int64_t)T.io_vchunks * T.io_fchunks;
        const int64_t items[kKinds] = {io,
                                       ((int64_t)T.tiles * T.cn_wpt + kWavesPerBlock - 1) / kWavesPerBlock,
                                       P->early ? (int64_t)T.tiles * T.red_chunks : 0,
                                       ((int64_t)T.tiles * T.vn_wpt + kWavesPerBlock - 1) / kWavesPerBlock,
                                       ((int64_t)T.tiles * g->m + kBlock - 1) / kBlock +
                                           (P->early && P->max_iters >= 2 ? (int64_t)T.tiles * T.red_chunks : 0),
                                       ((int64_t)T.gamma + kBlock - 1) / kBlock,
                                       io};
        for (int k = 0; k < kKinds; ++k) {
            A.items[k][c] = (int32_t)items[k];
            A.tk[k][c] = (int32_t)((items[k] + A.items_per_ticket - 1) / A.items_per_ticket);
        }
        T0 += A.tk[kKindIngest][c];
        Titer += A.tk[kKindCN][c] + A.tk[kKindUnsat][c] + A.tk[kKindVN][c];
        Ttail += A.tk[kKindSyn][c] + A.tk[kKindStatus][c] + A.tk[kKindOut][c];
    }
    uint64_t total = T0 + (uint64_t)P->max_iters * Titer + Ttail;
    for (int c = 0; c < P->ncodes; ++c)   // coherent accesses use 31-bit offsets within a code's region
        if (code_region(P->graphs[c], P->gammas[c], P->layouts[c], P->max_iters).total >= ((size_t)1 << 31))
            total = 0;
    A.T0 = (uint32_t)T0;
    A.Titer = (uint32_t)Titer;
    A.total = total < ((uint64_t)1 << 31) ? (uint32_t)total : 0u;   // 0: the launch cannot take this plan
    P->red_blocks = red;
    P->cn_waves = cn;
    P->vn_waves = vn;
    P->syn_threads = syn;
    P->st_threads = st;
    P->io_blocks = io;
}

bool same_buffers(const ldpc_plan* P, const PlanBuffers& B, const void* ws) {
    if (!P->table_valid || P->table_ws != ws) return false;
    if (P->onchip != onchip_choice(P)) return false;
    for (int c = 0; c < P->ncodes; ++c) {
        const PlanCode& T = P->table[c];
        if (T.llr != B.llr[c] || T.post != B.post[c] || T.bits_out != B.bits[c]) return false;
        if (T.iters != (B.iters ? B.iters[c] : nullptr)) return false;
        if (T.converged != (B.converged ? B.converged[c] : nullptr)) return false;
    }
    return true;
}

// make the device table describe (layouts, B, ws); synchronous when it changes
ldpc_status upload_table(ldpc_plan* P, const PlanBuffers& B, char* ws, hipStream_t st) {
    if (same_buffers(P, B, ws)) return LDPC_OK;
    build_table(P, B, ws);
    bool any = false;
    for (uint8_t o : P->onchip) any = any || o;
    if (any && !P->side) {
        // default priority, like every stream of the library
        if (hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking) != hipSuccess) {
            P->side = nullptr;
            return LDPC_EHIP;
        }
        if (hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&P->join_ev, hipEventDisableTiming) != hipSuccess)
            return LDPC_EHIP;
    }
    // the table, then the persistent launch's counters (zero)
    std::vector<char> host(P->state_off + sizeof(PersistState), 0);
    std::memcpy(host.data(), P->table.data(), P->table.size() * sizeof(PlanCode));
    if (hipMemcpyAsync(ws, host.data(), host.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return LDPC_EHIP;
    P->table_valid = true;
    P->table_ws = ws;
    P->generation += 1;
    return LDPC_OK;
}

unsigned blocks_for(int64_t units, int per_block) { return (unsigned)((units + per_block - 1) / per_block); }

void enqueue_phases(ldpc_plan* P, const PlanCode* T, hipStream_t st);

// enqueue one whole decode of the plan on st (table already on the device);
// false when an on-chip launch could not be made
bool enqueue(ldpc_plan* P, char* ws, hipStream_t st) {
    const PlanCode* T = reinterpret_cast<const PlanCode*>(ws);
    const int nc = P->ncodes;
    if (P->persistent) {
        PersistArgs A = P->pa;
        A.wait_ticks = P->wait_ticks;
        timing::Scope ts(22, st);
        plan_persistent_kernel<<<(unsigned)std::min<int64_t>(P->persist_grid, A.total), kBlock, 0, st>>>(
            T, reinterpret_cast<PersistState*>(ws + P->state_off), A);
        return true;
    }
    bool ok = true;
    // codes on chip: one launch each on the side stream, forked from st and
    // joined back at the end (under capture, a parallel branch of the graph)
    bool any_onchip = false;
    for (uint8_t o : P->onchip) any_onchip = any_onchip || o;
    if (any_onchip) {
        (void)hipEventRecord(P->fork_ev, st);
        (void)hipStreamWaitEvent(P->side, P->fork_ev, 0);
        for (int c = 0; c < nc; ++c) {
            if (!P->onchip[c]) continue;
            const PlanCode& H = P->table[c];
            ok = ok && onchip_decode(P->graphs[c], H.llr, H.gamma, P->max_iters, P->early, H.post, H.bits_out,
                                     H.iters, H.converged, P->side) > 0;
        }
        (void)hipEventRecord(P->join_ev, P->side);
    }
    if (P->cn_waves > 0) enqueue_phases(P, T, st);
    if (any_onchip) (void)hipStreamWaitEvent(st, P->join_ev, 0);
    return ok;
}

// the phase launches of the codes that are not decoded on chip
void enqueue_phases(ldpc_plan* P, const PlanCode* T, hipStream_t st) {
    const int nc = P->ncodes;
    PlanStep S{0, 0, P->early, P->max_iters};
    {
        timing::Scope ts(17, st);
        plan_ingest_kernel<<<(unsigned)P->io_blocks, 256, 0, st>>>(T, nc);
    }
    const unsigned cn_grid = blocks_for(P->cn_waves, kWavesPerBlock);
    const unsigned vn_grid = blocks_for(P->vn_waves, kWavesPerBlock);
    for (int it = 1; it <= P->max_iters; ++it) {
        S.iter = it;
        S.last = it == P->max_iters;
        {
            // with early stopping the check launch also reduces the check
            // words of iteration it - 2 (blocks after the check waves)
            timing::Scope ts(18, st);
            const unsigned red = (P->early && it >= 3) ? (unsigned)P->red_blocks : 0u;
            plan_cn_kernel<<<cn_grid + red, kBlock, 0, st>>>(T, nc, S, (int64_t)cn_grid);
        }
        {
            timing::Scope ts(19, st);
            plan_vn_kernel<<<vn_grid, kBlock, 0, st>>>(T, nc, S);
        }
    }
    timing::Scope ts(20, st);
    if (P->early && P->max_iters >= 2) {
        S.iter = P->max_iters - 1;   // the check words of the last-but-one iteration
        plan_unsat_kernel<<<(unsigned)P->red_blocks, 256, 0, st>>>(T, nc, S);
    }
    S.iter = P->max_iters;
    plan_syndrome_kernel<<<blocks_for(P->syn_threads, kBlock), kBlock, 0, st>>>(T, nc, S);
    plan_status_kernel<<<blocks_for(P->st_threads, kBlock), kBlock, 0, st>>>(T, nc, S);
    plan_output_kernel<<<(unsigned)P->io_blocks, 256, 0, st>>>(T, nc);
}

void drop_graph(ldpc_plan* P) {
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    P->exec = nullptr;
    P->graph = nullptr;
    P->graph_generation = 0;
}

PlanBuffers make_buffers(const float* const* llr, float* const* post, uint8_t* const* bits, int32_t* const* iters,
                         uint8_t* const* converged) {
    return PlanBuffers{llr, post, bits, iters, converged};
}

}  // namespace

extern "C" {

ldpc_status ldpc_plan_create(const ldpc_graph* const* graphs, const int32_t* gammas, int32_t ncodes,
                             int32_t max_iters, int32_t early_stop, ldpc_plan** out) {
    if (!out) return LDPC_EINVAL;
    *out = nullptr;
    if (!graphs || !gammas || ncodes < 1 || ncodes > LDPC_PLAN_MAX_CODES) return LDPC_EINVAL;
    if (max_iters < 1 || max_iters > LDPC_MAX_ITERS) return LDPC_EINVAL;
    for (int c = 0; c < ncodes; ++c) {
        if (!graphs[c] || graphs[c]->kind != LDPC_GRAPH_QC || gammas[c] < 1) return LDPC_EINVAL;
        if (graphs[c]->dc_max > kPlanMaxRowWeight) return LDPC_EUNSUPPORTED;
        if ((int64_t)gammas[c] * graphs[c]->n > ((int64_t)1 << 40)) return LDPC_EUNSUPPORTED;
    }
    ldpc_plan* P = new (std::nothrow) ldpc_plan();
    if (!P) return LDPC_ENOMEM;
    P->ncodes = ncodes;
    P->max_iters = max_iters;
    P->early = early_stop ? 1 : 0;
    P->graphs.assign(graphs, graphs + ncodes);
    P->gammas.assign(gammas, gammas + ncodes);
    P->layouts.resize(ncodes);
    P->state_off = align256((size_t)ncodes * sizeof(PlanCode));
    P->table_bytes = align256(P->state_off + sizeof(PersistState));
    size_t off = P->table_bytes;
    for (int c = 0; c < ncodes; ++c) {
        P->layouts[c] = default_layout(graphs[c], gammas[c]);
        size_t most = 0;
        for (int l = 0; l < kLayoutValues; ++l)
            if (layout_allowed(graphs[c], l)) most = std::max(most, code_region(graphs[c], gammas[c], l, max_iters).total);
        P->region_off.push_back(off);
        off = align256(off + most);
    }
    P->ws_bytes = off;
    *out = P;
    return LDPC_OK;
}

void ldpc_plan_destroy(ldpc_plan* P) {
    if (!P) return;
    drop_graph(P);
    if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
    if (P->side) (void)hipStreamDestroy(P->side);
    if (P->fork_ev) (void)hipEventDestroy(P->fork_ev);
    if (P->join_ev) (void)hipEventDestroy(P->join_ev);
    delete P;
}

ldpc_status ldpc_plan_workspace_size(const ldpc_plan* P, size_t* bytes) {
    if (!P || !bytes) return LDPC_EINVAL;
    *bytes = P->ws_bytes;
    return LDPC_OK;
}

ldpc_status ldpc_plan_set_layout(ldpc_plan* P, int32_t code, int32_t layout) {
    if (!P || code < 0 || code >= P->ncodes) return LDPC_EINVAL;
    if (layout == -1) layout = default_layout(P->graphs[code], P->gammas[code]);
    if (!layout_allowed(P->graphs[code], layout)) return LDPC_EINVAL;
    if (P->layouts[code] != layout) {
        P->layouts[code] = layout;
        P->table_valid = false;
    }
    return LDPC_OK;
}

ldpc_status ldpc_plan_get_layout(const ldpc_plan* P, int32_t code, int32_t* layout) {
    if (!P || !layout || code < 0 || code >= P->ncodes) return LDPC_EINVAL;
    *layout = P->layouts[code];
    return LDPC_OK;
}

ldpc_status ldpc_plan_decode(ldpc_plan* P, const float* const* llr, float* const* post, uint8_t* const* bits,
                             int32_t* const* iters, uint8_t* const* converged, void* workspace,
                             size_t workspace_bytes, void* stream) {
    if (!P) return LDPC_EINVAL;
    const PlanBuffers B = make_buffers(llr, post, bits, iters, converged);
    ldpc_status chk = check_buffers(P, B, workspace, workspace_bytes);
    if (chk != LDPC_OK) return chk;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(workspace);
    (void)hipGetLastError();
    ldpc_status up = upload_table(P, B, ws, st);
    if (up != LDPC_OK) return up;
    if (P->persistent && P->pa.total == 0) return LDPC_EUNSUPPORTED;
    const bool ok = enqueue(P, ws, st);
    return ok && hipGetLastError() == hipSuccess ? LDPC_OK : LDPC_EHIP;
}

ldpc_status ldpc_plan_capture(ldpc_plan* P, const float* const* llr, float* const* post, uint8_t* const* bits,
                              int32_t* const* iters, uint8_t* const* converged, void* workspace,
                              size_t workspace_bytes, void* stream) {
    if (!P) return LDPC_EINVAL;
    const PlanBuffers B = make_buffers(llr, post, bits, iters, converged);
    ldpc_status chk = check_buffers(P, B, workspace, workspace_bytes);
    if (chk != LDPC_OK) return chk;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(workspace);
    (void)hipGetLastError();
    ldpc_status up = upload_table(P, B, ws, st);
    if (up != LDPC_OK) return up;
    if (P->persistent && P->pa.total == 0) return LDPC_EUNSUPPORTED;
    if (!P->cap_stream && hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        P->cap_stream = nullptr;
        return LDPC_EHIP;
    }
    drop_graph(P);
    const bool timing_was = timing::set_enabled(false);
    hipError_t e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const bool ok = enqueue(P, ws, P->cap_stream);
        e = hipStreamEndCapture(P->cap_stream, &P->graph);
        if (e == hipSuccess && !ok) e = hipErrorLaunchFailure;
    }
    timing::set_enabled(timing_was);
    if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(P);
        (void)hipGetLastError();
        return LDPC_EHIP;
    }
    P->graph_generation = P->generation;
    return LDPC_OK;
}

ldpc_status ldpc_plan_replay(ldpc_plan* P, void* stream) {
    if (!P) return LDPC_EINVAL;
    if (!P->exec || P->graph_generation != P->generation || !P->table_valid) return LDPC_EINVAL;
    (void)hipGetLastError();
    if (hipGraphLaunch(P->exec, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return LDPC_EHIP;
    return LDPC_OK;
}

ldpc_status ldpc_plan_autotune(ldpc_plan* P, const float* const* llr, float* const* post, uint8_t* const* bits,
                               int32_t* const* iters, uint8_t* const* converged, void* workspace,
                               size_t workspace_bytes, int32_t trials, void* stream, double* best_ms) {
    if (!P || trials < 1) return LDPC_EINVAL;
    const PlanBuffers B = make_buffers(llr, post, bits, iters, converged);
    ldpc_status chk = check_buffers(P, B, workspace, workspace_bytes);
    if (chk != LDPC_OK) return chk;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(workspace);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return LDPC_EHIP;
    }
    const bool timing_was = timing::set_enabled(false);
    // time of one whole decode with the current layouts (after one warm-up)
    auto measure = [&](double& out) -> ldpc_status {
        (void)hipGetLastError();
        ldpc_status up = upload_table(P, B, ws, st);
        if (up != LDPC_OK) return up;
        if (P->persistent && P->pa.total == 0) return LDPC_EUNSUPPORTED;
        bool ok = enqueue(P, ws, st);
        float ms = 0.0f;
        if (hipEventRecord(e0, st) != hipSuccess) return LDPC_EHIP;
        for (int t = 0; t < trials; ++t) ok = enqueue(P, ws, st) && ok;
        if (!ok) return LDPC_EHIP;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess)
            return LDPC_EHIP;
        out = (double)ms / trials;
        return LDPC_OK;
    };
    // one pass of coordinate descent: each code in turn tries its other
    // layouts with the rest of the plan fixed, and keeps the fastest whole decode
    double best = 0.0;
    ldpc_status status = measure(best);
    for (int c = 0; c < P->ncodes && status == LDPC_OK; ++c) {
        if (P->onchip[c]) continue;   // decoded on chip: its lane layout is not used
        const int start = P->layouts[c];
        int keep = start;
        for (int l = 0; l < kLayoutValues && status == LDPC_OK; ++l) {
            if (l == start || !layout_allowed(P->graphs[c], l)) continue;
            const int tile = layout_g(l) * layout_fpl(l);
            if (tile > 8 && tile / 2 >= P->gammas[c]) continue;   // tiles at most the next power of two
            P->layouts[c] = l;
            P->table_valid = false;
            double ms = 0.0;
            status = measure(ms);
            if (status == LDPC_OK && ms < best) {
                best = ms;
                keep = l;
            }
        }
        P->layouts[c] = keep;
        P->table_valid = false;
    }
    timing::set_enabled(timing_was);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status == LDPC_OK && best_ms) *best_ms = best;
    return status;
}

ldpc_status ldpc_plan_set_persistent(ldpc_plan* P, int32_t on, int64_t wait_limit_us) {
    if (!P || (on != 0 && on != 1) || wait_limit_us < 0) return LDPC_EINVAL;
    const int64_t us = wait_limit_us ? wait_limit_us : 2000000;
    if (on) {
        int dev = 0, cus = 0, per_cu = 0, rate_khz = 0;
        (void)hipGetLastError();
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, plan_persistent_kernel, kBlock, 0) != hipSuccess ||
            cus < 1 || per_cu < 1 || rate_khz < 1) {
            (void)hipGetLastError();
            return LDPC_EHIP;
        }
        P->persist_grid = cus * per_cu;
        P->wait_ticks = (uint64_t)us * (uint64_t)rate_khz / 1000u;
        if (P->wait_ticks == 0) P->wait_ticks = 1;
    }
    P->wait_us = us;
    if (P->persistent != on) {
        P->persistent = on;
        P->generation += 1;   // a captured graph holds the other form
    }
    return LDPC_OK;
}

ldpc_status ldpc_plan_check(ldpc_plan* P, void* workspace, void* stream) {
    if (!P || !workspace) return LDPC_EINVAL;
    if (!P->table_valid || P->table_ws != workspace) return LDPC_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* w = reinterpret_cast<char*>(workspace) + P->state_off + offsetof(PersistState, err_sticky.v);
    uint32_t err = 0;
    (void)hipGetLastError();
    if (hipMemcpyAsync(&err, w, sizeof(err), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return LDPC_EHIP;
    if (!err) return LDPC_OK;
    const uint32_t zero = 0;
    if (hipMemcpyAsync(w, &zero, sizeof(zero), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return LDPC_EHIP;
    return LDPC_EHIP;
}

}  // extern "C"
