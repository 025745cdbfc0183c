// Internal descriptors shared by the host graph code and the HIP decoders.
//
// A graph is a host object.  What the kernels need of it fits in a few
// kilobytes and travels by value in the kernel arguments: per circulant block
// one column (or row) index and one shift.  Per-edge addresses are computed
// from those (row (j, s) of block (j, l) meets column (l, (s + a) mod p)), so
// no per-edge index table is read from memory.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <vector>

#include "../../include/ldpc.h"

namespace ldpc {

// Block code: the nonzero circulants ("edge blocks") of the J x L base are
// numbered row by row, left to right.  Edge block b holds the p packages of
// its p edges, package b*p + s belonging to check row s of the block.
struct QCDesc {
    int32_t J, L, p, n, m, E, nb;
    int32_t dc_max, dv_max;
    uint16_t rstart[LDPC_MAX_BASE_ROWS + 1];  // edge blocks of base row j: rstart[j] .. rstart[j+1]-1
    uint16_t cstart[LDPC_MAX_BASE_COLS + 1];  // cedge[cstart[l] .. cstart[l+1]-1]: edge blocks of base column l
    uint8_t ecol[LDPC_MAX_BLOCKS];            // base column of edge block b
    uint16_t cedge[LDPC_MAX_BLOCKS];          // edge blocks per base column, ascending base row
    int32_t eshift[LDPC_MAX_BLOCKS];          // circulant shift of edge block b
};

// Terminated periodic convolutional code, stored as syndrome-former shifts
// sf[i][d][rr][q] (class i = layer mod T, lag d = layer - position).
// Window decoding keeps the messages of R = W + ms positions in a ring; the
// edges of position t live in ring slot t mod R, grouped by (d, rr, q)
// blocks of p packages (package s of block (d, rr, q) = the edge of check
// row s of circulant row rr of layer t + d).
struct ConvDesc {
    int32_t T, ms, Jb, Lb, p, c, cb, positions, layers;
    int32_t dc_max, dv_max;
    int32_t sf[LDPC_MAX_BLOCKS];              // [T][ms+1][Jb][Lb], -1 = zero block
};

// Kernel timing (ldpc_timing_enable / ldpc_timing_read): while enabled, a
// Scope records a pair of events around the launches it brackets.
namespace timing {
struct Scope {
    int idx = -1;
    hipStream_t st;
    Scope(int cls, hipStream_t s);
    ~Scope();
};
// turns recording off (for stream capture) and returns the previous state
bool set_enabled(bool on);
}  // namespace timing

}  // namespace ldpc

struct ldpc_graph {
    int32_t kind;              // ldpc_graph_kind
    int32_t J, L, p;           // QC base (for a convolutional graph built from QC: that base, else 0)
    std::vector<int32_t> shifts;
    int32_t T, ms, Jb, Lb, positions, terminate, layers;
    std::vector<int32_t> sf;
    int32_t n, m, E, dv_max, dc_max;
    double rate;
    ldpc::QCDesc qc;
    ldpc::ConvDesc cv;
};
