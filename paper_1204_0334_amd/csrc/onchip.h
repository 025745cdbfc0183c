// Block decoder with one frame per workgroup, decoded on one compute unit
// without message traffic to HBM (onchip.hip).  Called by ldpc_decode when
// the code fits; the message-package decoder of decode.hip takes the rest.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "internal.h"

namespace ldpc {

// Whether a graph fits the on-chip decoder on the current device (QC graph,
// every base column nonzero, an instantiation for its base height, row
// weight and circulant size, and two posterior arrays of n floats in LDS).
bool onchip_fits(const ldpc_graph* g);

// Whether ldpc_decode decodes g on chip: the graph fits and the environment
// variable LDPC_BLOCK_PATH is not "packages" (the rule ldpc_decode applies).
bool onchip_selected(const ldpc_graph* g);

// Enqueues the whole decode (arguments as ldpc_decode; outputs written
// directly in the caller's layout; nms_w: NULL for sum-product, else the
// learned min-sum weights of ldpc_nms_decode).  Returns 1 once launched, 0
// (having enqueued nothing) when the graph does not fit, -1 when the launch
// failed.
int onchip_decode(const ldpc_graph* g, const float* llr, int gamma, int max_iters, int early, float* post,
                  uint8_t* bits, int32_t* iters, uint8_t* converged, hipStream_t st, const float* nms_w = nullptr);

}  // namespace ldpc
