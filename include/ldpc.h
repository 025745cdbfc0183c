/*
 * ldpc.h -- batched sum-product decoding of quasi-cyclic LDPC block codes and
 * of LDPC convolutional codes unwrapped from them, on one AMD Instinct MI355X
 * (gfx950).
 *
 * Method: Y. Zhao and F. C. M. Lau, "Implementation of Decoders for LDPC Block
 * Codes and LDPC Convolutional Codes Based on GPUs" (arXiv:1204.0334).
 * Gamma codewords that share one Tanner graph are decoded together (Sec. IV-A)
 * with the flooding belief-propagation of Algorithm 1: check-node update
 * (horizontal step), variable-node update and a-posteriori LLR (vertical
 * step), hard decision.
 *
 * Conventions for every entry point
 *   - Return value: LDPC_OK (0) or a negative ldpc_status.  Nothing throws
 *     across this interface.
 *   - All arguments are validated on the host before anything is enqueued; a
 *     call that returns an error has launched nothing and written nothing.
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary CPU memory.  The caller owns every buffer; the
 *     library never allocates device memory (the decoders take a caller
 *     workspace sized by ldpc_workspace_size).
 *   - Decoding is asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream): outputs are valid once the caller has synchronised the stream.
 *     Calls on different streams need different workspaces.
 *   - A graph is an immutable host object; it may be shared across threads
 *     and streams.
 *   - Tuning: the environment variable LDPC_FRAMES_PER_LANE (1, 2 or 4)
 *     overrides how many frames each GPU lane carries (frames are processed
 *     in tiles of 64 * that many).  It changes speed and workspace size, never
 *     results; read by ldpc_workspace_size and the decoders at each call.
 *   - Bit and LLR conventions (Sec. II-B): bit c maps to x = 1 - 2c; channel
 *     LLRs are mu = ln P(c=0|y)/P(c=1|y) = 2y/sigma^2; a hard decision is 0
 *     when the posterior LLR is >= 0 (Eq. 6; -0.0 decides 0).
 *   - Saturation (not stated in the paper): every variable-to-check message,
 *     including the initial one, is clipped to [-30, 30], and so is every
 *     returned posterior; decisions use the unclipped posterior.
 */
#ifndef LDPC_H
#define LDPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ldpc_graph ldpc_graph;

typedef enum {
    LDPC_OK = 0,
    LDPC_EINVAL = -1,        /* bad argument (NULL pointer, out-of-range value, wrong graph kind) */
    LDPC_EWORKSPACE = -2,    /* workspace NULL or smaller than ldpc_workspace_size */
    LDPC_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    LDPC_EUNSUPPORTED = -4,  /* valid code, but outside this build's limits (degrees, sizes) */
    LDPC_ENOMEM = -5         /* host allocation failed */
} ldpc_status;

typedef enum { LDPC_GRAPH_QC = 0, LDPC_GRAPH_CONV = 1 } ldpc_graph_kind;

typedef struct {
    int32_t kind;            /* ldpc_graph_kind */
    int32_t n, m, E;         /* variables, checks, edges (ones of H) */
    int32_t dv_max, dc_max;  /* largest column / row weight */
    int32_t J, L, p;         /* QC base: J x L circulants of size p (the QC code; for a
                                convolutional graph built from a QC base, that base) */
    int32_t ms, T;           /* convolutional: syndrome-former memory, period */
    int32_t Jb, Lb;          /* convolutional: circulant rows per check layer, columns per position */
    int32_t c, c_minus_b;    /* convolutional: bits per code position, checks per layer */
    int32_t positions;       /* convolutional: code positions kept (terminated chain) */
    int32_t layers;          /* convolutional: check layers kept */
    int32_t blocks;          /* nonzero circulants of the QC base (numbered row by row, left to
                                right) or of the syndrome-former table */
    double design_rate;      /* 1 - J/L (QC), b/c (convolutional) */
} ldpc_graph_info;

/* Limits of this build. */
#define LDPC_MAX_BLOCKS      256   /* nonzero circulants in a base / syndrome-former table */
#define LDPC_MAX_BASE_ROWS   32
#define LDPC_MAX_BASE_COLS   64
#define LDPC_MAX_ROW_WEIGHT  32
#define LDPC_MAX_COL_WEIGHT  16
#define LDPC_MAX_ITERS       100000

/*
 * Quasi-cyclic LDPC code of Eq. 2: H is J x L blocks of p x p circulants.
 * shifts: host, int32 [J][L] row-major.  Block (j,l) is the identity with its
 * columns shifted cyclically to the right shifts[j][l] times, i.e. row r of
 * the block has its one in column (r + shifts[j][l]) mod p; -1 is the zero
 * block (footnote of Sec. IV-B).  Requires 0 <= shift < p or shift == -1.
 * Check (j, s) is row j*p + s; variable (l, t) is column l*p + t.
 * The shift table is copied; *out receives a graph to release with
 * ldpc_graph_destroy.  Errors: EINVAL (NULL, J/L/p <= 0, shift out of range),
 * EUNSUPPORTED (beyond the limits above), ENOMEM.
 */
ldpc_status ldpc_graph_create_qc(const int32_t* shifts, int32_t J, int32_t L, int32_t p,
                                 ldpc_graph** out);

/*
 * LDPC convolutional code derived from a QC code by unwrapping (Sec. II-D):
 * Lambda = gcd(J, L); the base is cut into Lambda x Lambda sub-blocks
 * H_{i,j}; the lower part (j <= i) is kept on the block diagonal and the
 * strictly upper part pasted below it, and the pair repeats down the
 * diagonal.  Period T = Lambda, memory ms = Lambda - 1; a code position
 * (frame) holds c = p L / Lambda bits, a check layer c - b = p J / Lambda
 * checks.  Check layer tau meets position tau - d (d = 0..ms) through
 * sub-block H_{tau mod T, (tau - d) mod T}.
 * The chain holds `positions` code positions (variables indexed
 * position-major: variable q*p + u of position t is column t*c + q*p + u);
 * terminate = 1 keeps the ms tail layers that close the chain
 * (positions + ms layers), terminate = 0 keeps layers 0..positions-1.
 * Errors as ldpc_graph_create_qc, plus EINVAL for positions <= 0.
 */
ldpc_status ldpc_graph_create_ldpccc_from_qc(const int32_t* shifts, int32_t J, int32_t L, int32_t p,
                                             int32_t positions, int32_t terminate,
                                             ldpc_graph** out);

/*
 * Periodic LDPC convolutional code given by its syndrome-former components
 * (Eq. of H_[0,inf] in Sec. II-C): check layer tau of class i = tau mod T
 * meets position tau - d through H_d(tau), d = 0..ms, each a Jb x Lb array of
 * p x p circulants.  sf: host, int32 [T][ms+1][Jb][Lb] row-major, same shift
 * convention as ldpc_graph_create_qc.  positions / terminate as above.
 */
ldpc_status ldpc_graph_create_ldpccc_sf(const int32_t* sf, int32_t T, int32_t ms, int32_t Jb,
                                        int32_t Lb, int32_t p, int32_t positions, int32_t terminate,
                                        ldpc_graph** out);

/* Fills *info.  Errors: EINVAL for NULL arguments. */
ldpc_status ldpc_graph_get_info(const ldpc_graph* g, ldpc_graph_info* info);

/* Releases a graph; NULL is ignored. */
void ldpc_graph_destroy(ldpc_graph* g);

/*
 * Device workspace needed for `gamma` frames by ldpc_decode (QC graph,
 * window == 0, at most `max_iters` iterations), ldpc_decode_window
 * (convolutional graph, window = W >= ms + 1; max_iters is ignored but must be
 * >= 1) or ldpc_decode_pipeline (convolutional graph, window == 0, max_iters =
 * number of processors).  Errors: EINVAL, EUNSUPPORTED (a window on a QC
 * graph; W or processors above 64).
 */
ldpc_status ldpc_workspace_size(const ldpc_graph* g, int32_t gamma, int32_t max_iters,
                                int32_t window, size_t* bytes);

/*
 * Flooding sum-product decoding of `gamma` frames of a QC graph
 * (Algorithm 1: initialisation beta = mu; horizontal step Eq. 3; vertical
 * step Eq. 4; posterior Eq. 5; hard decision Eq. 6).
 *   llr        device, float [gamma][n]: channel LLRs; not modified
 *   max_iters  >= 1 iterations (one iteration = all check nodes, then all
 *              variable nodes)
 *   early_stop 0: run max_iters iterations.  1: test the syndrome of the
 *              hard decisions after every iteration and freeze a frame at
 *              the first iteration whose syndrome is zero (the paper always
 *              runs the full count; this is an addition)
 *   post       device, float [gamma][n]: clip(posterior LLR, +-30) of the
 *              returned iteration
 *   bits       device, uint8 [gamma][n]: hard decisions, 0/1
 *   iters      device, int32 [gamma] or NULL: iterations run per frame
 *   converged  device, uint8 [gamma] or NULL: 1 if the returned decisions
 *              satisfy every check
 *   workspace  device, >= ldpc_workspace_size(g, gamma, max_iters, 0) bytes,
 *              256-byte aligned; its contents on entry do not matter
 * Errors: EINVAL (NULL required pointer, gamma < 1, max_iters outside
 * [1, LDPC_MAX_ITERS], convolutional graph), EWORKSPACE, EHIP.
 */
ldpc_status ldpc_decode(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t max_iters,
                        int32_t early_stop, float* post, uint8_t* bits, int32_t* iters,
                        uint8_t* converged, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Which decoder ldpc_decode (and ldpc_decode_noalloc, ldpc_nms_decode) runs
 * for g on the current device: *onchip = 1 when each frame is decoded by one workgroup
 * on one compute unit, its check-to-variable messages in registers and its
 * posterior sums in LDS (a (3,6) code up to n = 18,432; codes whose base
 * has 3 rows of weight <= 9 or 4 rows of weight <= 8, no empty base column,
 * p <= 3072, two n-float arrays within the device's LDS per workgroup), 0
 * when it runs the message-package decoder (edge messages in the workspace,
 * one launch per half-iteration).  Both compute Algorithm 1 with the FP32
 * check rule in the (tanh, 1 - tanh) pair form; the on-chip decoder carries
 * the pairs unnormalised (no reciprocal per input) and forms each
 * variable-to-check message as clip(L - alpha) from the posterior sum
 * instead of summing the other edges, so the two agree within FP32
 * rounding, not bit for bit.  Setting
 * the environment variable LDPC_BLOCK_PATH=packages makes ldpc_decode use
 * the package decoder for every code (read at each call).  The workspace
 * argument of ldpc_decode is validated the same way on both paths.
 * Errors: EINVAL (NULL, convolutional graph).
 */
ldpc_status ldpc_decode_path(const ldpc_graph* g, int32_t* onchip);

/*
 * ldpc_decode for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  It
 * takes no workspace argument.  Its workspace is a static device array of
 * LDPC_NOALLOC_SCRATCH_BYTES that the library holds once on every device it
 * runs on, until the process ends; the first call on a device looks up that
 * device's copy (hipGetSymbolAddress), later calls reuse the address.  The
 * call itself allocates nothing (no hipMalloc, no hipFree, no events: kernel
 * timing is not recorded for it).  The caller still passes the inputs and
 * outputs, with the arguments, results and kernels of ldpc_decode; the
 * stream must belong to the current device.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (the decode clears what must start at zero with a kernel,
 * so no memset node is recorded under capture): calls that overlap on one
 * device (on different streams, or from different threads) race and return
 * garbage.  Serialise them.
 * Errors: those of ldpc_decode; EWORKSPACE when the decode needs more than
 * LDPC_NOALLOC_SCRATCH_BYTES (ldpc_workspace_size(g, gamma, max_iters, 0)
 * tells); EUNSUPPORTED for a device ordinal >= 64.
 */
#define LDPC_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
ldpc_status ldpc_decode_noalloc(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t max_iters,
                                int32_t early_stop, float* post, uint8_t* bits, int32_t* iters,
                                uint8_t* converged, void* stream);

/*
 * Learned min-sum decoding (an addition to the paper: the neural normalized
 * / offset min-sum of Nachmani et al. 2016/2018 and Lugosch & Gross 2017 on
 * the flooding schedule of Algorithm 1).  The horizontal step (Eq. 3) is
 * replaced, at iteration t on edge k of a check row, by
 *   alpha_k = w[t][e] * s_k * max(m_k - b[t][e], 0),
 * e = the edge's class: its circulant block (0 .. blocks-1, the base's
 * nonzero blocks numbered row by row, left to right; ldpc_graph_info.blocks),
 * m_k = min(|beta_k'|) over the row's other edges (|beta| clipped at 30),
 * s_k = product of their signs (negative iff beta < 0).  The vertical step
 * (Eq. 4), the posterior (Eq. 5), the decision (Eq. 6), the clip of beta at
 * +-30 and early stopping are those of ldpc_decode.
 *   weights  device, float [iters][blocks][2]: (w, b) per iteration and edge
 *            class
 *   iters    iterations, 1..LDPC_MAX_ITERS (the weight rows used)
 * Other arguments as for ldpc_decode (workspace from
 * ldpc_workspace_size(g, gamma, iters, 0)).  Like ldpc_decode it decodes a
 * code that fits one compute unit on chip (ldpc_decode_path; the rule above
 * in base-2 units there, within FP32 rounding of the package decoder's).
 * Errors: those of ldpc_decode, and EINVAL for NULL weights.
 */
ldpc_status ldpc_nms_decode(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t iters,
                            const float* weights, int32_t early_stop, float* post, uint8_t* bits,
                            int32_t* iters_out, uint8_t* converged, void* workspace, size_t workspace_bytes,
                            void* stream);

/*
 * Training the learned min-sum weights: loss and gradient through T = iters
 * unrolled iterations for frames of the all-zero codeword.  The loss of
 * iteration t is the binary cross-entropy of its (unclipped) posterior
 * against the transmitted bits, averaged over the gamma frames and n bits:
 *   loss[t] = mean_{g, v} log(1 + exp(-L_gv^(t))).
 *
 * ldpc_nms_train_forward runs the T iterations, writes loss (device float
 * [iters]) and keeps in the workspace the channel LLRs and the betas of
 * iterations ckpt_every, 2 ckpt_every, ... (< iters).
 *
 * ldpc_nms_train_backward, called after ldpc_nms_train_forward on the same
 * workspace with the same graph, gamma, iters, ckpt_every and weights,
 * writes grad (device float [iters][blocks][2]) = d(sum_t dloss[t] loss[t]) /
 * d weights, for dloss device float [iters] (the upstream gradient).  It
 * recomputes each segment of ckpt_every iterations from its checkpoint
 * and runs the hand-written backward of the vertical and horizontal steps
 * through the segment, last iteration first.  The gradient of the minimum
 * goes to the first edge holding it; the clips pass gradient inside
 * [-30, 30] (inclusive), the offset's max(., 0) at >= 0; the gradient sums
 * are reduced in a fixed order (deterministic for a given launch).
 *
 * ldpc_nms_train_workspace_size: bytes for (g, gamma, iters, ckpt_every).
 * Errors: EINVAL (NULL pointers, convolutional graph, gamma < 1, iters
 * outside [1, LDPC_MAX_ITERS], ckpt_every outside [1, iters], misaligned
 * buffers), EWORKSPACE, EHIP.
 */
ldpc_status ldpc_nms_train_workspace_size(const ldpc_graph* g, int32_t gamma, int32_t iters, int32_t ckpt_every,
                                          size_t* bytes);
ldpc_status ldpc_nms_train_forward(const ldpc_graph* g, const float* llr, int32_t gamma, int32_t iters,
                                   int32_t ckpt_every, const float* weights, float* loss, void* workspace,
                                   size_t workspace_bytes, void* stream);
ldpc_status ldpc_nms_train_backward(const ldpc_graph* g, int32_t gamma, int32_t iters, int32_t ckpt_every,
                                    const float* weights, const float* dloss, float* grad, void* workspace,
                                    size_t workspace_bytes, void* stream);

/*
 * Multi-code plan: frames of several QC graphs, each with its own batch size,
 * decoded together by the flooding sum-product decoders of ldpc_decode
 * (Algorithm 1, Eq. 3-6; same arithmetic, so each code's outputs equal
 * ldpc_decode's bit for bit, except in the split layouts below).  Codes that ldpc_decode would decode on chip
 * (ldpc_decode_path; not in persistent mode) run that decoder, one launch
 * per code on a stream forked from the caller's and joined back before the
 * decode ends; for the others, one check-node launch and one variable-node
 * launch per iteration cover all codes.  The whole decode can be captured
 * once into a HIP graph (the on-chip launches as a parallel branch) and
 * replayed; which codes run on chip is decided when the plan binds its
 * buffers, so a change of LDPC_BLOCK_PATH between calls rebuilds the table
 * and invalidates a captured graph.
 *
 * Layout of a code (frames per tile and rows per wavefront):
 *   LDPC_LAYOUT_G8, _G16, _G32: tiles of 8, 16 or 32 frames, a wavefront
 *     working on 8, 4 or 2 consecutive rows (variables) at once;
 *   LDPC_LAYOUT_G64: tiles of 64 frames, one row per wavefront;
 *   LDPC_LAYOUT_G64F4: tiles of 256 frames, 4 frames per lane (row weight
 *     <= 6 and column weight <= 8 only);
 *   LDPC_LAYOUT_G64F2: tiles of 128 frames, 2 frames per lane (row weight
 *     <= 12 and column weight <= 8 only);
 *   LDPC_LAYOUT_G8F2, _G8F4, _G16F2, _G16F4, _G32F2, _G32F4: groups of 8, 16
 *     or 32 lanes per row (variable), each lane carrying 2 or 4 consecutive
 *     frames (tiles of 16 to 128 frames; 64 * frames-per-lane / lanes rows
 *     per wavefront), so small batches still move 8 or 16 bytes per lane
 *     and access (same row and column weight limits as G64F2 / G64F4).
 * OR-ing LDPC_LAYOUT_VN2 or LDPC_LAYOUT_VN4 into a one-frame-per-lane
 * layout (G8 .. G64, column weight <= 8) makes each variable-node wavefront
 * handle 2 or 4 groups of variables (fewer, longer waves); LDPC_LAYOUT_CN2
 * (row weight <= 8) or LDPC_LAYOUT_CN4 (row weight <= 6) does the same for
 * the check-node wavefronts.  OR-ing LDPC_LAYOUT_SPLIT2, _SPLIT4 or _SPLIT8
 * into G8, G16 or G32 (lanes per group times lanes per row at most 64; row
 * weight at least twice the lanes per row) spreads each check row's edges
 * over 2, 4 or 8 lanes of the check-node wavefront (Eq. 3 with the (t, q)
 * products of each lane's edges combined across the lanes by shuffles), so
 * that a heavy row of a small batch is not one lane's chain; the
 * variable-node pass is that of the base layout.  These layouts form the
 * products of Eq. 3 in another order than ldpc_decode: their results equal
 * ldpc_decode's to FP32 rounding, not bit for bit (every other layout is
 * bit-equal).
 * Graphs in a plan have row weight <= 24 (EUNSUPPORTED otherwise): one
 * kernel serves all codes and carries the registers of its heaviest case.
 * The default is the smallest tile >= gamma (for large batches G64F4, else
 * G64F2, when allowed and padding stays under 1/8); ldpc_plan_autotune times every candidate per code and keeps the
 * fastest; ldpc_plan_set_layout sets one (-1 = the default).
 *
 * ldpc_plan_create: graphs (host array of ncodes QC graphs, which must
 * outlive the plan), gammas (host int32 [ncodes], >= 1), 1 <= ncodes <=
 * LDPC_PLAN_MAX_CODES, max_iters, early_stop as for ldpc_decode.
 * ldpc_plan_workspace_size: bytes for any choice of layouts; the workspace
 * (device, 256-byte aligned) starts with the plan's table of per-code
 * descriptors, written by the first call that uses new buffers or layouts
 * (that call synchronises `stream`).
 *
 * ldpc_plan_decode: per code c (host arrays of device pointers, ncodes
 * entries): llr[c] float [gamma_c][n_c], post[c] float [gamma_c][n_c],
 * bits[c] uint8 [gamma_c][n_c], iters[c] int32 [gamma_c] and converged[c]
 * uint8 [gamma_c] (the arrays `iters` and `converged`, or their entries, may
 * be NULL).  Outputs as for ldpc_decode.  Asynchronous on `stream`.
 *
 * ldpc_plan_capture: records the same decode for these buffers into a HIP
 * graph (on a stream of the plan's own; nothing runs); ldpc_plan_replay
 * launches it on `stream`.  Replay fails with EINVAL once another call has
 * bound other buffers or layouts (capture again).  The workspace must not be
 * used by anything else between capture and replay.
 *
 * ldpc_plan_autotune: one pass of coordinate descent over the codes: each
 * code in turn tries every other allowed layout value (tiles no larger than the
 * next power of two at or above its batch) while the others stay fixed; each
 * candidate is timed over `trials` whole decodes of the plan (after one
 * warm-up) on the given buffers (outputs are overwritten); the fastest is
 * kept.  Writes the final time per decode in ms to *best_ms (host, may be
 * NULL).  Synchronises `stream`.
 *
 * Errors: EINVAL (NULL pointers, bad counts, convolutional graphs, layout not
 * allowed, misaligned buffers), EWORKSPACE, EUNSUPPORTED, EHIP, ENOMEM.
 */
typedef struct ldpc_plan ldpc_plan;
#define LDPC_PLAN_MAX_CODES 16
enum { LDPC_LAYOUT_G8 = 0, LDPC_LAYOUT_G16 = 1, LDPC_LAYOUT_G32 = 2, LDPC_LAYOUT_G64 = 3, LDPC_LAYOUT_G64F4 = 4,
       LDPC_LAYOUT_G64F2 = 5, LDPC_LAYOUT_G8F2 = 6, LDPC_LAYOUT_G8F4 = 7, LDPC_LAYOUT_G16F2 = 8,
       LDPC_LAYOUT_G16F4 = 9, LDPC_LAYOUT_G32F2 = 10, LDPC_LAYOUT_G32F4 = 11, LDPC_LAYOUT_VN2 = 16,
       LDPC_LAYOUT_VN4 = 32, LDPC_LAYOUT_CN2 = 64, LDPC_LAYOUT_CN4 = 128, LDPC_LAYOUT_SPLIT2 = 256,
       LDPC_LAYOUT_SPLIT4 = 512, LDPC_LAYOUT_SPLIT8 = 768 };

ldpc_status ldpc_plan_create(const ldpc_graph* const* graphs, const int32_t* gammas, int32_t ncodes,
                             int32_t max_iters, int32_t early_stop, ldpc_plan** out);
void        ldpc_plan_destroy(ldpc_plan* plan);
ldpc_status ldpc_plan_workspace_size(const ldpc_plan* plan, size_t* bytes);
ldpc_status ldpc_plan_set_layout(ldpc_plan* plan, int32_t code, int32_t layout);
ldpc_status ldpc_plan_get_layout(const ldpc_plan* plan, int32_t code, int32_t* layout);
ldpc_status ldpc_plan_decode(ldpc_plan* plan, const float* const* llr, float* const* post, uint8_t* const* bits,
                             int32_t* const* iters, uint8_t* const* converged, void* workspace,
                             size_t workspace_bytes, void* stream);
ldpc_status ldpc_plan_capture(ldpc_plan* plan, const float* const* llr, float* const* post, uint8_t* const* bits,
                              int32_t* const* iters, uint8_t* const* converged, void* workspace,
                              size_t workspace_bytes, void* stream);
ldpc_status ldpc_plan_replay(ldpc_plan* plan, void* stream);
ldpc_status ldpc_plan_autotune(ldpc_plan* plan, const float* const* llr, float* const* post, uint8_t* const* bits,
                               int32_t* const* iters, uint8_t* const* converged, void* workspace,
                               size_t workspace_bytes, int32_t trials, void* stream, double* best_ms);

/*
 * Persistent launch of a plan (the paper's flexibility claim of its
 * Conclusion, with Algorithm 1 run for several codes at once): with `on` = 1,
 * ldpc_plan_decode, ldpc_plan_capture and ldpc_plan_autotune enqueue the
 * whole decode as ONE kernel instead of 2 * max_iters + 4 phase launches.
 * Inside it, workgroups take numbered tickets of work (a few wavefronts of
 * one step of one code); steps of one code run in order (ingest, then per
 * iteration the check-node pass, the flag reduction, the variable-node pass,
 * then the final syndrome, frame status and output), while different codes
 * advance independently.  A ticket waits only for tickets of lower numbers,
 * so the launch needs no co-residency of its workgroups.  Results equal the
 * phase launches' bit for bit (same device functions, same order within
 * each step).  Each wait is bounded by wait_limit_us (0: 2 s); if a wait
 * expires the kernel stops early and still exits normally, leaving the
 * outputs undefined, and the next ldpc_plan_check reports it.  Switching
 * the mode invalidates a captured graph.
 *   on             0 (the phase launches, the default) or 1
 *   wait_limit_us  >= 0
 * Errors: EINVAL (NULL plan, on not 0/1, negative limit), EHIP (device
 * queries).  ldpc_plan_decode / _capture return EUNSUPPORTED in persistent
 * mode when a decode would need 2^31 tickets or more, or a code's share of
 * the workspace is 2 GiB or more.
 *
 * ldpc_plan_check: synchronises `stream`, then returns EHIP if a persistent
 * decode on this workspace had a wait expire since the last check (and
 * clears that record), LDPC_OK otherwise.  workspace: the plan's workspace
 * (device), after at least one decode with the current buffers.
 */
ldpc_status ldpc_plan_set_persistent(ldpc_plan* plan, int32_t on, int64_t wait_limit_us);
ldpc_status ldpc_plan_check(ldpc_plan* plan, void* workspace, void* stream);

/*
 * Sliding-window decoding of `gamma` independent streams of a terminated
 * convolutional graph (Sec. II-E: checks span at most ms+1 positions).  For
 * target position s = 0..positions-1: the window holds check layers
 * s..s+W-1 and active positions s..s+W-1 (those that exist); a position
 * entering the window starts from beta = clip(mu) on its edges, messages of
 * the previous window are kept, and positions s-ms..s-1 keep the messages
 * they last sent; `iters_per_window` flooding iterations run over the window
 * (horizontal step on its layers, vertical step on its active positions,
 * summing only messages from window layers); position s is then decided
 * from mu plus the window layers' messages.
 *   llr   device, float [gamma][positions * c]
 *   post  device, float [gamma][positions * c]: clip(posterior, +-30)
 *   bits  device, uint8 [gamma][positions * c]
 *   W     window length in positions, ms + 1 <= W <= 64
 * Execution: when one stream's ring (the messages and channel LLRs of the
 * W + ms positions a window holds) fits the device's LDS per workgroup, each
 * stream is decoded from start to end by one workgroup out of LDS (one
 * launch); otherwise every phase is a launch over all streams, with the
 * ring in the workspace.  Both give the same results bit for bit; the
 * environment variable LDPC_WINDOW_PATH=launch (or =lds) selects one.  The
 * workspace size is that of the launch-per-phase form in either case.
 * Errors: EINVAL (QC graph, W < ms+1, iters_per_window < 1, NULL pointers),
 * EWORKSPACE, EHIP.
 */
ldpc_status ldpc_decode_window(const ldpc_graph* conv, const float* llr, int32_t gamma, int32_t W,
                               int32_t iters_per_window, float* post, uint8_t* bits,
                               void* workspace, size_t workspace_bytes, void* stream);

/*
 * Pipelined decoding of `gamma` independent streams of a terminated
 * convolutional graph with `iters` processors (Algorithm 2; Sec. IV-B): at
 * time slot t frame t enters processor 1 with beta = clip(mu); processor i
 * (i = 1..iters) updates check layer t - (i-1)(ms+1) (horizontal step, all
 * processors first) and then frame t - (i-1)(ms+1) - ms (vertical step); the
 * frame leaving the last processor is decided.  Slots continue until the
 * last frame has left.  Every check layer and every frame is thereby updated
 * exactly `iters` times, in flooding order, so the result equals `iters`
 * flooding iterations on the whole terminated chain while the decoder holds
 * only iters * (ms+1) frames, plus 7 it reads in ahead so that one launch
 * brings in 8 entering frames (workspace from
 * ldpc_workspace_size(conv, gamma, iters, 0)).
 *   llr, post, bits as for ldpc_decode_window; 1 <= iters <= 64.
 * Errors: EINVAL (QC graph, iters < 1, NULL pointers), EUNSUPPORTED
 * (iters > 64), EWORKSPACE, EHIP.
 */
ldpc_status ldpc_decode_pipeline(const ldpc_graph* conv, const float* llr, int32_t gamma, int32_t iters,
                                 float* post, uint8_t* bits, void* workspace, size_t workspace_bytes,
                                 void* stream);

/*
 * Simulation on the GPU (Sec. V-B: codewords and noise are generated on the
 * device, the host only reads error counts).  The codeword is all-zero (the
 * decoders treat every codeword alike: flipping the signs of a codeword's
 * LLRs flips the decisions and nothing else).
 *
 * ldpc_awgn_llr: llr (device, float [gamma][n]) = 2 y / sigma^2 with
 * y = 1 + sigma z, z ~ N(0, 1), for frames frame0 .. frame0+gamma-1.  Sample
 * (g, i) depends only on (seed, frame0 + g, i): Philox-4x32-10 with key =
 * seed (low word first) and counter (i / 4, frame, 0x4E5A, frame >> 32) gives
 * four uniforms (w + 0.5) / 2^32 and two Box-Muller pairs, in FP64.
 * Errors: EINVAL (NULL, n < 1, gamma < 1, sigma2 <= 0, frame0 < 0).
 *
 * ldpc_count_errors: for decisions bits (device, uint8 [gamma][n]) against the
 * all-zero codeword, writes each frame's bit-error count to frame_errors
 * (device int32 [gamma], or NULL) and adds the batch's bit errors to totals[0]
 * and its erroneous frames to totals[1] (device uint64 [2], or NULL; not
 * cleared).  Errors: EINVAL (NULL bits, both outputs NULL, gamma or n < 1,
 * misaligned totals).
 */
ldpc_status ldpc_awgn_llr(int64_t n, int32_t gamma, double sigma2, uint64_t seed, int64_t frame0, float* llr,
                          void* stream);
ldpc_status ldpc_count_errors(const uint8_t* bits, int32_t gamma, int64_t n, int32_t* frame_errors,
                              uint64_t* totals, void* stream);

/* Static description of a status code. */
const char* ldpc_status_str(ldpc_status s);

/*
 * Kernel timing for measurement.  While enabled, every kernel the decoders
 * enqueue is bracketed by a pair of HIP events on its stream, grouped by
 * kernel class; ldpc_timing_read synchronises those events and returns, per
 * class, the launch count and the summed device time in milliseconds, then
 * clears them.  Classes (index into the arrays, capacity >= LDPC_TIMING_CLASSES):
 *   0 ingest, 1 check-node, 2 variable-node, 3 syndrome, 4 output (the
 *   last variable-node pass of a decode without early stopping, which writes
 *   the outputs; with early stopping the final transpose),
 *   5 frame status, 6 window ingest, 7 window check-node,
 *   8 window variable-node, 9 pipeline ingest, 10 pipeline check-node,
 *   11 pipeline variable-node, 12 training check-node, 13 training
 *   variable-node, 14 training variable-node backward, 15 training
 *   check-node backward, 16 training loss and gradient reductions,
 *   17 plan ingest, 18 plan check-node, 19 plan variable-node, 20 plan
 *   final syndrome, frame status and output, 21 window decoding with the
 *   ring in LDS (one launch per call), 22 plan decode in one persistent
 *   launch, 23 block decode with each frame on one compute unit (one launch
 *   per call).
 * ldpc_kernel_class_name returns a static name for a class index.
 */
#define LDPC_TIMING_CLASSES 24
ldpc_status ldpc_timing_enable(int32_t enable);
ldpc_status ldpc_timing_read(int64_t* launches, double* total_ms, int32_t capacity);
const char* ldpc_kernel_class_name(int32_t cls);

#ifdef __cplusplus
}
#endif

#endif /* LDPC_H */
