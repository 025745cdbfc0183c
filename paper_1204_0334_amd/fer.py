"""Frame/bit error-rate simulation on the GPU, following the paper's
simulation loop (Sec. V-B): codewords and channel noise are generated on the
device, the decoded bits are checked on the device, and only error counts
come back to the host; the run stops after a fixed number of frame errors.

The transmitted codeword is all-zero (the decoders treat every codeword
alike).  Every step runs in the HIP library: `ldpc_awgn_llr` (channel),
`ldpc_decode` / `ldpc_nms_decode` / `ldpc_decode_pipeline` /
`ldpc_decode_window` (decoder) and
`ldpc_count_errors` (error counting); this module only loops and keeps time.
"""
from __future__ import annotations

import math

import torch

from . import ldpc


def ebn0_to_sigma2(ebn0_db: float, rate: float) -> float:
    """Unit-energy BPSK: sigma^2 = N0 / 2 = 1 / (2 R Eb/N0)."""
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def simulate(g: ldpc.Graph, ebn0_db: float, *, decoder: str = "block", gamma: int = 1024, iters: int = 30,
             early_stop: bool = False, window: int = 6, seed: int = 1, min_frame_errors: int = 100,
             max_frames: int = 1 << 20, weights=None, device=None) -> dict:
    """Simulate until `min_frame_errors` frame errors or `max_frames` frames.

    decoder: "block" (QC graph, `iters` flooding iterations), "nms" (QC
    graph, learned min-sum with `weights` [T, J, 2], T iterations), "pipeline"
    (convolutional graph, `iters` processors) or "window" (convolutional
    graph, window `window`, `iters` iterations per window).  A frame is one
    codeword of the block code, or one stream of the convolutional chain.
    Returns counts, rates and the GPU time of the whole loop (generation,
    decoding and counting)."""
    dev = torch.device(device or "cuda:0")
    info = g.info
    n = info["n"]
    rate = info["design_rate"]
    sigma2 = ebn0_to_sigma2(ebn0_db, rate)
    llr = torch.empty((gamma, n), dtype=torch.float32, device=dev)
    post = torch.empty((gamma, n), dtype=torch.float32, device=dev)
    bits = torch.empty((gamma, n), dtype=torch.uint8, device=dev)
    it = torch.empty((gamma,), dtype=torch.int32, device=dev)
    conv = torch.empty((gamma,), dtype=torch.uint8, device=dev)
    per_frame = torch.empty((gamma,), dtype=torch.int32, device=dev)
    totals = torch.zeros((2,), dtype=torch.int64, device=dev)
    iter_sum = torch.zeros((), dtype=torch.int64, device=dev)
    if decoder == "nms":
        if weights is None:
            raise ValueError("the learned decoder needs weights")
        iters = int(weights.shape[0])
    if decoder in ("block", "nms"):
        ws = ldpc.workspace(g, gamma, iters, 0, dev)
    elif decoder == "pipeline":
        ws = ldpc.workspace(g, gamma, iters, 0, dev)
    elif decoder == "window":
        ws = ldpc.workspace(g, gamma, 1, window, dev)
    else:
        raise ValueError(f"unknown decoder {decoder!r}")
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    frames = 0
    start.record()
    while frames < max_frames:
        ldpc.awgn_llr(n, gamma, sigma2, seed, frames, out=llr)
        if decoder == "block":
            ldpc.decode(g, llr, iters, early_stop, out=(post, bits, it, conv), ws=ws)
            iter_sum += it.sum()
        elif decoder == "nms":
            ldpc.nms_decode(g, llr, weights, early_stop, out=(post, bits, it, conv), ws=ws)
            iter_sum += it.sum()
        elif decoder == "pipeline":
            ldpc.decode_pipeline(g, llr, iters, out=(post, bits), ws=ws)
        else:
            ldpc.decode_window(g, llr, window, iters, out=(post, bits), ws=ws)
        ldpc.count_errors(bits, frame_errors=per_frame, totals=totals)
        frames += gamma
        if int(totals[1].item()) >= min_frame_errors:     # synchronises the stream
            break
    stop.record()
    torch.cuda.synchronize()
    seconds = start.elapsed_time(stop) * 1e-3
    bit_err, frame_err = (int(x) for x in totals.tolist())
    out = dict(frames=frames, frame_errors=frame_err, bit_errors=bit_err, fer=frame_err / frames,
               ber=bit_err / (frames * n), seconds=seconds, ms_per_frame=seconds * 1e3 / frames,
               coded_mbps=frames * n / seconds / 1e6, ebn0_db=ebn0_db, sigma2=sigma2, n=n, gamma=gamma,
               decoder=decoder, iters=iters)
    if decoder in ("block", "nms"):
        out["avg_iters"] = int(iter_sum.item()) / frames
    else:
        out["ms_per_code_frame"] = seconds * 1e3 / (frames * info["positions"])
    return out


def fer_interval(frame_errors: int, frames: int, z: float = 1.96):
    """Wilson score interval for the frame error rate."""
    if frames == 0:
        return (0.0, 1.0)
    p = frame_errors / frames
    d = 1 + z * z / frames
    c = (p + z * z / (2 * frames)) / d
    h = z * math.sqrt(p * (1 - p) / frames + z * z / (4 * frames * frames)) / d
    return (max(0.0, c - h), min(1.0, c + h))
