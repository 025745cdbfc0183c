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

import json
import math
import os

import torch

from . import ldpc


def ebn0_to_sigma2(ebn0_db: float, rate: float) -> float:
    """Unit-energy BPSK: sigma^2 = N0 / 2 = 1 / (2 R Eb/N0)."""
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def simulate(g: ldpc.Graph, ebn0_db: float, *, decoder: str = "block", gamma: int = 1024, iters: int = 30,
             early_stop: bool = False, window: int = 6, seed: int = 1, min_frame_errors: int = 100,
             max_frames: int = 1 << 20, weights=None, device=None, resume: dict | None = None,
             checkpoint=None, checkpoint_every: int = 64) -> dict:
    """Simulate until `min_frame_errors` frame errors or `max_frames` frames.

    decoder: "block" (QC graph, `iters` flooding iterations), "nms" (QC
    graph, learned min-sum with `weights` [T, blocks, 2], T iterations), "pipeline"
    (convolutional graph, `iters` processors) or "window" (convolutional
    graph, window `window`, `iters` iterations per window).  A frame is one
    codeword of the block code, or one stream of the convolutional chain.
    Returns counts, rates and the GPU time of the whole loop (generation,
    decoding and counting).

    Checkpoint / resume: the generator is counter-based (frame f's noise
    depends only on (seed, f)), so a run is fully described by its counters.
    `checkpoint(state)` is called every `checkpoint_every` batches with
    {frames, frame_errors, bit_errors, iter_sum, seconds}; passing such a
    state as `resume` continues the run exactly where it stopped."""
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
    frames, seconds0 = 0, 0.0
    if resume:
        frames = int(resume["frames"])
        seconds0 = float(resume.get("seconds", 0.0))
        totals[0] = int(resume["bit_errors"])
        totals[1] = int(resume["frame_errors"])
        iter_sum.fill_(int(resume.get("iter_sum", 0)))
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
    start.record()
    batches = 0
    done = int(totals[1].item()) >= min_frame_errors
    while frames < max_frames and not done:
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
        batches += 1
        done = int(totals[1].item()) >= min_frame_errors     # synchronises the stream
        if checkpoint is not None and (batches % checkpoint_every == 0 or done or frames >= max_frames):
            stop.record()
            torch.cuda.synchronize()
            checkpoint(dict(frames=frames, frame_errors=int(totals[1].item()), bit_errors=int(totals[0].item()),
                            iter_sum=int(iter_sum.item()), seconds=seconds0 + start.elapsed_time(stop) * 1e-3))
    stop.record()
    torch.cuda.synchronize()
    seconds = seconds0 + start.elapsed_time(stop) * 1e-3
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


def sweep(g: ldpc.Graph, points, log_path: str, *, key: str, **kw) -> list:
    """FER/BER over Eb/N0 points with the stopping rule of `simulate`,
    appending per-point records to the JSONL file `log_path` (one line per
    checkpoint; `key` names the code and decoder).  Points already finished
    in the log are not run again, and an interrupted point resumes from its
    last checkpoint."""
    last = {}
    if os.path.exists(log_path):
        with open(log_path) as f:
            for line in f:
                line = line.strip()
                if line:
                    r = json.loads(line)
                    last[(r["key"], r["ebn0_db"])] = r
    out = []
    for e in points:
        prev = last.get((key, e))
        if prev is not None and prev["done"]:
            out.append(prev["result"])
            continue

        def save(state, e=e):
            with open(log_path, "a") as f:
                f.write(json.dumps(dict(key=key, ebn0_db=e, done=False, state=state)) + "\n")

        res = simulate(g, e, resume=prev["state"] if prev else None, checkpoint=save, **kw)
        with open(log_path, "a") as f:
            f.write(json.dumps(dict(key=key, ebn0_db=e, done=True, state=None, result=res)) + "\n")
        out.append(res)
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
