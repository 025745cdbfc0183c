"""Throughput of the batched sum-product decoder on one MI355X.

One step = one ldpc_decode call on the paper-scale block code: the
(3,6)-regular QC-LDPC code with p = 3060 (n = 18360, m = 9180, 55080 edges),
1024 frames, 20 flooding iterations, no early stopping (fixed work), random
codewords over BPSK/AWGN at 1.5 dB, FP32 messages.  Inputs are resident in
device memory before timing starts.

Prints one JSON line: coded Mbit/s (1024 * 18360 bits per step, from the
timed region of K decodes), the roofline of the dominant kernel (from HIP
events recorded around every launch while the same K decodes run again
right after the timed region; the events are kept out of the timed region
because they add gaps between kernels), and the FP64 reference decoder timed
on the host cores on a bounded sample.  ldpc_decode runs this code on the
decoder that keeps each frame on one compute unit (one launch per decode,
bound by the FP32 vector ALUs: its roofline is algorithmic issue slots over
the launch time); the message-package decoder (edge messages through HBM,
bound by HBM bandwidth: algorithmic bytes over the launch time) is timed on
the same frames and reported beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "coded Mbit/s at 20 BP iters (n=18360, Γ=1024) + %HBM peak; FER learned vs plain"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_qc36_p3060.json")
TRAFFIC_FILE_4096 = os.path.join(ROOT, "profiles", "traffic_qc36_p3060_g4096.json")
TRAFFIC_FILE_PIPELINE = os.path.join(ROOT, "profiles", "traffic_cc36_p512_pipeline.json")
TRAFFIC_FILE_ONCHIP = os.path.join(ROOT, "profiles", "traffic_onchip_qc36_p3060.json")
TRAFFIC_FILE_ONCHIP_4096 = os.path.join(ROOT, "profiles", "traffic_onchip_qc36_p3060_g4096.json")
# counter summaries per batch size of the n = 18360 workload (none for others)
TRAFFIC_BY_GAMMA = {1024: TRAFFIC_FILE, 4096: TRAFFIC_FILE_4096}
TRAFFIC_ONCHIP_BY_GAMMA = {1024: TRAFFIC_FILE_ONCHIP, 4096: TRAFFIC_FILE_ONCHIP_4096}
# sources a counter record stays valid for: the package kernels (and the
# convolutional-code kernels) live in decode.hip, the on-chip decoder in onchip.hip
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1204_0334_amd", "csrc", f)
                  for f in ("decode.hip", "check2.h", "device.h", "internal.h")]
ONCHIP_SOURCES = [os.path.join(ROOT, "paper_1204_0334_amd", "csrc", f)
                  for f in ("onchip.hip", "check2.h", "device.h", "internal.h")]


def kernel_source_hash(files=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for p in files:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n: int, E: int, gamma: int):
    """Bytes flooding FP32 sum-product must move per launch with its state in
    HBM: the check-node pass reads and writes every edge message (8 E per
    frame); the variable-node pass reads every message and the channel LLR and
    writes every message (8 E + 4 n per frame)."""
    return {"check_node": 8 * E * gamma, "variable_node": (8 * E + 4 * n) * gamma}


def measured_traffic(kernel: str, path: str = TRAFFIC_FILE, files=KERNEL_SOURCES):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash(files):
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def window_algorithmic_bytes(info, W: int, gamma: int):
    """Average algorithmic bytes per window launch over the whole chain.
    Check-node launch: read beta on every edge of the window layers, write
    alpha on the edges whose position is active.  Variable-node launch: read
    alpha on the edges to window layers, mu of every active variable, write
    beta on every edge of the active positions."""
    import numpy as np
    c, cb, ms, L = info["c"], info["c_minus_b"], info["ms"], info["positions"]
    layers = info["layers"]
    # edges per (layer, position) pair of the unwrapped (J/Lambda x L/Lambda) base: Jb * Lb circulants
    per_pair = info["Jb"] * info["Lb"] * info["p"]
    cn = vn = 0
    for s in range(L):
        lay = range(s, min(s + W, layers))
        act = range(s, min(s + W, L))
        edges = sum(per_pair for t in lay for d in range(ms + 1) if 0 <= t - d < L)
        wr = sum(per_pair for t in lay for d in range(ms + 1) if s <= t - d < L)
        cn += 4 * (edges + wr)
        contrib = sum(per_pair for t in act for d in range(ms + 1) if t + d < layers and t + d <= lay[-1])
        alle = sum(per_pair for t in act for d in range(ms + 1) if t + d < layers)
        vn += 4 * (contrib + alle + c * len(act))
    return {"window_check_node": cn * gamma / L, "window_variable_node": vn * gamma / L}


# Issue slots of the FP32 vector ALUs (a transcendental -- exp2, log2,
# reciprocal -- issues at a quarter of the rate, so it counts 4) for the
# check rules the decoders run, Eq. 3 in base-2 units.  Convolutional-code
# decoders, (t, q) form: a row of weight d takes, over its edges, the input
# pairs 4d (1 + e, e * r, q = 2 e r, t = 1 - q), the sign product d - 1, the
# suffix sweep 2 (d - 2), the prefix sweep with the exclusive complements
# 3 (d - 2), the output pairs 2d (1 + P, times 1/Q), the output signs 2d:
# 14d - 11 plain operations, and 4d transcendentals (2^-|x| and 1/(1 + e) of
# each input, 1/Q and log2 of each output): 30d - 11 slots.  On-chip block
# decoder, the same pairs unnormalised, (u, w, s) = (1 - e, 2e, 1 + e): the
# input triples 3d, the sign product d - 1, the suffix sweep 4 (d - 2) - 1
# (U, W, S; the last S is not needed), the prefix sweep with the exclusive
# triples 6 (d - 2), the outputs 2d (2U + W, times 1/W), the output signs 2d:
# 18d - 22 plain operations, and 3d transcendentals (2^-|x| of each input,
# 1/W and log2 of each output): 30d - 22 slots.  Variable side per edge: the
# on-chip block decoder forms L = mu + sum alpha and beta = clip(L - alpha)
# (3: the addition, the subtraction, the clip); the window decoder sums the
# other edges by prefix and suffix (4: two partial sums, mu + sum, the clip).
def check_row_slots(d: int) -> int:
    return 30 * d - 11


def onchip_check_row_slots(d: int) -> int:
    return 30 * d - 22


VN_EDGE_SLOTS = 4
ONCHIP_VN_EDGE_SLOTS = 3
# FP32 vector issue rate: 256 CUs x 128 FP32 lanes x 2.4 GHz = 78.6 T lane
# operations/s (MI355X's 157.3 TFLOP/s FP32 vector figure counts an FMA as
# two).  The kernels use no packed-FP32 instructions; plain VOP2/VOP3 FP32
# instructions of wave64 issue at this rate on gfx950 (a multiply-only loop
# measured 61 T lane-ops/s), transcendentals at a quarter of it (18.6 T/s).
ALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12


def window_algorithmic_ops(info, W: int, K: int, gamma: int):
    """ALU issue slots (lane operations) of one sliding-window decode: K
    iterations per window position over the edges of the window layers
    (check) and of the active positions (variable)."""
    c, ms, L = info["c"], info["ms"], info["positions"]
    layers = info["layers"]
    per_pair = info["Jb"] * info["Lb"] * info["p"]
    total = 0
    for s in range(L):
        lay = range(s, min(s + W, layers))
        act = range(s, min(s + W, L))
        e_cn = sum(per_pair for t in lay for d in range(ms + 1) if 0 <= t - d < L)
        e_vn = sum(per_pair for t in act for d in range(ms + 1) if t + d < layers)
        # rows of the full weight (ms + 1) Lb; rows at the chain's ends have
        # fewer edges and are counted at the full rows' cost per edge
        dfull = (ms + 1) * info["Lb"]
        total += K * (check_row_slots(dfull) * e_cn / dfull + VN_EDGE_SLOTS * e_vn)
    return total * gamma


def pipeline_algorithmic_bytes(info, I: int, gamma: int):
    """Average algorithmic bytes per pipelined-decoder launch: a check-node
    launch reads beta and writes alpha on every edge of its layers, a
    variable-node launch reads alpha and mu and writes beta on every edge of
    its frames (averaged over all slots, start-up and drain included)."""
    c, ms, L, layers = info["c"], info["ms"], info["positions"], info["layers"]
    per_pair = info["Jb"] * info["Lb"] * info["p"]
    last = L - 1 + ms + (I - 1) * (ms + 1)
    cn = vn = ncn = nvn = 0
    for t in range(last + 1):
        lays = [t - (i - 1) * (ms + 1) for i in range(1, I + 1)]
        lays = [x for x in lays if 0 <= x < layers]
        frames = [x - ms for x in [t - (i - 1) * (ms + 1) for i in range(1, I + 1)]]
        frames = [f for f in frames if 0 <= f < L]
        e_cn = sum(per_pair for x in lays for d in range(ms + 1) if 0 <= x - d < L)
        e_vn = sum(per_pair for f in frames for d in range(ms + 1) if f + d < layers)
        if lays:
            cn += 8 * e_cn
            ncn += 1
        if frames:
            vn += 8 * e_vn + 4 * c * len(frames)
            nvn += 1
    return {"pipeline_check_node": cn * gamma / ncn, "pipeline_variable_node": vn * gamma / nvn}


def conv_cpu_baseline(w, spec, pipeline: bool, streams: int):
    """The FP64 reference window (or pipelined) decoder on the host, on the
    first `streams` streams of the same batch, OpenMP over streams."""
    import numpy as np

    import oracle
    threads = max(1, min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1))
    H, info = oracle.unwrap_qc(w["shifts"], spec["p"], spec["positions"], True)
    x = np.ascontiguousarray(w["llr"][:streams])
    t0 = time.perf_counter()
    if pipeline:
        oracle.decode_pipeline(H, x, spec["pipeline_iters"], info["ms"], nthreads=threads)
        what = f"pipelined decoder, {spec['pipeline_iters']} processors"
    else:
        oracle.decode_window(H, x, spec["window"], spec["iters_per_window"], nthreads=threads)
        what = f"window {spec['window']}, {spec['iters_per_window']} iterations per window"
    dt = time.perf_counter() - t0
    return {"value": round(streams * H.n / dt / 1e6, 4), "unit": "coded Mbit/s", "cores": threads, "kind": "oracle",
            "sample": f"{streams} of the {w['llr'].shape[0]} streams (whole chains), {what}, FP64, {threads} "
                      f"OpenMP threads over streams, {dt:.2f} s wall",
            "host": {"model": host_cpu_model(), "logical_cpus": os.cpu_count()}}


def bench_window(args, pipeline: bool = False):
    """The LDPC convolutional code unwrapped from the 3x6 base at p = 512:
    128 positions (c = 1024 bits) + 2 tail layers, 512 streams; sliding-window
    decoding with W = 6 and 10 iterations per window, or the pipelined decoder
    with 20 processors."""
    import torch

    import synth
    from paper_1204_0334_amd import ldpc
    gamma = args.gamma if args.gamma != 1024 else 512
    w = synth.workload_inputs("cc36_p512", gamma=gamma)
    spec = w["spec"]
    g = ldpc.Graph.ldpccc_from_qc(w["shifts"], spec["p"], spec["positions"], True)
    W, K = spec["window"], spec["iters_per_window"]
    n = g.info["n"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    llr = torch.from_numpy(w["llr"]).to(dev)
    post = torch.empty((gamma, n), dtype=torch.float32, device=dev)
    bits = torch.empty((gamma, n), dtype=torch.uint8, device=dev)
    ws = ldpc.workspace(g, gamma, 1, W, dev)

    I = spec["pipeline_iters"]
    if pipeline:
        ws = ldpc.workspace(g, gamma, I, 0, dev)

    def step():
        if pipeline:
            ldpc.decode_pipeline(g, llr, I, out=(post, bits), ws=ws)
        else:
            ldpc.decode_window(g, llr, W, K, out=(post, bits), ws=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms_per_step = start.elapsed_time(stop) / args.steps
    ldpc.timing_read()
    ldpc.timing_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ldpc.timing_enable(False)
    per_kernel = ldpc.timing_read()
    if not pipeline and per_kernel["window_lds"][0]:
        # one workgroup per stream with the ring in LDS: no message traffic
        # through HBM; the bound is the ALUs
        launches, ms = per_kernel["window_lds"]
        avg_s = ms / launches * 1e-3
        ops = window_algorithmic_ops(g.info, W, K, gamma)
        achieved = ops / avg_s / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(ALU_PEAK_TOPS, 2), "unit": "Top/s",
                    "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": None, "kernel": "window_lds",
                    "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_ops_per_launch": ops,
                    "note": "FP32 vector issue slots (transcendentals count 4) against the FP32 vector "
                            "issue rate (256 CUs x 128 lanes x 2.4 GHz); messages stay in LDS"}
    elif pipeline:
        # the ring of 68 frames x 512 streams (about 74 MB) stays in the
        # L2 / Infinity Cache, so algorithmic bytes overstate what crosses the
        # fabric: the achieved rate is the counted fabric bytes (FETCH_SIZE +
        # WRITE_SIZE, calibrated) per launch over the launch time
        algo = pipeline_algorithmic_bytes(g.info, I, gamma)
        dom = max(algo, key=lambda k: per_kernel[k][1])
        launches, ms = per_kernel[dom]
        avg_s = ms / launches * 1e-3
        traffic = measured_traffic(dom, TRAFFIC_FILE_PIPELINE)
        achieved = None if traffic is None else traffic / avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": None if achieved is None else round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": None if achieved is None else round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": dom, "avg_launch_us": round(avg_s * 1e6, 2),
                    "algorithmic_bytes_per_launch": round(algo[dom]),
                    "algorithmic_gbs": round(algo[dom] / avg_s / 1e9, 1),
                    "note": "achieved = counted fabric bytes per launch / launch time (the ring is cache-resident: "
                            "algorithmic bytes overstate HBM traffic); null when the counters predate the kernels"}
    else:
        algo = window_algorithmic_bytes(g.info, W, gamma)
        dom = max(algo, key=lambda k: per_kernel[k][1])
        launches, ms = per_kernel[dom]
        avg_s = ms / launches * 1e-3
        achieved = algo[dom] / avg_s / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                    "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": round(algo[dom]),
                    "note": "fraction of HBM peak; the decoder's ring is cache-resident"}
    ber = float(bits.float().mean().item())
    if pipeline:
        metric = "coded Mbit/s, pipelined LDPC-CC decoding (p=512, 128 positions, 20 processors, 512 streams)"
        sched = f"pipelined decoder with {I} processors"
    else:
        metric = "coded Mbit/s, sliding-window LDPC-CC decoding (p=512, 128 positions, W=6, 10 iterations/window, 512 streams)"
        sched = f"window {W}, {K} iterations per window"
    line = {
        "metric": metric,
        "value": round(gamma * n / (ms_per_step * 1e-3) / 1e6, 2), "unit": "coded Mbit/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"LDPC convolutional code unwrapped from the 3x6 base at p=512: {spec['positions']} "
                               f"positions x c={g.info['c']} bits + {g.info['ms']} tail layers; {gamma} streams; "
                               f"{sched}; all-zero codeword, BPSK/AWGN {spec['ebn0_db']} dB",
                   "n": n, "gamma": gamma, "schedule": "pipeline" if pipeline else "window",
                   "window": None if pipeline else W, "iters_per_window": None if pipeline else K,
                   "processors": I if pipeline else None, "bit_error_rate": ber},
        "roofline": roofline,
        "cpu_baseline": None if args.no_cpu else conv_cpu_baseline(w, spec, pipeline, args.cpu_streams),
        "kernels": {k: {"launches": v[0], "avg_us": round(v[1] / v[0] * 1e3, 2)} for k, v in per_kernel.items() if v[0]},
    }
    print(json.dumps(line), flush=True)


def paper_tables(args):
    """Analogue of the paper's Tables III and V on one MI355X: the 4 x 24
    (rate 5/6) code shapes A-D of Table II with seeded 4-cycle-free shifts
    (the paper's shifts are not printed).  Table III: block decoding, 30
    iterations, 3.2 dB, until 100 frame errors.  Table V: the convolutional
    codes A'-D' unwrapped from them, pipelined decoder with 20 processors,
    3.1 dB.  GPU times cover channel generation, decoding and error counting
    (as the paper's do); CPU times are the FP64 reference decoder on the host."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_1204_0334_amd import fer, ldpc
    torch.cuda.set_device(0)
    threads = max(1, min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1))
    codes = [("A", 422), ("B", 632), ("C", 768), ("D", 1024)]
    rows3, rows5 = [], []
    # one untimed batch of each decoder first: module loading and the first
    # allocations are not part of any code's time
    g0 = ldpc.Graph.qc(synth.draw_qc_shifts(4, 24, codes[0][1], 40 + codes[0][1]), codes[0][1])
    fer.simulate(g0, 3.2, gamma=args.gamma, iters=30, seed=1, max_frames=args.gamma)
    for name, p in codes:
        a = synth.draw_qc_shifts(4, 24, p, 40 + p)
        g = ldpc.Graph.qc(a, p)
        r = fer.simulate(g, 3.2, gamma=args.gamma, iters=30, seed=7, min_frame_errors=100,
                         max_frames=args.max_frames)
        H = oracle.qc_parity_check(a, p)
        llr = synth.bpsk_awgn_llr(None, fer.ebn0_to_sigma2(3.2, 5 / 6), 7, gamma=2, n=H.n)
        t0 = time.perf_counter()
        oracle.decode_block(H, llr, 30, nthreads=1)
        t_cpu = (time.perf_counter() - t0) / 2 * 1e3
        rows3.append(dict(code=name, n=H.n, E=H.ne, frames=r["frames"], frame_errors=r["frame_errors"],
                          fer=r["fer"], T_gpu_s=r["seconds"], t_gpu_ms=r["ms_per_frame"], t_cpu_ms=t_cpu,
                          speedup=t_cpu / r["ms_per_frame"], coded_mbps=r["coded_mbps"]))
        print(json.dumps({"table": "III", **rows3[-1]}), flush=True)
    positions, I, streams = args.chain_positions, 20, args.streams
    g0 = ldpc.Graph.ldpccc_from_qc(synth.draw_qc_shifts(4, 24, codes[0][1], 40 + codes[0][1]), codes[0][1],
                                   positions, True)
    fer.simulate(g0, 3.1, decoder="pipeline", gamma=streams, iters=I, seed=1, max_frames=streams)
    for name, p in codes:
        a = synth.draw_qc_shifts(4, 24, p, 40 + p)
        g = ldpc.Graph.ldpccc_from_qc(a, p, positions, True)
        r = fer.simulate(g, 3.1, decoder="pipeline", gamma=streams, iters=I, seed=9, min_frame_errors=100,
                         max_frames=args.max_streams)
        Hc, info = oracle.unwrap_qc(a, p, positions)
        llr = synth.bpsk_awgn_llr(None, fer.ebn0_to_sigma2(3.1, 5 / 6), 9, gamma=threads, n=Hc.n)
        t0 = time.perf_counter()
        oracle.decode_pipeline(Hc, llr[:1], I, info["ms"], nthreads=1)
        t1 = (time.perf_counter() - t0) * 1e3 / positions
        t0 = time.perf_counter()
        oracle.decode_pipeline(Hc, llr, I, info["ms"], nthreads=threads)
        tn = (time.perf_counter() - t0) * 1e3 / (positions * threads)
        rows5.append(dict(code=name + "'", c=info["c"], streams=r["frames"], code_frames=r["frames"] * positions,
                          stream_errors=r["frame_errors"], ber=r["ber"], T_gpu_s=r["seconds"],
                          t_gpu_ms=r["ms_per_code_frame"], t_cpu1_ms=t1, t_cpun_ms=tn, cpu_threads=threads,
                          speedup1=t1 / r["ms_per_code_frame"], speedupn=tn / r["ms_per_code_frame"],
                          coded_mbps=r["coded_mbps"]))
        print(json.dumps({"table": "V", **rows5[-1]}), flush=True)
    print()
    print(f"Table III analogue: 4x24 QC-LDPC (rate 5/6), 30 iterations, 3.2 dB, {args.gamma} frames per batch, "
          f"stop after 100 frame errors")
    print()
    print("| code | N | edges | frames | frame errors | FER | T_GPU (s) | t_GPU (ms/codeword) | t_CPU 1 thread (ms) | speed-up | coded Mbit/s |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for r in rows3:
        print(f"| {r['code']} | {r['n']} | {r['E']} | {r['frames']} | {r['frame_errors']} | {r['fer']:.2e} | "
              f"{r['T_gpu_s']:.3f} | {r['t_gpu_ms']:.5f} | {r['t_cpu_ms']:.1f} | {r['speedup']:.0f} | "
              f"{r['coded_mbps']:.0f} |")
    print()
    print(f"Table V analogue: LDPC-CC unwrapped from the same codes (Lambda = 4, m_s = 3), pipelined decoder with "
          f"{I} processors, 3.1 dB, {positions} code frames per stream, {streams} streams per batch")
    print()
    print(f"| code | c | code frames | BER | T_GPU (s) | t_GPU (ms/frame) | t_CPU 1 thread (ms/frame) | "
          f"t_CPU {threads} threads (ms/frame) | speed-up vs 1 | speed-up vs {threads} | coded Mbit/s |")
    print("|---|---|---|---|---|---|---|---|---|---|---|")
    for r in rows5:
        print(f"| {r['code']} | {r['c']} | {r['code_frames']} | {r['ber']:.2e} | {r['T_gpu_s']:.3f} | "
              f"{r['t_gpu_ms']:.5f} | {r['t_cpu1_ms']:.2f} | {r['t_cpun_ms']:.3f} | {r['speedup1']:.0f} | "
              f"{r['speedupn']:.0f} | {r['coded_mbps']:.0f} |")


def train_algorithmic_bytes(n: int, E: int, gamma: int, T: int):
    """Average bytes per launch of the training kernels with their state in
    HBM (per frame): check node 8 E (read beta or gather mu, write alpha);
    variable node 8 E + 4 n when it writes beta, 4 E + 4 n when it does not
    (the last iteration, and the end of a recomputed segment); variable-node
    backward 12 E + 4 n (alpha, dbeta, mu in; dalpha out), 8 E + 4 n at
    iteration T (no dbeta); check-node backward 12 E (beta, dalpha in; dbeta
    out), 8 E at iteration 1 (gathers mu, writes no dbeta)."""
    return {"train_variable_node_backward": ((T - 1) * (12 * E + 4 * n) + 8 * E + 4 * n) * gamma / T,
            "train_check_node_backward": ((T - 1) * 12 * E + 8 * E) * gamma / T,
            "train_check_node": 8 * E * gamma}


def bench_train(args):
    """Training throughput of the learned min-sum decoder on the paper-scale
    code: one step = forward (T = 12 iterations, checkpoints every 4), the
    hand-written backward, and an Adam update, on 1024 resident frames."""
    import torch

    import synth
    from paper_1204_0334_amd import fer, ldpc, nnms
    spec = synth.WORKLOADS["qc36_p3060"]
    g = ldpc.Graph.qc(synth.draw_qc_shifts(3, 6, spec["p"], spec["shift_seed"]), spec["p"])
    n, E, nb = g.info["n"], g.info["E"], g.info["blocks"]
    gamma, T, k = args.gamma, 12, 4
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    llr = ldpc.awgn_llr(n, gamma, fer.ebn0_to_sigma2(1.75, 0.5), 11, 0, device=dev)
    W = nnms.initial_weights(T, nb, 0.8, 0.0, device=dev).requires_grad_(True)
    opt = torch.optim.Adam([W], lr=0.01)
    ws = ldpc.nms_train_workspace(g, gamma, T, k, dev)

    def step():
        per = nnms.iteration_losses(W, g, llr, k, ws)
        loss = per.mean()
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        with torch.no_grad():
            W.clamp_(min=0.0)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms_per_step = start.elapsed_time(stop) / args.steps
    ldpc.timing_read()
    ldpc.timing_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ldpc.timing_enable(False)
    per_kernel = ldpc.timing_read()
    no_recompute = None
    if args.extras:
        # the same step keeping every iteration's messages (one segment of
        # T): no recomputation in the backward pass, at the cost of a larger
        # workspace; the gradient does not depend on the checkpoint interval
        kk = T
        ws_all = ldpc.nms_train_workspace(g, gamma, T, kk, dev)

        def step_all():
            per = nnms.iteration_losses(W, g, llr, kk, ws_all)
            loss = per.mean()
            opt.zero_grad(set_to_none=True)
            loss.backward()
            opt.step()
            with torch.no_grad():
                W.clamp_(min=0.0)

        for _ in range(args.warmup):
            step_all()
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.steps):
            step_all()
        stop.record()
        torch.cuda.synchronize()
        ms_all = start.elapsed_time(stop) / args.steps
        no_recompute = {"ckpt_every": kk, "ms_per_step": round(ms_all, 4),
                        "frames_per_s": round(gamma / (ms_all * 1e-3), 1),
                        "workspace_gb": round(ws_all.numel() * ws_all.element_size() / 1e9, 2),
                        "workspace_gb_ckpt4": round(ws.numel() * ws.element_size() / 1e9, 2)}
        del ws_all
    algo = train_algorithmic_bytes(n, E, gamma, T)
    dom = max(algo, key=lambda c: per_kernel[c][1])
    launches, ms = per_kernel[dom]
    avg_s = ms / launches * 1e-3
    achieved = algo[dom] / avg_s / 1e9
    line = {
        "metric": "learned min-sum training frames/s (forward + backward + Adam)",
        "value": round(gamma / (ms_per_step * 1e-3), 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"learned normalized/offset min-sum on the (3,6)-regular QC-LDPC code p=3060 "
                               f"(n={n}, E={E}); {gamma} frames at 1.75 dB; T={T} unrolled iterations, "
                               f"checkpoints every {k}; BCE on every iteration's posterior",
                   "n": n, "gamma": gamma, "T": T, "ckpt_every": k},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, os.path.join(ROOT, "profiles", "traffic_nnms_train_p3060.json")),
                     "kernel": dom,
                     "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": round(algo[dom])},
        "cpu_baseline": None,
        "kernels": {c: {"launches": v[0], "avg_us": round(v[1] / v[0] * 1e3, 2)} for c, v in per_kernel.items()
                    if v[0]},
        "without_recompute": no_recompute,
    }
    print(json.dumps(line), flush=True)


def bench_plan(args):
    """Mixed batch through the multi-code plan: 7 QC codes (3 x 6, 3 x 9,
    3 x 18 bases; p from 27 to 3600; 8 to 1024 frames each; 1.75-3.5 dB), 20
    iterations with early stop, one HIP graph per decode (layouts autotuned
    before timing; codes that fit a compute unit run the on-chip decoder in a
    parallel branch).  Also times the same batch decoded code by code with
    ldpc_decode, and the fixed-work (no early stop) plan for the roofline."""
    import torch

    import synth
    from paper_1204_0334_amd import ldpc
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    specs = synth.MIXED_CODES
    graphs, llrs, shifts = [], [], []
    for i, c in enumerate(specs):
        a = synth.mixed_shifts(i)
        g = ldpc.Graph.qc(a, c["p"])
        shifts.append(a)
        graphs.append(g)
        s2 = synth.ebn0_to_sigma2(c["ebn0_db"], 1.0 - c["J"] / c["L"])
        llrs.append(ldpc.awgn_llr(g.n, c["gamma"], s2, 7100 + i, 0, device=dev))
    gammas = [c["gamma"] for c in specs]
    bits = sum(g.n * x for g, x in zip(graphs, gammas))
    iters = 20

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    plan = ldpc.Plan(graphs, gammas, iters, early_stop=True)
    ws = plan.workspace(dev)
    outs = plan.outputs(dev)
    tuned_ms = plan.autotune(llrs, outs, ws, trials=3)
    layouts = [ldpc.layout_name(plan.layout(c)) for c in range(len(graphs))]
    plan.capture(llrs, outs, ws)
    ms = timed(plan.replay, args.steps, args.warmup)
    conv = sum(int(o[3].sum()) for o in outs) / sum(gammas)
    # the same decode as one persistent launch: with the layouts tuned for the
    # phase launches, then with layouts tuned for itself (graph replay both)
    per = ldpc.Plan(graphs, gammas, iters, early_stop=True)
    per.set_persistent(True)
    for c in range(len(graphs)):
        per.set_layout(c, plan.layout(c))
    pws = per.workspace(dev)
    pouts = per.outputs(dev)
    per.decode(llrs, outs=pouts, ws=pws)
    per.check(pws)
    # same layouts, same device functions: bit for bit the phase launches'
    # outputs for the codes both run in the message-package kernels (the
    # phase launches decode the codes that fit a compute unit on chip, the
    # persistent launch does not; after its own autotuning the persistent plan
    # may also pick other layouts, and a split layout agrees only to FP32
    # rounding)
    torch.cuda.synchronize()
    pkg = [c for c, g in enumerate(graphs) if ldpc.decode_path(g) != "onchip"]
    same = all(torch.equal(a, b) for c in pkg for a, b in zip(outs[c], pouts[c]))
    per.capture(llrs, pouts, pws)
    per_same_ms = timed(per.replay, args.steps, args.warmup)
    per_tuned_ms = per.autotune(llrs, pouts, pws, trials=3)
    per_layouts = [ldpc.layout_name(per.layout(c)) for c in range(len(graphs))]
    per.capture(llrs, pouts, pws)
    per_ms = timed(per.replay, args.steps, args.warmup)
    per.check(pws)
    del pws, pouts
    # the same frames code by code
    wss = [ldpc.workspace(g, x, iters, 0, dev) for g, x in zip(graphs, gammas)]
    souts = [ldpc.decode(g, x, iters, True, ws=w) for g, x, w in zip(graphs, llrs, wss)]
    seq_ms = timed(lambda: [ldpc.decode(g, x, iters, True, out=o, ws=w)
                            for g, x, o, w in zip(graphs, llrs, souts, wss)], args.steps, args.warmup)
    # fixed work (no early stop), same layouts: per-kernel times for the roofline
    fixed = ldpc.Plan(graphs, gammas, iters, early_stop=False)
    for c in range(len(graphs)):
        fixed.set_layout(c, plan.layout(c))
    fws = fixed.workspace(dev)
    fouts = fixed.outputs(dev)
    fixed.decode(llrs, outs=fouts, ws=fws)
    torch.cuda.synchronize()
    ldpc.timing_read()
    ldpc.timing_enable(True)
    for _ in range(args.steps):
        fixed.decode(llrs, outs=fouts, ws=fws)
    torch.cuda.synchronize()
    ldpc.timing_enable(False)
    per_kernel = ldpc.timing_read()
    # the phase launches carry only the codes that do not run on chip
    paths = [ldpc.decode_path(g) for g in graphs]
    pk = [i for i, q in enumerate(paths) if q == "packages"]
    E = [g.info["E"] for g in graphs]
    ns = [g.n for g in graphs]
    algo = {"plan_check_node": sum(8 * E[i] * gammas[i] for i in pk),
            "plan_variable_node": sum(((iters - 1) * (8 * E[i] + 4 * ns[i]) + 4 * E[i] + 8 * ns[i] + ns[i] / 8)
                                      * gammas[i] / iters for i in pk)}
    dom = max(algo, key=lambda k: per_kernel[k][1])
    launches, kms = per_kernel[dom]
    avg_s = kms / launches * 1e-3
    achieved = algo[dom] / avg_s / 1e9
    onchip = None
    oc = [i for i, q in enumerate(paths) if q == "onchip"]
    if oc and per_kernel["onchip_decode"][0]:
        # fixed work: every iteration of every frame of the on-chip codes,
        # over their launches' summed time (they run beside the phase launches)
        slots = sum(iters * gammas[i] * (onchip_row_slots(shifts[i], specs[i]["p"]) + ONCHIP_VN_EDGE_SLOTS * E[i])
                    for i in oc)
        t_s = per_kernel["onchip_decode"][1] * 1e-3 / args.steps
        onchip = {"bound": "alu", "codes": [i for i in oc], "achieved": round(slots / t_s / 1e12, 2),
                  "peak": round(ALU_PEAK_TOPS, 2), "unit": "Top/s",
                  "frac": round(slots / t_s / 1e12 / ALU_PEAK_TOPS, 4),
                  "launch_us_per_decode": round(t_s * 1e6, 1)}
    cpu = None
    if not args.no_cpu:
        import oracle
        threads = max(1, min(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), os.cpu_count() or 1))
        t0 = time.perf_counter()
        nb = 0
        for a, c, x in zip(shifts, specs, llrs):
            k = min(c["gamma"], 16)
            H = oracle.qc_parity_check(a, c["p"])
            oracle.decode_block(H, x[:k].cpu().numpy(), iters, early_stop=True, nthreads=threads)
            nb += k * H.n
        dt = time.perf_counter() - t0
        cpu = {"value": round(nb / dt / 1e6, 4), "unit": "coded Mbit/s", "cores": threads, "kind": "oracle",
               "sample": f"the first min(gamma, 16) frames of each of the 7 codes, {iters} iterations with early "
                         f"stop, FP64, {threads} OpenMP threads over frames, {dt:.2f} s wall"}
    line = {
        "metric": "coded Mbit/s of a mixed multi-code batch (20 BP iterations, early stop)",
        "value": round(bits / (ms * 1e-3) / 1e6, 2), "unit": "coded Mbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "7 QC-LDPC codes in one plan: " + ", ".join(
            f"{c['J']}x{c['L']} p={c['p']} x{c['gamma']} @{c['ebn0_db']}dB" for c in specs) +
            "; 20 flooding sum-product iterations with early stop; HIP graph replay",
                   "coded_bits_per_step": bits, "layouts": layouts, "autotuned_ms": round(tuned_ms, 4),
                   "frames_converged": round(conv, 4)},
        "persistent": {"ms_per_step": round(per_ms, 4), "value": round(bits / (per_ms * 1e-3) / 1e6, 2),
                       "vs_phase_launches": round(ms / per_ms, 3), "layouts": per_layouts,
                       "autotuned_ms": round(per_tuned_ms, 4),
                       "ms_with_phase_launch_layouts": round(per_same_ms, 4),
                       "outputs_equal_phase_launches": bool(same), "codes_compared": pkg,
                       "how": "one persistent launch per decode (ldpc_plan_set_persistent), HIP graph replay; outputs compared bit for bit with the phase launches in the same layouts, for the codes both decode in the message-package kernels"},
        "sequential": {"ms_per_step": round(seq_ms, 4), "value": round(bits / (seq_ms * 1e-3) / 1e6, 2),
                       "speedup_of_plan": round(seq_ms / ms, 3),
                       "how": "the same frames decoded code by code with ldpc_decode (early stop)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                     "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": round(algo[dom]),
                     "codes": pk, "onchip": onchip,
                     "note": "fixed-work pass (no early stop) with the tuned layouts, over the codes of the phase "
                             "launches; codes that fit a compute unit run the on-chip decoder beside them"},
        "cpu_baseline": cpu,
        "kernels": {c: {"launches": v[0], "avg_us": round(v[1] / v[0] * 1e3, 2)} for c, v in per_kernel.items()
                    if v[0]},
    }
    print(json.dumps(line), flush=True)


def learned_vs_plain(g, points, *, train_frames: int, eval_frames: int, T: int = 12, ckpt_every=None,
                     extra: bool = False, log=None):
    """Train the learned min-sum decoder (T iterations, scale and offset per
    iteration and base row, Adam on `train_frames` GPU-generated frames at
    Eb/N0 uniform in 1.0-2.5 dB, BCE on every iteration's posterior,
    checkpoints every `ckpt_every` iterations, None: nnms.choose_ckpt_every),
    then decode the same fresh
    frames at each Eb/N0 with it and with plain sum-product (up to 30
    iterations, early stop).  `extra` adds sum-product with T iterations and
    the untrained normalised min-sum (scale 0.8) for context."""
    import torch

    from paper_1204_0334_amd import fer, nnms
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    if ckpt_every is None:
        ckpt_every = nnms.choose_ckpt_every(g, 1024, T, dev)
    W, hist = nnms.train(g, T=T, ckpt_every=ckpt_every, frames=train_frames, batch=1024, lr=0.01, seed=7,
                         init=nnms.initial_weights(T, g.info["blocks"], 0.8, 0.0, device=dev), log_every=128)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    rows = []
    for k, e in enumerate(points):
        seed = 1_000_003 + 7919 * k

        def run(decoder, **kw):
            r = fer.simulate(g, e, decoder=decoder, gamma=1024, seed=seed, early_stop=True,
                             min_frame_errors=1 << 62, max_frames=eval_frames, **kw)
            return {"fer": r["fer"], "frame_errors": r["frame_errors"], "frames": r["frames"], "ber": r["ber"],
                    "avg_iters": round(r["avg_iters"], 3), "coded_mbps": round(r["coded_mbps"], 1)}

        row = {"ebn0_db": e, "learned_nms": run("nms", weights=W), "sp30": run("block", iters=30)}
        if extra:
            row["sp_T"] = run("block", iters=T)
            row["nms_untrained"] = run("nms", weights=nnms.initial_weights(T, g.info["blocks"], 0.8, 0.0, device=dev))
        rows.append(row)
        if log:
            log(row)
    return {"T": T, "ckpt_every": ckpt_every, "train_frames": train_frames, "train_s": round(train_s, 2),
            "train_frames_per_s": round(train_frames / train_s, 1),
            "loss_first_last": [round(hist[0][1], 5), round(hist[-1][1], 5)],
            "weights": {"scale": W[..., 0].cpu().numpy().round(4).tolist(),
                        "offset": W[..., 1].cpu().numpy().round(4).tolist()},
            "eval_frames_per_point": eval_frames, "points": rows}


def nnms_report(args):
    """Learned min-sum against plain sum-product on the paper-scale code:
    training on 2^20 frames, 10^6 fresh frames per Eb/N0 point."""
    import torch

    import synth
    from paper_1204_0334_amd import ldpc
    torch.cuda.set_device(0)
    spec = synth.WORKLOADS["qc36_p3060"]
    g = ldpc.Graph.qc(synth.draw_qc_shifts(3, 6, spec["p"], spec["shift_seed"]), spec["p"])
    points = [1.0, 1.25, 1.5, 1.75, 2.0, 2.25, 2.5]
    T = args.nnms_iters
    res = learned_vs_plain(g, points, train_frames=args.train_frames, eval_frames=args.eval_frames, T=T,
                           extra=True, log=lambda r: print(json.dumps(r), flush=True))
    print(json.dumps({k: v for k, v in res.items() if k != "points"}), flush=True)
    print()
    print(f"Learned min-sum (T = {res['T']}, trained on {res['train_frames']} frames in {res['train_s']} s) "
          f"against sum-product, n = 18360, {res['eval_frames_per_point']} frames per point, early stop")
    print()
    print(f"| Eb/N0 (dB) | SP-30 FER | SP-30 avg iters | learned NMS-{T} FER | NMS-{T} avg iters | SP-{T} FER | "
          f"untrained NMS-{T} FER |")
    print("|---|---|---|---|---|---|---|")
    for r in res["points"]:
        print(f"| {r['ebn0_db']} | {r['sp30']['fer']:.3e} | {r['sp30']['avg_iters']:.2f} | "
              f"{r['learned_nms']['fer']:.3e} | {r['learned_nms']['avg_iters']:.2f} | {r['sp_T']['fer']:.3e} | "
              f"{r['nms_untrained']['fer']:.3e} |")


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(shifts, p, llr, iters, sample, single_sample=8):
    """The FP64 reference decoder on the host: `sample` frames on all host
    threads (OpenMP over frames) -- the value -- and `single_sample` frames on
    one thread (the paper's serial-CPU analogue), same LLRs, no early stop."""
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    H = oracle.qc_parity_check(shifts, p)
    x = np.ascontiguousarray(llr[:sample])
    t0 = time.perf_counter()
    oracle.decode_block(H, x, iters, early_stop=False, nthreads=threads)
    dt = time.perf_counter() - t0
    k = min(single_sample, sample)
    t1 = time.perf_counter()
    oracle.decode_block(H, np.ascontiguousarray(llr[:k]), iters, early_stop=False, nthreads=1)
    d1 = time.perf_counter() - t1
    return {"value": round(sample * H.n / dt / 1e6, 4), "unit": "coded Mbit/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sample} of the {llr.shape[0]} frames, {iters} iterations, no early stop, FP64, "
                      f"{threads} OpenMP threads over frames, {dt:.2f} s wall ({dt * threads:.1f} thread-s)",
            "single_thread": {"value": round(k * H.n / d1 / 1e6, 4), "frames": k, "seconds": round(d1, 3),
                              "ms_per_frame": round(d1 * 1e3 / k, 2)},
            "host": {"model": host_cpu_model(), "logical_cpus": os.cpu_count()}}


def early_stop_sweep(g, gamma, iters, points, steps=5):
    """Throughput of the benchmark code with early stopping at each Eb/N0
    (GPU channel, all-zero codeword: the decoder treats every codeword alike),
    with the average iteration count."""
    import torch

    from paper_1204_0334_amd import fer, ldpc
    dev = torch.device("cuda:0")
    n = g.n
    ws = ldpc.workspace(g, gamma, iters, 0, dev)
    out = (torch.empty((gamma, n), dtype=torch.float32, device=dev),
           torch.empty((gamma, n), dtype=torch.uint8, device=dev),
           torch.empty((gamma,), dtype=torch.int32, device=dev),
           torch.empty((gamma,), dtype=torch.uint8, device=dev))
    rows = []
    for k, e in enumerate(points):
        llr = ldpc.awgn_llr(n, gamma, fer.ebn0_to_sigma2(e, g.info["design_rate"]), 900 + k, 0, device=dev)
        ldpc.decode(g, llr, iters, True, out=out, ws=ws)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            ldpc.decode(g, llr, iters, True, out=out, ws=ws)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        rows.append({"ebn0_db": e, "coded_mbps": round(gamma * n / (ms * 1e-3) / 1e6, 1), "ms": round(ms, 4),
                     "avg_iters": round(float(out[2].float().mean().item()), 3),
                     "frames_converged": round(float(out[3].float().mean().item()), 4)})
    return rows


def gamma_control(g, shifts, llr_dev, iters, gamma, steps=5):
    """The benchmark decode at a larger batch (frames repeated from the
    benchmark batch) on the decoder ldpc_decode currently selects.  For the
    message-package decoder its working set exceeds the 256 MB Infinity
    Cache, and the roofline of its variable-node pass is the HBM-resident
    figure."""
    import torch

    from paper_1204_0334_amd import ldpc
    dev = llr_dev.device
    reps = (gamma + llr_dev.shape[0] - 1) // llr_dev.shape[0]
    x = llr_dev.repeat(reps, 1)[:gamma].contiguous()
    ws = ldpc.workspace(g, gamma, iters, 0, dev)
    out = ldpc.decode(g, x, iters, False, ws=ws)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        ldpc.decode(g, x, iters, False, out=out, ws=ws)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    ldpc.timing_read()
    ldpc.timing_enable(True)
    for _ in range(steps):
        ldpc.decode(g, x, iters, False, out=out, ws=ws)
    torch.cuda.synchronize()
    ldpc.timing_enable(False)
    per_kernel = ldpc.timing_read()
    del out, ws, x
    if per_kernel["onchip_decode"][0]:
        roof = onchip_roofline(per_kernel, shifts, g.info["p"], g.info["E"], iters, gamma,
                               traffic_path=TRAFFIC_ONCHIP_BY_GAMMA.get(gamma))
    else:
        algo = algorithmic_bytes(g.n, g.info["E"], gamma)["variable_node"]
        launches, kms = per_kernel["variable_node"]
        avg_s = kms / launches * 1e-3
        achieved = algo / avg_s / 1e9
        roof = {"kernel": "variable_node", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "avg_launch_us": round(avg_s * 1e6, 2),
                "algorithmic_bytes_per_launch": algo,
                "traffic": measured_traffic("variable_node", TRAFFIC_FILE_4096)}
    return {"gamma": gamma, "ms_per_step": round(ms, 4), "coded_mbps": round(gamma * g.n / (ms * 1e-3) / 1e6, 1),
            "roofline": roof}


def onchip_row_slots(shifts, p: int) -> int:
    """Check-rule issue slots of one iteration of one frame of the QC code
    with this shift table: p rows of each base row, onchip_check_row_slots(weight)
    each (the weight: the base row's nonzero blocks)."""
    import numpy as np
    return sum(p * onchip_check_row_slots(int(d)) for d in (np.asarray(shifts) >= 0).sum(1))


def onchip_roofline(per_kernel, shifts, p: int, E: int, iters: int, gamma: int, traffic_path=TRAFFIC_FILE_ONCHIP):
    """ALU roofline of the block decoder that keeps each frame on one compute
    unit (one launch per decode, no message traffic to HBM): FP32 vector issue
    slots of Eq. 3-5 per launch (onchip_check_row_slots per row, 3 per variable
    edge; every iteration, every frame) over the launch time, against the
    FP32 vector issue rate."""
    launches, ms = per_kernel["onchip_decode"]
    avg_s = ms / launches * 1e-3
    ops = iters * gamma * (onchip_row_slots(shifts, p) + ONCHIP_VN_EDGE_SLOTS * E)
    achieved = ops / avg_s / 1e12
    return {"bound": "alu", "achieved": round(achieved, 2), "peak": round(ALU_PEAK_TOPS, 2), "unit": "Top/s",
            "frac": round(achieved / ALU_PEAK_TOPS, 4),
            "traffic": measured_traffic("onchip_decode", traffic_path, ONCHIP_SOURCES) if traffic_path else None,
            "kernel": "onchip_decode",
            "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_ops_per_launch": ops,
            "note": "FP32 vector issue slots of the check rule (30 d - 22 per row of weight d, transcendentals "
                    "count 4) and 3 per variable edge, against the FP32 vector issue rate (256 CUs x 128 lanes x "
                    "2.4 GHz); each frame's messages stay in registers and LDS of one compute unit"}


def package_roofline(per_kernel, n: int, E: int, gamma: int):
    """HBM roofline of the message-package decoder's dominant kernel."""
    algo = algorithmic_bytes(n, E, gamma)
    dom = max(algo, key=lambda k: per_kernel[k][1])
    launches, ms = per_kernel[dom]
    avg_s = ms / launches * 1e-3
    achieved = algo[dom] / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": dom,
            "traffic": measured_traffic(dom, TRAFFIC_BY_GAMMA[gamma]) if gamma in TRAFFIC_BY_GAMMA else None,
            "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": algo[dom]}


WARM_S = 0.25


def warm_seconds(fn, torch, seconds: float = WARM_S):
    """Runs fn (untimed) until about `seconds` of GPU time have passed, in
    batches timed by events, so that the timed steps start from the GPU's
    steady clocks rather than from an idle one."""
    spent, batch = 0.0, 1
    while spent < seconds:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(batch):
            fn()
        b.record()
        torch.cuda.synchronize()
        spent += a.elapsed_time(b) * 1e-3
        batch = min(batch * 2, 64)


def time_block_decode(g, llr, iters, gamma, steps, warmup):
    """After WARM_S seconds of untimed decodes and W warm-up steps, K whole
    fixed-iteration decodes timed with one event pair (nothing else enqueued
    in between), then the same K decodes again with a HIP event pair around
    every kernel launch on the decode stream (per-kernel averages)."""
    import torch

    from paper_1204_0334_amd import ldpc
    dev = llr.device
    n = g.n
    out = (torch.empty((gamma, n), dtype=torch.float32, device=dev),
           torch.empty((gamma, n), dtype=torch.uint8, device=dev),
           torch.empty((gamma,), dtype=torch.int32, device=dev),
           torch.empty((gamma,), dtype=torch.uint8, device=dev))
    ws = ldpc.workspace(g, gamma, iters, 0, dev)

    def step():
        ldpc.decode(g, llr, iters, early_stop=False, out=out, ws=ws)

    # the GPU's first ~50 decodes in a process run 3-6 % slower (clock ramp):
    # decode untimed for WARM_S of GPU time before the W warm-up steps
    warm_seconds(step, torch)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms_per_step = start.elapsed_time(stop) / steps
    ldpc.timing_read()
    ldpc.timing_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ldpc.timing_enable(False)
    per_kernel = ldpc.timing_read()
    conv_rate = float(out[3].float().mean().item())
    return ms_per_step, per_kernel, conv_rate


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--gamma", type=int, default=1024, help="frames per step (1024 is the benchmark workload)")
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--cpu-sample", type=int, default=1024, help="frames decoded by the FP64 reference")
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="benchmark line: skip the early-stop sweep over Eb/N0 and the 4096-frame control")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-streams", type=int, default=16,
                    help="convolutional workloads: streams decoded by the FP64 reference")
    ap.add_argument("--workload", default="qc36_p3060",
                    choices=["qc36_p3060", "cc36_p512", "cc36_p512_pipeline", "nnms_train_p3060", "mixed_plan"],
                    help="qc36_p3060: the block-code benchmark; cc36_p512: the convolutional-code window "
                         "decoder; cc36_p512_pipeline: the pipelined convolutional-code decoder; "
                         "nnms_train_p3060: training steps of the learned min-sum decoder; "
                         "mixed_plan: seven codes decoded together by the multi-code plan")
    ap.add_argument("--paper-tables", action="store_true",
                    help="run the analogue of the paper's Tables III and V instead of the benchmark line")
    ap.add_argument("--max-frames", type=int, default=1 << 19, help="--paper-tables: frame cap per code")
    ap.add_argument("--chain-positions", type=int, default=64, help="--paper-tables: code frames per stream")
    ap.add_argument("--streams", type=int, default=256, help="--paper-tables: streams per batch")
    ap.add_argument("--max-streams", type=int, default=4096, help="--paper-tables: stream cap per code")
    ap.add_argument("--nnms", action="store_true",
                    help="run the learned min-sum against sum-product FER comparison instead of the benchmark line")
    ap.add_argument("--train-frames", type=int, default=1 << 20, help="learned min-sum: training frames")
    ap.add_argument("--eval-frames", type=int, default=1_000_000, help="--nnms: frames per Eb/N0 point")
    ap.add_argument("--nnms-iters", type=int, default=12, help="--nnms: unrolled iterations T of the learned decoder")
    ap.add_argument("--fer-frames", type=int, default=1 << 17,
                    help="benchmark line: frames per Eb/N0 point of its learned-vs-plain FER check (0: skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run 6 device-to-device copies of BYTES (counter calibration and the copy "
                         "bandwidth ceiling; the last 5 are timed) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(5):
            dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 5
        nbytes = src.numel() * 4
        # a copy reads and writes every byte once
        print(json.dumps({"copy_bytes": nbytes, "copies": 6, "ms_per_copy": round(ms, 4),
                          "read_plus_write_gbs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this decoder runs on a single MI355X; a batch of frames "
              "would shard over GPUs with no exchange during decoding (each GPU takes a share of the frames), "
              "but no multi-GPU run is made.",
              file=sys.stderr)
        sys.exit(2)

    if args.paper_tables:
        paper_tables(args)
        return
    if args.nnms:
        nnms_report(args)
        return
    if args.workload == "nnms_train_p3060":
        bench_train(args)
        return
    if args.workload == "mixed_plan":
        bench_plan(args)
        return
    if args.workload in ("cc36_p512", "cc36_p512_pipeline"):
        bench_window(args, pipeline=args.workload.endswith("pipeline"))
        return

    import numpy as np
    import torch

    import synth
    from paper_1204_0334_amd import ldpc

    w = synth.workload_inputs("qc36_p3060", gamma=args.gamma)
    spec, shifts, llr_h = w["spec"], w["shifts"], w["llr"]
    p, gamma, iters = spec["p"], args.gamma, args.iters
    g = ldpc.Graph.qc(shifts, p)
    n, E = g.info["n"], g.info["E"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    llr = torch.from_numpy(llr_h).to(dev)
    os.environ.pop("LDPC_BLOCK_PATH", None)
    path = ldpc.decode_path(g)
    # timed region: K whole decodes on the decoder ldpc_decode selects
    ms_per_step, per_kernel, conv_rate = time_block_decode(g, llr, iters, gamma, args.steps, args.warmup)
    value = gamma * n / (ms_per_step * 1e-3) / 1e6
    if path == "onchip":
        roofline = onchip_roofline(per_kernel, shifts, p, E, iters, gamma, traffic_path=TRAFFIC_ONCHIP_BY_GAMMA.get(gamma))
    else:
        roofline = package_roofline(per_kernel, n, E, gamma)
    kernels = {k: {"launches": v[0], "avg_us": round(v[1] / v[0] * 1e3, 2)} for k, v in per_kernel.items() if v[0]}
    # the message-package decoder on the same frames (LDPC_BLOCK_PATH=packages)
    packages = None
    if path == "onchip":
        os.environ["LDPC_BLOCK_PATH"] = "packages"
        pk_ms, pk_kernels, _ = time_block_decode(g, llr, iters, gamma, args.steps, args.warmup)
        packages = {"ms_per_step": round(pk_ms, 4), "coded_mbps": round(gamma * n / (pk_ms * 1e-3) / 1e6, 1),
                    "roofline": package_roofline(pk_kernels, n, E, gamma),
                    "kernels": {k: {"launches": v[0], "avg_us": round(v[1] / v[0] * 1e3, 2)}
                                for k, v in pk_kernels.items() if v[0]}}
        if args.extras:
            packages["gamma_control"] = gamma_control(g, shifts, llr, iters, 4096)
        os.environ.pop("LDPC_BLOCK_PATH", None)

    learned = None
    if args.fer_frames > 0:
        learned = learned_vs_plain(g, [1.5, 1.75, 2.0, 2.25], train_frames=args.train_frames,
                                   eval_frames=args.fer_frames)
        learned = {"T": learned["T"], "train_frames": learned["train_frames"], "train_s": learned["train_s"],
                   "frames_per_point": learned["eval_frames_per_point"],
                   "points": [{"ebn0_db": r["ebn0_db"], "fer_learned_nms12": r["learned_nms"]["fer"],
                               "fer_sp30": r["sp30"]["fer"], "avg_iters_learned": r["learned_nms"]["avg_iters"],
                               "avg_iters_sp30": r["sp30"]["avg_iters"]} for r in learned["points"]]}
    sweep = early_stop_sweep(g, gamma, iters, [1.0, 1.25, 1.5, 1.75, 2.0, 2.25, 2.5]) if args.extras else None
    control = gamma_control(g, shifts, llr, iters, 4096) if args.extras else None
    if control is not None and path != "onchip":
        roofline["gamma_4096"] = control["roofline"]
    if packages is not None and "gamma_control" in packages:
        packages["roofline"]["gamma_4096"] = packages["gamma_control"]["roofline"]
    cpu = None if args.no_cpu else cpu_baseline(shifts, p, llr_h, iters, min(args.cpu_sample, gamma))
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "coded Mbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "gpu_warm_s": WARM_S, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"(3,6)-regular QC-LDPC, p=3060, n={n}, m={g.info['m']}, E={E}; {gamma} frames; "
                               f"{iters} flooding sum-product iterations, no early stop; random codewords, "
                               f"BPSK/AWGN {spec['ebn0_db']} dB",
                   "n": n, "gamma": gamma, "iterations": iters, "early_stop": False, "decoder": path,
                   "frames_converged": round(conv_rate, 4)},
        "roofline": roofline, "cpu_baseline": cpu, "kernels": kernels,
        "package_decoder": packages,
        "fer_learned_vs_plain": learned,
        "early_stop_per_ebn0": sweep,
        "gamma_control": control,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
