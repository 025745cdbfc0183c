"""Throughput of the batched sum-product decoder on one MI355X.

One step = one ldpc_decode call on the paper-scale block code: the
(3,6)-regular QC-LDPC code with p = 3060 (n = 18360, m = 9180, 55080 edges),
1024 frames, 20 flooding iterations, no early stopping (fixed work), random
codewords over BPSK/AWGN at 1.5 dB, FP32 messages.  Inputs are resident in
device memory before timing starts.

Prints one JSON line: coded Mbit/s (1024 * 18360 bits per step, from the
timed region of K decodes), the roofline of the dominant kernel (algorithmic
bytes / average launch time, from HIP events recorded around every launch
while the same K decodes run again right after the timed region; the events
are kept out of the timed region because they add gaps between kernels), and
the FP64 reference decoder timed on the host cores on a bounded sample.
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
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1204_0334_amd", "csrc", "decode.hip"),
                  os.path.join(ROOT, "paper_1204_0334_amd", "csrc", "internal.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n: int, E: int, gamma: int):
    """Bytes flooding FP32 sum-product must move per launch with its state in
    HBM: the check-node pass reads and writes every edge message (8 E per
    frame); the variable-node pass reads every message and the channel LLR and
    writes every message (8 E + 4 n per frame)."""
    return {"check_node": 8 * E * gamma, "variable_node": (8 * E + 4 * n) * gamma}


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(shifts, p, llr, iters, sample):
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    H = oracle.qc_parity_check(shifts, p)
    x = np.ascontiguousarray(llr[:sample])
    t0 = time.perf_counter()
    oracle.decode_block(H, x, iters, early_stop=False, nthreads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(sample * H.n / dt / 1e6, 4), "unit": "coded Mbit/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sample} of the {llr.shape[0]} frames, {iters} iterations, no early stop, FP64, "
                      f"{threads} OpenMP threads over frames, {dt:.2f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--gamma", type=int, default=1024, help="frames per step (1024 is the benchmark workload)")
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--cpu-sample", type=int, default=96, help="frames decoded by the FP64 reference")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run 5 device-to-device copies of BYTES (counter calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(args.calibrate_copy // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 5}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this decoder runs on a single MI355X; a batch of frames "
              "would shard over GPUs with no exchange (see DESIGN.md), but no multi-GPU run is made.",
              file=sys.stderr)
        sys.exit(2)

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
    post = torch.empty((gamma, n), dtype=torch.float32, device=dev)
    bits = torch.empty((gamma, n), dtype=torch.uint8, device=dev)
    it = torch.empty((gamma,), dtype=torch.int32, device=dev)
    conv = torch.empty((gamma,), dtype=torch.uint8, device=dev)
    ws = ldpc.workspace(g, gamma, iters, 0, dev)
    out = (post, bits, it, conv)

    def step():
        ldpc.decode(g, llr, iters, early_stop=False, out=out, ws=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: K whole decodes, nothing else enqueued in between
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ms_per_step = total_ms / args.steps
    # the same K decodes again with a HIP event pair around every kernel launch
    # (on the decode stream): per-kernel average durations for the roofline
    ldpc.timing_read()
    ldpc.timing_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ldpc.timing_enable(False)
    per_kernel = ldpc.timing_read()
    value = gamma * n / (ms_per_step * 1e-3) / 1e6

    # dominant kernel and its roofline
    algo = algorithmic_bytes(n, E, gamma)
    dom = max(algo, key=lambda k: per_kernel[k][1])
    launches, ms = per_kernel[dom]
    avg_s = ms / launches * 1e-3
    achieved = algo[dom] / avg_s / 1e9
    traffic = measured_traffic(dom)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "avg_launch_us": round(avg_s * 1e6, 2), "algorithmic_bytes_per_launch": algo[dom]}
    kernels = {k: {"launches": v[0], "avg_us": round(v[1] / v[0] * 1e3, 2)} for k, v in per_kernel.items() if v[0]}

    conv_rate = float(conv.float().mean().item())
    cpu = None if args.no_cpu else cpu_baseline(shifts, p, llr_h, iters, min(args.cpu_sample, gamma))
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "coded Mbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"(3,6)-regular QC-LDPC, p=3060, n={n}, m={g.info['m']}, E={E}; {gamma} frames; "
                               f"{iters} flooding sum-product iterations, no early stop; random codewords, "
                               f"BPSK/AWGN {spec['ebn0_db']} dB",
                   "n": n, "gamma": gamma, "iterations": iters, "early_stop": False,
                   "frames_converged": round(conv_rate, 4)},
        "roofline": roofline, "cpu_baseline": cpu, "kernels": kernels,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
