"""Command line: FER/BER sweeps on the GPU with the paper's stopping rule.

    python -m paper_1204_0334_amd sweep --code qc36_p3060 --ebn0 1.0 1.5 2.0 \\
        --iters 30 --log sweep.jsonl
    python -m paper_1204_0334_amd sweep --code cc36_p512 --decoder pipeline --iters 20 --ebn0 1.5
    python -m paper_1204_0334_amd codes

Codes are the named presets (QC shift tables drawn by the seeded 4-cycle-free
generator: the benchmark workloads and the paper's Table II shapes
table2_A..D; `--positions` unwraps a block preset into a convolutional code)
or `--shifts FILE` (a JSON list of rows, -1 = zero block) with `--p`.  Each Eb/N0 point runs until `--min-errors` frame errors or
`--max-frames` frames; results are appended to the JSONL log, and a rerun
with the same log resumes unfinished points and skips finished ones.
"""
from __future__ import annotations

import argparse
import json
import sys


def _presets():
    """Named codes: the benchmark workloads, and the 4 x 24 (rate 5/6) shapes
    of the paper's Table II (codes A-D, p = 422, 632, 768, 1024) with the
    seeded 4-cycle-free shifts the paper-table analogue of bench.py uses
    (the paper does not print its shifts)."""
    import synth
    out = {k: dict(w) for k, w in synth.WORKLOADS.items()}
    for name, p in (("A", 422), ("B", 632), ("C", 768), ("D", 1024)):
        out[f"table2_{name}"] = dict(J=4, L=24, p=p, shift_seed=40 + p)
    return out


def _graph(args):
    import synth

    from . import ldpc
    if args.shifts:
        if args.p is None:
            raise SystemExit("--shifts needs --p")
        with open(args.shifts) as f:
            shifts = json.load(f)
        key = f"{args.shifts}:p{args.p}"
        if args.positions:
            return ldpc.Graph.ldpccc_from_qc(shifts, args.p, args.positions, True), key
        return ldpc.Graph.qc(shifts, args.p), key
    presets = _presets()
    if args.code not in presets:
        raise SystemExit(f"unknown code {args.code!r}; see `codes`")
    w = presets[args.code]
    shifts = synth.draw_qc_shifts(w["J"], w["L"], w["p"], w["shift_seed"])
    if "positions" in w or args.positions:
        return ldpc.Graph.ldpccc_from_qc(shifts, w["p"], args.positions or w["positions"], True), args.code
    return ldpc.Graph.qc(shifts, w["p"]), args.code


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_1204_0334_amd")
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("codes", help="list the named code presets")
    sw = sub.add_parser("sweep", help="FER/BER over Eb/N0 points")
    sw.add_argument("--code", default="qc36_p3060")
    sw.add_argument("--shifts", help="JSON shift table (rows of circulant shifts, -1 = zero block)")
    sw.add_argument("--p", type=int, help="circulant size for --shifts")
    sw.add_argument("--positions", type=int, help="convolutional code: unwrap to this many positions")
    sw.add_argument("--decoder", default="block", choices=["block", "window", "pipeline"])
    sw.add_argument("--iters", type=int, default=30, help="iterations (window: per window; pipeline: processors)")
    sw.add_argument("--window", type=int, default=6)
    sw.add_argument("--early-stop", action="store_true")
    sw.add_argument("--ebn0", type=float, nargs="+", required=True)
    sw.add_argument("--gamma", type=int, default=1024, help="frames (streams) per batch")
    sw.add_argument("--min-errors", type=int, default=100)
    sw.add_argument("--max-frames", type=int, default=1 << 20)
    sw.add_argument("--seed", type=int, default=1)
    sw.add_argument("--log", default="fer_sweep.jsonl")
    args = ap.parse_args(argv)
    if args.cmd == "codes":
        for k, w in _presets().items():
            print(k, json.dumps({a: b for a, b in w.items() if a != "noise_seed"}))
        return 0
    from . import fer
    g, key = _graph(args)
    key = f"{key}:{args.decoder}:{args.iters}:{'es' if args.early_stop else 'fixed'}:w{args.window}:s{args.seed}"
    res = fer.sweep(g, args.ebn0, args.log, key=key, decoder=args.decoder, gamma=args.gamma, iters=args.iters,
                    early_stop=args.early_stop, window=args.window, seed=args.seed,
                    min_frame_errors=args.min_errors, max_frames=args.max_frames)
    for r in res:
        lo, hi = fer.fer_interval(r["frame_errors"], r["frames"])
        print(json.dumps({"ebn0_db": r["ebn0_db"], "frames": r["frames"], "frame_errors": r["frame_errors"],
                          "fer": r["fer"], "fer_95": [lo, hi], "ber": r["ber"],
                          "coded_mbps": round(r["coded_mbps"], 1)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
