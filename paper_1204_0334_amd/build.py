"""Build step for the HIP library: compiles csrc/ into libldpc_hip.so (gfx950).

Each source is compiled to its own object in parallel (the device code of the
two .hip files dominates the build time), then the objects are linked."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libldpc_hip.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("graph.cpp", "decode.hip", "plan.hip", "onchip.hip")]
ARCH = os.environ.get("LDPC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_flags() -> list:
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
            # keep the compiler from forming packed-FP32 VALU instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="ldpc_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in SOURCES]
        cmds = [[cc, *compile_flags(), "-c", s, "-o", o] for s, o in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), file=sys.stderr)
        with ThreadPoolExecutor(max_workers=len(cmds)) as pool:
            procs = list(pool.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
        for c, p in zip(cmds, procs):
            if p.stderr:
                sys.stderr.write(p.stderr)
            if p.returncode != 0:
                raise subprocess.CalledProcessError(p.returncode, c)
        tmp = LIB + ".tmp"
        link = [cc, f"--offload-arch={ARCH}", "-fPIC", "-shared", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), file=sys.stderr)
        subprocess.check_call(link)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
