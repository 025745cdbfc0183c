"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the C ABI's graph construction and validation (graph.cpp, which makes
no HIP call) on random and invalid inputs, and the FP64 reference decoders on
random banded codes, built with g++/gcc and run by tests/host/
sanitize_harness.cpp."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


@pytest.mark.skipif(not (shutil.which("g++") and shutil.which("gcc")), reason="needs g++ and gcc")
def test_graph_builders_and_reference_under_sanitizers(tmp_path):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    bp = str(tmp_path / "bp.o")
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", *SAN, "-c", os.path.join(ROOT, "oracle", "bp.c"),
                           "-o", bp])
    exe = str(tmp_path / "harness")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fopenmp", *SAN, *inc,
                           os.path.join(ROOT, "paper_1204_0334_amd", "csrc", "graph.cpp"),
                           os.path.join(ROOT, "tests", "host", "sanitize_harness.cpp"), bp, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout[-2000:] + r.stderr[-4000:]
