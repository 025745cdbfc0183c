"""GPU parity of the block decoder that keeps each frame on one compute unit
(through the C ABI), against the FP64 reference with the tolerances and gates
of test_gpu_decode: circulant sizes that give each thread 1, 2 or 3 rows of
every base row with a ragged last group, rows of weight 6, 9 and an
irregular 4-row base, one iteration with early stopping, and which decoder
ldpc_decode picks.  The block-code tests of test_gpu_decode run on this
decoder as well as on the message-package decoder."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1204_0334_amd import ldpc

from test_gpu_decode import check_parity, gpu_decode, qc_case

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(autouse=True)
def default_path(monkeypatch):
    monkeypatch.delenv("LDPC_BLOCK_PATH", raising=False)


def test_which_codes_run_on_chip(monkeypatch):
    on = [(synth.draw_qc_shifts(3, 6, 3060, 2), 3060), (synth.draw_qc_shifts(3, 6, 64, 1), 64),
          (synth.draw_qc_shifts(3, 9, 72, 53), 72), (synth.draw_qc_shifts(3, 6, 2049, 3), 2049),
          (np.array([[0, 5, -1, 7, 2, -1, 11, 3], [9, -1, 4, 1, -1, 6, 0, -1],
                     [-1, 2, 8, -1, 10, 12, -1, 5], [3, 7, -1, -1, 1, -1, 9, 0]]), 13)]
    off = [(synth.draw_qc_shifts(3, 18, 36, 1), 36),          # rows of weight 18
           (synth.draw_qc_shifts(3, 6, 3600, 1), 3600),       # 2n floats beyond the LDS of a workgroup
           (np.array([[0, -1], [3, -1]]), 5),                 # a base column without edges
           (np.array([[0, 2, 1]]), 40)]                       # one base row
    for a, p in on:
        assert ldpc.decode_path(ldpc.Graph.qc(a, p)) == "onchip", (a.shape, p)
    for a, p in off:
        assert ldpc.decode_path(ldpc.Graph.qc(a, p)) == "packages", (a.shape, p)
    monkeypatch.setenv("LDPC_BLOCK_PATH", "packages")
    assert ldpc.decode_path(ldpc.Graph.qc(*on[0])) == "packages"


def test_the_kernel_that_runs_is_the_on_chip_one():
    a, llr, _ = qc_case(3, 6, 64, 1, 64, 2.0, 101)
    g = ldpc.Graph.qc(a, 64)
    x = torch.from_numpy(llr).to(DEV)
    ldpc.timing_enable(True)
    try:
        ldpc.decode(g, x, 5, early_stop=True)
        t = ldpc.timing_read()
    finally:
        ldpc.timing_enable(False)
    assert t["onchip_decode"][0] == 1
    assert t["check_node"][0] == 0 and t["variable_node"][0] == 0


# p: rows per thread and base row 1 (p = 130: 192 threads), 2 (p = 1100: 576
# threads, the last 52 with one row), 3 (p = 2049: 704 threads, ragged)
@pytest.mark.parametrize("p", [130, 1100, 2049])
@pytest.mark.parametrize("iters", [1, 2, 3])
def test_rows_per_thread_fixed_iterations_all_frames(p, iters):
    a, llr, _ = qc_case(3, 6, p, 7, 24, 1.75, 500 + p)
    g = ldpc.Graph.qc(a, p)
    assert ldpc.decode_path(g) == "onchip"
    ref = oracle.decode_block(oracle.qc_parity_check(a, p), llr, iters)
    check_parity(gpu_decode(g, llr, iters, False), ref, True, f"p={p} I={iters}")


@pytest.mark.parametrize("p", [130, 1100, 2049])
def test_rows_per_thread_early_stop_exact_iterations(p):
    a, llr, _ = qc_case(3, 6, p, 7, 40, 2.25, 600 + p)
    g = ldpc.Graph.qc(a, p)
    H = oracle.qc_parity_check(a, p)
    ref = oracle.decode_block(H, llr, 25, early_stop=True)
    gpu = gpu_decode(g, llr, 25, True)
    check_parity(gpu, ref, False, f"p={p} early stop")
    assert np.array_equal(gpu["converged"].astype(bool), ~H.syndrome(gpu["bits"]).any(1))
    assert len(set(gpu["iters"].tolist())) >= 3


@pytest.mark.parametrize("iters", [1, 3])
def test_rate_two_thirds_two_rows_per_thread(iters):
    # 3 x 9 base with p = 1030: the 9-edge rows with 2 rows per thread
    a, llr, _ = qc_case(3, 9, 1030, 55, 16, 3.0, 404)
    g = ldpc.Graph.qc(a, 1030)
    assert ldpc.decode_path(g) == "onchip"
    ref = oracle.decode_block(oracle.qc_parity_check(a, 1030), llr, iters)
    check_parity(gpu_decode(g, llr, iters, False), ref, True, f"3x9 p=1030 I={iters}")


def test_rate_two_thirds_two_rows_per_thread_early_stop():
    a, llr, _ = qc_case(3, 9, 1030, 55, 32, 2.75, 405)
    g = ldpc.Graph.qc(a, 1030)
    H = oracle.qc_parity_check(a, 1030)
    ref = oracle.decode_block(H, llr, 20, early_stop=True)
    gpu = gpu_decode(g, llr, 20, True)
    check_parity(gpu, ref, False, "3x9 p=1030 early stop")
    assert gpu["converged"].sum() >= 16


def test_one_iteration_with_early_stop():
    # the only syndrome test is the one after the loop
    a, llr, _ = qc_case(3, 6, 64, 1, 64, 6.0, 102)   # 43 of 64 frames converge after one iteration
    g = ldpc.Graph.qc(a, 64)
    H = oracle.qc_parity_check(a, 64)
    gpu = gpu_decode(g, llr, 1, True)
    ref = oracle.decode_block(H, llr, 1, early_stop=True)
    check_parity(gpu, ref, True, "I=1 early stop")
    assert np.all(gpu["iters"] == 1)
    assert np.array_equal(gpu["converged"].astype(bool), ~H.syndrome(gpu["bits"]).any(1))
    assert 0 < gpu["converged"].sum() < 64


def test_outputs_are_optional_and_match():
    # iteration counts and convergence flags may be omitted (NULL)
    a, llr, _ = qc_case(3, 6, 64, 1, 50, 2.0, 103)
    g = ldpc.Graph.qc(a, 64)
    x = torch.from_numpy(llr).to(DEV)
    full = ldpc.decode(g, x, 20, early_stop=True)
    post = torch.empty_like(x)
    bits = torch.empty(x.shape, dtype=torch.uint8, device=DEV)
    ws = ldpc.workspace(g, 50, 20, 0, DEV)
    st = ldpc._decode(g.handle, x.data_ptr(), 50, 20, 1, post.data_ptr(), bits.data_ptr(), None, None,
                      ws.data_ptr(), ws.numel(), ldpc._stream_handle(None))
    assert st == ldpc.OK
    torch.cuda.synchronize()
    assert torch.equal(post, full[0]) and torch.equal(bits, full[1])


def test_against_the_package_decoder_at_full_size(monkeypatch):
    # n = 18360, 1024 frames, 20 iterations: the two decoders differ only in
    # FP32 rounding (beta from the posterior sum or from the other edges)
    w = synth.workload_inputs("qc36_p3060")
    g = ldpc.Graph.qc(w["shifts"], 3060)
    on = gpu_decode(g, w["llr"], 20, True)
    monkeypatch.setenv("LDPC_BLOCK_PATH", "packages")
    pk = gpu_decode(g, w["llr"], 20, True)
    both = (on["converged"] == 1) & (pk["converged"] == 1)
    assert both.mean() > 0.8
    same_iters = on["iters"] == pk["iters"]
    assert same_iters.mean() > 0.99
    sel = both & same_iters
    assert np.array_equal(on["bits"][sel], pk["bits"][sel])
    err = np.abs(on["post"][sel].astype(np.float64) - pk["post"][sel]) / np.maximum(np.abs(pk["post"][sel]), 1.0)
    assert err.max() <= 2e-4


@pytest.mark.parametrize("J,L,p", [(3, 9, 72), (3, 6, 64)])
def test_zero_llrs_of_either_sign_decide_zero(J, L, p):
    # a posterior of exactly zero, +0 or -0, is decision 0 (L < 0 is false):
    # frames of all-zero channel LLRs of either sign decode to the all-zero
    # word and stop after one iteration, also with odd row weights, where
    # counting -0 as negative would make every row unsatisfied; frames at a
    # good SNR beside them against the FP64 reference
    a = synth.draw_qc_shifts(J, L, p, 77)
    g = ldpc.Graph.qc(a, p)
    assert ldpc.decode_path(g) == "onchip"
    n = L * p
    _, llr, _ = qc_case(J, L, p, 77, 6, 4.0, 808)
    llr = llr.copy()
    llr[0] = -0.0
    llr[1] = 0.0
    llr[2, : n // 2] = -0.0
    assert np.signbit(llr[0]).all() and not np.signbit(llr[1]).any()
    gpu = gpu_decode(g, llr, 10, True)
    for f in (0, 1):
        assert gpu["iters"][f] == 1 and gpu["converged"][f] == 1, f
        assert not gpu["bits"][f].any() and not gpu["post"][f].any()
    H = oracle.qc_parity_check(a, p)
    ref = oracle.decode_block(H, llr, 10, early_stop=True)
    check_parity({k: v[2:] for k, v in gpu.items()}, {k: v[2:] for k, v in ref.items()}, False, "zero LLRs beside")
