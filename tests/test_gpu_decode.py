"""GPU parity: the HIP decoder (through the C ABI) against the FP64 reference
on the same seeded inputs.

Tolerance (FP32 GPU vs FP64 reference, LLRs clipped at 30):
|clip(gpu) - clip(ref)| <= 1e-4 * max(|clip(ref)|, 1) -- relative, with a
floor of 1 so that it is 1e-4 absolute for |L| < 1.  Decisions take part in
the result only through the syndrome test (which iteration is returned) and
the returned bits, so:
  * iteration counts and convergence flags are exact on every frame where no
    decision with |L| < 1e-3 could have changed whether the syndrome is zero
    (the reference's `fragile` diagnostic is 0);
  * decisions are exact on frames that converged on both sides and on frames
    whose every decision had |L| >= 1e-3;
  * posteriors are gated on every frame after 1-3 iterations and on frames
    that converged on both sides; on frames that never converge, BP amplifies
    the rounding difference between FP32 and FP64, so they are not gated.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1204_0334_amd import ldpc

pytestmark = pytest.mark.gpu

TOL = 1e-4
DEV = "cuda:0"


def rel_err(gpu, ref):
    g = np.clip(np.asarray(gpu, dtype=np.float64), -30, 30)
    r = np.clip(np.asarray(ref, dtype=np.float64), -30, 30)
    return np.abs(g - r) / np.maximum(np.abs(r), 1.0)


@pytest.fixture(params=["onchip", "packages"])
def block_path(request, monkeypatch):
    """Runs a block-code test on both decoders behind ldpc_decode: the
    default (each frame on one compute unit where the code fits) and the
    message-package decoder (LDPC_BLOCK_PATH=packages, read at each call)."""
    if request.param == "packages":
        monkeypatch.setenv("LDPC_BLOCK_PATH", "packages")
    else:
        monkeypatch.delenv("LDPC_BLOCK_PATH", raising=False)
    return request.param


def gpu_decode(g, llr, iters, early):
    print(f"[gpu] decode n={g.n} gamma={llr.shape[0]} iters={iters} early={early} path={ldpc.decode_path(g)}",
          flush=True)
    x = torch.from_numpy(np.ascontiguousarray(llr)).to(DEV)
    post, bits, it, conv = ldpc.decode(g, x, iters, early_stop=early)
    torch.cuda.synchronize()
    return dict(post=post.cpu().numpy(), bits=bits.cpu().numpy(), iters=it.cpu().numpy(),
                converged=conv.cpu().numpy())


def qc_case(J, L, p, seed, gamma, ebn0, noise_seed, codeword="zero"):
    a = synth.draw_qc_shifts(J, L, p, seed)
    rate = 1.0 - J / L
    s2 = synth.ebn0_to_sigma2(ebn0, rate)
    if codeword == "zero":
        cw = None
        llr = synth.bpsk_awgn_llr(None, s2, noise_seed, gamma=gamma, n=L * p)
    else:
        cw = synth.encoder_for(a, p).random_codewords(gamma, seed=noise_seed + 1)
        llr = synth.bpsk_awgn_llr(cw, s2, noise_seed)
    return a, llr, cw


def check_parity(gpu, ref, gate_all_posteriors, what):
    """Returns the number of frames whose posteriors were gated."""
    robust = ref["fragile"] == 0
    assert np.array_equal(gpu["iters"][robust], ref["iters"][robust]), f"{what}: iteration counts differ"
    assert np.array_equal(gpu["converged"][robust], ref["converged"][robust]), f"{what}: convergence flags differ"
    both = robust & (gpu["converged"] == 1) & (ref["converged"] == 1)
    bitgate = both | (ref["min_abs"] >= 1e-3)
    assert np.array_equal(gpu["bits"][bitgate], ref["bits"][bitgate]), f"{what}: hard decisions differ"
    err = rel_err(gpu["post"], ref["post"])
    gate = np.ones(len(err), dtype=bool) if gate_all_posteriors else both
    worst = err[gate].max() if gate.any() else 0.0
    assert worst <= TOL, f"{what}: posterior error {worst:.3e} > {TOL}"
    return int(gate.sum())


# ----------------------------------------------------------------------------
# the small (3,6) QC code: n = 384, 64 frames, 2.0 dB
# ----------------------------------------------------------------------------

@pytest.mark.usefixtures("block_path")
@pytest.mark.parametrize("iters", [1, 2, 3])
def test_qc_p64_fixed_iterations_all_frames(iters):
    a, llr, _ = qc_case(3, 6, 64, 1, 64, 2.0, 101)
    g = ldpc.Graph.qc(a, 64)
    ref = oracle.decode_block(oracle.qc_parity_check(a, 64), llr, iters)
    gpu = gpu_decode(g, llr, iters, False)
    check_parity(gpu, ref, True, f"I={iters}")


@pytest.mark.usefixtures("block_path")
def test_qc_p64_twenty_iterations_early_stop():
    a, llr, _ = qc_case(3, 6, 64, 1, 64, 2.0, 101)
    g = ldpc.Graph.qc(a, 64)
    H = oracle.qc_parity_check(a, 64)
    ref = oracle.decode_block(H, llr, 20, early_stop=True)
    gpu = gpu_decode(g, llr, 20, True)
    check_parity(gpu, ref, False, "I=20 early stop")
    # every frame reported converged satisfies every check (independent syndrome)
    syn = H.syndrome(gpu["bits"])
    assert np.array_equal(gpu["converged"].astype(bool), ~syn.any(1))
    assert gpu["converged"].sum() >= 40


@pytest.mark.usefixtures("block_path")
def test_qc_p64_twenty_iterations_no_early_stop():
    a, llr, _ = qc_case(3, 6, 64, 1, 64, 2.0, 101)
    ref = oracle.decode_block(oracle.qc_parity_check(a, 64), llr, 20)
    gpu = gpu_decode(ldpc.Graph.qc(a, 64), llr, 20, False)
    check_parity(gpu, ref, False, "I=20")
    assert np.all(gpu["iters"] == 20)


@pytest.mark.usefixtures("block_path")
def test_frozen_frames_keep_their_stopping_iteration():
    # a frame stopped at iteration i returns exactly what a fixed i-iteration run returns
    a, llr, _ = qc_case(3, 6, 64, 1, 64, 1.5, 77)
    g = ldpc.Graph.qc(a, 64)
    es = gpu_decode(g, llr, 20, True)
    for i in sorted(set(es["iters"].tolist()))[:6]:
        sel = np.nonzero((es["iters"] == i) & (es["converged"] == 1))[0]
        if len(sel) == 0:
            continue
        fixed = gpu_decode(g, llr, int(i), False)
        assert np.array_equal(fixed["post"][sel], es["post"][sel])
        assert np.array_equal(fixed["bits"][sel], es["bits"][sel])


# ----------------------------------------------------------------------------
# ragged batches, several tiles, irregular codes, degenerate cases
# ----------------------------------------------------------------------------

@pytest.mark.usefixtures("block_path")
@pytest.mark.parametrize("gamma", [1, 63, 65, 100, 130, 257, 700])
def test_ragged_batches(gamma):
    a, llr, _ = qc_case(3, 6, 37, 1, gamma, 1.75, 300 + gamma)
    ref = oracle.decode_block(oracle.qc_parity_check(a, 37), llr, 4)
    gpu = gpu_decode(ldpc.Graph.qc(a, 37), llr, 4, False)
    check_parity(gpu, ref, True, f"gamma={gamma}")


@pytest.mark.usefixtures("block_path")
def test_irregular_qc_with_zero_blocks():
    a = np.array([[0, 5, -1, 7, 2, -1, 11, 3],
                  [9, -1, 4, 1, -1, 6, 0, -1],
                  [-1, 2, 8, -1, 10, 12, -1, 5],
                  [3, 7, -1, -1, 1, -1, 9, 0]])
    p = 13
    s2 = synth.ebn0_to_sigma2(2.5, 0.5)
    llr = synth.bpsk_awgn_llr(None, s2, 5, gamma=96, n=8 * p)
    H = oracle.qc_parity_check(a, p)
    g = ldpc.Graph.qc(a, p)
    check_parity(gpu_decode(g, llr, 3, False), oracle.decode_block(H, llr, 3), True, "irregular I=3")
    check_parity(gpu_decode(g, llr, 15, True), oracle.decode_block(H, llr, 15, early_stop=True), False,
                 "irregular I=15 early")


def test_wide_rows_use_narrow_tiles():
    # row weight 18 (rate 5/6) and 24 (rate 5/6, the paper's 4 x 24 shape)
    for J, L, p in ((3, 18, 17), (4, 24, 13)):
        a = np.random.default_rng(J * L).integers(0, p, size=(J, L))
        s2 = synth.ebn0_to_sigma2(4.0, 1 - J / L)
        llr = synth.bpsk_awgn_llr(None, s2, 9, gamma=300, n=L * p)
        ref = oracle.decode_block(oracle.qc_parity_check(a, p), llr, 3)
        check_parity(gpu_decode(ldpc.Graph.qc(a, p), llr, 3, False), ref, True, f"{J}x{L}")


@pytest.fixture
def two_frames_per_lane(monkeypatch):
    # LDPC_FRAMES_PER_LANE is read at every call; 2 is the most the tiling
    # allows for rows of weight 9..16
    monkeypatch.setenv("LDPC_FRAMES_PER_LANE", "2")


@pytest.mark.usefixtures("block_path")
@pytest.mark.parametrize("iters", [1, 2, 3])
def test_rate_two_thirds_fixed_iterations_all_frames(iters, two_frames_per_lane):
    # 3 x 9 base: rows of weight 9 (the 12-slot row class, 2 frames per
    # lane, tiles of 128 frames); 370 frames = 3 tiles, the last one ragged
    a, llr, _ = qc_case(3, 9, 72, 53, 370, 3.0, 401)
    g = ldpc.Graph.qc(a, 72)
    ref = oracle.decode_block(oracle.qc_parity_check(a, 72), llr, iters)
    check_parity(gpu_decode(g, llr, iters, False), ref, True, f"3x9 I={iters}")


@pytest.mark.usefixtures("block_path")
def test_rate_two_thirds_twenty_iterations_early_stop(two_frames_per_lane):
    a, llr, _ = qc_case(3, 9, 72, 53, 370, 2.5, 402)
    g = ldpc.Graph.qc(a, 72)
    H = oracle.qc_parity_check(a, 72)
    ref = oracle.decode_block(H, llr, 20, early_stop=True)
    gpu = gpu_decode(g, llr, 20, True)
    check_parity(gpu, ref, False, "3x9 I=20 early stop")
    assert np.array_equal(gpu["converged"].astype(bool), ~H.syndrome(gpu["bits"]).any(1))
    assert gpu["converged"].sum() >= 300 and len(set(gpu["iters"].tolist())) >= 3


@pytest.mark.usefixtures("block_path")
def test_rate_two_thirds_one_frame_per_lane():
    # the same rows with one frame per lane (the default tiling for 300 frames)
    a, llr, _ = qc_case(3, 9, 40, 54, 300, 3.0, 403)
    ref = oracle.decode_block(oracle.qc_parity_check(a, 40), llr, 3)
    check_parity(gpu_decode(ldpc.Graph.qc(a, 40), llr, 3, False), ref, True, "3x9 one frame per lane")


def test_degenerate_codes_and_inputs():
    # a variable in no check, weight-1 checks (alpha = +inf), all-zero and saturated LLRs
    a = np.array([[0, -1], [3, -1]])
    p = 5
    llr = np.zeros((70, 2 * p), dtype=np.float32)
    llr[1] = 100.0
    llr[2] = -100.0
    llr[3, :p] = -0.0
    llr[4] = np.linspace(-40, 40, 2 * p)
    ref = oracle.decode_block(oracle.qc_parity_check(a, p), llr, 3)
    gpu = gpu_decode(ldpc.Graph.qc(a, p), llr, 3, False)
    np.testing.assert_array_equal(gpu["post"], np.clip(ref["post"], -30, 30).astype(np.float32))
    np.testing.assert_array_equal(gpu["bits"], ref["bits"])


def test_forest_protographs_are_exact_map():
    # base protographs that are trees lift to forests: BP = bitwise MAP
    rng = np.random.default_rng(11)
    for base, p, iters in ((np.array([[0, 2, 1]]), 40, 1), (np.array([[0, 0, -1], [-1, 0, 0]]), 40, 3)):
        J, L = base.shape
        llr = rng.normal(0.8, 2.0, size=(64, L * p)).astype(np.float32)
        gpu = gpu_decode(ldpc.Graph.qc(base, p), llr, iters, False)
        # MAP per tree component: components of 5 columns (one circulant index each)
        H = oracle.qc_parity_check(base, p).dense()
        seen = np.zeros(L * p, dtype=bool)
        for v0 in range(L * p):
            if seen[v0]:
                continue
            comp, frontier = {v0}, [v0]
            while frontier:
                v = frontier.pop()
                for r in np.nonzero(H[:, v])[0]:
                    for u in np.nonzero(H[r])[0]:
                        if u not in comp:
                            comp.add(u)
                            frontier.append(u)
            cols = sorted(comp)
            seen[cols] = True
            rows = np.nonzero(H[:, cols].any(1))[0]
            ref = oracle.map_decode(H[np.ix_(rows, cols)], llr[:, cols])
            np.testing.assert_allclose(gpu["post"][:, cols], np.clip(ref, -30, 30), rtol=1e-5, atol=1e-5)


# ----------------------------------------------------------------------------
# batch semantics and invariants (bit-exact)
# ----------------------------------------------------------------------------

@pytest.mark.usefixtures("block_path")
def test_batch_and_permutation_invariance_and_determinism():
    a, llr, _ = qc_case(3, 6, 64, 1, 320, 1.5, 55)
    g = ldpc.Graph.qc(a, 64)
    full = gpu_decode(g, llr, 12, True)
    again = gpu_decode(g, llr, 12, True)
    for k in full:
        assert np.array_equal(full[k], again[k]), f"non-deterministic {k}"
    sub = gpu_decode(g, llr[:70], 12, True)                 # another tiling
    perm = np.random.default_rng(0).permutation(320)
    shuf = gpu_decode(g, llr[perm], 12, True)
    for k in full:
        assert np.array_equal(sub[k], full[k][:70]), k
        assert np.array_equal(shuf[k], full[k][perm]), k


@pytest.mark.usefixtures("block_path")
def test_decode_on_another_stream_with_buffers_allocated_by_the_binding():
    # workspace and outputs allocated by the binding on the current stream,
    # the decode enqueued on a second stream (default priority): the same
    # results as on the current stream, also while other work churns the
    # allocator in between
    a, llr, _ = qc_case(3, 6, 64, 1, 300, 1.75, 61)
    g = ldpc.Graph.qc(a, 64)
    x = torch.from_numpy(llr).to(DEV)
    ref = [t.clone() for t in ldpc.decode(g, x, 15, early_stop=True)]
    torch.cuda.synchronize()
    side = torch.cuda.Stream(device=DEV)
    outs = []
    for rep in range(3):
        outs.append(ldpc.decode(g, x, 15, early_stop=True, stream=side))
        junk = torch.empty(1 << 22, device=DEV).fill_(float(rep))   # reuses freed allocator blocks
        del junk
    side.synchronize()
    torch.cuda.synchronize()
    for o in outs:
        for a_, b_ in zip(o, ref):
            assert torch.equal(a_, b_)


@pytest.mark.usefixtures("block_path")
def test_codeword_symmetry():
    a, llr, cw = qc_case(3, 6, 64, 1, 128, 2.0, 21, codeword="random")
    g = ldpc.Graph.qc(a, 64)
    s = (1 - 2 * cw.astype(np.int64)).astype(np.float32)
    x = gpu_decode(g, llr, 20, True)
    y = gpu_decode(g, (llr * s).astype(np.float32), 20, True)
    assert np.array_equal(y["post"], x["post"] * s)
    assert np.array_equal(y["bits"], x["bits"] ^ cw)
    assert np.array_equal(y["iters"], x["iters"]) and np.array_equal(y["converged"], x["converged"])


# ----------------------------------------------------------------------------
# paper scale: n = 18360, 1024 frames, 20 iterations (the benchmark's call)
# ----------------------------------------------------------------------------

@pytest.mark.usefixtures("block_path")
def test_n18360_full_batch_sampled_frames():
    w = synth.workload_inputs("qc36_p3060")
    a, llr = w["shifts"], w["llr"]
    g = ldpc.Graph.qc(a, 3060)
    gpu = gpu_decode(g, llr, 20, False)
    H = oracle.qc_parity_check(a, 3060)
    # properties at full size
    assert np.array_equal(gpu["bits"], (gpu["post"] < 0).astype(np.uint8))
    syn = H.syndrome(gpu["bits"][:64])
    assert np.array_equal(gpu["converged"][:64].astype(bool), ~syn.any(1))
    # sampled frames against the reference, decoded one by one
    pick = np.array([0, 1, 255, 256, 511, 700, 1022, 1023])
    ref = oracle.decode_block(H, llr[pick], 20)
    sub = {k: v[pick] for k, v in gpu.items()}
    assert check_parity(sub, ref, False, "n=18360 sampled") >= 4
    # the codewords were random: converged frames reproduce them, except for
    # rare undetected errors -- other codewords (QC codes with weight-1
    # circulants and three block rows have minimum distance at most 24)
    ok = gpu["converged"] == 1
    assert ok.mean() > 0.5
    wrong = ok & (gpu["bits"] != w["codewords"]).any(1)
    assert wrong.sum() <= 0.01 * ok.sum()
    assert not H.syndrome(gpu["bits"][wrong]).any()


@pytest.mark.usefixtures("block_path")
def test_n18360_early_stop_sampled_frames():
    w = synth.workload_inputs("qc36_p3060", gamma=256, ebn0_db=1.25)
    a, llr = w["shifts"], w["llr"]
    gpu = gpu_decode(ldpc.Graph.qc(a, 3060), llr, 30, True)
    pick = np.array([0, 3, 40, 77, 100, 130, 160, 200, 230, 255])
    ref = oracle.decode_block(oracle.qc_parity_check(a, 3060), llr[pick], 30, early_stop=True)
    assert check_parity({k: v[pick] for k, v in gpu.items()}, ref, False, "n=18360 early stop") >= 4


# ----------------------------------------------------------------------------
# convolutional code, sliding window
# ----------------------------------------------------------------------------

def gpu_window(g, llr, W, K):
    print(f"[gpu] window n={g.n} gamma={llr.shape[0]} W={W} K={K}", flush=True)
    x = torch.from_numpy(np.ascontiguousarray(llr)).to(DEV)
    post, bits = ldpc.decode_window(g, x, W, K)
    torch.cuda.synchronize()
    return dict(post=post.cpu().numpy(), bits=bits.cpu().numpy())


def window_parity(gpu, ref, what, c, back=8, ahead=5):
    """Per code frame (chain position of c bits), as the paper's frames:
    decisions exact at every position whose neighbourhood (`back` positions
    before it, `ahead` after: the positions that share its windows or feed
    them frozen messages) holds no reference posterior with |L| < 1e-3;
    posteriors gated at every position whose neighbourhood decoded the
    all-zero codeword on both sides (inside error bursts BP amplifies the
    FP32/FP64 rounding difference).  Returns the fraction of positions whose
    posteriors were gated."""
    s = gpu["post"].shape[0]
    P = gpu["post"].shape[1] // c
    post_r = ref["post"].reshape(s, P, c)
    close = (np.abs(post_r) < 1e-3).any(2)
    wrong = gpu["bits"].reshape(s, P, c).any(2) | ref["bits"].reshape(s, P, c).any(2)

    def spread(m):
        out = np.zeros_like(m)
        for d in range(-back, ahead + 1):
            lo, hi = max(0, -d), min(P, P - d)
            if lo < hi:
                out[:, lo:hi] |= m[:, lo + d:hi + d]
        return out

    bitgate = np.repeat(~spread(close), c, axis=1)
    assert np.array_equal(gpu["bits"][bitgate], ref["bits"][bitgate]), f"{what}: decisions differ"
    gate = ~spread(close | wrong)
    err = rel_err(gpu["post"], ref["post"]).reshape(s, P, c).max(2)
    worst = err[gate].max() if gate.any() else 0.0
    assert worst <= TOL, f"{what}: posterior error {worst:.3e}"
    print(f"{what}: posteriors gated at {gate.sum()} of {gate.size} positions, decisions at "
          f"{bitgate.sum() // c} of {gate.size}", flush=True)
    return gate.mean()


@pytest.mark.parametrize("p,positions,W,K,gamma,terminate", [(32, 16, 6, 10, 64, True), (17, 12, 3, 4, 100, True),
                                                             (24, 9, 12, 5, 70, True), (16, 10, 4, 3, 65, False),
                                                             (16, 8, 3, 2, 1, True)])
def test_window_decoder_small(p, positions, W, K, gamma, terminate):
    a = synth.draw_qc_shifts(3, 6, p, 2)
    Hc, info = oracle.unwrap_qc(a, p, positions, terminate=terminate)
    llr = synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(1.5, 0.5), 103, gamma=gamma, n=Hc.n)
    ref = oracle.decode_window(Hc, llr, W, K)
    gpu = gpu_window(ldpc.Graph.ldpccc_from_qc(a, p, positions, terminate), llr, W, K)
    window_parity(gpu, ref, f"window p={p}", 2 * p)


def test_window_decoder_single_position_window_tight():
    # few iterations: every frame gated on posteriors
    a = synth.draw_qc_shifts(3, 6, 20, 2)
    Hc, _ = oracle.unwrap_qc(a, 20, 8)
    llr = synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(1.0, 0.5), 5, gamma=64, n=Hc.n)
    ref = oracle.decode_window(Hc, llr, 3, 1)
    gpu = gpu_window(ldpc.Graph.ldpccc_from_qc(a, 20, 8), llr, 3, 1)
    assert rel_err(gpu["post"], ref["post"]).max() <= TOL


def test_window_decoder_paper_scale_sampled_streams():
    w = synth.workload_inputs("cc36_p512")
    spec = w["spec"]
    a, llr = w["shifts"], w["llr"]
    g = ldpc.Graph.ldpccc_from_qc(a, spec["p"], spec["positions"], True)
    gpu = gpu_window(g, llr, spec["window"], spec["iters_per_window"])
    Hc, _ = oracle.unwrap_qc(a, spec["p"], spec["positions"])
    pick = np.array([0, 257, 511])
    ref = oracle.decode_window(Hc, llr[pick], spec["window"], spec["iters_per_window"])
    gated = window_parity({k: v[pick] for k, v in gpu.items()}, ref, "cc p=512 sampled", 2 * spec["p"])
    assert gated >= 0.15
    # a 6-position window leaves residual errors at 1.5 dB (the full chain
    # decodes under flooding BP); the bit error rate stays low
    assert gpu["bits"].mean() < 1e-2


def window_path(path, g, x, W, K):
    # LDPC_WINDOW_PATH is read by ldpc_decode_window at every call
    old = os.environ.get("LDPC_WINDOW_PATH")
    os.environ["LDPC_WINDOW_PATH"] = path
    try:
        ldpc.timing_read()
        ldpc.timing_enable(True)
        post, bits = ldpc.decode_window(g, x, W, K)
        torch.cuda.synchronize()
        ldpc.timing_enable(False)
        t = ldpc.timing_read()
    finally:
        if old is None:
            del os.environ["LDPC_WINDOW_PATH"]
        else:
            os.environ["LDPC_WINDOW_PATH"] = old
    return post, bits, t


@pytest.mark.parametrize("p,positions,W,K,gamma,terminate", [(32, 16, 6, 10, 64, True), (17, 12, 3, 4, 100, True),
                                                             (24, 9, 12, 5, 70, True), (16, 10, 4, 3, 65, False),
                                                             (16, 8, 3, 2, 1, True), (512, 128, 6, 10, 512, True)])
def test_window_lds_and_launch_paths_agree_bit_for_bit(p, positions, W, K, gamma, terminate):
    # one workgroup per stream with the ring in LDS vs one launch per phase
    # with the ring in the workspace: same arithmetic in the same order
    a = synth.draw_qc_shifts(3, 6, p, 2)
    g = ldpc.Graph.ldpccc_from_qc(a, p, positions, terminate)
    print(f"[gpu] window paths n={g.n} gamma={gamma} W={W} K={K}", flush=True)
    s2 = synth.ebn0_to_sigma2(1.5, 0.5)
    x = ldpc.awgn_llr(g.n, gamma, s2, 7 + p, 0, device=DEV)
    post_l, bits_l, t_l = window_path("lds", g, x, W, K)
    post_m, bits_m, t_m = window_path("launch", g, x, W, K)
    assert t_l["window_lds"][0] == 1 and t_l["window_check_node"][0] == 0, t_l
    assert t_m["window_lds"][0] == 0 and t_m["window_check_node"][0] > 0, t_m
    assert torch.equal(bits_l, bits_m)
    assert torch.equal(post_l, post_m)


def test_window_ring_too_big_for_lds_takes_the_launch_path():
    # p = 1024: a stream's ring is 8 x (6144 + 2048) floats = 256 KiB, more
    # than a workgroup's LDS, so every phase is a launch; results against
    # the FP64 reference as for the other windows
    p, positions, W, K, gamma = 1024, 6, 4, 3, 4
    a = synth.draw_qc_shifts(3, 6, p, 2)
    Hc, _ = oracle.unwrap_qc(a, p, positions)
    llr = synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(1.5, 0.5), 17, gamma=gamma, n=Hc.n)
    g = ldpc.Graph.ldpccc_from_qc(a, p, positions, True)
    ldpc.timing_read()
    ldpc.timing_enable(True)
    gpu = gpu_window(g, llr, W, K)
    ldpc.timing_enable(False)
    t = ldpc.timing_read()
    assert t["window_lds"][0] == 0 and t["window_check_node"][0] > 0, t
    window_parity(gpu, oracle.decode_window(Hc, llr, W, K), "window p=1024", 2 * p)


# ----------------------------------------------------------------------------
# convolutional code, pipelined decoder (Algorithm 2)
# ----------------------------------------------------------------------------

def gpu_pipeline(g, llr, I):
    print(f"[gpu] pipeline n={g.n} gamma={llr.shape[0]} I={I}", flush=True)
    x = torch.from_numpy(np.ascontiguousarray(llr)).to(DEV)
    post, bits = ldpc.decode_pipeline(g, x, I)
    torch.cuda.synchronize()
    return dict(post=post.cpu().numpy(), bits=bits.cpu().numpy())


@pytest.mark.parametrize("p,positions,I,gamma,terminate", [(32, 16, 1, 64, True), (32, 16, 3, 70, True),
                                                           (17, 12, 8, 100, True), (24, 9, 20, 65, False),
                                                           (16, 30, 12, 257, True), (16, 8, 4, 1, True)])
def test_pipeline_decoder_small(p, positions, I, gamma, terminate):
    a = synth.draw_qc_shifts(3, 6, p, 2)
    Hc, info = oracle.unwrap_qc(a, p, positions, terminate=terminate)
    llr = synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(1.5, 0.5), 107, gamma=gamma, n=Hc.n)
    ref = oracle.decode_pipeline(Hc, llr, I, info["ms"])
    gpu = gpu_pipeline(ldpc.Graph.ldpccc_from_qc(a, p, positions, terminate), llr, I)
    if I <= 3:
        assert rel_err(gpu["post"], ref["post"]).max() <= TOL
    window_parity(gpu, ref, f"pipeline p={p} I={I}", 2 * p)


def test_pipeline_matches_flooding_reference_on_the_chain():
    # the pipelined decoder computes I flooding iterations on the whole chain
    a = synth.draw_qc_shifts(3, 6, 20, 2)
    Hc, info = oracle.unwrap_qc(a, 20, 10)
    llr = synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(2.0, 0.5), 9, gamma=64, n=Hc.n)
    ref = oracle.decode_block(Hc, llr, 6)
    gpu = gpu_pipeline(ldpc.Graph.ldpccc_from_qc(a, 20, 10), llr, 6)
    window_parity(gpu, ref, "pipeline vs flooding", 40)


def test_pipeline_paper_scale_sampled_streams():
    w = synth.workload_inputs("cc36_p512")
    spec = w["spec"]
    a, llr = w["shifts"], w["llr"]
    I = spec["pipeline_iters"]
    g = ldpc.Graph.ldpccc_from_qc(a, spec["p"], spec["positions"], True)
    gpu = gpu_pipeline(g, llr, I)
    Hc, info = oracle.unwrap_qc(a, spec["p"], spec["positions"])
    pick = np.array([0, 300, 511])
    ref = oracle.decode_pipeline(Hc, llr[pick], I, info["ms"])
    gated = window_parity({k: v[pick] for k, v in gpu.items()}, ref, "pipeline p=512 sampled", 2 * spec["p"])
    assert gated >= 0.5
    assert gpu["bits"].mean() < 1e-3


# ----------------------------------------------------------------------------
# simulation on the GPU: channel generator, error counting, FER loop
# ----------------------------------------------------------------------------

def test_gpu_channel_matches_the_cpu_generator():
    n, gamma, s2, seed, f0 = 1001, 37, synth.ebn0_to_sigma2(1.3, 0.5), 0x1234_5678_9ABC, 77
    gpu = ldpc.awgn_llr(n, gamma, s2, seed, f0, device=DEV).cpu().numpy()
    cpu = synth.bpsk_awgn_llr(None, s2, seed, frame0=f0, gamma=gamma, n=n)
    ulp = np.abs(gpu.view(np.int32).astype(np.int64) - cpu.view(np.int32).astype(np.int64))
    assert ulp.max() <= 1
    assert (ulp == 0).mean() > 0.999


def test_gpu_error_counts():
    rng = np.random.default_rng(3)
    b = (rng.random((50, 333)) < 0.01).astype(np.uint8)
    b[7] = 0
    bits = torch.from_numpy(b).to(DEV)
    totals = torch.zeros((2,), dtype=torch.int64, device=DEV)
    pf = ldpc.count_errors(bits, totals=totals)
    ldpc.count_errors(bits, totals=totals)
    assert np.array_equal(pf.cpu().numpy(), b.sum(1))
    assert totals.cpu().tolist() == [2 * int(b.sum()), 2 * int((b.sum(1) > 0).sum())]


def test_fer_loop_counts_match_the_reference():
    from paper_1204_0334_amd import fer
    a = synth.draw_qc_shifts(3, 6, 37, 1)
    g = ldpc.Graph.qc(a, 37)
    r = fer.simulate(g, 0.5, gamma=64, iters=10, seed=5, min_frame_errors=10, max_frames=256)
    assert r["frame_errors"] >= 10 and r["frames"] % 64 == 0
    s2 = fer.ebn0_to_sigma2(0.5, 0.5)
    llr = synth.bpsk_awgn_llr(None, s2, 5, frame0=0, gamma=r["frames"], n=g.n)
    ref = oracle.decode_block(oracle.qc_parity_check(a, 37), llr, 10)
    errs = ref["bits"].sum(1)
    exempt = ref["min_abs"] < 1e-3
    lo = int(((errs > 0) & ~exempt).sum())
    hi = int(((errs > 0) | exempt).sum())
    assert lo <= r["frame_errors"] <= hi
    # high SNR: no errors in the frames simulated
    r2 = fer.simulate(g, 8.0, gamma=64, iters=10, seed=5, max_frames=512)
    assert r2["frames"] == 512 and r2["frame_errors"] == 0


def test_fer_loop_pipeline_decoder():
    from paper_1204_0334_amd import fer
    a = synth.draw_qc_shifts(3, 6, 24, 2)
    g = ldpc.Graph.ldpccc_from_qc(a, 24, 12)
    r = fer.simulate(g, 0.0, decoder="pipeline", gamma=64, iters=5, seed=3, min_frame_errors=5, max_frames=128)
    Hc, info = oracle.unwrap_qc(a, 24, 12)
    llr = synth.bpsk_awgn_llr(None, fer.ebn0_to_sigma2(0.0, 0.5), 3, frame0=0, gamma=r["frames"], n=Hc.n)
    ref = oracle.decode_pipeline(Hc, llr, 5, info["ms"])
    close = (np.abs(ref["post"]) < 1e-3).any(1)
    errs = ref["bits"].sum(1)
    assert int(((errs > 0) & ~close).sum()) <= r["frame_errors"] <= int(((errs > 0) | close).sum())


def test_fer_simulation_resumes_exactly(tmp_path):
    # an interrupted FER run resumed from its last checkpoint gives the same
    # counters as an uninterrupted one (counter-based generator)
    from paper_1204_0334_amd import fer
    a = synth.draw_qc_shifts(3, 6, 64, 1)
    g = ldpc.Graph.qc(a, 64)
    print("[gpu] fer resume", flush=True)
    kw = dict(gamma=256, iters=10, early_stop=True, seed=5, min_frame_errors=1 << 30, max_frames=8 * 256)
    full = fer.simulate(g, 2.0, **kw)
    states = []
    fer.simulate(g, 2.0, checkpoint=states.append, checkpoint_every=3, **dict(kw, max_frames=3 * 256))
    assert states[-1]["frames"] == 3 * 256
    rest = fer.simulate(g, 2.0, resume=states[-1], **kw)
    for k in ("frames", "frame_errors", "bit_errors", "avg_iters"):
        assert rest[k] == full[k], k
    # the JSONL sweep skips finished points and resumes unfinished ones
    log = str(tmp_path / "sweep.jsonl")
    r1 = fer.sweep(g, [2.0, 2.5], log, key="p64", **kw)
    r2 = fer.sweep(g, [2.0, 2.5], log, key="p64", **kw)
    assert [x["frame_errors"] for x in r1] == [x["frame_errors"] for x in r2]
    assert r1[0]["frame_errors"] == full["frame_errors"]
