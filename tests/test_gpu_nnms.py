"""GPU parity of the learned min-sum decoder and of its hand-written backward
pass (through the C ABI) against the FP64 reference (torch float64 autograd
on the CPU), on the same seeded inputs.

Tolerances.  Decoding: the min-sum rule itself is exact in FP32 (minimum,
sign, scale and offset round once), so the posteriors differ from FP64 only
by the rounding of the sums: |clip(gpu) - clip(ref)| <= 1e-4 max(|ref|, 1),
decisions exact except where the reference posterior is below 1e-3 in
magnitude.  Loss: 1e-5 relative.  Gradient: each entry is a sum over all
frames and rows in FP32 of terms with FP32 exponentials, so
|gpu - ref| <= 2e-3 |ref| + 2e-4 max|ref|.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import nnms as ref_nnms
from paper_1204_0334_amd import ldpc
from paper_1204_0334_amd import nnms

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-4


def case(J, L, p, seed, gamma, ebn0, noise_seed):
    a = synth.draw_qc_shifts(J, L, p, seed)
    s2 = synth.ebn0_to_sigma2(ebn0, 1.0 - J / L)
    llr = synth.bpsk_awgn_llr(None, s2, noise_seed, gamma=gamma, n=L * p)
    return a, llr


def rand_weights(T, classes, seed):
    """[T, classes, 2]: (scale, offset) per iteration and edge class."""
    rng = np.random.default_rng(seed)
    w = np.stack([rng.uniform(0.55, 1.0, size=(T, classes)), rng.uniform(0.0, 0.6, size=(T, classes))], axis=-1)
    return w.astype(np.float32)


def ref_graph(a, p):
    return ref_nnms.EdgeGraph(oracle.qc_parity_check(a, p), ref_nnms.qc_edge_class(a, p))


NB36, NB318 = 18, 54   # edge classes (circulant blocks) of the 3 x 6 and 3 x 18 bases


@pytest.fixture(params=["onchip", "packages"])
def block_path(request, monkeypatch):
    """Runs a decoding test on both decoders behind ldpc_nms_decode: the
    default (each frame on one compute unit where the code fits) and the
    message-package decoder (LDPC_BLOCK_PATH=packages, read at each call)."""
    if request.param == "packages":
        monkeypatch.setenv("LDPC_BLOCK_PATH", "packages")
    else:
        monkeypatch.delenv("LDPC_BLOCK_PATH", raising=False)
    return request.param


def gpu_nms(g, llr, w, early=False):
    print(f"[gpu] nms_decode n={g.n} gamma={llr.shape[0]} T={w.shape[0]} early={early} path={ldpc.decode_path(g)}",
          flush=True)
    x = torch.from_numpy(np.ascontiguousarray(llr)).to(DEV)
    wt = torch.from_numpy(np.ascontiguousarray(w)).to(DEV)
    post, bits, it, conv = ldpc.nms_decode(g, x, wt, early_stop=early)
    torch.cuda.synchronize()
    return dict(post=post.cpu().numpy(), bits=bits.cpu().numpy(), iters=it.cpu().numpy(),
                converged=conv.cpu().numpy())


def check_decode(gpu, ref, what):
    raw = ref["raw"]
    ok = np.abs(raw) >= 1e-3
    assert np.array_equal(gpu["bits"][ok], ref["bits"][ok]), f"{what}: decisions differ"
    g = np.clip(gpu["post"].astype(np.float64), -30, 30)
    r = ref["post"]
    err = np.abs(g - r) / np.maximum(np.abs(r), 1.0)
    assert err.max() <= TOL, f"{what}: posterior error {err.max():.3e}"


@pytest.mark.usefixtures("block_path")
@pytest.mark.parametrize("T,gamma", [(1, 64), (3, 64), (12, 64), (12, 200), (4, 1), (5, 65)])
def test_nms_decode_matches_reference(T, gamma):
    a, llr = case(3, 6, 64, 1, gamma, 2.0, 101)
    w = rand_weights(T, NB36, T)
    ref = ref_nnms.decode(ref_graph(a, 64), llr.astype(np.float64), w[..., 0], w[..., 1], T)
    gpu = gpu_nms(ldpc.Graph.qc(a, 64), llr, w)
    check_decode(gpu, ref, f"T={T} gamma={gamma}")
    assert np.all(gpu["iters"] == T)


def test_nms_decode_wide_rows():
    # 3 x 18 base (row weight 18): one frame per lane, row-weight class 24
    a, llr = case(3, 18, 36, 3, 96, 3.5, 55)
    w = rand_weights(8, NB318, 5)
    ref = ref_nnms.decode(ref_graph(a, 36), llr.astype(np.float64), w[..., 0], w[..., 1], 8)
    check_decode(gpu_nms(ldpc.Graph.qc(a, 36), llr, w), ref, "3x18")


@pytest.mark.usefixtures("block_path")
def test_nms_early_stop_returns_the_stopping_iteration():
    a, llr = case(3, 6, 64, 1, 64, 2.0, 101)
    g = ldpc.Graph.qc(a, 64)
    H = oracle.qc_parity_check(a, 64)
    T = 12
    w = rand_weights(T, NB36, 9)
    gpu = gpu_nms(g, llr, w, early=True)
    syn = H.syndrome(gpu["bits"])
    assert np.array_equal(gpu["converged"].astype(bool), ~syn.any(1))
    assert gpu["converged"].sum() >= 40
    G = ref_graph(a, 64)
    for i in sorted(set(gpu["iters"].tolist())):
        sel = np.nonzero(gpu["iters"] == i)[0]
        ref = ref_nnms.decode(G, llr[sel].astype(np.float64), w[:i, :, 0], w[:i, :, 1], int(i))
        sub = {k: v[sel] for k, v in gpu.items()}
        check_decode(sub, ref, f"frames stopped at {i}")
        if i < T:
            assert np.all(gpu["converged"][sel] == 1)


def gpu_grad(g, llr, w, ckpt, dloss=None):
    print(f"[gpu] nms_train n={g.n} gamma={llr.shape[0]} T={w.shape[0]} ckpt={ckpt}", flush=True)
    T = w.shape[0]
    x = torch.from_numpy(np.ascontiguousarray(llr)).to(DEV)
    wt = torch.from_numpy(np.ascontiguousarray(w)).to(DEV)
    ws = ldpc.nms_train_workspace(g, llr.shape[0], T, ckpt, DEV)
    loss = ldpc.nms_train_forward(g, x, wt, ckpt, ws)
    dl = torch.full((T,), 1.0 / T, dtype=torch.float32, device=DEV) if dloss is None else \
        torch.from_numpy(np.asarray(dloss, dtype=np.float32)).to(DEV)
    grad = ldpc.nms_train_backward(g, llr.shape[0], wt, ckpt, dl, ws)
    torch.cuda.synchronize()
    return loss.cpu().numpy().astype(np.float64), grad.cpu().numpy().astype(np.float64)


def check_grad(gg, gw, gb, what):
    ref = np.stack([gw, gb], axis=-1)
    err = np.abs(gg - ref)
    bound = 2e-3 * np.abs(ref) + 2e-4 * np.abs(ref).max()
    worst = (err / bound).max()
    assert worst <= 1.0, f"{what}: gradient off by {worst:.2f} x tolerance"


@pytest.mark.parametrize("gamma,T,ckpt", [(64, 6, 2), (200, 5, 2), (256, 12, 4)])
def test_gradient_matches_fp64_autograd(gamma, T, ckpt):
    a, llr = case(3, 6, 64, 1, gamma, 1.5, 303)
    w = rand_weights(T, NB36, 11)
    g = ldpc.Graph.qc(a, 64)
    loss, gg = gpu_grad(g, llr, w, ckpt)
    G = ref_graph(a, 64)
    x = np.ones_like(llr, dtype=np.float64)
    per = ref_nnms.iteration_losses(G, llr.astype(np.float64), x, torch.tensor(w[..., 0], dtype=torch.float64),
                                    torch.tensor(w[..., 1], dtype=torch.float64), T).numpy()
    np.testing.assert_allclose(loss, per, rtol=1e-5)
    _, gw, gb = ref_nnms.grad(G, llr.astype(np.float64), x, w[..., 0].astype(np.float64),
                              w[..., 1].astype(np.float64), T)
    check_grad(gg, gw, gb, f"gamma={gamma} T={T} ckpt={ckpt}")


def test_gradient_with_per_iteration_upstream():
    a, llr = case(3, 6, 64, 1, 128, 1.5, 304)
    T = 4
    w = rand_weights(T, NB36, 12)
    coef = np.array([0.0, 2.0, -0.5, 1.0])
    g = ldpc.Graph.qc(a, 64)
    _, gg = gpu_grad(g, llr, w, 2, dloss=coef)
    x = np.ones_like(llr, dtype=np.float64)
    _, gw, gb = ref_nnms.grad(ref_graph(a, 64), llr.astype(np.float64), x, w[..., 0].astype(np.float64),
                              w[..., 1].astype(np.float64), T, coef=coef)
    check_grad(gg, gw, gb, "upstream coefficients")


def test_gradient_independent_of_checkpoint_interval():
    a, llr = case(3, 6, 64, 1, 256, 1.5, 305)
    T = 6
    w = rand_weights(T, NB36, 13)
    g = ldpc.Graph.qc(a, 64)
    grads = [gpu_grad(g, llr, w, k)[1] for k in (1, 2, 4, 6)]
    for k, gk in zip((2, 4, 6), grads[1:]):
        assert np.array_equal(gk, grads[0]), f"checkpoint every {k} changes the gradient"
    assert np.array_equal(gpu_grad(g, llr, w, 4)[1], grads[2]), "gradient is not deterministic"


def test_gradient_wide_rows():
    a, llr = case(3, 18, 36, 3, 64, 3.5, 56)
    T = 4
    w = rand_weights(T, NB318, 14)
    _, gg = gpu_grad(ldpc.Graph.qc(a, 36), llr, w, 2)
    x = np.ones_like(llr, dtype=np.float64)
    _, gw, gb = ref_nnms.grad(ref_graph(a, 36), llr.astype(np.float64), x, w[..., 0].astype(np.float64),
                              w[..., 1].astype(np.float64), T)
    check_grad(gg, gw, gb, "3x18")


@pytest.mark.usefixtures("block_path")
def test_irregular_base_decode_and_gradient():
    # zero blocks: base rows with 4 and 5 blocks, columns with 1 to 3, so an
    # edge slot of a row is not its block's base column
    a = np.array([[0, 5, -1, 7, 2, -1], [9, -1, 4, 1, -1, 6], [-1, 2, 8, -1, 10, 12]])
    p = 13
    g = ldpc.Graph.qc(a, p)
    nb = int((a >= 0).sum())
    assert g.info["blocks"] == nb
    llr = synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(2.0, 0.5), 57, gamma=96, n=6 * p)
    T = 5
    w = rand_weights(T, nb, 16)
    ref = ref_nnms.decode(ref_graph(a, p), llr.astype(np.float64), w[..., 0], w[..., 1], T)
    check_decode(gpu_nms(g, llr, w), ref, "irregular base")
    _, gg = gpu_grad(g, llr, w, 2)
    x = np.ones_like(llr, dtype=np.float64)
    _, gw, gb = ref_nnms.grad(ref_graph(a, p), llr.astype(np.float64), x, w[..., 0].astype(np.float64),
                              w[..., 1].astype(np.float64), T)
    check_grad(gg, gw, gb, "irregular base")


def test_paper_scale_gradient():
    # n = 18360 (p = 3060), T = 12, checkpoints every 4: 16 frames against the
    # reference; at the training batch of 1024 frames, the gradient is the
    # mean of the gradients of its four quarters (the loss is a mean over frames)
    spec = synth.WORKLOADS["qc36_p3060"]
    a = synth.draw_qc_shifts(3, 6, 3060, spec["shift_seed"])
    s2 = synth.ebn0_to_sigma2(1.75, 0.5)
    g = ldpc.Graph.qc(a, 3060)
    T, ckpt = 12, 4
    w = rand_weights(T, NB36, 15)
    llr = synth.bpsk_awgn_llr(None, s2, 909, gamma=16, n=18360)
    _, gg = gpu_grad(g, llr, w, ckpt)
    x = np.ones_like(llr, dtype=np.float64)
    _, gw, gb = ref_nnms.grad(ref_graph(a, 3060), llr.astype(np.float64), x, w[..., 0].astype(np.float64),
                              w[..., 1].astype(np.float64), T)
    check_grad(gg, gw, gb, "n=18360, 16 frames")
    dev_llr = ldpc.awgn_llr(18360, 1024, s2, 910, 0, device=DEV)
    torch.cuda.synchronize()
    big = dev_llr.cpu().numpy()
    _, gfull = gpu_grad(g, big, w, ckpt)
    quarters = [gpu_grad(g, big[i * 256:(i + 1) * 256], w, ckpt)[1] for i in range(4)]
    mean = np.mean(quarters, axis=0)
    err = np.abs(gfull - mean)
    assert np.all(err <= 1e-4 * np.abs(mean) + 1e-5 * np.abs(mean).max())


def test_training_improves_on_plain_min_sum():
    a = synth.draw_qc_shifts(3, 6, 64, 1)
    g = ldpc.Graph.qc(a, 64)
    T = 6
    print("[gpu] nnms.train p=64", flush=True)
    plain = nnms.initial_weights(T, NB36, scale=1.0, offset=0.0, device=DEV)
    W, hist = nnms.train(g, T=T, ckpt_every=2, frames=64 * 1024, batch=1024, lr=0.02, log_every=8, init=plain)
    assert torch.all(W >= 0)
    assert not torch.allclose(W[..., 0], plain[..., 0])
    # on the same 8192 fresh frames at 2.5 dB the learned weights decode
    # better than plain min-sum (about 0.33 against 0.47 frame error rate)
    learned = nnms.compare_fer(g, W, [2.5], sp_iters=20, frames=8192, gamma=1024)[0]["learned"]
    base = nnms.compare_fer(g, plain, [2.5], sp_iters=20, frames=8192, gamma=1024)[0]["learned"]
    assert learned["frames"] == base["frames"] == 8192
    assert learned["fer"] < base["fer"] - 0.05


def test_training_resumes_from_checkpoint(tmp_path):
    # 6 steps in one run equal 3 steps, a checkpoint, and 3 resumed steps
    a = synth.draw_qc_shifts(3, 6, 64, 1)
    g = ldpc.Graph.qc(a, 64)
    T = 4
    init = nnms.initial_weights(T, NB36, 0.8, 0.1, device=DEV)
    print("[gpu] nnms.train checkpoint", flush=True)
    W_full, h_full = nnms.train(g, T=T, ckpt_every=2, frames=6 * 512, batch=512, lr=0.02, init=init, log_every=1)
    path = str(tmp_path / "nnms.pt")
    nnms.train(g, T=T, ckpt_every=2, frames=3 * 512, batch=512, lr=0.02, init=init, log_every=1,
               checkpoint_path=path, checkpoint_every=2)
    W_res, h_res = nnms.train(g, T=T, ckpt_every=2, frames=6 * 512, batch=512, lr=0.02, init=init, log_every=1,
                              checkpoint_path=path, checkpoint_every=2)
    assert torch.equal(W_full, W_res)
    assert h_full == h_res


def test_default_keeps_every_iteration_and_trains_identically():
    # with room on the device the default keeps every iteration's messages
    # (no recomputation); the trained weights are those of checkpointing
    # every 2 iterations, bit for bit
    a = synth.draw_qc_shifts(3, 6, 64, 1)
    g = ldpc.Graph.qc(a, 64)
    T = 5
    assert nnms.choose_ckpt_every(g, 512, T, DEV) == T
    init = nnms.initial_weights(T, NB36, 0.8, 0.1, device=DEV)
    print("[gpu] nnms.train default checkpoint interval", flush=True)
    W_all, h_all = nnms.train(g, T=T, frames=3 * 512, batch=512, lr=0.02, init=init, log_every=1)
    W_ck, h_ck = nnms.train(g, T=T, ckpt_every=2, frames=3 * 512, batch=512, lr=0.02, init=init, log_every=1)
    assert torch.equal(W_all, W_ck)
    assert h_all == h_ck
