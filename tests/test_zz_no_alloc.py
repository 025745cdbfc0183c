"""ldpc_decode_noalloc (the entry point whose workspace is the library's
static per-device array) through the C ABI, against ldpc_decode on the same
inputs: the two run the same kernels, so every output must be equal bit for
bit.  Two calls in a row on one device, the second with a smaller batch (the
array keeps the first call's contents), then another code."""
import numpy as np
import pytest
import torch

import synth
from paper_1204_0334_amd import ldpc

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def same_as_decode(g, llr, iters, early):
    gamma, n = llr.shape
    print(f"[gpu] noalloc n={n} gamma={gamma} iters={iters} early={early}", flush=True)
    x = torch.from_numpy(np.ascontiguousarray(llr)).to(DEV)
    ref = ldpc.decode(g, x, iters, early_stop=early)
    # outputs pre-filled with values the decoder never writes
    out = (torch.full((gamma, n), float("nan"), device=DEV),
           torch.full((gamma, n), 7, dtype=torch.uint8, device=DEV),
           torch.full((gamma,), -1, dtype=torch.int32, device=DEV),
           torch.full((gamma,), 9, dtype=torch.uint8, device=DEV))
    got = ldpc.decode_noalloc(g, x, iters, early_stop=early, out=out)
    torch.cuda.synchronize()
    for name, a, b in zip(("post", "bits", "iters", "converged"), ref, got):
        assert torch.equal(a, b), f"{name} differs from ldpc_decode (n={n}, gamma={gamma})"
    return got


@pytest.fixture(params=["packages", "onchip"])
def block_path(request, monkeypatch):
    # both decoders behind ldpc_decode; the package decoder is the one whose
    # kernels use the workspace (the static array), the on-chip one needs none
    if request.param == "packages":
        monkeypatch.setenv("LDPC_BLOCK_PATH", "packages")
    else:
        monkeypatch.delenv("LDPC_BLOCK_PATH", raising=False)
    return request.param


def test_noalloc_two_calls_in_a_row_then_another_code(block_path):
    a = synth.draw_qc_shifts(3, 6, 3060, 2)
    g = ldpc.Graph.qc(a, 3060)
    assert ldpc.decode_path(g) == block_path
    assert g.workspace_size(100, 20) <= ldpc.NOALLOC_SCRATCH_BYTES
    s2 = synth.ebn0_to_sigma2(1.5, 0.5)
    first = same_as_decode(g, synth.bpsk_awgn_llr(None, s2, 301, gamma=100, n=g.n), 20, True)
    assert (first[2] >= 1).all() and (first[2] <= 20).all()
    # smaller batch: frames 0..36 must not be taken from the first call's state
    second = same_as_decode(g, synth.bpsk_awgn_llr(None, s2, 302, gamma=37, n=g.n), 20, True)
    assert second[0].shape == (37, g.n)
    # fixed iterations, then a small code with another tiling
    same_as_decode(g, synth.bpsk_awgn_llr(None, s2, 303, gamma=20, n=g.n), 5, False)
    b = synth.draw_qc_shifts(3, 6, 64, 1)
    small = ldpc.Graph.qc(b, 64)
    same_as_decode(small, synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(2.0, 0.5), 101, gamma=300, n=384), 20, True)


def test_noalloc_rejects_a_batch_beyond_its_array():
    g = ldpc.Graph.qc(synth.draw_qc_shifts(3, 6, 3060, 2), 3060)
    x = torch.zeros((1024, g.n), dtype=torch.float32, device=DEV)
    with pytest.raises(ldpc.LdpcError) as e:
        ldpc.decode_noalloc(g, x, 20)
    assert e.value.status == ldpc.EWORKSPACE
