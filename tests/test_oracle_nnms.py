"""Pins for the FP64 reference of the learned min-sum decoder and its
gradient: max-log MAP by enumeration on cycle-free graphs and on single
checks (with a scale and offset per edge), special cases that switch parts of
the rule off, per-edge-class and per-iteration indexing (a base row switched
off, base columns permuted), exact codeword symmetry, and finite differences
of the loss."""
import itertools

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import nnms
from test_oracle import _random_tree_code


def _max_log_map(H, llr):
    """For each bit: max over codewords with the bit 0 minus max over
    codewords with the bit 1 of sum_k (1 - 2 c_k) mu_k / 2, by enumerating
    all 2^n words."""
    H = np.asarray(H)
    n = H.shape[1]
    words = np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.int64)
    cw = words[np.all((words @ H.T) % 2 == 0, axis=1)]
    y = np.atleast_2d(np.asarray(llr, dtype=np.float64))
    metric = y @ (1.0 - 2.0 * cw).T / 2.0                     # [F, codewords]
    out = np.empty_like(y)
    for v in range(n):
        out[:, v] = metric[:, cw[:, v] == 0].max(1) - metric[:, cw[:, v] == 1].max(1)
    return out


def _weights(T, J, w, b):
    return np.full((T, J), w, dtype=np.float64), np.full((T, J), b, dtype=np.float64)


@pytest.mark.parametrize("seed", range(6))
def test_min_sum_on_trees_is_max_log_map(seed):
    rng = np.random.default_rng(seed)
    H = _random_tree_code(rng, int(rng.integers(6, 13)))
    G = nnms.EdgeGraph(oracle.SparseH.from_dense(H))
    llr = rng.normal(1.0, 1.5, size=(3, H.shape[1]))
    T = 2 * H.shape[1]
    w, b = _weights(T, 1, 1.0, 0.0)
    out = nnms.decode(G, llr, w, b, T, lmax=np.inf)
    np.testing.assert_allclose(out["raw"], _max_log_map(H, llr), rtol=1e-12, atol=1e-12)


def test_single_check_scale_and_offset_per_edge():
    # every edge of one check in its own class: edge k takes its own (w, b)
    rng = np.random.default_rng(17)
    for d in (2, 3, 6):
        H = np.ones((1, d), dtype=np.uint8)
        G = nnms.EdgeGraph(oracle.SparseH.from_dense(H), np.arange(d))
        llr = rng.normal(0.3, 2.0, size=(4, d))
        ext = _max_log_map(H, llr) - llr
        w, b = rng.uniform(0.3, 1.0, size=d), rng.uniform(0.0, 1.0, size=d)
        got = nnms.decode(G, llr, w[None], b[None], 1, lmax=np.inf)["raw"] - llr
        want = w * np.sign(ext) * np.maximum(np.abs(ext) - b, 0.0)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_single_check_scale_and_offset():
    # on one parity check the max-log MAP extrinsic of bit k is the minimum
    # of the others with their sign product; scale and offset act on it
    rng = np.random.default_rng(7)
    for d in (2, 3, 5, 8):
        H = np.ones((1, d), dtype=np.uint8)
        G = nnms.EdgeGraph(oracle.SparseH.from_dense(H))
        llr = rng.normal(0.3, 2.0, size=(5, d))
        ext = _max_log_map(H, llr) - llr
        for w, b in ((1.0, 0.0), (0.7, 0.0), (1.0, 0.4), (0.55, 0.9)):
            W, B = _weights(1, 1, w, b)
            got = nnms.decode(G, llr, W, B, 1, lmax=np.inf)["raw"] - llr
            want = w * np.sign(ext) * np.maximum(np.abs(ext) - b, 0.0)
            np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


NB = 18   # edge classes of the 3 x 6 base: its circulant blocks


def _qc_graph(J=3, L=6, p=7, seed=1):
    a = synth.draw_qc_shifts(J, L, p, seed)
    H = oracle.qc_parity_check(a, p)
    return a, H, nnms.EdgeGraph(H, nnms.qc_edge_class(a, p))


def test_qc_edge_classes_are_the_circulant_blocks():
    # edge of row j*p + s in column l*p + t belongs to block (j, l), numbered
    # row by row over the nonzero blocks
    a = np.array([[3, -1, 0, 5], [-1, 2, 6, -1], [1, 4, -1, 0]])
    p = 7
    H = oracle.qc_parity_check(a, p)
    cls = nnms.qc_edge_class(a, p)
    number = {(j, l): k for k, (j, l) in enumerate((j, l) for j in range(3) for l in range(4) if a[j, l] >= 0)}
    rows = np.repeat(np.arange(H.m), np.diff(H.row_ptr))
    for e in range(H.ne):
        j, l = rows[e] // p, H.col_idx[e] // p
        assert cls[e] == number[(j, l)]
        assert H.col_idx[e] % p == (rows[e] % p + a[j, l]) % p


def test_zero_scale_or_large_offset_leaves_channel_llrs():
    _, H, G = _qc_graph()
    rng = np.random.default_rng(1)
    llr = rng.normal(1.0, 2.0, size=(4, H.n))
    x = np.ones_like(llr)
    for w, b in ((0.0, 0.0), (1.0, 31.0)):
        W, B = _weights(3, NB, w, b)
        for L in nnms.run(G, llr, torch.tensor(W), torch.tensor(B), 3):
            assert np.array_equal(L.numpy(), llr)
        per = nnms.iteration_losses(G, llr, x, torch.tensor(W), torch.tensor(B), 3).numpy()
        np.testing.assert_allclose(per, np.log1p(np.exp(-llr)).mean(), rtol=1e-14)


def test_edge_classes_select_their_weights():
    # the six classes of base row 0 switched off (w = 0) must equal decoding
    # the code without base row 0, whose classes are the remaining twelve
    a, H, G = _qc_graph()
    p = 7
    rng = np.random.default_rng(2)
    llr = rng.normal(0.8, 2.0, size=(3, H.n))
    T = 4
    W = rng.uniform(0.6, 1.0, size=(T, NB))
    B = rng.uniform(0.0, 0.4, size=(T, NB))
    W[:, :6] = 0.0
    got = nnms.decode(G, llr, W, B, T)["raw"]
    a2 = a[1:]
    H2 = oracle.qc_parity_check(a2, p)
    G2 = nnms.EdgeGraph(H2, nnms.qc_edge_class(a2, p))
    want = nnms.decode(G2, llr, W[:, 6:], B[:, 6:], T)["raw"]
    np.testing.assert_allclose(got, want, rtol=0, atol=0)


def test_permuted_base_columns_carry_their_classes():
    # permuting the base columns (and the bits, and the classes with their
    # blocks) permutes the decoder's output; an edge that took the weights
    # of another edge of its row (by position in the row) would break this
    a, H, G = _qc_graph()
    p = 7
    perm = np.array([3, 0, 5, 1, 4, 2])
    a2 = a[:, perm]
    H2 = oracle.qc_parity_check(a2, p)
    G2 = nnms.EdgeGraph(H2, nnms.qc_edge_class(a2, p))
    rng = np.random.default_rng(9)
    llr = rng.normal(0.8, 2.0, size=(3, H.n))
    T = 3
    W = rng.uniform(0.5, 1.0, size=(T, NB))
    B = rng.uniform(0.0, 0.6, size=(T, NB))
    # block (j, l) of a is block (j, position of l in perm) of a2
    inv = np.argsort(perm)
    cls2 = np.array([j * 6 + inv[l] for j in range(3) for l in range(6)])   # a2 class of a's block (j, l)
    W2, B2 = np.empty_like(W), np.empty_like(B)
    W2[:, cls2] = W
    B2[:, cls2] = B
    bitperm = (perm[:, None] * p + np.arange(p)[None, :]).reshape(-1)        # a2 column c <- a column bitperm[c]
    out = nnms.decode(G, llr, W, B, T)["raw"]
    out2 = nnms.decode(G2, llr[:, bitperm], W2, B2, T)["raw"]
    np.testing.assert_allclose(out2, out[:, bitperm], rtol=0, atol=0)


def test_iteration_selects_its_weights():
    # a first iteration with w = 0 sends nothing, so iteration 2 equals
    # iteration 1 of a run that starts with iteration 2's weights
    _, H, G = _qc_graph()
    rng = np.random.default_rng(3)
    llr = rng.normal(0.8, 2.0, size=(3, H.n))
    W = np.vstack([np.zeros(NB), rng.uniform(0.6, 0.9, size=(2, NB))])
    B = np.vstack([np.full(NB, 0.5), rng.uniform(0.0, 0.3, size=(2, NB))])
    full = nnms.run(G, llr, torch.tensor(W), torch.tensor(B), 3)
    short = nnms.run(G, llr, torch.tensor(W[1:]), torch.tensor(B[1:]), 2)
    assert np.array_equal(full[1].numpy(), short[0].numpy())
    assert np.array_equal(full[2].numpy(), short[1].numpy())


def test_codeword_symmetry_is_exact():
    a, H, G = _qc_graph(p=16)
    cw = synth.QCEncoder(a, 16).random_codewords(4, seed=5).astype(np.int64)
    rng = np.random.default_rng(4)
    llr = rng.normal(1.0, 1.5, size=(4, H.n))
    s = 1.0 - 2.0 * cw
    W, B = rng.uniform(0.5, 1.0, size=(5, NB)), rng.uniform(0.0, 0.6, size=(5, NB))
    a0 = nnms.decode(G, llr, W, B, 5)
    a1 = nnms.decode(G, llr * s, W, B, 5)
    assert np.array_equal(a1["raw"], a0["raw"] * s)
    # the loss against the transmitted word is the same for both
    l0 = nnms.iteration_losses(G, llr, np.ones_like(llr), torch.tensor(W), torch.tensor(B), 5)
    l1 = nnms.iteration_losses(G, llr * s, s, torch.tensor(W), torch.tensor(B), 5)
    np.testing.assert_allclose(l1.numpy(), l0.numpy(), rtol=1e-14)


def test_messages_stay_clipped():
    _, H, G = _qc_graph()
    rng = np.random.default_rng(5)
    llr = rng.normal(20.0, 30.0, size=(3, H.n))
    W, B = _weights(6, NB, 1.0, 0.0)
    mu = torch.tensor(llr)
    beta = torch.clamp(mu[:, G.col], -30, 30)
    for t in range(6):
        alpha = nnms.check_step(G, beta, torch.tensor(W[t]), torch.tensor(B[t]))
        assert float(alpha.abs().max()) <= 30.0
        beta, _ = nnms.variable_step(G, mu, alpha, 30.0)
        assert float(beta.abs().max()) <= 30.0


def test_gradient_matches_finite_differences():
    _, H, G = _qc_graph()
    rng = np.random.default_rng(6)
    sigma2 = synth.ebn0_to_sigma2(1.5, 0.5)
    llr = 2.0 / sigma2 * (1.0 + np.sqrt(sigma2) * rng.normal(size=(6, H.n)))
    x = np.ones_like(llr)
    T = 4
    W, B = rng.uniform(0.5, 1.0, size=(T, NB)), rng.uniform(0.0, 0.5, size=(T, NB))
    coef = rng.uniform(0.2, 1.0, size=T)
    _, gw, gb = nnms.grad(G, llr, x, W, B, T, coef=coef)
    h = 1e-6

    def f(Wp, Bp):
        return float(nnms.loss(G, llr, x, torch.tensor(Wp), torch.tensor(Bp), T, coef=coef))

    for t in range(T):
        for j in range(NB):
            E = np.zeros_like(W)
            E[t, j] = h
            fw = (f(W + E, B) - f(W - E, B)) / (2 * h)
            fb = (f(W, B + E) - f(W, B - E)) / (2 * h)
            assert abs(fw - gw[t, j]) <= 1e-6 * max(1.0, abs(fw))
            assert abs(fb - gb[t, j]) <= 1e-6 * max(1.0, abs(fb))


def test_gradient_is_causal_and_vanishes_when_switched_off():
    _, H, G = _qc_graph()
    rng = np.random.default_rng(8)
    llr = rng.normal(1.0, 2.0, size=(4, H.n))
    x = np.ones_like(llr)
    T = 4
    W, B = rng.uniform(0.5, 1.0, size=(T, NB)), rng.uniform(0.0, 0.5, size=(T, NB))
    # the loss of iteration 2 does not depend on the weights of iterations 3, 4
    _, gw, gb = nnms.grad(G, llr, x, W, B, T, coef=[0.0, 1.0, 0.0, 0.0])
    assert np.all(gw[2:] == 0) and np.all(gb[2:] == 0)
    assert np.all(np.abs(gw[:2]) > 0)
    # an offset above every magnitude turns the check rule off: no gradient
    B2 = np.full((T, NB), 40.0)
    _, gw, gb = nnms.grad(G, llr, x, W, B2, T)
    assert np.all(gw == 0) and np.all(gb == 0)
