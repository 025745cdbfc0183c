"""Pins for the FP64 reference decoder: values the paper prints, exact MAP on
cycle-free graphs, closed forms, invariants and special cases.  None of these
re-derive the reference's own formulas."""
import math

import numpy as np
import pytest

import oracle
import synth
from conftest import read_golden

INF = float("inf")


# ----------------------------------------------------------------------------
# graph construction against the paper's worked examples
# ----------------------------------------------------------------------------

def test_lookup_tables_of_worked_example():
    g = read_golden("paper_example_lut.txt")
    lut_c, lut_v = oracle.edge_lookup_tables(np.array(g["H"]))
    assert lut_c == g["LUT_c"]
    assert lut_v == g["LUT_v"]


def test_circulants_match_golden():
    gold = read_golden("circulant_p4.txt")
    for key, rows in gold.items():
        assert oracle.circulant(int(key), 4).tolist() == rows
        H = oracle.qc_parity_check(np.array([[int(key)]]), 4)
        assert H.dense().tolist() == rows


def test_qc_matrix_is_block_of_circulants():
    a = np.array([[0, 3, -1], [2, -1, 1]])
    p = 5
    H = oracle.qc_parity_check(a, p).dense()
    for j in range(2):
        for l in range(3):
            assert np.array_equal(H[j * p:(j + 1) * p, l * p:(l + 1) * p], oracle.circulant(a[j, l], p))


def test_table2_counts():
    # E = J*L*p edges; c = (L/Lambda) p bits per code frame; c-b = (J/Lambda) p
    for code, J, L, p, c, cb, edges in read_golden("table2_codes.txt")[None]:
        a = synth.draw_qc_shifts(J, L, p, 11)
        H = oracle.qc_parity_check(a, p)
        assert H.ne == edges and H.n == L * p and H.m == J * p
        Hc, info = oracle.unwrap_qc(a, p, positions=16)
        assert info["c"] == c and info["cb"] == cb
        # one period (Lambda positions) of the unwrapped code carries all E edges
        lam = info["Lambda"]
        rows = np.repeat(np.arange(Hc.m), np.diff(Hc.row_ptr))
        lay = Hc.layer_of_row[rows]
        steady = (lay >= 2 * lam) & (lay < 3 * lam)
        assert int(steady.sum()) == edges


def _label_table(J, L, p):
    """Unwrap a Lambda x Lambda base whose sub-blocks are single circulants
    with distinct shifts, then read back which sub-block of H_QC each block of
    the convolutional matrix came from."""
    lam = math.gcd(J, L)
    base = np.arange(J * L).reshape(J, L)          # distinct shifts, label = shift
    Hc, info = oracle.unwrap_qc(base, p, positions=4 * lam)
    D = Hc.dense()
    c, cb = info["c"], info["cb"]
    lut_c, lut_v = [], []
    for cls in range(lam):
        tau = 2 * lam + cls                          # a steady-state check layer
        labels = []
        for t in range(tau - info["ms"], tau + 1):   # oldest frame first
            blk = D[tau * cb:(tau + 1) * cb, t * c:(t + 1) * c]
            hit = [s for s in range(J * L) if np.array_equal(blk, oracle.circulant(s, p))]
            assert len(hit) == 1
            labels.append(hit[0])
        lut_c.append(labels)
    for cls in range(lam):
        t = 2 * lam + cls
        labels = []
        for tau in range(t, t + info["ms"] + 1):     # earliest layer first
            blk = D[tau * cb:(tau + 1) * cb, t * c:(t + 1) * c]
            hit = [s for s in range(J * L) if np.array_equal(blk, oracle.circulant(s, p))]
            assert len(hit) == 1
            labels.append(hit[0])
        lut_v.append(labels)
    return lut_c, lut_v


def test_ldpccc_unwrapping_reproduces_printed_tables():
    gold = read_golden("ldpccc_example_lut.txt")
    lut_c, lut_v = _label_table(4, 4, 17)
    assert lut_c == gold["LUT_c"]
    assert lut_v == gold["LUT_v"]


def test_ldpccc_degrees_and_memory():
    # regular (m_s, J, K) code: J ones per column; K ones per row after the start;
    # no check spans more than m_s + 1 code positions (Sec. II-E)
    a = synth.draw_qc_shifts(3, 6, 16, 2)
    Hc, info = oracle.unwrap_qc(a, 16, positions=12)
    assert np.all(np.bincount(Hc.col_idx, minlength=Hc.n) == 3)
    deg = np.diff(Hc.row_ptr)
    lay = Hc.layer_of_row
    ms = info["ms"]
    assert np.all(deg[(lay >= ms) & (lay < 12)] == 6)
    assert np.all(deg[lay == 0] == 2) and np.all(deg[lay == 1] == 4)
    assert np.all(deg[lay == 12] == 4) and np.all(deg[lay == 13] == 2)
    for r in range(Hc.m):
        pos = Hc.pos_of_col[Hc.col_idx[Hc.row_ptr[r]:Hc.row_ptr[r + 1]]]
        assert pos.max() - pos.min() <= ms
        assert lay[r] - ms <= pos.min() and pos.max() <= lay[r]
    # every terminated check has even degree, so the all-ones word is a codeword
    assert np.all(deg % 2 == 0)


# ----------------------------------------------------------------------------
# decoder pins
# ----------------------------------------------------------------------------

def _random_tree_code(rng, n_target):
    """Random cycle-free Tanner graph: grow a tree by hanging a new check with
    1-3 fresh variables on an existing variable."""
    n = 1
    rows = []
    while n < n_target:
        v = int(rng.integers(0, n))
        k = int(min(rng.integers(1, 4), n_target - n))
        rows.append([v] + list(range(n, n + k)))
        n += k
    H = np.zeros((len(rows), n), dtype=np.uint8)
    for r, cols in enumerate(rows):
        H[r, cols] = 1
    return H


@pytest.mark.parametrize("seed", range(8))
def test_tree_codes_reach_exact_map(seed):
    rng = np.random.default_rng(seed)
    H = _random_tree_code(rng, int(rng.integers(6, 15)))
    llr = rng.normal(1.0, 1.5, size=(3, H.shape[1])).astype(np.float32)
    ref = oracle.map_decode(H, llr)
    out = oracle.decode_block(oracle.SparseH.from_dense(H), llr, max_iters=2 * H.shape[1],
                              lmax=INF)
    np.testing.assert_allclose(out["post"], ref, rtol=1e-9, atol=1e-9)
    assert np.array_equal(out["bits"], (ref < 0).astype(np.uint8))


def test_single_parity_check_one_iteration_is_map():
    rng = np.random.default_rng(3)
    for d in (2, 3, 6, 9):
        H = np.ones((1, d), dtype=np.uint8)
        llr = rng.normal(0.5, 2.0, size=(4, d)).astype(np.float32)
        out = oracle.decode_block(oracle.SparseH.from_dense(H), llr, max_iters=1, lmax=INF)
        np.testing.assert_allclose(out["post"], oracle.map_decode(H, llr), rtol=1e-10, atol=1e-10)


def test_qc_forest_protographs_are_exact():
    # a single block row (p disjoint parity checks) and a path protograph lift to forests
    rng = np.random.default_rng(5)
    for base, p in ((np.array([[0, 2, 1]]), 5), (np.array([[0, 0, -1], [-1, 0, 0]]), 5)):
        H = oracle.qc_parity_check(base, p)
        llr = rng.normal(0.8, 2.0, size=(2, H.n)).astype(np.float32)
        out = oracle.decode_block(H, llr, max_iters=4, lmax=INF)
        np.testing.assert_allclose(out["post"], oracle.map_decode(H.dense(), llr), rtol=1e-9, atol=1e-9)


def test_repetition_chain_sums_all_llrs():
    # checks x_k + x_{k+1} = 0: the only codewords are 0...0 and 1...1, so the
    # MAP LLR of every bit is the sum of all channel LLRs
    n = 9
    H = np.zeros((n - 1, n), dtype=np.uint8)
    for k in range(n - 1):
        H[k, k] = H[k, k + 1] = 1
    rng = np.random.default_rng(1)
    llr = rng.normal(0.3, 1.0, size=(5, n)).astype(np.float32)
    out = oracle.decode_block(oracle.SparseH.from_dense(H), llr, max_iters=n, lmax=INF)
    want = np.repeat(llr.astype(np.float64).sum(1, keepdims=True), n, axis=1)
    np.testing.assert_allclose(out["post"], want, rtol=1e-9, atol=1e-9)


def test_check_output_bounded_by_weakest_other_input():
    # J = 1: every variable has degree one, so after one iteration L_n - mu_n is
    # the single check-to-variable message, bounded by min |beta| of the others
    a = np.array([[0, 1, 2, 3, 4, 5]])
    p = 7
    H = oracle.qc_parity_check(a, p)
    rng = np.random.default_rng(2)
    llr = rng.normal(0.0, 8.0, size=(6, H.n)).astype(np.float32)
    out = oracle.decode_block(H, llr, max_iters=1)
    alpha = out["post"] - llr.astype(np.float64)
    mu = np.clip(llr.astype(np.float64), -30, 30)
    for r in range(H.m):
        cols = H.col_idx[H.row_ptr[r]:H.row_ptr[r + 1]]
        for k, v in enumerate(cols):
            others = np.delete(cols, k)
            bound = np.abs(mu[:, others]).min(axis=1)
            assert np.all(np.abs(alpha[:, v]) <= bound + 1e-12)
            assert np.all(np.sign(alpha[:, v]) == np.prod(np.sign(mu[:, others]), axis=1))


def test_codeword_symmetry_is_exact():
    p = 64
    a = synth.draw_qc_shifts(3, 6, p, 1)
    H = oracle.qc_parity_check(a, p)
    cw = synth.QCEncoder(a, p).random_codewords(16, seed=4)
    sigma2 = synth.ebn0_to_sigma2(2.0, 0.5)
    llr0 = synth.bpsk_awgn_llr(None, sigma2, 101, gamma=16, n=H.n)
    s = (1 - 2 * cw.astype(np.int64)).astype(np.float32)
    a0 = oracle.decode_block(H, llr0, 20, early_stop=True)
    a1 = oracle.decode_block(H, llr0 * s, 20, early_stop=True)
    assert np.array_equal(a1["post"], a0["post"] * s)
    assert np.array_equal(a1["bits"], a0["bits"] ^ cw)
    assert np.array_equal(a1["iters"], a0["iters"])
    assert np.array_equal(a1["converged"], a0["converged"])


def test_early_stop_rule():
    p = 64
    a = synth.draw_qc_shifts(3, 6, p, 1)
    H = oracle.qc_parity_check(a, p)
    llr = synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(1.5, 0.5), 7, gamma=48, n=H.n)
    es = oracle.decode_block(H, llr, 20, early_stop=True)
    full = oracle.decode_block(H, llr, 20, early_stop=False, trace=True)
    syn = H.syndrome(es["bits"])
    for g in range(llr.shape[0]):
        zero = not syn[g].any()
        assert bool(es["converged"][g]) == zero
        tr = full["syn_trace"][g]
        first = int(np.argmax(tr)) + 1 if tr.any() else 20
        assert es["iters"][g] == first
        if es["converged"][g]:
            # the stopped frame equals a fixed-iteration run of that length
            again = oracle.decode_block(H, llr[g:g + 1], int(es["iters"][g]), early_stop=False)
            assert np.array_equal(again["post"][0], es["post"][g])
    assert es["converged"].sum() > 10          # the SNR lets most frames decode
    assert np.all(full["iters"] == 20)
    assert np.array_equal(full["converged"], (~H.syndrome(full["bits"]).any(1)).astype(np.uint8))


def syndrome_outcome_can_change(Hd, c, Z):
    """Brute force: does flipping some nonempty subset of the decisions Z
    change whether H c^T is zero?"""
    zero = not (Hd @ c % 2).any()
    for mask in range(1, 1 << len(Z)):
        cc = c.copy()
        for i, v in enumerate(Z):
            if (mask >> i) & 1:
                cc[v] ^= 1
        if (not (Hd @ cc % 2).any()) != zero:
            return True
    return False


@pytest.mark.parametrize("near", [1e-3, 0.4, 1.5])
def test_fragile_iteration_follows_its_rule_and_misses_no_change(near):
    # the fragile diagnostic (first iteration at which decisions with
    # |L| < near could change whether the syndrome is zero), recomputed from
    # the per-iteration L trace; and where few decisions are near zero, brute
    # force over every subset of them: whenever a flip changes the outcome,
    # the rule says fragile (it may say fragile more often, never less)
    p = 12
    a = synth.draw_qc_shifts(3, 6, p, 3)
    H = oracle.qc_parity_check(a, p)
    Hd = H.dense().astype(np.int64)
    llr = synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(1.0, 0.5), 31, gamma=48, n=H.n)
    out = oracle.decode_block(H, llr, 12, early_stop=True, L_trace=True, near=near)
    checked = fragile_seen = 0
    for g in range(llr.shape[0]):
        expect = 0
        for it in range(int(out["iters"][g])):
            L = out["L_trace"][g, it]
            c = (L < 0).astype(np.int64)
            Z = np.nonzero(np.abs(L) < near)[0]
            if len(Z) == 0:
                continue
            syn = Hd @ c % 2
            touched = Hd[:, Z].any(1)
            rule = bool(np.all(touched[syn == 1])) if syn.any() else bool(touched.any())
            if len(Z) <= 10:
                checked += 1
                if syndrome_outcome_can_change(Hd, c, Z):
                    assert rule, (g, it)
            if rule and expect == 0:
                expect = it + 1
        assert out["fragile"][g] == expect, g
        fragile_seen += expect > 0
    assert checked > 0
    if near >= 0.4:
        assert fragile_seen > 0
    # the trace ends at the returned iteration, whose L is the posterior
    for g in range(llr.shape[0]):
        it = int(out["iters"][g])
        assert np.array_equal(np.clip(out["L_trace"][g, it - 1], -30, 30), out["post"][g])
        assert np.all(np.isnan(out["L_trace"][g, it:]))


def test_threads_do_not_change_results():
    p = 32
    a = synth.draw_qc_shifts(3, 6, p, 1)
    H = oracle.qc_parity_check(a, p)
    llr = synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(1.0, 0.5), 8, gamma=16, n=H.n)
    a1 = oracle.decode_block(H, llr, 10, nthreads=1)
    a4 = oracle.decode_block(H, llr, 10, nthreads=4)
    for k in a1:
        assert np.array_equal(a1[k], a4[k])


def test_hard_decision_tie_goes_to_zero():
    # Eq. 6: c_n = 0 when the posterior is >= 0, so an exact zero (also -0.0)
    # decides 0.  Variables 2 and 3 take part in no check, so L = mu exactly.
    H = np.array([[1, 1, 0, 0]], dtype=np.uint8)
    llr = np.array([[1.0, 2.0, 0.0, -0.0], [-1.0, 3.0, -0.0, 0.0]], dtype=np.float32)
    out = oracle.decode_block(oracle.SparseH.from_dense(H), llr, max_iters=2)
    assert out["bits"][:, 2:].tolist() == [[0, 0], [0, 0]]
    assert out["post"][:, 2:].tolist() == [[0.0, 0.0], [0.0, 0.0]]


def test_saturation_keeps_messages_finite():
    # all inputs at the clip level: the FP64 product stays below one, so every
    # message and posterior is finite (reading: clip beta and the output at 30)
    H = oracle.qc_parity_check(np.array([[0, 1, 2, 3, 4, 5]] * 3) + np.arange(3)[:, None] * 0, 11)
    llr = np.full((2, H.n), 100.0, dtype=np.float32)
    out = oracle.decode_block(H, llr, 3)
    assert np.all(np.isfinite(out["post"])) and np.all(out["post"] == 30.0)


# ----------------------------------------------------------------------------
# window decoder pins
# ----------------------------------------------------------------------------

def _conv_inputs(p=16, positions=10, ebn0=1.5, gamma=6, seed=3):
    a = synth.draw_qc_shifts(3, 6, p, 2)
    Hc, info = oracle.unwrap_qc(a, p, positions)
    llr = synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(ebn0, 0.5), seed, gamma=gamma, n=Hc.n)
    return a, Hc, info, llr


def test_window_covering_the_chain_is_flooding_bp():
    # a window at least as long as the whole terminated chain: the first target
    # position is decided after K flooding iterations on the whole matrix
    a, Hc, info, llr = _conv_inputs()
    K = 7
    win = oracle.decode_window(Hc, llr, W=info["nlayers"], K=K)
    blk = oracle.decode_block(Hc, llr, K)
    first = Hc.pos_of_col == 0
    np.testing.assert_allclose(win["post"][:, first], blk["post"][:, first], rtol=0, atol=1e-12)


def test_window_on_decoupled_positions_counts_iterations():
    # block-diagonal sub-blocks: every check layer touches only its own code
    # position, so position s is an independent code decoded with warm-started
    # flooding for K iterations in each of the min(s+1, W) windows it was in
    p, positions, W, K = 8, 7, 3, 2
    # Lambda = 2; the off-diagonal sub-blocks are zero and each diagonal one
    # (2 x 3 circulants) has cycles, so iterations matter
    base = np.array([[0, 1, 3, -1, -1, -1], [2, 5, 0, -1, -1, -1],
                     [-1, -1, -1, 3, 0, 4], [-1, -1, -1, 6, 2, 1]])
    Hc, info = oracle.unwrap_qc(base, p, positions)
    rng = np.random.default_rng(0)
    llr = rng.normal(1.0, 1.6, size=(3, Hc.n)).astype(np.float32)
    assert info["Lambda"] == 2
    win = oracle.decode_window(Hc, llr, W=W, K=K)
    c = info["c"]
    for s in range(positions):
        cls = s % 2
        sub = oracle.qc_parity_check(base[2 * cls:2 * cls + 2, 3 * cls:3 * cls + 3], p)
        cols = slice(s * c, (s + 1) * c)
        ref = oracle.decode_block(sub, llr[:, cols], K * min(s + 1, W))
        np.testing.assert_allclose(win["post"][:, cols], ref["post"], rtol=0, atol=1e-12)


def test_window_all_ones_symmetry():
    # every terminated check has even degree, so flipping all channel LLRs
    # flips every decision and negates every posterior exactly
    a, Hc, info, llr = _conv_inputs(ebn0=1.0)
    w0 = oracle.decode_window(Hc, llr, W=4, K=5)
    w1 = oracle.decode_window(Hc, -llr, W=4, K=5)
    assert np.array_equal(w1["post"], -w0["post"])
    assert np.array_equal(w1["bits"], 1 - w0["bits"])


def test_window_single_layer_is_a_forward_recursion():
    # W = 1: only check layer s and position s take part in window s, earlier
    # positions hold the messages they sent when they were decided.  With
    # K = 1 this unrolls into a forward recursion over positions, written
    # here directly from that description on a dense matrix.
    p, positions = 7, 6
    a = synth.draw_qc_shifts(3, 6, p, 2)
    Hc, info = oracle.unwrap_qc(a, p, positions)
    rng = np.random.default_rng(1)
    llr = rng.normal(1.0, 2.0, size=(2, Hc.n)).astype(np.float32)
    win = oracle.decode_window(Hc, llr, W=1, K=1)
    D = Hc.dense()
    lay, pos = Hc.layer_of_row, Hc.pos_of_col
    for g in range(llr.shape[0]):
        mu = llr[g].astype(np.float64)
        sent = {}   # (row, col) -> message variable col sends to check row
        post = np.zeros(Hc.n)
        for s in range(positions):
            rows = np.nonzero(lay == s)[0]
            msg_in = {}
            for r in rows:
                cols = np.nonzero(D[r])[0]
                vals = [sent[(r, v)] if pos[v] < s else np.clip(mu[v], -30, 30) for v in cols]
                for k, v in enumerate(cols):
                    if pos[v] == s:
                        prod = np.prod([math.tanh(x / 2) for i, x in enumerate(vals) if i != k])
                        msg_in[(r, v)] = 2 * math.atanh(prod)
            for v in np.nonzero(pos == s)[0]:
                inc = [msg_in[(r, v)] for r in rows if D[r, v]]
                post[v] = mu[v] + sum(inc)
                for r in np.nonzero(D[:, v])[0]:
                    if lay[r] > s:
                        sent[(r, v)] = np.clip(mu[v] + sum(inc), -30, 30)
        np.testing.assert_allclose(win["post"][g], np.clip(post, -30, 30), rtol=1e-12, atol=1e-12)


# ----------------------------------------------------------------------------
# pipelined decoder (Algorithm 2) pins
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("I,positions,terminate", [(1, 9, True), (2, 9, True), (5, 12, True), (20, 12, True),
                                                   (3, 10, False)])
def test_pipeline_equals_flooding_on_the_chain(I, positions, terminate):
    # each layer and each frame is updated I times, every check update seeing
    # the previous round's variable messages: I flooding iterations on the
    # terminated chain, bit for bit (same arithmetic, same summation order)
    a = synth.draw_qc_shifts(3, 6, 16, 2)
    Hc, info = oracle.unwrap_qc(a, 16, positions, terminate=terminate)
    llr = synth.bpsk_awgn_llr(None, synth.ebn0_to_sigma2(1.0, 0.5), 11, gamma=4, n=Hc.n)
    pipe = oracle.decode_pipeline(Hc, llr, I, info["ms"])
    flood = oracle.decode_block(Hc, llr, I)
    assert np.array_equal(pipe["post"], flood["post"])
    assert np.array_equal(pipe["bits"], flood["bits"])


def test_pipeline_on_decoupled_positions_is_block_bp():
    # block-diagonal sub-blocks: every frame is its own code, decoded with I iterations
    p, positions, I = 8, 7, 4
    base = np.array([[0, 1, 3, -1, -1, -1], [2, 5, 0, -1, -1, -1],
                     [-1, -1, -1, 3, 0, 4], [-1, -1, -1, 6, 2, 1]])
    Hc, info = oracle.unwrap_qc(base, p, positions)
    rng = np.random.default_rng(4)
    llr = rng.normal(1.0, 1.6, size=(3, Hc.n)).astype(np.float32)
    pipe = oracle.decode_pipeline(Hc, llr, I, info["ms"])
    c = info["c"]
    for s in range(positions):
        cls = s % 2
        sub = oracle.qc_parity_check(base[2 * cls:2 * cls + 2, 3 * cls:3 * cls + 3], p)
        ref = oracle.decode_block(sub, llr[:, s * c:(s + 1) * c], I)
        np.testing.assert_allclose(pipe["post"][:, s * c:(s + 1) * c], ref["post"], rtol=0, atol=1e-12)


def test_pipeline_all_ones_symmetry():
    a, Hc, info, llr = _conv_inputs(ebn0=1.0)
    p0 = oracle.decode_pipeline(Hc, llr, 6, info["ms"])
    p1 = oracle.decode_pipeline(Hc, -llr, 6, info["ms"])
    assert np.array_equal(p1["post"], -p0["post"])
    assert np.array_equal(p1["bits"], 1 - p0["bits"])
