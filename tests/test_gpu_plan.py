"""GPU tests of the multi-code plan (through the C ABI): every code of a
plan decodes exactly as ldpc_decode decodes it alone (same arithmetic and
edge order, so bit for bit: posteriors, decisions, iteration counts,
convergence flags), in every lane layout but the split ones, eagerly and by
graph replay; codes of a plan against the FP64 reference with the tolerances
of test_gpu_decode, the split layouts (each check row's edges over several
lanes, FP32 rounding of another order) among them."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1204_0334_amd import ldpc

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def package_decoder(monkeypatch):
    # the plan runs the message-package kernels; ldpc_decode is compared with
    # it bit for bit, so it must run them too (LDPC_BLOCK_PATH, read per call)
    monkeypatch.setenv("LDPC_BLOCK_PATH", "packages")


DEV = "cuda:0"

RAGGED = [dict(J=3, L=6, p=27, gamma=1, ebn0_db=2.5), dict(J=3, L=6, p=27, gamma=7, ebn0_db=2.5),
          dict(J=3, L=9, p=72, gamma=9, ebn0_db=3.0), dict(J=3, L=18, p=36, gamma=33, ebn0_db=3.5),
          dict(J=3, L=6, p=81, gamma=65, ebn0_db=2.0), dict(J=3, L=6, p=64, gamma=300, ebn0_db=2.0),
          dict(J=3, L=9, p=40, gamma=200, ebn0_db=3.0)]


def make_case(specs, seed):
    graphs, llrs = [], []
    for i, c in enumerate(specs):
        g = ldpc.Graph.qc(synth.draw_qc_shifts(c["J"], c["L"], c["p"], 50 + i), c["p"])
        s2 = synth.ebn0_to_sigma2(c["ebn0_db"], 1.0 - c["J"] / c["L"])
        graphs.append(g)
        llrs.append(ldpc.awgn_llr(g.n, c["gamma"], s2, seed + i, 0, device=DEV))
    return graphs, llrs


def single_code(graphs, llrs, iters, early):
    return [ldpc.decode(g, x, iters, early_stop=early) for g, x in zip(graphs, llrs)]


def assert_same(outs, refs, what):
    torch.cuda.synchronize()
    for c, (o, r) in enumerate(zip(outs, refs)):
        for name, a, b in zip(("post", "bits", "iters", "converged"), o, r):
            assert torch.equal(a, b), f"{what}: code {c} {name} differs"


def assert_close_to_single_code(out, ref, what):
    """A code decoded in a split layout against ldpc_decode: the same
    iteration count on nearly every frame; where both converged after the same
    number of iterations, the same decisions and posteriors within 2e-4
    relative (floor 1): the two form the products of Eq. 3 in different
    orders, so they agree to FP32 rounding, not bit for bit."""
    post, bits, it, conv = (t.cpu().numpy() for t in out)
    rpost, rbits, rit, rconv = (t.cpu().numpy() for t in ref)
    same = it == rit
    assert same.mean() > 0.95, f"{what}: iteration counts"
    sel = same & (conv == 1) & (rconv == 1)
    assert sel.any(), f"{what}: no frame converged on both sides"
    assert np.array_equal(bits[sel], rbits[sel]), f"{what}: decisions"
    err = np.abs(post[sel].astype(np.float64) - rpost[sel]) / np.maximum(np.abs(rpost[sel]), 1.0)
    assert err.max() <= 2e-4, f"{what}: posterior difference {err.max():.3e}"


@pytest.mark.parametrize("early", [True, False])
def test_mixed_plan_matches_single_code_decoder(early):
    specs = synth.MIXED_CODES
    print(f"[gpu] mixed plan early={early}", flush=True)
    graphs, llrs = make_case(specs, 1000)
    plan = ldpc.Plan(graphs, [c["gamma"] for c in specs], 20, early_stop=early)
    outs = plan.decode(llrs)
    assert_same(outs, single_code(graphs, llrs, 20, early), "mixed")
    if early:
        assert sum(int(o[3].sum()) for o in outs) > 0


def test_every_layout_matches_single_code_decoder():
    graphs, llrs = make_case(RAGGED, 2000)
    gammas = [c["gamma"] for c in RAGGED]
    refs = single_code(graphs, llrs, 12, True)
    ws = None
    for layout in list(range(ldpc.PLAN_LAYOUTS)) + [ldpc.LAYOUT_G8 | ldpc.LAYOUT_VN2, ldpc.LAYOUT_G32 | ldpc.LAYOUT_VN4,
                                     ldpc.LAYOUT_G64 | ldpc.LAYOUT_VN2, ldpc.LAYOUT_G64 | ldpc.LAYOUT_VN4,
                                     ldpc.LAYOUT_G8 | ldpc.LAYOUT_CN2, ldpc.LAYOUT_G16 | ldpc.LAYOUT_CN4,
                                     ldpc.LAYOUT_G64 | ldpc.LAYOUT_CN4 | ldpc.LAYOUT_VN4]:
        plan = ldpc.Plan(graphs, gammas, 12, early_stop=True)
        for c in range(len(graphs)):
            try:
                plan.set_layout(c, layout)
            except ldpc.LdpcError:
                pass                       # 2 or 4 frames per lane where rows are too heavy
        print(f"[gpu] ragged plan layout={ldpc.layout_name(layout)}", flush=True)
        ws = plan.workspace(DEV) if ws is None else ws
        assert_same(plan.decode(llrs, ws=ws), refs, f"layout {ldpc.layout_name(layout)}")


def test_fixed_iterations_every_layout():
    graphs, llrs = make_case(RAGGED[:5], 3000)
    gammas = [c["gamma"] for c in RAGGED[:5]]
    refs = single_code(graphs, llrs, 3, False)
    for layout in (0, 2, 3, ldpc.LAYOUT_G64 | ldpc.LAYOUT_VN4, ldpc.LAYOUT_G32 | ldpc.LAYOUT_CN2, ldpc.LAYOUT_G8F4,
                   ldpc.LAYOUT_G16F2, ldpc.LAYOUT_G32F4):
        plan = ldpc.Plan(graphs, gammas, 3, early_stop=False)
        for c in range(len(graphs)):
            try:
                plan.set_layout(c, layout)
            except ldpc.LdpcError:
                pass                       # row groups where rows are too heavy
        print(f"[gpu] fixed-iteration plan layout={ldpc.layout_name(layout)}", flush=True)
        assert_same(plan.decode(llrs), refs, f"3 iterations, layout {ldpc.layout_name(layout)}")


def cpu_case(specs, seed):
    """Graphs and channel LLRs drawn on the host (synth), so that nothing the
    FP64 reference reads comes from the HIP library."""
    graphs, shifts, llrs = [], [], []
    for i, c in enumerate(specs):
        a = synth.draw_qc_shifts(c["J"], c["L"], c["p"], 50 + i)
        s2 = synth.ebn0_to_sigma2(c["ebn0_db"], 1.0 - c["J"] / c["L"])
        shifts.append(a)
        graphs.append(ldpc.Graph.qc(a, c["p"]))
        llrs.append(synth.bpsk_awgn_llr(None, s2, seed + i, gamma=c["gamma"], n=c["L"] * c["p"]))
    return graphs, shifts, llrs


def reference_parity(out, H, llr, iters, early, gate_all, what):
    """One code's plan outputs (sampled frames) against the FP64 reference,
    with the gates of test_gpu_decode.check_parity: iteration counts and flags
    exact where no decision with |L| < 1e-3 could change the syndrome test;
    decisions exact on frames converged on both sides and on frames without
    such decisions; posteriors within 1e-4 relative (floor 1) on every frame
    (gate_all) or on frames that converged on both sides.  Returns the number
    of frames whose posteriors were gated."""
    ref = oracle.decode_block(H, llr, iters, early_stop=early)
    post, bits, it, conv = out
    robust = ref["fragile"] == 0
    assert np.array_equal(it[robust], ref["iters"][robust]), f"{what}: iteration counts"
    assert np.array_equal(conv[robust], ref["converged"][robust]), f"{what}: convergence flags"
    both = robust & (conv == 1) & (ref["converged"] == 1)
    bitgate = both | (ref["min_abs"] >= 1e-3)
    assert np.array_equal(bits[bitgate], ref["bits"][bitgate]), f"{what}: decisions"
    gate = np.ones(len(robust), dtype=bool) if gate_all else both
    r = np.clip(ref["post"][gate], -30, 30)
    err = np.abs(np.clip(post[gate].astype(np.float64), -30, 30) - r) / np.maximum(np.abs(r), 1.0)
    assert err.size == 0 or err.max() <= 1e-4, f"{what}: posterior error {err.max():.3e}"
    return int(gate.sum())


def test_plan_code_against_fp64_reference():
    spec = [dict(J=3, L=6, p=27, gamma=20, ebn0_db=2.5), dict(J=3, L=18, p=36, gamma=40, ebn0_db=3.5)]
    graphs, shifts, llr_np = cpu_case(spec, 4000)
    llrs = [torch.from_numpy(x).to(DEV) for x in llr_np]
    plan = ldpc.Plan(graphs, [20, 40], 20, early_stop=True)
    print("[gpu] plan vs reference", flush=True)
    outs = plan.decode(llrs)
    torch.cuda.synchronize()
    for i, c in enumerate(spec):
        H = oracle.qc_parity_check(shifts[i], c["p"])
        o = tuple(t.cpu().numpy() for t in outs[i])
        reference_parity(o, H, llr_np[i], 20, True, False, f"code {i}")
        assert np.array_equal(o[3].astype(bool), ~H.syndrome(o[1]).any(1))


SPLIT_LAYOUTS = [ldpc.LAYOUT_G8 | ldpc.LAYOUT_SPLIT2, ldpc.LAYOUT_G8 | ldpc.LAYOUT_SPLIT4,
                 ldpc.LAYOUT_G8 | ldpc.LAYOUT_SPLIT8, ldpc.LAYOUT_G16 | ldpc.LAYOUT_SPLIT2,
                 ldpc.LAYOUT_G16 | ldpc.LAYOUT_SPLIT4, ldpc.LAYOUT_G32 | ldpc.LAYOUT_SPLIT2,
                 ldpc.LAYOUT_G8 | ldpc.LAYOUT_VN2 | ldpc.LAYOUT_SPLIT4]
# rows of weight 18 and 9 (ragged last tiles in every group size), and a
# 3 x 6 code that keeps its default layout in the same plan
SPLIT_SPEC = [dict(J=3, L=18, p=36, gamma=21, ebn0_db=3.5), dict(J=3, L=9, p=72, gamma=9, ebn0_db=3.0),
              dict(J=3, L=6, p=27, gamma=20, ebn0_db=2.5)]


@pytest.mark.parametrize("layout", SPLIT_LAYOUTS, ids=ldpc.layout_name)
def test_split_layouts_against_fp64_reference(layout):
    # each check row's edges over 2, 4 or 8 lanes: 1-3 iterations with every
    # posterior gated, 20 with early stopping and exact iteration counts
    graphs, shifts, llr_np = cpu_case(SPLIT_SPEC, 4500)
    llrs = [torch.from_numpy(x).to(DEV) for x in llr_np]
    gammas = [c["gamma"] for c in SPLIT_SPEC]
    for iters, early in [(1, False), (2, False), (3, False), (20, True)]:
        plan = ldpc.Plan(graphs, gammas, iters, early_stop=early)
        split = []
        for c in range(2):
            try:
                plan.set_layout(c, layout)
                split.append(c)
            except ldpc.LdpcError:
                pass                       # 8 lanes need rows of weight >= 16
        assert 0 in split
        print(f"[gpu] split layout {ldpc.layout_name(layout)} on codes {split}, I={iters} early={early}", flush=True)
        outs = plan.decode(llrs)
        torch.cuda.synchronize()
        for i, c in enumerate(SPLIT_SPEC):
            H = oracle.qc_parity_check(shifts[i], c["p"])
            o = tuple(t.cpu().numpy() for t in outs[i])
            gated = reference_parity(o, H, llr_np[i], iters, early, not early, f"code {i} I={iters}")
            assert gated > 0
            if early:
                assert np.array_equal(o[3].astype(bool), ~H.syndrome(o[1]).any(1))
        # the code in its default layout: bit for bit what ldpc_decode returns
        ref = ldpc.decode(graphs[2], llrs[2], iters, early_stop=early)
        assert_same([outs[2]], [ref], f"default-layout code beside {ldpc.layout_name(layout)}")


@pytest.mark.parametrize("iters,early", [(3, False), (20, True)])
def test_split_layouts_persistent_launch_matches_phase_launches(iters, early):
    # the persistent kernel carries the split bodies too: same layouts, same
    # device functions, so bit for bit the phase launches' outputs
    graphs, llrs = make_case(SPLIT_SPEC, 4600)
    gammas = [c["gamma"] for c in SPLIT_SPEC]
    layouts = [ldpc.LAYOUT_G8 | ldpc.LAYOUT_SPLIT4, ldpc.LAYOUT_G16 | ldpc.LAYOUT_SPLIT2, None]
    outs = []
    for persistent in (False, True):
        plan = ldpc.Plan(graphs, gammas, iters, early_stop=early)
        if persistent:
            plan.set_persistent(True)
        for c, l in enumerate(layouts):
            if l is not None:
                plan.set_layout(c, l)
        ws = plan.workspace(DEV)
        print(f"[gpu] split layouts persistent={persistent} I={iters} early={early}", flush=True)
        outs.append(plan.decode(llrs, ws=ws))
        torch.cuda.synchronize()
        if persistent:
            plan.check(ws)
    assert_same(outs[1], outs[0], "persistent against phase launches, split layouts")


def test_split_layouts_full_size_heavy_codes_against_reference():
    # the mixed workload's rate-5/6 and rate-2/3 codes at their real sizes
    # (3 x 18 p = 3600 with 8 frames, p = 36 with 128; 3 x 9 p = 2400 with
    # 32, p = 72 with 512) in split layouts; sampled frames against the FP64
    # reference
    specs = [c for c in synth.MIXED_CODES if c["L"] in (9, 18) and c["p"] >= 36]
    graphs, shifts, llr_np = cpu_case(specs, 7500)
    llrs = [torch.from_numpy(x).to(DEV) for x in llr_np]
    for iters, early in [(3, False), (20, True)]:
        plan = ldpc.Plan(graphs, [c["gamma"] for c in specs], iters, early_stop=early)
        for c, spec in enumerate(specs):
            plan.set_layout(c, ldpc.LAYOUT_G8 | (ldpc.LAYOUT_SPLIT4 if spec["L"] == 18 else ldpc.LAYOUT_SPLIT2))
        print(f"[gpu] split layouts at full size I={iters} early={early}: "
              f"{[(c['L'], c['p'], ldpc.layout_name(plan.layout(i))) for i, c in enumerate(specs)]}", flush=True)
        outs = plan.decode(llrs)
        torch.cuda.synchronize()
        gated = 0
        for i, c in enumerate(specs):
            pick = sampled_frames(c["gamma"])
            H = oracle.qc_parity_check(shifts[i], c["p"])
            o = tuple(t.cpu().numpy()[pick] for t in outs[i])
            gated += reference_parity(o, H, llr_np[i][pick], iters, early, not early, f"{c['L']} p={c['p']}")
        assert gated >= 6


def sampled_frames(gamma):
    return np.unique(np.array([0, 1, gamma // 3, gamma // 2, gamma - 2, gamma - 1]).clip(0, gamma - 1))


@pytest.mark.parametrize("iters,early,persistent", [(3, False, False), (20, True, False), (20, True, True)])
def test_mixed_workload_codes_at_full_size_against_reference(iters, early, persistent):
    # the seven codes of the mixed workload at their real circulant sizes
    # (rate 1/2: p = 27, 81, 2700; rate 2/3: p = 72, 2400; rate 5/6: p = 36,
    # 3600) and batch sizes, decoded together by one plan with the layouts
    # the autotuner picks; sampled frames of every code against the FP64
    # reference.  3 iterations without early stopping gate every posterior of
    # the sampled frames; 20 with early stopping gate exact iteration counts.
    specs = synth.MIXED_CODES
    graphs, shifts, llr_np = cpu_case(specs, 7000)
    llrs = [torch.from_numpy(x).to(DEV) for x in llr_np]
    plan = ldpc.Plan(graphs, [c["gamma"] for c in specs], iters, early_stop=early)
    if persistent:
        plan.set_persistent(True)
    ws = plan.workspace(DEV)
    outs = plan.outputs(DEV)
    print(f"[gpu] mixed plan at full size iters={iters} early={early} persistent={persistent}: autotune",
          flush=True)
    plan.autotune(llrs, outs, ws, trials=1)
    print(f"[gpu] layouts {[ldpc.layout_name(plan.layout(c)) for c in range(len(specs))]}", flush=True)
    outs = plan.decode(llrs, outs=outs, ws=ws)
    torch.cuda.synchronize()
    gated = 0
    for i, c in enumerate(specs):
        pick = sampled_frames(c["gamma"])
        H = oracle.qc_parity_check(shifts[i], c["p"])
        o = tuple(t.cpu().numpy()[pick] for t in outs[i])
        gated += reference_parity(o, H, llr_np[i][pick], iters, early, not early,
                                  f"{c['J']}x{c['L']} p={c['p']}")
        if early:
            assert np.array_equal(o[3].astype(bool), ~H.syndrome(o[1]).any(1))
    assert gated >= 30
    if persistent:
        plan.check(ws)


def test_graph_replay_matches_eager_decode():
    graphs, llrs = make_case(synth.MIXED_CODES, 5000)
    gammas = [c["gamma"] for c in synth.MIXED_CODES]
    plan = ldpc.Plan(graphs, gammas, 20, early_stop=True)
    ws = plan.workspace(DEV)
    eager = plan.decode(llrs, ws=ws)
    torch.cuda.synchronize()
    eager = [tuple(t.clone() for t in o) for o in eager]
    outs = plan.outputs(DEV)
    print("[gpu] plan capture", flush=True)
    plan.capture(llrs, outs, ws)
    scratch = torch.zeros(1 << 20, device=DEV)
    for rep in range(3):
        for o in outs:
            for t in o:
                t.zero_()
        scratch.add_(1.0)                  # eager work between replays
        torch.cuda.synchronize()
        print(f"[gpu] plan replay {rep}", flush=True)
        plan.replay()
        torch.cuda.synchronize()
        assert_same(outs, eager, f"replay {rep}")
    # binding other buffers invalidates the graph
    plan.decode(llrs, ws=ws)
    with pytest.raises(ldpc.LdpcError):
        plan.replay()


def test_autotune_keeps_results():
    graphs, llrs = make_case(synth.MIXED_CODES, 6000)
    gammas = [c["gamma"] for c in synth.MIXED_CODES]
    plan = ldpc.Plan(graphs, gammas, 20, early_stop=True)
    ws = plan.workspace(DEV)
    outs = plan.outputs(DEV)
    print("[gpu] plan autotune", flush=True)
    best = plan.autotune(llrs, outs, ws, trials=2)
    assert best > 0
    split = []
    for c, g in enumerate(graphs):
        l = plan.layout(c)
        base = l & 15
        fpl = {ldpc.LAYOUT_G64F4: 4, ldpc.LAYOUT_G8F4: 4, ldpc.LAYOUT_G16F4: 4, ldpc.LAYOUT_G32F4: 4,
               ldpc.LAYOUT_G64F2: 2, ldpc.LAYOUT_G8F2: 2, ldpc.LAYOUT_G16F2: 2, ldpc.LAYOUT_G32F2: 2}.get(base, 1)
        lanes = 1 << ((l >> 8) & 3)
        assert 0 <= base < ldpc.PLAN_LAYOUTS and l < 1024
        assert fpl != 4 or g.info["dc_max"] <= 6
        assert fpl != 2 or g.info["dc_max"] <= 12
        assert (l >> 4) & 15 == 0 or base in (0, 1, 2, 3)
        assert (l >> 6) & 3 == 0 or g.info["dc_max"] <= 8
        assert lanes == 1 or (base in (0, 1, 2) and (l >> 6) & 3 == 0 and g.info["dc_max"] >= 2 * lanes)
        if lanes > 1:
            split.append(c)
    print(f"[gpu] autotuned layouts {[ldpc.layout_name(plan.layout(c)) for c in range(len(graphs))]}", flush=True)
    outs = plan.decode(llrs, outs=outs, ws=ws)
    refs = single_code(graphs, llrs, 20, True)
    torch.cuda.synchronize()
    # bit for bit in every layout but the split ones; those agree to FP32 rounding
    assert_same([o for c, o in enumerate(outs) if c not in split],
                [r for c, r in enumerate(refs) if c not in split], "after autotune")
    for c in split:
        assert_close_to_single_code(outs[c], refs[c], f"code {c} after autotune")


def test_plan_at_the_code_limit_with_irregular_and_degenerate_codes():
    # LDPC_PLAN_MAX_CODES codes: regular ones, an irregular code with zero
    # blocks, a code with an unchecked variable and weight-1 checks, rows of
    # weight 18 and 24, and batches of 1 .. 300 frames
    irregular = np.array([[0, 5, -1, 7, 2, -1, 11, 3], [9, -1, 4, 1, -1, 6, 0, -1],
                          [-1, 2, 8, -1, 10, 12, -1, 5], [3, 7, -1, -1, 1, -1, 9, 0]])
    degenerate = np.array([[0, -1], [3, -1]])
    tables = [(irregular, 13), (degenerate, 5),
              (np.random.default_rng(54).integers(0, 17, size=(3, 18)), 17),
              (np.random.default_rng(96).integers(0, 13, size=(4, 24)), 13)]
    for i, c in enumerate(RAGGED + synth.MIXED_CODES[:5]):
        tables.append((synth.draw_qc_shifts(c["J"], c["L"], c["p"], 70 + i), c["p"]))
    assert len(tables) == 16
    gammas = [1, 70, 300, 2, 64, 65, 3, 129, 31, 256, 5, 1, 200, 17, 8, 97]
    graphs = [ldpc.Graph.qc(a, p) for a, p in tables]
    llrs = []
    for i, (g, n_frames) in enumerate(zip(graphs, gammas)):
        s2 = synth.ebn0_to_sigma2(3.0, 0.5)
        x = ldpc.awgn_llr(g.n, n_frames, s2, 3000 + i, 0, device=DEV)
        if i == 1:
            x[1] = 100.0
            x[2] = -100.0
            x[3] = 0.0
        llrs.append(x)
    for early in (True, False):
        print(f"[gpu] 16-code plan early={early}", flush=True)
        plan = ldpc.Plan(graphs, gammas, 12, early_stop=early)
        outs = plan.decode(llrs)
        assert_same(outs, single_code(graphs, llrs, 12, early), f"16 codes early={early}")
    with pytest.raises(Exception):
        ldpc.Plan(graphs + graphs[:1], gammas + [1], 12)


# ----------------------------------------------------------------------------
# one persistent launch per decode
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("early,items", [(True, "2"), (False, "2"), (True, "1"), (True, "7")])
def test_persistent_launch_matches_single_code_decoder(early, items, monkeypatch):
    # LDPC_PLAN_TICKET_ITEMS is read when the plan's table is built
    monkeypatch.setenv("LDPC_PLAN_TICKET_ITEMS", items)
    specs = synth.MIXED_CODES
    graphs, llrs = make_case(specs, 1100)
    plan = ldpc.Plan(graphs, [c["gamma"] for c in specs], 20, early_stop=early)
    plan.set_persistent(True)
    ws = plan.workspace(DEV)
    print(f"[gpu] persistent mixed plan early={early} items={items}", flush=True)
    ldpc.timing_read()
    ldpc.timing_enable(True)
    outs = plan.decode(llrs, ws=ws)
    torch.cuda.synchronize()
    ldpc.timing_enable(False)
    t = ldpc.timing_read()
    assert t["plan_persistent"][0] == 1 and t["plan_check_node"][0] == 0, t
    plan.check(ws)
    assert_same(outs, single_code(graphs, llrs, 20, early), f"persistent early={early} items={items}")
    # twice in a row on the same workspace (the launch resets its counters)
    again = plan.decode(llrs, ws=ws)
    plan.check(ws)
    assert_same(again, outs, "second persistent decode")


def test_persistent_launch_at_the_code_limit():
    irregular = np.array([[0, 5, -1, 7, 2, -1, 11, 3], [9, -1, 4, 1, -1, 6, 0, -1],
                          [-1, 2, 8, -1, 10, 12, -1, 5], [3, 7, -1, -1, 1, -1, 9, 0]])
    tables = [(irregular, 13), (np.array([[0, -1], [3, -1]]), 5),
              (np.random.default_rng(54).integers(0, 17, size=(3, 18)), 17),
              (np.random.default_rng(96).integers(0, 13, size=(4, 24)), 13)]
    for i, c in enumerate(RAGGED + synth.MIXED_CODES[:5]):
        tables.append((synth.draw_qc_shifts(c["J"], c["L"], c["p"], 70 + i), c["p"]))
    gammas = [1, 70, 300, 2, 64, 65, 3, 129, 31, 256, 5, 1, 200, 17, 8, 97]
    graphs = [ldpc.Graph.qc(a, p) for a, p in tables]
    llrs = [ldpc.awgn_llr(g.n, k, synth.ebn0_to_sigma2(3.0, 0.5), 3100 + i, 0, device=DEV)
            for i, (g, k) in enumerate(zip(graphs, gammas))]
    for early in (True, False):
        print(f"[gpu] persistent 16-code plan early={early}", flush=True)
        plan = ldpc.Plan(graphs, gammas, 12, early_stop=early)
        plan.set_persistent(True)
        ws = plan.workspace(DEV)
        outs = plan.decode(llrs, ws=ws)
        plan.check(ws)
        assert_same(outs, single_code(graphs, llrs, 12, early), f"persistent 16 codes early={early}")


def test_persistent_graph_replay_matches_eager_decode():
    graphs, llrs = make_case(synth.MIXED_CODES, 5100)
    gammas = [c["gamma"] for c in synth.MIXED_CODES]
    plan = ldpc.Plan(graphs, gammas, 20, early_stop=True)
    plan.set_persistent(True)
    ws = plan.workspace(DEV)
    eager = [tuple(t.clone() for t in o) for o in plan.decode(llrs, ws=ws)]
    torch.cuda.synchronize()
    outs = plan.outputs(DEV)
    print("[gpu] persistent plan capture", flush=True)
    plan.capture(llrs, outs, ws)
    scratch = torch.zeros(1 << 20, device=DEV)
    for rep in range(3):
        for o in outs:
            for t in o:
                t.zero_()
        scratch.add_(1.0)                  # eager work between replays
        torch.cuda.synchronize()
        print(f"[gpu] persistent plan replay {rep}", flush=True)
        plan.replay()
        torch.cuda.synchronize()
        assert_same(outs, eager, f"persistent replay {rep}")
    plan.check(ws)
    # switching back to the phase launches invalidates the graph
    plan.set_persistent(False)
    with pytest.raises(ldpc.LdpcError):
        plan.replay()


def test_persistent_wait_expiry_is_reported_and_the_next_decode_is_exact():
    # a wait limit of 1 us makes the waits for the other workgroups' steps
    # expire: the launch stops early but exits normally, and the check reports
    # it; with the default limit the same plan and workspace decode exactly
    graphs, llrs = make_case(synth.MIXED_CODES, 5200)
    gammas = [c["gamma"] for c in synth.MIXED_CODES]
    plan = ldpc.Plan(graphs, gammas, 20, early_stop=True)
    ws = plan.workspace(DEV)
    plan.set_persistent(True, wait_limit_us=1)
    print("[gpu] persistent plan with 1 us waits", flush=True)
    plan.decode(llrs, ws=ws)
    with pytest.raises(ldpc.LdpcError) as e:
        plan.check(ws)
    assert e.value.status == ldpc.EHIP
    plan.check(ws)                          # the record was cleared
    plan.set_persistent(True)
    print("[gpu] persistent plan with the default wait limit", flush=True)
    outs = plan.decode(llrs, ws=ws)
    plan.check(ws)
    assert_same(outs, single_code(graphs, llrs, 20, True), "after an expired wait")


# ----------------------------------------------------------------------------
# codes that fit one compute unit run the on-chip block decoder inside the
# plan (a parallel branch next to the phase launches), as ldpc_decode runs
# them: the plan's outputs equal ldpc_decode's, bit for bit, on both decoders
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("early", [True, False])
def test_plan_runs_on_chip_codes_as_the_single_code_decoder(early, monkeypatch):
    monkeypatch.delenv("LDPC_BLOCK_PATH", raising=False)
    specs = synth.MIXED_CODES
    print(f"[gpu] mixed plan with on-chip codes early={early}", flush=True)
    graphs, llrs = make_case(specs, 7000)
    paths = [ldpc.decode_path(g) for g in graphs]
    assert paths.count("onchip") >= 3 and paths.count("packages") >= 2
    plan = ldpc.Plan(graphs, [c["gamma"] for c in specs], 20, early_stop=early)
    ws = plan.workspace(DEV)
    outs = plan.decode(llrs, ws=ws)
    refs = single_code(graphs, llrs, 20, early)
    assert_same(outs, refs, "mixed, on-chip codes")
    # graph replay: three replays with eager work and synchronisation between
    outs2 = [tuple(torch.empty_like(t) for t in o) for o in outs]
    plan.capture(llrs, outs2, ws)
    for rep in range(3):
        for o in outs2:
            for t in o:
                t.zero_()
        plan.replay()
        torch.cuda.synchronize()
        assert_same(outs2, refs, f"replay {rep}")
        junk = torch.randn(1 << 20, device=DEV).sum()
        torch.cuda.synchronize()
        del junk
    # the same plan after forcing the package decoder: every code in the phase launches
    monkeypatch.setenv("LDPC_BLOCK_PATH", "packages")
    assert_same(plan.decode(llrs, ws=ws), single_code(graphs, llrs, 20, early), "mixed, package decoder")


def test_plan_of_on_chip_codes_only(monkeypatch):
    # no code left for the phase launches: the plan is the on-chip launches alone
    monkeypatch.delenv("LDPC_BLOCK_PATH", raising=False)
    specs = [c for c in synth.MIXED_CODES if c["L"] == 6][:2]
    graphs, llrs = make_case(specs, 8000)
    assert all(ldpc.decode_path(g) == "onchip" for g in graphs)
    plan = ldpc.Plan(graphs, [c["gamma"] for c in specs], 15, early_stop=True)
    assert_same(plan.decode(llrs), single_code(graphs, llrs, 15, True), "on-chip codes only")
