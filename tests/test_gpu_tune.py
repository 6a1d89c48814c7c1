"""Autotuner on the GPU (MI355X only): every choice the tuning table can hold
gives the oracle's results, on shapes where the grid cap binds (more tiles than
capped workgroups, so every workgroup drains its queue repeatedly), and `tune`
installs an accepted choice that later calls use.

Tolerances as in the parity tests: log-likelihood 1e-5 relative, counts 1e-4
norm-wise, Viterbi scores 1e-5 relative with paths checked like the Viterbi tests.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1310_3322_amd import hmm, tune, workloads

pytestmark = pytest.mark.gpu

LL_TOL = 1e-5
GRAD_TOL = 1e-4
CAPS = (0, 1, 2)


@pytest.fixture(autouse=True)
def _clean_table():
    hmm.load_library()
    hmm.select_kernel(hmm.KERNEL_AUTO)
    hmm.tune_clear()
    yield
    hmm.tune_clear()
    hmm.select_kernel(hmm.KERNEL_AUTO)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def problem(w, own):
    return hmm.Problem(dev(w.pi), dev(w.A), dev(w.B), dev(w.symbols), dev(w.offsets), dev(w.lengths),
                       dev(w.owner) if own else None, max_len=w.max_len, total_symbols=w.total_symbols)


def rel_err(gpu, ref):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert np.array_equal(np.isnan(gpu), np.isnan(ref)), "NaN pattern differs"
    assert np.array_equal(gpu[np.isinf(ref)], ref[np.isinf(ref)]), "infinities differ"
    fin = np.isfinite(ref)
    if not fin.any():
        return 0.0
    return float(np.max(np.abs(gpu[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1.0)))


def counts_err(gpu, ref):
    worst = 0.0
    for g, r in zip(gpu, ref):
        g = np.asarray(g, dtype=np.float64)
        r = np.asarray(r, dtype=np.float64)
        for k in range(r.shape[0]):
            nr = np.linalg.norm(r[k])
            worst = max(worst, np.linalg.norm(g[k] - r[k]) / nr if nr > 0 else np.linalg.norm(g[k]))
    return worst


def short_workload(seed, K, N, M, S, tmax, all_pairs, conc=0.6):
    rng = np.random.default_rng([31, seed])
    lengths = rng.integers(1, tmax + 1, size=S)
    lengths[:3] = [0, 1, tmax]
    return workloads.random_lengths_workload(rng, K=K, N=N, M=M, lengths=lengths, all_pairs=all_pairs, conc=conc)


@pytest.mark.parametrize("N,all_pairs", [(16, True), (32, True), (32, False), (64, True)])
def test_every_forward_table_choice(N, all_pairs):
    """K=64 models: 64 x 38 tiles of 16 (all pairs), or 1127 tiles of 16 own-model,
    outnumber the capped grids."""
    print(f"[case] tune forward choices N={N} all_pairs={all_pairs}", flush=True)
    S = 600 if all_pairs else 17000
    w = short_workload(N, K=64, N=N, M=16, S=S, tmax=40, all_pairs=all_pairs)
    ref = O.forward(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, None if all_pairs else w.owner)
    p = problem(w, not all_pairs)
    key = hmm.tune_key(p.bank, p.batch, hmm.OP_FORWARD)
    ran = 0
    for kind in tune.FORWARD_KINDS:
        for cap in CAPS:
            hmm.tune_set(key, kind, cap)
            try:
                ll = hmm.forward_loglik(p).cpu().numpy()
            except hmm.HMMError as e:
                assert e.status == -4, (kind, cap)
                continue
            ran += 1
            assert rel_err(ll, ref) <= LL_TOL, (kind, cap)
    assert ran >= 3


@pytest.mark.parametrize("N,S", [(32, 17000), (64, 8400)])
def test_every_gradient_table_choice(N, S):
    """N=32: 16-sequence tiles, 4 per workgroup (1070 tiles); N=64: one
    cooperative workgroup per tile (533 tiles): both exceed the capped grids."""
    print(f"[case] tune gradient choices N={N} S={S}", flush=True)
    w = short_workload(100 + N, K=8, N=N, M=24, S=S, tmax=12, all_pairs=False)
    ll_ref, *cnt_ref = O.counts(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner)
    p = problem(w, True)
    key = hmm.tune_key(p.bank, p.batch, hmm.OP_GRAD)
    for cap in CAPS:
        hmm.tune_set(key, hmm.KERNEL_BATCHED, cap)
        ll, cnt, _ = hmm.forward_backward_grad(p)
        assert rel_err(ll.cpu().numpy(), ll_ref) <= LL_TOL, cap
        assert counts_err([c.cpu().numpy() for c in cnt], cnt_ref) <= GRAD_TOL, cap


@pytest.mark.parametrize("N,S", [(32, 4100), (200, 700)])
def test_every_viterbi_table_choice(N, S):
    """N=32: 8 sequences per workgroup, 4100 sequences -> 513 units per cap-1 grid of 256;
    N=200: the workgroup decoder, one sequence per workgroup, 700 sequences on grids of
    256 to 1024 workgroups."""
    print(f"[case] tune viterbi choices N={N}", flush=True)
    w = short_workload(7, K=4, N=N, M=20, S=S, tmax=30, all_pairs=False)
    rs, rp, rm = O.viterbi(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner)
    p = problem(w, True)
    key = hmm.tune_key(p.bank, p.batch, hmm.OP_VITERBI)
    first = None
    for cap in CAPS:
        hmm.tune_set(key, hmm.KERNEL_BATCHED, cap)
        sc, path = hmm.viterbi(p)
        sc, path = sc.cpu().numpy(), path.cpu().numpy()
        assert rel_err(sc, rs) <= LL_TOL, cap
        if first is None:
            first = (sc, path)
        else:  # the decoding of a sequence does not depend on the grid
            assert np.array_equal(sc, first[0]) and np.array_equal(path, first[1]), cap
        # where the oracle's decision margins are clear, the paths agree
        clear = np.repeat(rm > 1e-5 * np.maximum(np.abs(rs), 1.0) + 1e-4, w.lengths)
        assert np.array_equal(path[clear], rp[clear]), cap


@pytest.mark.parametrize("op", [hmm.OP_FORWARD, hmm.OP_CLASSIFY, hmm.OP_GRAD, hmm.OP_VITERBI])
def test_tune_installs_an_accepted_choice(op):
    print(f"[case] tune op={op}", flush=True)
    own = op in (hmm.OP_GRAD, hmm.OP_VITERBI)
    N = 64 if op == hmm.OP_GRAD else 16
    w = short_workload(200 + op, K=6, N=N, M=12, S=300, tmax=120, all_pairs=not own)
    p = problem(w, own)
    r = tune.tune(p, op, warmup=1, reps=2)
    assert r["op"] == tune.OP_NAMES[op]
    chosen = (tune._KERNEL_IDS[r["choice"]["kernel"]], r["choice"]["wg_per_cu"], r["choice"]["flags"])
    key = hmm.TuneKey(**r["key"])
    assert hmm.tune_get(key) == chosen
    ok = [c for c in r["candidates"] if c["ok"]]
    assert any((c["kernel"], c["wg_per_cu"], c["flags"]) ==
               (r["choice"]["kernel"], r["choice"]["wg_per_cu"], r["choice"]["flags"]) for c in ok)
    # the second stage tried the flags exactly where the chosen family reads them (the tile
    # forwards; the gradient with 64 states runs the cooperative kernels, Viterbi its own)
    fam = hmm.call_kernel(p.bank, p.batch, op)
    tile = fam in (hmm.KERNEL_TILE16, hmm.KERNEL_TILE32) and op != hmm.OP_VITERBI
    assert any(c["flags"] != 0 for c in r["candidates"]) == tile, (fam, r["candidates"])
    if op in (hmm.OP_FORWARD, hmm.OP_CLASSIFY):
        assert tile
    # no accepted candidate beat the choice by more than the tuner's margin
    assert min(c["ms"] for c in ok) >= r["ms"] * (1.0 - tune.MIN_GAIN)
    assert all(c["reason"] in ("unsupported", "default", "") for c in r["candidates"]), r["candidates"]
    # a call after tuning takes the installed choice and still matches the oracle
    if op == hmm.OP_FORWARD:
        ref = O.forward(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, None)
        assert rel_err(hmm.forward_loglik(p).cpu().numpy(), ref) <= LL_TOL
    elif op == hmm.OP_CLASSIFY:
        ref = O.forward(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, None)
        ll = torch.empty((p.S, p.K), dtype=torch.float32, device="cuda")
        labels = hmm.classify(p, loglik=ll).cpu().numpy()
        assert rel_err(ll.cpu().numpy(), ref) <= LL_TOL
        top = np.sort(ref, axis=1)
        clear = (top[:, -1] - top[:, -2]) > 1e-3 * np.maximum(np.abs(top[:, -1]), 1.0)
        assert np.array_equal(labels[clear], np.argmax(ref, axis=1)[clear])
    elif op == hmm.OP_GRAD:
        ll_ref, *cnt_ref = O.counts(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner)
        ll, cnt, _ = hmm.forward_backward_grad(p)
        assert rel_err(ll.cpu().numpy(), ll_ref) <= LL_TOL
        assert counts_err([c.cpu().numpy() for c in cnt], cnt_ref) <= GRAD_TOL
    else:
        rs, _, _ = O.viterbi(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner)
        assert rel_err(hmm.viterbi(p)[0].cpu().numpy(), rs) <= LL_TOL


@pytest.mark.parametrize("kind,N,M,all_pairs,S", [(hmm.KERNEL_TILE32, 32, 500, True, 20000),
                                                 (hmm.KERNEL_TILE16, 16, 1000, True, 20000),
                                                 (hmm.KERNEL_TILE16, 16, 2000, True, 4000),
                                                 (hmm.KERNEL_TILE32, 32, 500, False, 3000),
                                                 (hmm.KERNEL_TILE16, 48, 300, False, 3000)])
def test_tune_flags_change_no_result(kind, N, M, all_pairs, S):
    """Where the tile kernels keep the emission table (LDS up to 128 KB, global memory) and
    whether all-pairs tiles are split over the XCDs (20,000 sequences of 4 models fill a
    grid that allows the split) change no result: log-likelihoods bit-identical to the
    built-in choice (the tables here take 64-75 KB, so the default reads them from global
    memory; with 2000 symbols and 16 states the padded table would not fit beside the symbol
    buffers, and the LDS flag falls back to global memory), and within the oracle's
    tolerance."""
    print(f"[case] tune flags kind={kind} N={N} all_pairs={all_pairs}", flush=True)
    w = short_workload(300 + N, K=4, N=N, M=M, S=S, tmax=24, all_pairs=all_pairs)
    p = problem(w, not all_pairs)
    key = hmm.tune_key(p.bank, p.batch, hmm.OP_FORWARD)
    sets = [0, hmm.TUNE_BT_GLOBAL, hmm.TUNE_BT_LDS]
    if all_pairs:
        sets += [hmm.TUNE_XCD_OFF, hmm.TUNE_XCD_OFF | hmm.TUNE_BT_LDS]
    base = None
    try:
        for flags in sets:
            hmm.tune_set(key, kind, 0, flags)
            ll = hmm.forward_loglik(p).cpu().numpy()
            if base is None:
                base = ll
                ref = O.forward(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, None if all_pairs else w.owner)
                assert rel_err(ll, ref) <= LL_TOL
            else:
                assert np.array_equal(ll, base, equal_nan=True), flags
    finally:
        hmm.tune_set(key, None)


def test_tune_flags_gradient_counts_identical():
    """The gradient's checkpointing forward (16-sequence tiles, N = 32) with its emission
    table in LDS or in global memory: identical log-likelihoods and counts."""
    print("[case] tune flags gradient", flush=True)
    w = short_workload(5, K=3, N=32, M=700, S=400, tmax=60, all_pairs=False)
    p = problem(w, True)
    key = hmm.tune_key(p.bank, p.batch, hmm.OP_GRAD)
    outs = []
    try:
        for flags in (0, hmm.TUNE_BT_LDS, hmm.TUNE_BT_GLOBAL):
            hmm.tune_set(key, hmm.KERNEL_BATCHED, 0, flags)
            ll, cnt, _ = hmm.forward_backward_grad(p)
            outs.append([ll.cpu().numpy()] + [c.cpu().numpy() for c in cnt])
    finally:
        hmm.tune_set(key, None)
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b, equal_nan=True)


def test_selector_overrides_table():
    """A forced family ignores the table: an entry naming a family that does not
    take the shape fails only while the selector is AUTO."""
    w = short_workload(9, K=3, N=100, M=8, S=40, tmax=30, all_pairs=True)
    p = problem(w, False)
    key = hmm.tune_key(p.bank, p.batch, hmm.OP_FORWARD)
    hmm.tune_set(key, hmm.KERNEL_TILE16, 0)  # one wave per tile takes at most 64 states
    with pytest.raises(hmm.HMMError) as e:
        hmm.forward_loglik(p)
    assert e.value.status == -4
    hmm.select_kernel(hmm.KERNEL_BATCHED)
    ref = O.forward(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, None)
    assert rel_err(hmm.forward_loglik(p).cpu().numpy(), ref) <= LL_TOL


def _replay_matches_eager(fn, outs):
    """Captures fn(stream) once and replays it three times with eager work in between;
    every replay must reproduce the eager outputs bit for bit."""
    fn(torch.cuda.current_stream())
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn(s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for o in outs:
            o.fill_(-3)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r), rep
        _ = (outs[0].float() * 2).sum().item()


def test_tuned_choices_replay_from_a_graph():
    """Tuned entries are read on the host when a call is captured: a graph of a
    call whose entry picks the time-parallel forward, one with capped 16-sequence
    tiles and one with a capped decoder all replay to the eager results."""
    print("[case] tuned choices in graphs", flush=True)
    w = short_workload(11, K=2, N=8, M=10, S=3, tmax=300, all_pairs=False)
    p = problem(w, True)
    hmm.tune_set(hmm.tune_key(p.bank, p.batch, hmm.OP_FORWARD), hmm.KERNEL_SCAN, 0)
    assert hmm.call_kernel(p.bank, p.batch, hmm.OP_FORWARD) == hmm.KERNEL_SCAN
    ws = p.workspace(hmm.OP_FORWARD)
    ll = torch.empty(p.S, device="cuda")
    _replay_matches_eager(lambda st: hmm.forward_loglik(p, out=ll, ws=ws, stream=st), [ll])
    ref = O.forward(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner)
    assert rel_err(ll.cpu().numpy(), ref) <= LL_TOL

    w2 = short_workload(12, K=12, N=16, M=20, S=2000, tmax=60, all_pairs=True)
    p2 = problem(w2, False)
    b2 = p2.batch_without_models()
    hmm.tune_set(hmm.tune_key(p2.bank, b2, hmm.OP_CLASSIFY), hmm.KERNEL_TILE16, 2)
    ws2 = p2.workspace(hmm.OP_CLASSIFY, b2)
    lab = torch.empty(p2.S, dtype=torch.int32, device="cuda")
    ll2 = torch.empty((p2.S, p2.K), device="cuda")
    _replay_matches_eager(lambda st: hmm.classify(p2, labels=lab, loglik=ll2, ws=ws2, stream=st), [lab, ll2])
    ref2 = O.forward(w2.pi, w2.A, w2.B, w2.symbols, w2.offsets, w2.lengths, None)
    assert rel_err(ll2.cpu().numpy(), ref2) <= LL_TOL

    w3 = short_workload(13, K=3, N=32, M=20, S=900, tmax=80, all_pairs=False)
    p3 = problem(w3, True)
    hmm.tune_set(hmm.tune_key(p3.bank, p3.batch, hmm.OP_VITERBI), hmm.KERNEL_BATCHED, 1)
    ws3 = p3.workspace(hmm.OP_VITERBI)
    sc = torch.empty(p3.S, device="cuda")
    pa = torch.empty(p3.total_symbols, dtype=torch.int32, device="cuda")
    _replay_matches_eager(lambda st: hmm.viterbi(p3, score=sc, path=pa, ws=ws3, stream=st), [sc, pa])
    rs, _, _ = O.viterbi(w3.pi, w3.A, w3.B, w3.symbols, w3.offsets, w3.lengths, w3.owner)
    assert rel_err(sc.cpu().numpy(), rs) <= LL_TOL
