"""The gradient keeps the scaled forward variables (alphahat, Sec. 2.7) between
its passes in one of two storages: every step (the forward pass stores each
step's row, the backward pass reads it back) or sqrt(T) checkpoints (the
backward pass recomputes each segment).  Both must give the same
log-likelihoods and counts bit for bit, and those must match the FP64 oracle.
The storage follows the workspace: rows for every step of the batch, else
checkpoints, found on the device, so that sequences overlapping in the symbol
array (more rows than symbols) fall back to checkpoints."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1310_3322_amd import hmm, workloads

pytestmark = pytest.mark.gpu

LL_TOL = 2e-5
GRAD_TOL = 2e-4


@pytest.fixture(scope="module", autouse=True)
def _lib():
    hmm.load_library()
    yield
    hmm.select_kernel(hmm.KERNEL_AUTO)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def problem(w, symbols=None, offsets=None, lengths=None, total=None):
    sym = w.symbols if symbols is None else symbols
    off = w.offsets if offsets is None else offsets
    lens = w.lengths if lengths is None else lengths
    return hmm.Problem(dev(w.pi), dev(w.A), dev(w.B), dev(sym), dev(off), dev(lens), dev(w.owner),
                       max_len=int(max(int(lens.max()) if lens.size else 0, w.max_len)),
                       total_symbols=w.total_symbols if total is None else total)


def grad(p, rows, wts=None):
    ws = p.grad_workspace(rows)
    ll, c, _ = hmm.forward_backward_grad(p, seq_weight=None if wts is None else dev(wts), ws=ws)
    torch.cuda.synchronize()
    return ll.clone(), [x.clone() for x in c], ws


def bits(t):
    return t.contiguous().view(torch.int32)


def assert_same(a, b, label):
    (lla, ca), (llb, cb) = a, b
    assert torch.equal(bits(lla), bits(llb)), f"{label}: log-likelihoods differ"
    for name, x, y in zip(("n_pi", "n_A", "n_B"), ca, cb):
        assert torch.equal(bits(x), bits(y)), f"{label}: {name} differs"


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
    for k in range(ref.shape[0]):
        den = np.linalg.norm(ref[k])
        if den == 0:
            assert np.linalg.norm(gpu[k]) == 0
            continue
        worst = max(worst, np.linalg.norm(gpu[k] - ref[k]) / den)
    return worst


def check_oracle(ll, c, w, symbols, offsets, lengths, wts):
    rll, rpi, rA, rB = O.counts(w.pi, w.A, w.B, symbols, offsets, lengths, w.owner, weights=wts)
    assert rel_err(ll.cpu().numpy(), rll) <= LL_TOL
    for got, ref in zip(c, (rpi, rA, rB)):
        assert counts_err(got.cpu().numpy(), ref) <= GRAD_TOL
    return rll


@pytest.mark.parametrize("N,M", [(49, 17), (64, 17), (64, 700), (96, 17), (128, 700), (129, 17), (200, 40),
                                 (256, 1024)])
def test_every_step_equals_checkpoints(N, M):
    """Ragged lengths (0, 1, 2, a square, several tiles per model) with weights: every
    count path of the cooperative shapes (LDS partial and slab, global sums, streamed
    fragments)."""
    print(f"[case] grad storage N={N} M={M}", flush=True)
    rng = np.random.default_rng([31, N, M])
    lengths = rng.integers(1, 300, size=53).astype(np.int32)
    lengths[:5] = [0, 1, 2, 64, 301]
    w = workloads.random_lengths_workload(rng, K=3, N=N, M=M, lengths=lengths, all_pairs=False, conc=0.5)
    wts = rng.uniform(0.5, 1.5, size=w.S).astype(np.float32)
    p = problem(w)
    ck = grad(p, 0, wts)
    ev = grad(p, w.total_symbols, wts)
    assert_same(ck[:2], ev[:2], f"N={N} M={M}")
    check_oracle(ev[0], ev[1], w, w.symbols, w.offsets, w.lengths, wts)
    # the default workspace of such a batch stores every step
    assert p.workspace(hmm.OP_GRAD).numel() == p.grad_workspace_size(w.total_symbols)


def test_every_step_invalid_inputs():
    """An impossible observation, an invalid symbol and an empty sequence take the same
    values and the same error word in both storages."""
    rng = np.random.default_rng(33)
    lengths = np.array([0, 1, 3, 40, 41, 1, 200, 17, 5, 90], np.int32)
    w = workloads.random_lengths_workload(rng, K=2, N=72, M=6, lengths=lengths, all_pairs=False)
    w.B[1, :, 5] = 0.0
    w.B[1] /= w.B[1].sum(axis=1, keepdims=True)
    s_dead = int(np.flatnonzero(w.owner == 1)[-1])
    sym = w.symbols.copy()
    sym[sym == 5] = 0
    sym[w.offsets[s_dead] + w.lengths[s_dead] - 1] = 5  # impossible at its last step
    s_bad = 4
    sym[w.offsets[s_bad] + 2] = 9  # invalid symbol
    p = problem(w, symbols=sym)
    ck = grad(p, 0)
    ev = grad(p, w.total_symbols)
    assert_same(ck[:2], ev[:2], "invalid inputs")
    assert hmm.workspace_error(ck[2]) == s_bad and hmm.workspace_error(ev[2]) == s_bad
    rll = check_oracle(ev[0], ev[1], w, sym, w.offsets, w.lengths, None)
    assert np.isneginf(rll[s_dead]) and np.isnan(rll[s_bad])


def test_overlapping_sequences_fall_back():
    """Sequences that share symbols need more rows than the symbol array holds: with
    room for total_symbols rows the device falls back to checkpoints, with room for
    S max_len rows it stores every step; all three runs agree bit for bit."""
    rng = np.random.default_rng(35)
    lengths = np.array([120, 80, 200, 33, 7, 150, 64], np.int32)
    w = workloads.random_lengths_workload(rng, K=2, N=64, M=9, lengths=lengths, all_pairs=False)
    # sequence i starts where the previous one did plus a third of its length
    offsets = np.zeros(w.S, np.int64)
    for i in range(1, w.S):
        offsets[i] = offsets[i - 1] + max(1, int(lengths[i - 1]) // 3)
    total = int(max(offsets[i] + lengths[i] for i in range(w.S)))
    sym = rng.integers(0, 9, size=total).astype(np.int32)
    assert int(lengths.sum()) > total
    p = problem(w, symbols=sym, offsets=offsets, lengths=lengths, total=total)
    ck = grad(p, 0)
    short = grad(p, total)
    ev = grad(p, int(lengths.sum()))
    assert_same(ck[:2], short[:2], "overlap, rows = total_symbols")
    assert_same(ck[:2], ev[:2], "overlap, rows = sum of lengths")
    check_oracle(ev[0], ev[1], w, sym, offsets, lengths, None)


@pytest.mark.parametrize("cfg,scale", [("c4", 0.02), ("c5", 0.005)])
def test_every_step_phase_split(cfg, scale):
    """Phase 1 then phase 2 (twice) from one workspace that stores every step equals the
    fused call bit for bit.  On c5 (global counts) the fused call sums the emission counts
    from the gamma it leaves in the rows, phase 2 with per-step atomics and without
    touching the rows, so that the second phase 2 still reads the forward's."""
    print(f"[case] grad storage phases {cfg} scale={scale}", flush=True)
    w = workloads.make_workload(cfg, scale=scale)
    p = problem(w)
    wt = dev(np.linspace(0.2, 2.0, w.S).astype(np.float32))
    ws0 = p.grad_workspace(w.total_symbols)
    ll0, c0, _ = hmm.forward_backward_grad(p, seq_weight=wt, phase=0, ws=ws0)
    ws = p.grad_workspace(w.total_symbols)
    ll1, _, _ = hmm.forward_backward_grad(p, phase=1, ws=ws)
    for _ in range(2):
        _, c2, _ = hmm.forward_backward_grad(p, seq_weight=wt, phase=2, ws=ws)
        assert torch.equal(ll0, ll1)
        for a, b in zip(c0, c2):
            assert torch.equal(bits(a), bits(b))


@pytest.mark.parametrize("cfg,scale", [("c4", 1.0), ("c5", 0.02)])
def test_every_step_benchmark_shapes(cfg, scale):
    """The benchmarked gradient shapes (c4 at full size, a c5 sample of 328 sequences of up
    to 4096 steps): both storages agree bit for bit."""
    print(f"[case] grad storage {cfg} scale={scale}", flush=True)
    w = workloads.make_workload(cfg, scale=scale)
    rng = np.random.default_rng(37)
    wts = rng.uniform(0.5, 1.5, size=w.S).astype(np.float32)
    p = problem(w)
    ck = grad(p, 0, wts)
    ev = grad(p, w.total_symbols, wts)
    assert_same(ck[:2], ev[:2], cfg)
    assert torch.isfinite(ev[0]).all()


def test_every_step_c5_full_size_masked_weights():
    """The N=256 gradient as the benchmark runs it: all 16,384 sequences with every step
    stored (38 GB of workspace), sequence weights nonzero on 32 sampled sequences only, so
    that the counts are the sample's and the oracle computes them; the checkpoint storage
    gives the same counts bit for bit."""
    print("[case] grad storage c5 full size, masked weights", flush=True)
    w = workloads.make_workload("c5")
    rng = np.random.default_rng(39)
    order = np.argsort(-w.lengths, kind="stable")
    pick = np.unique(np.concatenate([order[:6], order[-6:], rng.choice(w.S, 20, replace=False)]))
    wts = np.zeros(w.S, np.float32)
    wts[pick] = rng.uniform(0.5, 1.5, size=pick.size).astype(np.float32)
    p = problem(w)
    ev = grad(p, w.total_symbols, wts)
    ll = ev[0].cpu().numpy()
    assert np.all(np.isfinite(ll))
    sub = w.subset(pick)
    rll, rpi, rA, rB = O.counts(sub.pi, sub.A, sub.B, sub.symbols, sub.offsets, sub.lengths, sub.owner,
                                weights=wts[pick])
    assert rel_err(ll[pick], rll) <= LL_TOL
    for got, ref in zip(ev[1], (rpi, rA, rB)):
        assert counts_err(got.cpu().numpy(), ref) <= GRAD_TOL
    ws_bytes = ev[2].numel()
    ev = ev[:2]  # the 38 GB workspace is released
    ck = grad(p, 0, wts)
    assert ck[2].numel() < ws_bytes
    assert_same(ck[:2], ev, "c5 full size")


def test_every_step_invalid_model_index():
    """Sequences whose model index is out of range (K and -1) take NaN log-likelihoods, add
    no counts and set the error word (the smallest such index) in both storages; the counts
    are the valid sequences' (the oracle on that subset)."""
    rng = np.random.default_rng(41)
    lengths = rng.integers(1, 120, size=23).astype(np.int32)
    w = workloads.random_lengths_workload(rng, K=3, N=70, M=9, lengths=lengths, all_pairs=False)
    owner = w.owner.copy()
    owner[5] = 3
    owner[9] = -1
    p = hmm.Problem(dev(w.pi), dev(w.A), dev(w.B), dev(w.symbols), dev(w.offsets), dev(w.lengths), dev(owner),
                    max_len=w.max_len, total_symbols=w.total_symbols)
    ck = grad(p, 0)
    ev = grad(p, w.total_symbols)
    assert_same(ck[:2], ev[:2], "invalid model index")
    assert hmm.workspace_error(ck[2]) == 5 and hmm.workspace_error(ev[2]) == 5
    ll = ev[0].cpu().numpy()
    assert np.isnan(ll[5]) and np.isnan(ll[9])
    valid = np.array([s for s in range(w.S) if s not in (5, 9)])
    sub = w.subset(valid)
    rll, rpi, rA, rB = O.counts(sub.pi, sub.A, sub.B, sub.symbols, sub.offsets, sub.lengths, sub.owner)
    assert rel_err(ll[valid], rll) <= LL_TOL
    for got, ref in zip(ev[1], (rpi, rA, rB)):
        assert counts_err(got.cpu().numpy(), ref) <= GRAD_TOL
