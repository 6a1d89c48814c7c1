"""The planner's work list (hmm_plan_order) against a stable sort on the host (MI355X only).

The list must equal, entry for entry, the sequence indices ordered by (group, decreasing
length, increasing index), where the group is the owning model for own-model calls and
one group for all-pairs calls and for Viterbi decoding (whose list holds every sequence,
longest first, whatever its model), and an invalid sequence counts as length 0 of its
group (group 0 when its model index is out of range).  Integer work: bit-exact.
"""
import numpy as np
import pytest
import torch

from paper_1310_3322_amd import hmm, workloads

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def expected(lengths, offsets, owner, K, max_len, total, own, M=None, symbols=None):
    S = len(lengths)
    T = lengths.astype(np.int64)
    bad = (T < 0) | (T > max_len) | (offsets < 0) | (offsets + T > total)
    g = np.zeros(S, dtype=np.int64)
    if own:
        g = owner.astype(np.int64).copy()
        inval = (g < 0) | (g >= K)
        bad |= inval
        g[inval] = 0
    te = np.where(bad, 0, T)
    order = np.lexsort((np.arange(S), -te, g))  # last key is the primary one
    groups = K if own else 1
    gstart = np.searchsorted(g[order], np.arange(groups + 1), side="left").astype(np.int32)
    gstart[-1] = S
    return order.astype(np.int32), gstart


def run(w, op, own, max_len=None, lengths=None, owner=None):
    lengths = w.lengths if lengths is None else lengths
    owner = w.owner if owner is None else owner
    ml = w.max_len if max_len is None else max_len
    p = hmm.Problem(dev(w.pi), dev(w.A), dev(w.B), dev(w.symbols), dev(w.offsets), dev(lengths),
                    dev(owner) if own else None, max_len=ml, total_symbols=w.total_symbols)
    order, gstart = hmm.plan_order(p, op)
    torch.cuda.synchronize()
    eo, eg = expected(lengths, w.offsets, owner, w.K, ml, w.total_symbols, own and op != hmm.OP_VITERBI)
    assert np.array_equal(gstart.cpu().numpy(), eg)
    assert np.array_equal(order.cpu().numpy(), eo)
    return order


@pytest.mark.parametrize("cfg,scale,op,own", [("c2", 1.0, hmm.OP_CLASSIFY, False), ("c3", 0.1, hmm.OP_CLASSIFY, False),
                                              ("c4", 1.0, hmm.OP_GRAD, True), ("c5", 0.1, hmm.OP_GRAD, True),
                                              ("c5", 0.1, hmm.OP_VITERBI, True), ("paper", 1.0, hmm.OP_FORWARD, True)])
def test_plan_matches_stable_sort(cfg, scale, op, own):
    print(f"[case] plan {cfg} scale={scale} op={op}", flush=True)
    run(workloads.make_workload(cfg, scale=scale), op, own)


def test_plan_large_bins_and_invalid_entries():
    """Few distinct lengths (bins far larger than a sort block), invalid lengths and model
    indices, and a bin count that makes the chunks span several sort blocks."""
    print("[case] plan large bins", flush=True)
    rng = np.random.default_rng(17)
    S = 20000
    lengths = rng.choice(np.array([0, 1, 3, 40], dtype=np.int32), size=S)
    w = workloads.random_lengths_workload(rng, K=64, N=8, M=5, lengths=lengths, all_pairs=False)
    lengths = w.lengths.copy()
    owner = w.owner.copy()
    lengths[5] = -1                 # negative length
    lengths[7] = 1 << 20            # beyond max_len
    owner[11] = 64                  # model index out of range
    owner[13] = -3
    # max_len 65535: 64 x 65536 bins, so the 20,000 sequences form 4 chunks of 5120 (3 sort blocks each)
    run(w, hmm.OP_GRAD, True, max_len=65535, lengths=lengths, owner=owner)
    run(w, hmm.OP_FORWARD, False, max_len=65535, lengths=lengths, owner=owner)


def test_plan_empty_batch_and_repeatability():
    print("[case] plan empty / repeat", flush=True)
    w = workloads.make_workload("c4", scale=0.3)
    a = run(w, hmm.OP_GRAD, True)
    b = run(w, hmm.OP_GRAD, True)
    assert torch.equal(a, b)
    e = w.subset(np.array([], dtype=np.int64))
    run(e, hmm.OP_GRAD, True, max_len=10)
