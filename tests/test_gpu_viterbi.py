"""Viterbi decoding on the GPU vs the FP64 oracle, through the C ABI (MI355X only).

score  |s_gpu - s_oracle| / max(|s_oracle|, 1) <= 1e-5, infinities and NaNs equal
path   equal to the oracle's wherever the oracle's smallest decision margin on its
       path exceeds the FP32 rounding of the decoder (1e-5 |score| + 1e-4); elsewhere
       (near-ties, where several paths are optimal to rounding) the GPU path must be a
       valid state path whose FP64 log-probability is within the score tolerance of the
       oracle's optimum.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1310_3322_amd import hmm, workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _lib():
    hmm.load_library()
    yield


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def problem(w, symbols=None):
    sym = w.symbols if symbols is None else symbols
    return hmm.Problem(dev(w.pi), dev(w.A), dev(w.B), dev(sym), dev(w.offsets), dev(w.lengths), dev(w.owner),
                       max_len=w.max_len, total_symbols=w.total_symbols)


def path_logprob(w, s, q, sym):
    k, T, off = int(w.owner[s]), int(w.lengths[s]), int(w.offsets[s])
    o = sym[off:off + T]
    with np.errstate(divide="ignore"):
        lp = np.log(w.pi[k].astype(np.float64))[q[0]] + np.log(w.B[k].astype(np.float64))[q, o].sum()
        if T > 1:
            lp += np.log(w.A[k].astype(np.float64))[q[:-1], q[1:]].sum()
    return lp


def check(w, symbols=None):
    sym = w.symbols if symbols is None else symbols
    sc, path = hmm.viterbi(problem(w, sym))
    sc, path = sc.cpu().numpy().astype(np.float64), path.cpu().numpy()
    rs, rp, rm = O.viterbi(w.pi, w.A, w.B, sym, w.offsets, w.lengths, w.owner)
    assert np.array_equal(np.isnan(sc), np.isnan(rs))
    assert np.array_equal(sc[np.isinf(rs)], rs[np.isinf(rs)])
    fin = np.isfinite(rs)
    if fin.any():
        err = np.max(np.abs(sc[fin] - rs[fin]) / np.maximum(np.abs(rs[fin]), 1.0))
        assert err <= TOL, err
    exact = 0
    for s in range(w.S):
        T, off = int(w.lengths[s]), int(w.offsets[s])
        g, r = path[off:off + T], rp[off:off + T]
        if not np.isfinite(rs[s]):
            if np.isnan(rs[s]):
                assert np.all(g == -1), s
            continue
        if rm[s] > 1e-5 * max(1.0, abs(rs[s])) + 1e-4:
            assert np.array_equal(g, r), (s, T)
            exact += 1
        else:
            assert np.all((g >= 0) & (g < w.N)), s
            lp = path_logprob(w, s, g, sym)
            assert abs(lp - rs[s]) <= TOL * max(1.0, abs(rs[s])), (s, lp, rs[s])
    return exact


@pytest.mark.parametrize("cfg,scale", [("brute", 1.0), ("c1", 1.0), ("paper", 1.0), ("c2", 0.1), ("c3", 0.004)])
def test_viterbi_parity_workloads(cfg, scale):
    print(f"[case] viterbi {cfg} scale={scale}", flush=True)
    w = workloads.make_workload(cfg, scale=scale)
    if w.all_pairs:
        w.all_pairs = False
    n = check(w)
    print(f"  {n} of {w.S} paths compared exactly", flush=True)
    if w.S >= 10:
        assert n > 0  # the exact comparison is exercised


@pytest.mark.parametrize("N", [1, 2, 5, 16, 17, 31, 32, 33, 48, 64, 65, 100, 128, 129, 200, 256])
def test_viterbi_state_counts_and_ragged_lengths(N):
    """Every padding of the state axis (lane groups up to 64 states, workgroups of 4 threads
    per state above); lengths around the shift period (16) and the workgroup decoder's
    symbol chunk (64), T = 0 and 1."""
    print(f"[case] viterbi N={N}", flush=True)
    rng = np.random.default_rng([31, N])
    lengths = np.concatenate([[0, 1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 129, 300], rng.integers(1, 120, size=26)])
    w = workloads.random_lengths_workload(rng, K=3, N=N, M=11, lengths=lengths, all_pairs=False, conc=0.4)
    check(w)


@pytest.mark.parametrize("N", [6, 150])
def test_viterbi_special_inputs(N):
    """An impossible observation (score -inf), an invalid symbol (NaN, path -1, error word),
    T = 0 (score 0), for the per-wave decoder (N=6) and the workgroup decoder (N=150)."""
    print(f"[case] viterbi special inputs N={N}", flush=True)
    rng = np.random.default_rng(41)
    lengths = np.array([0, 1, 5, 40, 7, 12, 3], np.int32)
    w = workloads.random_lengths_workload(rng, K=2, N=N, M=5, lengths=lengths, all_pairs=False)
    w.B[1, :, 4] = 0.0
    w.B[1] /= w.B[1].sum(axis=1, keepdims=True)
    sym = w.symbols.copy()
    s_imp = int(np.flatnonzero(w.owner == 1)[0])
    if w.lengths[s_imp] == 0:
        s_imp = int(np.flatnonzero((w.owner == 1) & (w.lengths > 0))[0])
    sym[w.offsets[s_imp]] = 4                     # impossible under model 1
    sym[w.offsets[3] + 7] = 99                    # invalid symbol in sequence 3
    p = problem(w, sym)
    ws = p.workspace(hmm.OP_VITERBI)
    sc, path = hmm.viterbi(p, ws=ws)
    assert hmm.workspace_error(ws) == 3
    sc = sc.cpu().numpy()
    assert np.isneginf(sc[s_imp]) and np.isnan(sc[3]) and sc[0] == 0.0
    check(w, sym)


def test_viterbi_full_c3_sampled():
    """The c3 bank and full batch, each sequence decoded with its owner; sampled sequences vs the oracle."""
    print("[case] viterbi c3 full", flush=True)
    w = workloads.make_workload("c3")
    w.all_pairs = False
    sc, path = hmm.viterbi(problem(w))
    sc, path = sc.cpu().numpy(), path.cpu().numpy()
    assert np.all(np.isfinite(sc))
    order = np.argsort(-w.lengths, kind="stable")
    rng = np.random.default_rng(9)
    pick = np.unique(np.concatenate([order[:8], order[-8:], rng.choice(w.S, 40, replace=False)]))
    sub = w.subset(pick)
    rs, rp, rm = O.viterbi(sub.pi, sub.A, sub.B, sub.symbols, sub.offsets, sub.lengths, sub.owner)
    err = np.max(np.abs(sc[pick] - rs) / np.maximum(np.abs(rs), 1.0))
    assert err <= TOL, err
    for i, s in enumerate(pick):
        T, off, so = int(w.lengths[s]), int(w.offsets[s]), int(sub.offsets[i])
        if rm[i] > 1e-5 * max(1.0, abs(rs[i])) + 1e-4:
            assert np.array_equal(path[off:off + T], rp[so:so + T]), s


def test_viterbi_determinism():
    """Repeated calls give identical scores and paths, for the per-wave decoder (c2) and
    the workgroup decoder (65 states)."""
    rng = np.random.default_rng(3)
    big = workloads.random_lengths_workload(rng, K=2, N=65, M=4, lengths=np.array([5, 6, 70, 0, 1]), all_pairs=False)
    check(big)
    w = workloads.make_workload("c2", scale=0.05)
    w.all_pairs = False
    for x in (w, big):
        p = problem(x)
        a = hmm.viterbi(p)
        b = hmm.viterbi(p)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_viterbi_c5_bank_sampled():
    """The c5 bank (256 states, 1024 symbols, banded transitions) on a 5 % sample of its
    sequences (lengths 256..4096), each with its owner: sampled sequences vs the oracle."""
    print("[case] viterbi c5 sample", flush=True)
    w = workloads.make_workload("c5", scale=0.05)
    w.all_pairs = False
    sc, path = hmm.viterbi(problem(w))
    sc, path = sc.cpu().numpy(), path.cpu().numpy()
    assert np.all(np.isfinite(sc))
    order = np.argsort(-w.lengths, kind="stable")
    rng = np.random.default_rng(5)
    pick = np.unique(np.concatenate([order[:2], order[-2:], rng.choice(w.S, 6, replace=False)]))
    sub = w.subset(pick)
    rs, rp, rm = O.viterbi(sub.pi, sub.A, sub.B, sub.symbols, sub.offsets, sub.lengths, sub.owner)
    err = np.max(np.abs(sc[pick] - rs) / np.maximum(np.abs(rs), 1.0))
    assert err <= TOL, err
    exact = 0
    for i, s in enumerate(pick):
        T, off, so = int(w.lengths[s]), int(w.offsets[s]), int(sub.offsets[i])
        g = path[off:off + T]
        if rm[i] > 1e-5 * max(1.0, abs(rs[i])) + 1e-4:
            assert np.array_equal(g, rp[so:so + T]), s
            exact += 1
        else:
            assert np.all((g >= 0) & (g < w.N)), s
            lp = path_logprob(sub, i, g, sub.symbols)
            assert abs(lp - rs[i]) <= TOL * max(1.0, abs(rs[i])), (s, lp, rs[i])
    print(f"  {exact} of {len(pick)} paths compared exactly", flush=True)
