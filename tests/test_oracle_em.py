"""Pins of the oracle's Baum-Welch EM (CPU): the M-step and the EM loop.

The re-estimation divides expected counts (pinned elsewhere against path
enumeration) by their row sums.  Checked here: the M-step from enumerated
counts on a tiny model, the EM theorem (the likelihood never decreases), the
stationary point of a one-state model, and rows without counts.
"""
import math

import numpy as np

from oracle import bruteforce
from paper_1310_3322_amd import workloads


def test_mstep_from_enumerated_counts(oracle_mod):
    rng = np.random.default_rng(51)
    N, M, T = 3, 4, 6
    pi = workloads.dirichlet_rows(rng, (1,), N, 0.8)
    A = workloads.dirichlet_rows(rng, (1, N), N, 0.8)
    B = workloads.dirichlet_rows(rng, (1, N), M, 0.8)
    o = rng.integers(0, M, size=T).astype(np.int32)
    _, bpi, bA, bB = bruteforce.expected_counts(pi[0].tolist(), A[0].tolist(), B[0].tolist(), o.tolist())
    hist, _ = oracle_mod.baum_welch(pi, A, B, o, np.zeros(1, np.int64), np.array([T], np.int32),
                                    np.zeros(1, np.int32), iters=1)
    npi, nA, nB = hist[0]
    bA, bB = np.array(bA), np.array(bB)
    assert np.allclose(npi[0], np.array(bpi) / sum(bpi), rtol=1e-12)
    assert np.allclose(nA[0], bA / bA.sum(axis=1, keepdims=True), rtol=1e-12)
    assert np.allclose(nB[0], bB / bB.sum(axis=1, keepdims=True), rtol=1e-12)
    # one sequence: pi' is the posterior of q_1, which sums to one
    assert abs(npi[0].sum() - 1.0) < 1e-14


def test_em_likelihood_never_decreases(oracle_mod):
    w = workloads.make_workload("c2", scale=0.02)
    hist, lls = oracle_mod.baum_welch(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner, iters=6)
    assert all(b >= a - 1e-9 * abs(a) for a, b in zip(lls, lls[1:])), lls
    assert lls[-1] > lls[0]
    for pi, A, B in hist:  # every iterate is a proper model
        assert np.allclose(pi.sum(-1), 1) and np.allclose(A.sum(-1), 1) and np.allclose(B.sum(-1), 1)


def test_em_one_state_is_symbol_frequencies(oracle_mod):
    """N = 1: one M-step gives B = empirical symbol frequencies over the model's sequences."""
    rng = np.random.default_rng(52)
    lengths = np.array([7, 0, 13, 4], np.int32)
    w = workloads.random_lengths_workload(rng, K=1, N=1, M=5, lengths=lengths, all_pairs=False)
    hist, _ = oracle_mod.baum_welch(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner, iters=1)
    freq = np.bincount(w.symbols, minlength=5) / len(w.symbols)
    assert np.allclose(hist[0][2][0, 0], freq, rtol=1e-13)
    assert hist[0][0][0, 0] == 1.0 and hist[0][1][0, 0, 0] == 1.0


def test_em_rows_without_counts_keep_old_values(oracle_mod):
    """A model with no sequences, and a state that can never be reached, keep their rows."""
    rng = np.random.default_rng(53)
    lengths = np.array([9, 11, 6], np.int32)
    w = workloads.random_lengths_workload(rng, K=2, N=3, M=4, lengths=lengths, all_pairs=False)
    w.owner[:] = 0                               # model 1 gets no sequences
    w.pi[0] = [0.5, 0.5, 0.0]
    w.A[0, :, 2] = 0.0                           # state 2 unreachable in model 0
    w.A[0] /= w.A[0].sum(axis=1, keepdims=True)
    hist, _ = oracle_mod.baum_welch(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner, iters=1)
    pi, A, B = hist[0]
    assert np.array_equal(pi[1], w.pi[1].astype(np.float64))
    assert np.array_equal(A[1], w.A[1].astype(np.float64)) and np.array_equal(B[1], w.B[1].astype(np.float64))
    assert np.array_equal(A[0, 2], w.A[0, 2].astype(np.float64))
    assert np.array_equal(B[0, 2], w.B[0, 2].astype(np.float64))
    assert pi[0, 2] == 0.0 and np.all(A[0, :, 2] == 0.0)
