"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

The paper names the forward and Baum-Welch functions of its activity
recognition stage (Sec. 2.7) but prints no formula or worked example, so the
oracle follows the textbook discrete HMM and is pinned here by:
  * exact rational values from path enumeration (tests/golden/exact_small.json);
  * brute-force enumeration of all N^T state paths on random models;
  * the probability axiom sum_O P(O) = 1 over all symbol strings;
  * the scaled-variable invariant sum_i alphahat_t(i) betahat_t(i) = 1 for all t;
  * closed forms (N = 1, uniform B, i.i.d. chains, identity A);
  * an independent log-space forward written here;
  * count totals and flow conservation of the expected counts;
  * central finite differences of the log-likelihood for the logit gradient;
  * the arg-max tie and NaN rules of recognition.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import bruteforce
from paper_1310_3322_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "exact_small.json")


def _rng(tag):
    return np.random.default_rng([1310, 3322, 77, tag])


def _dir(rng, shape, n, conc=1.0):
    return workloads.dirichlet_rows(rng, shape, n, conc)


def _one(K_pi, o):
    """Pack one sequence as a batch."""
    o = np.asarray(o, dtype=np.int32)
    return o, np.zeros(1, np.int64), np.array([len(o)], np.int32)


# --------------------------------------------------------------------------- exact rationals
def test_golden_exact_rationals(oracle_mod):
    data = json.load(open(GOLDEN))
    for case in data["cases"]:
        pi = np.array([[float(Fraction(x)) for x in case["pi"]]])
        A = np.array([[[float(Fraction(x)) for x in r] for r in case["A"]]])
        B = np.array([[[float(Fraction(x)) for x in r] for r in case["B"]]])
        for seq in case["sequences"]:
            o, off, lens = _one(pi, seq["symbols"])
            P = Fraction(seq["P"])
            ll = oracle_mod.forward(pi, A, B, o, off, lens, np.zeros(1, np.int32))[0]
            assert ll == pytest.approx(math.log(P), rel=1e-13, abs=1e-13), case["name"]
            _, npi, nA, nB = oracle_mod.counts(pi, A, B, o, off, lens, np.zeros(1, np.int32))
            np.testing.assert_allclose(npi[0], [float(Fraction(x)) for x in seq["n_pi"]], rtol=1e-12, atol=1e-14)
            np.testing.assert_allclose(nA[0], [[float(Fraction(x)) for x in r] for r in seq["n_A"]],
                                       rtol=1e-12, atol=1e-14)
            np.testing.assert_allclose(nB[0], [[float(Fraction(x)) for x in r] for r in seq["n_B"]],
                                       rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------------------- brute force
@pytest.mark.parametrize("N,M,T", [(1, 3, 5), (2, 2, 6), (2, 4, 1), (3, 4, 6), (3, 2, 4), (3, 3, 2)])
def test_forward_matches_path_enumeration(oracle_mod, N, M, T):
    rng = _rng(N * 100 + M * 10 + T)
    for rep in range(3):
        pi = _dir(rng, (1,), N)
        A = _dir(rng, (1, N), N, 0.7)
        B = _dir(rng, (1, N), M, 0.7)
        o = rng.integers(0, M, size=T)
        P = bruteforce.likelihood(pi[0].tolist(), A[0].tolist(), B[0].tolist(), o.tolist())
        sym, off, lens = _one(pi, o)
        ll = oracle_mod.forward(pi, A, B, sym, off, lens, np.zeros(1, np.int32))[0]
        assert ll == pytest.approx(math.log(P), rel=1e-12, abs=1e-12)


def test_counts_match_path_enumeration(oracle_mod):
    rng = _rng(5)
    for N, M, T in [(2, 3, 5), (3, 4, 6), (3, 2, 1), (1, 2, 4), (3, 3, 3)]:
        pi = _dir(rng, (1,), N)
        A = _dir(rng, (1, N), N, 0.8)
        B = _dir(rng, (1, N), M, 0.8)
        o = rng.integers(0, M, size=T)
        P, bpi, bA, bB = bruteforce.expected_counts(pi[0].tolist(), A[0].tolist(), B[0].tolist(), o.tolist())
        sym, off, lens = _one(pi, o)
        w = np.array([1.75])
        ll, npi, nA, nB = oracle_mod.counts(pi, A, B, sym, off, lens, np.zeros(1, np.int32), weights=w)
        assert ll[0] == pytest.approx(math.log(P), rel=1e-12)
        np.testing.assert_allclose(npi[0], 1.75 * np.array(bpi), rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(nA[0], 1.75 * np.array(bA), rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(nB[0], 1.75 * np.array(bB), rtol=1e-11, atol=1e-14)


def test_brute_workload_matches_enumeration(oracle_mod):
    w = workloads.make_workload("brute")
    P = bruteforce.likelihood(w.pi[0].astype(np.float64).tolist(), w.A[0].astype(np.float64).tolist(),
                              w.B[0].astype(np.float64).tolist(), w.symbols.tolist())
    ll = oracle_mod.forward(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner)[0]
    assert ll == pytest.approx(math.log(P), rel=1e-12)


# --------------------------------------------------------------------------- probability axiom
@pytest.mark.parametrize("N,M,T", [(1, 4, 5), (2, 3, 4), (3, 4, 6), (3, 2, 6), (2, 4, 1)])
def test_probability_axiom_all_strings(oracle_mod, N, M, T):
    rng = _rng(1000 + N * 100 + M * 10 + T)
    pi = _dir(rng, (1,), N)
    A = _dir(rng, (1, N), N)
    B = _dir(rng, (1, N), M)
    strings = np.array(np.meshgrid(*[np.arange(M)] * T, indexing="ij")).reshape(T, -1).T
    S = strings.shape[0]
    sym = strings.astype(np.int32).ravel()
    off = (np.arange(S) * T).astype(np.int64)
    lens = np.full(S, T, np.int32)
    ll = oracle_mod.forward(pi, A, B, sym, off, lens, np.zeros(S, np.int32))
    assert math.fsum(np.exp(ll)) == pytest.approx(1.0, abs=1e-12)


# --------------------------------------------------------------------------- scaled invariants
def test_alpha_beta_product_is_one_every_step(oracle_mod):
    rng = _rng(11)
    for N, M, T in [(4, 6, 40), (8, 16, 200), (16, 5, 64)]:
        pi = _dir(rng, (1,), N)[0]
        A = _dir(rng, (N,), N, 0.5)
        B = _dir(rng, (N,), M, 0.5)
        o = rng.integers(0, M, size=T)
        ll, ah, bh, c = oracle_mod.trace(pi, A, B, o)
        np.testing.assert_allclose((ah * bh).sum(axis=1), 1.0, rtol=1e-12)
        np.testing.assert_allclose(ah.sum(axis=1), 1.0, rtol=1e-13)
        assert ll == pytest.approx(np.log(c).sum(), rel=1e-14)
        # unscaled alpha_t . beta_t = P for every t:  alpha_t = alphahat_t prod_{s<=t} c_s,
        # beta_t = betahat_t prod_{s>t} c_s
        logc = np.log(c)
        for t in range(T):
            la = logc[:t + 1].sum()
            lb = logc[t + 1:].sum()
            assert la + lb + np.log((ah[t] * bh[t]).sum()) == pytest.approx(ll, rel=1e-12, abs=1e-12)


def test_count_totals_and_flow_conservation(oracle_mod):
    w = workloads.random_lengths_workload(_rng(12), K=3, N=6, M=7, lengths=[1, 2, 5, 17, 33, 60, 0, 9],
                                          all_pairs=False)
    ll, npi, nA, nB = oracle_mod.counts(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner)
    for k in range(w.K):
        mine = (w.owner == k) & (w.lengths > 0)
        assert npi[k].sum() == pytest.approx(mine.sum(), rel=1e-12)
        assert nA[k].sum() == pytest.approx((w.lengths[mine] - 1).sum(), rel=1e-12)
        assert nB[k].sum() == pytest.approx(w.lengths[mine].sum(), rel=1e-12)
        # every visit to state j either starts the chain or is entered by a transition
        np.testing.assert_allclose(nB[k].sum(axis=1) - nA[k].sum(axis=0), npi[k], atol=1e-10)
        # emission counts of symbol o sum to the number of times o was observed
        sym_counts = np.zeros(w.M)
        for s in np.nonzero(mine)[0]:
            np.add.at(sym_counts, w.symbols[w.offsets[s]:w.offsets[s] + w.lengths[s]], 1.0)
        np.testing.assert_allclose(nB[k].sum(axis=0), sym_counts, atol=1e-10)


def test_counts_zero_where_parameter_zero(oracle_mod):
    rng = _rng(13)
    N, M = 5, 6
    pi = _dir(rng, (1,), N)
    A = _dir(rng, (1, N), N)
    B = _dir(rng, (1, N), M)
    A[0, 1, 3] = 0.0
    A[0, 1] /= A[0, 1].sum()
    B[0, 2, 4] = 0.0
    B[0, 2] /= B[0, 2].sum()
    o = rng.integers(0, M, size=50).astype(np.int32)
    _, npi, nA, nB = oracle_mod.counts(pi, A, B, o, np.zeros(1, np.int64), np.array([50], np.int32),
                                       np.zeros(1, np.int32))
    assert nA[0, 1, 3] == 0.0 and nB[0, 2, 4] == 0.0


# --------------------------------------------------------------------------- closed forms
def test_closed_forms(oracle_mod):
    rng = _rng(14)
    M, T = 9, 37
    o = rng.integers(0, M, size=T).astype(np.int32)
    off, lens, own = np.zeros(1, np.int64), np.array([T], np.int32), np.zeros(1, np.int32)
    # N = 1: log P = sum_t ln B(o_t)
    B1 = _dir(rng, (1, 1), M)
    ll = oracle_mod.forward(np.ones((1, 1)), np.ones((1, 1, 1)), B1, o, off, lens, own)[0]
    assert ll == pytest.approx(np.log(B1[0, 0, o]).sum(), rel=1e-13)
    # uniform emissions: log P = -T ln M for any pi, A
    N = 6
    pi = _dir(rng, (1,), N)
    A = _dir(rng, (1, N), N)
    Bu = np.full((1, N, M), 1.0 / M)
    ll = oracle_mod.forward(pi, A, Bu, o, off, lens, own)[0]
    assert ll == pytest.approx(-T * math.log(M), rel=1e-13)
    # all rows of A equal r and pi = r: i.i.d. states, log P = sum_t ln sum_i r_i B_i(o_t)
    r = _dir(rng, (1,), N)[0]
    B = _dir(rng, (1, N), M)
    ll = oracle_mod.forward(r[None], np.tile(r, (1, N, 1)), B, o, off, lens, own)[0]
    assert ll == pytest.approx(np.log(r @ B[0][:, o]).sum(), rel=1e-13)
    # identity A: the first state persists, P = sum_i pi_i prod_t B_i(o_t)
    ll = oracle_mod.forward(pi, np.eye(N)[None], B, o, off, lens, own)[0]
    expect = np.log(np.sum(pi[0] * np.exp(np.log(B[0][:, o]).sum(axis=1))))
    assert ll == pytest.approx(expect, rel=1e-12)


def _logspace_forward(pi, A, B, o):
    """Independent check: unscaled forward recursion carried in log space."""
    lpi, lA, lB = np.log(pi), np.log(A), np.log(B)
    la = lpi + lB[:, o[0]]
    for t in range(1, len(o)):
        z = la[:, None] + lA
        m = z.max(axis=0)
        la = m + np.log(np.exp(z - m).sum(axis=0)) + lB[:, o[t]]
    m = la.max()
    return m + np.log(np.exp(la - m).sum())


def test_independent_logspace_forward(oracle_mod):
    rng = _rng(15)
    for N, M, T in [(4, 4, 300), (8, 16, 64), (16, 64, 400), (32, 256, 500), (5, 6, 200)]:
        pi = _dir(rng, (1,), N)
        A = _dir(rng, (1, N), N, 0.5)
        B = _dir(rng, (1, N), M, 0.5)
        o = rng.integers(0, M, size=T).astype(np.int32)
        ll = oracle_mod.forward(pi, A, B, o, np.zeros(1, np.int64), np.array([T], np.int32),
                                np.zeros(1, np.int32))[0]
        ref = _logspace_forward(pi[0], A[0], B[0], o)
        assert ll == pytest.approx(ref, rel=1e-11)


def test_all_pairs_layout(oracle_mod):
    w = workloads.make_workload("paper", scale=0.2)
    full = oracle_mod.forward(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, None)
    for k in range(w.K):
        own = oracle_mod.forward(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, np.full(w.S, k, np.int32))
        np.testing.assert_array_equal(full[:, k], own)


# --------------------------------------------------------------------------- special cases
def test_special_lengths_and_bad_symbols(oracle_mod):
    rng = _rng(16)
    N, M = 3, 4
    pi = _dir(rng, (1,), N)
    A = _dir(rng, (1, N), N)
    B = _dir(rng, (1, N), M)
    B[0, :, 3] = 0.0          # symbol 3 is impossible
    B[0] /= B[0].sum(axis=1, keepdims=True)
    sym = np.array([0, 1, 2, 3, 0, 4, 1, -1], np.int32)
    off = np.array([0, 0, 0, 2, 4, 6, 0], np.int64)
    lens = np.array([0, 1, 2, 2, 2, 2, -1], np.int32)
    ll = oracle_mod.forward(pi, A, B, sym, off, lens, np.zeros(7, np.int32))
    assert ll[0] == 0.0                                   # T = 0
    assert ll[1] == pytest.approx(math.log(pi[0] @ B[0][:, 0]), rel=1e-14)   # T = 1
    assert np.isfinite(ll[2])
    assert ll[3] == -np.inf                               # contains the impossible symbol 3
    assert np.isnan(ll[4])                                # symbol 4 >= M
    assert np.isnan(ll[5])                                # symbol -1
    assert np.isnan(ll[6])                                # negative length
    l2, npi, nA, nB = oracle_mod.counts(pi, A, B, sym, off, lens, np.zeros(7, np.int32))
    np.testing.assert_array_equal(np.isnan(l2), np.isnan(ll))
    assert npi[0].sum() == pytest.approx(2.0)             # only the T=1 and T=2 valid sequences count
    assert nA[0].sum() == pytest.approx(1.0)


def test_classify_rules(oracle_mod):
    nan, inf = np.nan, np.inf
    ll = np.array([[1.0, 3.0, 3.0, 2.0],
                   [nan, -5.0, nan, -5.0],
                   [nan, nan, nan, nan],
                   [-inf, -inf, -inf, -inf],
                   [-inf, nan, -7.0, -inf],
                   [0.0, -0.0, 0.0, 0.0]])
    expect = np.array([1, 1, -1, 0, 2, 0], np.int32)
    np.testing.assert_array_equal(oracle_mod.classify(ll), expect)
    np.testing.assert_array_equal(oracle_mod.classify(ll.astype(np.float32)), expect)


# --------------------------------------------------------------------------- gradient
def test_softmax_gradient_rows_sum_to_zero(oracle_mod):
    w = workloads.make_workload("c4", scale=0.002)
    lpi, lA, lB = w.logits
    ll, gpi, gA, gB = oracle_mod.loglik_grad_from_logits(lpi, lA, lB, w.symbols, w.offsets, w.lengths, w.owner)
    for g in (gpi, gA, gB):
        scale = np.abs(g).max()
        np.testing.assert_allclose(g.sum(axis=-1), 0.0, atol=1e-10 * max(scale, 1.0) * g.shape[-1])


def test_gradient_matches_central_differences(oracle_mod):
    rng = _rng(17)
    K, N, M = 2, 4, 5
    lpi = rng.standard_normal((K, N))
    lA = rng.standard_normal((K, N, N))
    lB = rng.standard_normal((K, N, M))
    pi, A, B = oracle_mod.softmax(lpi), oracle_mod.softmax(lA), oracle_mod.softmax(lB)
    lengths = np.array([7, 1, 12, 30, 3, 18], np.int32)
    owner = (np.arange(6) % K).astype(np.int32)
    sym, off = workloads.sample_sequences(rng, pi.astype(np.float32), A.astype(np.float32),
                                          B.astype(np.float32), owner, lengths)
    wts = rng.uniform(0.5, 2.0, size=6)
    _, gpi, gA, gB = oracle_mod.loglik_grad_from_logits(lpi, lA, lB, sym, off, lengths, owner, weights=wts)
    h = 1e-3

    def f(a, b, c):
        return oracle_mod.objective_from_logits(a, b, c, sym, off, lengths, owner, weights=wts)

    for which, (arr, g) in enumerate([(lpi, gpi), (lA, gA), (lB, gB)]):
        fd = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            args = [lpi.copy(), lA.copy(), lB.copy()]
            args[which][idx] += h
            fp = f(*args)
            args[which][idx] -= 2 * h
            fm = f(*args)
            fd[idx] = (fp - fm) / (2 * h)
        np.testing.assert_allclose(g, fd, rtol=1e-5, atol=2e-6)


def test_oracle_thread_count_does_not_change_results(oracle_mod):
    w = workloads.make_workload("c2", scale=0.02)
    a = oracle_mod.forward(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, None, nthreads=1)
    b = oracle_mod.forward(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, None, nthreads=4)
    np.testing.assert_array_equal(a, b)
