"""Pins of the oracle's Viterbi decoder (CPU): the most likely state path.

The Viterbi function of the paper's HMM stage (Sec. 2.7) is checked against
path enumeration (exact rationals and floats), closed forms, the tie rule
(smallest index), bounds against the forward likelihood, and special inputs.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import bruteforce
from paper_1310_3322_amd import workloads


def one(oracle_mod, pi, A, B, o):
    o = np.asarray(o, np.int32)
    sc, path, mg = oracle_mod.viterbi(np.asarray(pi)[None], np.asarray(A)[None], np.asarray(B)[None], o,
                                      np.zeros(1, np.int64), np.array([len(o)], np.int32), np.zeros(1, np.int32))
    return sc[0], path, mg[0]


def joint_log(pi, A, B, q, o):
    s = math.log(pi[q[0]]) + math.log(B[q[0]][o[0]])
    for t in range(1, len(o)):
        s += math.log(A[q[t - 1]][q[t]]) + math.log(B[q[t]][o[t]])
    return s


@pytest.mark.parametrize("N,M,T", [(3, 4, 6), (2, 3, 7), (3, 2, 1), (1, 3, 5), (3, 3, 2)])
def test_viterbi_matches_path_enumeration(oracle_mod, N, M, T):
    rng = np.random.default_rng([17, N, M, T])
    for rep in range(4):
        pi = workloads.dirichlet_rows(rng, (1,), N, 0.6)[0]
        A = workloads.dirichlet_rows(rng, (N,), N, 0.6)
        B = workloads.dirichlet_rows(rng, (N,), M, 0.6)
        o = rng.integers(0, M, size=T).astype(np.int32)
        best, args = bruteforce.best_paths(pi.tolist(), A.tolist(), B.tolist(), o.tolist())
        sc, path, mg = one(oracle_mod, pi, A, B, o)
        assert abs(sc - math.log(best)) <= 1e-12 * max(1.0, abs(sc))
        assert tuple(path.tolist()) in args
        if len(args) == 1:
            assert tuple(path.tolist()) == args[0]


@pytest.mark.parametrize("N,M,T", [(3, 4, 6), (2, 3, 7), (3, 2, 1), (3, 3, 2), (2, 2, 5)])
def test_viterbi_margin_matches_second_best_path(oracle_mod, N, M, T):
    """The margin the oracle reports (smallest gap over the final choice and every
    backtracking choice on its path) equals, by enumeration of all N^T paths, the
    log-probability of the decoded path minus that of the best other path."""
    rng = np.random.default_rng([29, N, M, T])
    for rep in range(6):
        conc = 0.3 if rep % 2 else 1.0
        pi = workloads.dirichlet_rows(rng, (1,), N, conc)[0]
        A = workloads.dirichlet_rows(rng, (N,), N, conc)
        B = workloads.dirichlet_rows(rng, (N,), M, conc)
        o = rng.integers(0, M, size=T).astype(np.int32)
        sc, path, mg = one(oracle_mod, pi, A, B, o)
        ref = bruteforce.path_margin(pi.tolist(), A.tolist(), B.tolist(), o.tolist(), path.tolist())
        assert ref >= 0.0
        assert abs(mg - ref) <= 1e-10 * max(1.0, abs(sc)), (rep, mg, ref)


def test_viterbi_margin_special_cases(oracle_mod):
    """Zero where the best path is not unique (a tie at the final state or at one
    backtracking step), +inf for one state, and the exact gap of a model whose two
    best paths differ by a known factor."""
    # tie at the final choice only: two end states equally likely, predecessors unique
    pi = np.array([0.6, 0.4])
    A = np.array([[0.5, 0.5], [0.5, 0.5]])
    B = np.array([[0.5, 0.5], [0.5, 0.5]])
    _, path, mg = one(oracle_mod, pi, A, B, [0, 1])
    assert mg == 0.0 and path.tolist() == [0, 0]
    # tie at a backtracking choice only: both predecessors of state 1 give the same value
    pi = np.array([0.5, 0.5])
    A = np.array([[0.2, 0.8], [0.2, 0.8]])
    B = np.array([[0.5, 0.5], [0.5, 0.5]])
    _, path, mg = one(oracle_mod, pi, A, B, [0, 0])
    assert mg == 0.0 and path.tolist() == [0, 1]
    # one state: the only path, infinite margin
    _, _, mg = one(oracle_mod, np.array([1.0]), np.array([[1.0]]), np.array([[0.25, 0.75]]), [1, 0, 1])
    assert mg == math.inf
    # dyadic bank: best path 0,0 has P = 1/2 * 3/4 * 1/2 * 1/2, second best differs by ln 3 exactly
    pi = np.array([0.5, 0.5])
    A = np.array([[0.75, 0.25], [0.5, 0.5]])
    B = np.array([[0.5, 0.5], [0.25, 0.75]])
    sc, path, mg = one(oracle_mod, pi, A, B, [0, 0])
    ref = bruteforce.path_margin(pi.tolist(), A.tolist(), B.tolist(), [0, 0], path.tolist())
    assert path.tolist() == [0, 0]
    assert abs(mg - math.log(3.0)) <= 1e-14 and abs(ref - math.log(3.0)) <= 1e-14


def test_viterbi_exact_rational_enumeration(oracle_mod):
    """A bank of small dyadic rationals (exact in FP64): the max over paths is exact."""
    pi = [Fraction(1, 4), Fraction(1, 2), Fraction(1, 4)]
    A = [[Fraction(1, 2), Fraction(1, 4), Fraction(1, 4)], [Fraction(1, 8), Fraction(5, 8), Fraction(1, 4)],
         [Fraction(3, 4), Fraction(1, 8), Fraction(1, 8)]]
    B = [[Fraction(1, 2), Fraction(1, 2)], [Fraction(7, 8), Fraction(1, 8)], [Fraction(1, 16), Fraction(15, 16)]]
    o = [0, 1, 1, 0, 0]
    best, args = bruteforce.best_paths(pi, A, B, o)
    f = lambda X: np.array([[float(x) for x in row] for row in X]) if isinstance(X[0], list) else np.array(
        [float(x) for x in X])
    sc, path, _ = one(oracle_mod, f(pi), f(A), f(B), o)
    assert len(args) == 1
    assert tuple(path.tolist()) == args[0]
    assert abs(sc - math.log(float(best))) <= 1e-14 * abs(sc)


def test_viterbi_tie_rule_smallest_index(oracle_mod):
    """Uniform model: every path ties; the rule yields the all-zero path."""
    N, M, T = 4, 3, 6
    pi = np.full(N, 1.0 / N)
    A = np.full((N, N), 1.0 / N)
    B = np.full((N, M), 1.0 / M)
    sc, path, mg = one(oracle_mod, pi, A, B, [2, 0, 1, 1, 0, 2])
    assert path.tolist() == [0] * T
    assert abs(sc - T * (math.log(1.0 / N) + math.log(1.0 / M))) < 1e-12
    assert mg == 0.0
    # two equally good final states, the smaller one wins; the path follows its predecessors
    pi = np.array([0.5, 0.5])
    A = np.array([[0.5, 0.5], [0.5, 0.5]])
    B = np.array([[0.9, 0.1], [0.9, 0.1]])
    sc, path, _ = one(oracle_mod, pi, A, B, [0, 0, 0])
    assert path.tolist() == [0, 0, 0]


def test_viterbi_closed_forms(oracle_mod):
    rng = np.random.default_rng(23)
    # N = 1: the only path
    B = workloads.dirichlet_rows(rng, (1,), 5, 1.0)
    o = rng.integers(0, 5, size=9)
    sc, path, mg = one(oracle_mod, np.array([1.0]), np.array([[1.0]]), B, o)
    assert path.tolist() == [0] * 9 and mg == math.inf
    assert abs(sc - sum(math.log(B[0][x]) for x in o)) < 1e-12
    # A = I: the path is constant at argmax_i ln pi_i + sum_t ln B_i(o_t)
    N, M, T = 5, 6, 12
    pi = workloads.dirichlet_rows(rng, (1,), N, 1.0)[0]
    B = workloads.dirichlet_rows(rng, (N,), M, 1.0)
    o = rng.integers(0, M, size=T)
    sc, path, _ = one(oracle_mod, pi, np.eye(N), B, o)
    per = [math.log(pi[i]) + sum(math.log(B[i][x]) for x in o) for i in range(N)]
    best = int(np.argmax(per))
    assert path.tolist() == [best] * T
    assert abs(sc - per[best]) < 1e-12 * abs(sc)
    # one-hot emissions (state i emits symbol i): the path is the symbol string
    N = 4
    A = workloads.dirichlet_rows(rng, (N,), N, 1.0)
    pi = workloads.dirichlet_rows(rng, (1,), N, 1.0)[0]
    o = rng.integers(0, N, size=15)
    sc, path, _ = one(oracle_mod, pi, A, np.eye(N), o)
    assert path.tolist() == o.tolist()
    assert abs(sc - joint_log(pi, A, np.eye(N), o.tolist(), o.tolist())) < 1e-12


def test_viterbi_bounded_by_forward(oracle_mod):
    """max_Q P(Q, O) <= P(O) <= N^T max_Q P(Q, O), and the decoded path attains the score."""
    w = workloads.make_workload("paper")
    own = w.subset(np.arange(40))
    sc, path, mg = oracle_mod.viterbi(own.pi, own.A, own.B, own.symbols, own.offsets, own.lengths, own.owner)
    ll = oracle_mod.forward(own.pi, own.A, own.B, own.symbols, own.offsets, own.lengths, own.owner)
    assert np.all(sc <= ll + 1e-9)
    assert np.all(ll <= sc + own.lengths * math.log(own.N) + 1e-9)
    A64, B64, p64 = (np.asarray(x, np.float64) for x in (own.A, own.B, own.pi))
    for s in range(own.S):
        k, T, off = own.owner[s], own.lengths[s], own.offsets[s]
        q = path[off:off + T].tolist()
        o = own.symbols[off:off + T].tolist()
        assert abs(joint_log(p64[k], A64[k], B64[k], q, o) - sc[s]) <= 1e-9 * abs(sc[s])
        assert mg[s] >= 0.0


def test_viterbi_special_inputs(oracle_mod):
    pi = np.array([[0.5, 0.5]])
    A = np.array([[[0.5, 0.5], [0.5, 0.5]]])
    B = np.array([[[1.0, 0.0], [1.0, 0.0]]])
    sym = np.array([0, 1, 0, 0, 5, 0], np.int32)
    off = np.array([0, 2, 2, 4], np.int64)
    lens = np.array([2, 0, 2, 2], np.int32)
    sc, path, mg = oracle_mod.viterbi(pi, A, B, sym, off, lens, np.zeros(4, np.int32))
    assert sc[0] == -math.inf                       # impossible observation
    assert sc[1] == 0.0                             # empty sequence
    assert abs(sc[2] - (math.log(0.5) + math.log(0.5))) < 1e-15 and path[2:4].tolist() == [0, 0]
    assert math.isnan(sc[3]) and path[4:6].tolist() == [-1, -1]   # invalid symbol
    assert path[0:2].tolist() == [0, 0]             # all -inf: smallest index everywhere


def test_viterbi_thread_count_invariant(oracle_mod):
    w = workloads.make_workload("c2", scale=0.02)
    a = oracle_mod.viterbi(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner, nthreads=1)
    b = oracle_mod.viterbi(w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths, w.owner, nthreads=4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
