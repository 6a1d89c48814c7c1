"""The plain definitions, by enumeration (TEST INFRASTRUCTURE ONLY).

These functions write the discrete-HMM quantities out as sums over every
hidden state path, with no recursion at all, so that the forward / backward
oracle in hmm_oracle.c can be checked against something other than itself.
They accept Python floats or fractions.Fraction (exact arithmetic); they are
exponential in T and meant for N <= 3, T <= 6.

  P(O | lambda) = sum_Q pi[q_1] B[q_1][o_1] prod_{t>=2} A[q_{t-1}][q_t] B[q_t][o_t]

Expected counts under the posterior P(Q | O) = P(Q, O) / P(O):
  n_pi[i]   = E[ [q_1 = i] ]
  n_A[i][j] = E[ #{t < T : q_t = i, q_{t+1} = j} ]
  n_B[i][o] = E[ #{t : q_t = i, o_t = o} ]
These are the gradient of log P(O | lambda) with respect to ln pi, ln A, ln B.
"""
from __future__ import annotations

import itertools


def joint(pi, A, B, q, o):
    """P(Q = q, O = o | lambda) for one state path q."""
    p = pi[q[0]] * B[q[0]][o[0]]
    for t in range(1, len(o)):
        p = p * A[q[t - 1]][q[t]] * B[q[t]][o[t]]
    return p


def likelihood(pi, A, B, o):
    """P(O = o | lambda) as the sum over all N^T state paths (1 for T = 0)."""
    N = len(pi)
    T = len(o)
    if T == 0:
        return 1 if not isinstance(pi[0], float) else 1.0
    total = 0
    for q in itertools.product(range(N), repeat=T):
        total = total + joint(pi, A, B, q, o)
    return total


def total_over_strings(pi, A, B, M, T):
    """sum over all M^T symbol strings of P(O | lambda) (equals 1 for a proper model)."""
    total = 0
    for o in itertools.product(range(M), repeat=T):
        total = total + likelihood(pi, A, B, o)
    return total


def expected_counts(pi, A, B, o):
    """(P(O), n_pi[N], n_A[N][N], n_B[N][M]) by enumerating every state path."""
    N = len(pi)
    M = len(B[0])
    T = len(o)
    zero = 0 * pi[0]
    n_pi = [zero] * N
    n_A = [[zero] * N for _ in range(N)]
    n_B = [[zero] * M for _ in range(N)]
    P = zero
    for q in itertools.product(range(N), repeat=T):
        w = joint(pi, A, B, q, o)
        P = P + w
        n_pi[q[0]] = n_pi[q[0]] + w
        for t in range(T):
            n_B[q[t]][o[t]] = n_B[q[t]][o[t]] + w
            if t + 1 < T:
                n_A[q[t]][q[t + 1]] = n_A[q[t]][q[t + 1]] + w
    n_pi = [x / P for x in n_pi]
    n_A = [[x / P for x in row] for row in n_A]
    n_B = [[x / P for x in row] for row in n_B]
    return P, n_pi, n_A, n_B


def best_paths(pi, A, B, o):
    """(max_Q P(Q, O), every state path attaining it) by enumerating all N^T paths.

    This is the quantity the Viterbi function of the paper's HMM stage decodes: the most
    likely hidden state path for an observed symbol string."""
    N = len(pi)
    T = len(o)
    best = None
    arg = []
    for q in itertools.product(range(N), repeat=T):
        p = joint(pi, A, B, q, o)
        if best is None or p > best:
            best, arg = p, [q]
        elif p == best:
            arg.append(q)
    return best, arg


def path_margin(pi, A, B, o, q):
    """ln P(Q = q, O) minus the largest ln P(Q, O) over every other state path Q != q
    (+inf when q is the only path, -inf .. 0 when another path is at least as likely).

    For q the decoded most likely path this is the decoding margin: how much the
    log-probability would have to move before another path wins.  It is zero when the
    most likely path is not unique.  Floats only (logarithms)."""
    import math

    N = len(pi)
    T = len(o)
    q = tuple(q)
    own = joint(pi, A, B, q, o)
    other = None
    for p in itertools.product(range(N), repeat=T):
        if p == q:
            continue
        v = joint(pi, A, B, p, o)
        if other is None or v > other:
            other = v
    if other is None:
        return math.inf
    lo = math.log(own) if own > 0 else -math.inf
    lx = math.log(other) if other > 0 else -math.inf
    if lo == -math.inf and lx == -math.inf:
        return 0.0
    return lo - lx
