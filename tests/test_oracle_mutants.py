"""The pins are sharp: each plausible mistake planted in a copy of the oracle fails one.

Each mutant is a textual edit of oracle/hmm_oracle.c (a transposed operand, a
dropped term, a wrong time index, a wrong log base, a missing weight ...),
compiled with gcc into a temporary library.  The checks below are the same
mathematical pins as in test_oracle_pins.py, phrased as predicates; every
mutant must violate at least one of them while the real oracle passes all.
"""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import bruteforce
from oracle import oracle as O
from paper_1310_3322_amd import workloads

SRC = os.path.join(os.path.dirname(O.__file__), "hmm_oracle.c")

MUTANTS = {
    "transpose_A_forward": ("u += ahat[i] * A[(size_t)i * N + j];", "u += ahat[i] * A[(size_t)j * N + i];"),
    "transpose_A_trace": ("u += ap[i] * A[(size_t)i * N + j];", "u += ap[i] * A[(size_t)j * N + i];"),
    "drop_pi_forward": ("atil[i] = pi[i] * B[(size_t)i * M + o[0]];", "atil[i] = B[(size_t)i * M + o[0]];"),
    "drop_pi_trace": ("at[i] = pi[i] * B[(size_t)i * M + o[0]];", "at[i] = B[(size_t)i * M + o[0]];"),
    "emission_time_shift": ("atil[j] = u * B[(size_t)j * M + o[t]];", "atil[j] = u * B[(size_t)j * M + o[t - 1]];"),
    "emission_row_col_swap": ("atil[j] = u * B[(size_t)j * M + o[t]];", "atil[j] = u * B[(size_t)o[t] * N + j];"),
    "log_base2": ("loglik += log(c);", "loglik += log2(c);"),
    "no_renormalise": ("ahat[i] = atil[i] / c;", "ahat[i] = atil[i];"),
    "backward_scale_index": ("* bn[j] / c[t + 1]);", "* bn[j] / c[t]);"),
    "backward_transpose_A": ("acc += A[(size_t)i * N + j] * (B", "acc += A[(size_t)j * N + i] * (B"),
    "xi_transpose_A": ("ws * at[i] * Ak[(size_t)i * N + j] * w;", "ws * at[i] * Ak[(size_t)j * N + i] * w;"),
    "xi_drop_A": ("ws * at[i] * Ak[(size_t)i * N + j] * w;", "ws * at[i] * w;"),
    "gamma_emission_time": ("nB[(size_t)i * M + o[t]] += ws * g;", "nB[(size_t)i * M + o[t > 0 ? t - 1 : 0]] += ws * g;"),
    "pi_count_unweighted": ("if (t == 0) npi[i] += ws * g;", "if (t == 0) npi[i] += g;"),
    "pi_count_last_step": ("if (t == 0) npi[i] += ws * g;", "if (t == T - 1) npi[i] += ws * g;"),
    "zero_prob_not_inf": ("if (c == 0.0) return -INFINITY;", "if (c == 0.0) return 0.0;"),
    "argmax_last_tie": ("if (best < 0 || v > bv) {\n                best = k;\n                bv = v;\n            }\n        }\n        labels[s] = best;\n    }\n}\n\n/* Same",
                        "if (best < 0 || v >= bv) {\n                best = k;\n                bv = v;\n            }\n        }\n        labels[s] = best;\n    }\n}\n\n/* Same"),
    "viterbi_transpose_A": ("const double cand = dp[i] + log(Ak[(size_t)i * N + j]);",
                            "const double cand = dp[i] + log(Ak[(size_t)j * N + i]);"),
    "viterbi_drop_first_emission": ("delta[i] = log(pk[i]) + log(Bk[(size_t)i * M + o[0]]);",
                                    "delta[i] = log(pk[i]);"),
    "viterbi_emission_time_shift": ("dt[j] = best + log(Bk[(size_t)j * M + o[t]]);",
                                    "dt[j] = best + log(Bk[(size_t)j * M + o[t - 1]]);"),
    "viterbi_step_tie_last": ("if (cand > best) {", "if (cand >= best) {"),
    "viterbi_final_tie_last": ("if (dl[j] > best) {", "if (dl[j] >= best) {"),
    "viterbi_margin_drop_A": ("const double chosen = dp[c] + log(Ak[(size_t)c * N + j]);",
                              "const double chosen = dp[c];"),
    "viterbi_margin_final_only": ("for (int32_t t = T - 1; t > 0; --t) {\n                    const double *dp",
                                  "for (int32_t t = 0; t > 0; --t) {\n                    const double *dp"),
    "viterbi_margin_row_index": ("const double *dp = delta + (size_t)(t - 1) * N;\n                    const int j = q[t]",
                                 "const double *dp = delta + (size_t)t * N;\n                    const int j = q[t]"),
}


def _build_mutant(name, tmpdir):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    path_c = os.path.join(tmpdir, f"{name}.c")
    path_so = os.path.join(tmpdir, f"{name}.so")
    open(path_c, "w").write(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", path_so, path_c, "-lm"])
    return O.load_library(path_so)


def _rng(tag):
    return np.random.default_rng([1310, 3322, 99, tag])


def pin_bruteforce(lib):
    rng = _rng(1)
    for N, M, T in [(3, 4, 6), (2, 3, 5), (3, 2, 1)]:
        pi = workloads.dirichlet_rows(rng, (1,), N, 0.7)
        A = workloads.dirichlet_rows(rng, (1, N), N, 0.7)
        B = workloads.dirichlet_rows(rng, (1, N), M, 0.7)
        o = rng.integers(0, M, size=T).astype(np.int32)
        P = bruteforce.likelihood(pi[0].tolist(), A[0].tolist(), B[0].tolist(), o.tolist())
        ll = O.forward(pi, A, B, o, np.zeros(1, np.int64), np.array([T], np.int32), np.zeros(1, np.int32), lib=lib)[0]
        if not abs(ll - math.log(P)) <= 1e-12 * max(1.0, abs(ll)):
            return False
        P2, bpi, bA, bB = bruteforce.expected_counts(pi[0].tolist(), A[0].tolist(), B[0].tolist(), o.tolist())
        w = np.array([1.5])
        _, npi, nA, nB = O.counts(pi, A, B, o, np.zeros(1, np.int64), np.array([T], np.int32),
                                  np.zeros(1, np.int32), weights=w, lib=lib)
        for got, ref in ((npi[0], bpi), (nA[0], bA), (nB[0], bB)):
            if not np.allclose(got, 1.5 * np.array(ref), rtol=1e-10, atol=1e-13):
                return False
    return True


def pin_trace_invariant(lib):
    rng = _rng(2)
    N, M, T = 5, 7, 30
    pi = workloads.dirichlet_rows(rng, (1,), N, 1.0)[0]
    A = workloads.dirichlet_rows(rng, (N,), N, 0.5)
    B = workloads.dirichlet_rows(rng, (N,), M, 0.5)
    o = rng.integers(0, M, size=T).astype(np.int32)
    ll, ah, bh, c = O.trace(pi, A, B, o, lib=lib)
    P = O.forward(pi[None], A[None], B[None], o, np.zeros(1, np.int64), np.array([T], np.int32),
                  np.zeros(1, np.int32), lib=lib)[0]
    return bool(np.allclose((ah * bh).sum(axis=1), 1.0, rtol=1e-12) and abs(ll - P) < 1e-10 * abs(P))


def pin_axiom(lib):
    rng = _rng(3)
    N, M, T = 3, 3, 4
    pi = workloads.dirichlet_rows(rng, (1,), N, 1.0)
    A = workloads.dirichlet_rows(rng, (1, N), N, 1.0)
    B = workloads.dirichlet_rows(rng, (1, N), M, 1.0)
    strings = np.array(np.meshgrid(*[np.arange(M)] * T, indexing="ij")).reshape(T, -1).T
    S = strings.shape[0]
    ll = O.forward(pi, A, B, strings.astype(np.int32).ravel(), (np.arange(S) * T).astype(np.int64),
                   np.full(S, T, np.int32), np.zeros(S, np.int32), lib=lib)
    return abs(math.fsum(np.exp(ll)) - 1.0) < 1e-12


def pin_impossible(lib):
    pi = np.array([[0.5, 0.5]])
    A = np.array([[[0.5, 0.5], [0.5, 0.5]]])
    B = np.array([[[1.0, 0.0], [1.0, 0.0]]])
    ll = O.forward(pi, A, B, np.array([0, 1], np.int32), np.zeros(1, np.int64), np.array([2], np.int32),
                   np.zeros(1, np.int32), lib=lib)[0]
    return ll == -np.inf


def pin_classify(lib):
    ll = np.array([[1.0, 3.0, 3.0, 2.0], [np.nan, -5.0, np.nan, -5.0]])
    S, K = ll.shape
    labels = np.empty(S, dtype=np.int32)
    lib.oracle_classify(S, K, O._ptr(np.ascontiguousarray(ll), O._dp), O._ptr(labels, O._i32p))
    return labels.tolist() == [1, 1]


def pin_viterbi(lib):
    rng = _rng(4)
    for N, M, T in [(3, 4, 6), (2, 3, 5), (3, 3, 1)]:
        pi = workloads.dirichlet_rows(rng, (1,), N, 0.7)
        A = workloads.dirichlet_rows(rng, (1, N), N, 0.7)
        B = workloads.dirichlet_rows(rng, (1, N), M, 0.7)
        o = rng.integers(0, M, size=T).astype(np.int32)
        best, args = bruteforce.best_paths(pi[0].tolist(), A[0].tolist(), B[0].tolist(), o.tolist())
        sc, path, _ = O.viterbi(pi, A, B, o, np.zeros(1, np.int64), np.array([T], np.int32), np.zeros(1, np.int32),
                                lib=lib)
        if not abs(sc[0] - math.log(best)) <= 1e-12 * max(1.0, abs(sc[0])) or tuple(path.tolist()) not in args:
            return False
    # every path ties under a uniform model: the smallest-index rule gives all zeros
    N, M, T = 3, 2, 4
    u = lambda *shape: np.full(shape, 1.0 / shape[-1])
    _, path, _ = O.viterbi(u(1, N), u(1, N, N), u(1, N, M), np.array([0, 1, 1, 0], np.int32), np.zeros(1, np.int64),
                           np.array([T], np.int32), np.zeros(1, np.int32), lib=lib)
    return path.tolist() == [0] * T


def pin_viterbi_margin(lib):
    rng = _rng(5)
    for N, M, T in [(3, 4, 6), (2, 3, 5), (3, 3, 4)]:
        for _ in range(3):
            pi = workloads.dirichlet_rows(rng, (1,), N, 0.5)
            A = workloads.dirichlet_rows(rng, (1, N), N, 0.5)
            B = workloads.dirichlet_rows(rng, (1, N), M, 0.5)
            o = rng.integers(0, M, size=T).astype(np.int32)
            sc, path, mg = O.viterbi(pi, A, B, o, np.zeros(1, np.int64), np.array([T], np.int32),
                                     np.zeros(1, np.int32), lib=lib)
            ref = bruteforce.path_margin(pi[0].tolist(), A[0].tolist(), B[0].tolist(), o.tolist(), path.tolist())
            if not abs(mg[0] - ref) <= 1e-10 * max(1.0, abs(sc[0])):
                return False
    return True


PINS = [pin_bruteforce, pin_trace_invariant, pin_axiom, pin_impossible, pin_classify, pin_viterbi,
        pin_viterbi_margin]


def test_real_oracle_passes_every_predicate():
    lib = O.load_library(O.build(force=False))
    for pin in PINS:
        assert pin(lib), pin.__name__


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    with tempfile.TemporaryDirectory() as d:
        lib = _build_mutant(name, d)
        failed = [p.__name__ for p in PINS if not p(lib)]
        assert failed, f"mutant {name} passed every pin"
