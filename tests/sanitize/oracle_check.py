"""Runs the FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer on
small workloads and special inputs, and compares every output with the ordinary
build (run by tests/test_sanitizers.py in a process that preloads the sanitizer
runtime).

    python tests/sanitize/oracle_check.py SANITIZED_LIB
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1310_3322_amd import workloads  # noqa: E402


def same(a, b, what):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, what
    assert np.array_equal(np.isnan(a), np.isnan(b)), what
    fin = ~np.isnan(a)
    assert np.array_equal(a[fin], b[fin]), what


def special(w):
    """Copies of w's symbols and lengths with an empty sequence and an invalid symbol."""
    sym = w.symbols.copy()
    lengths = w.lengths.copy()
    owner = w.owner.copy()
    if w.S > 3:
        lengths[0] = 0
        sym[w.offsets[1]] = w.M          # symbol outside [0, M)
    return sym, lengths, owner


def main(path):
    san = O.load_library(path)
    ref = O.load_library(O.build(force=False))
    cases = [workloads.make_workload("brute"), workloads.make_workload("c1"), workloads.make_workload("paper"),
             workloads.make_workload("c2", scale=0.02), workloads.make_workload("c4", scale=0.001),
             workloads.random_lengths_workload(np.random.default_rng(5), K=2, N=130, M=17,
                                               lengths=[0, 1, 5, 33, 40, 2], all_pairs=False, conc=0.3)]
    n = 0
    for w in cases:
        for sym, lengths, owner in ((w.symbols, w.lengths, w.owner), special(w)):
            args = (w.pi, w.A, w.B, sym, w.offsets, lengths)
            same(O.forward(*args, None, lib=san), O.forward(*args, None, lib=ref), f"{w.name} forward all pairs")
            same(O.forward(*args, owner, lib=san), O.forward(*args, owner, lib=ref), f"{w.name} forward own")
            wts = np.linspace(-1.0, 2.0, w.S)
            for a, b in zip(O.counts(*args, owner, wts, lib=san), O.counts(*args, owner, wts, lib=ref)):
                same(a, b, f"{w.name} counts")
            for a, b in zip(O.viterbi(*args, owner, lib=san), O.viterbi(*args, owner, lib=ref)):
                same(a, b, f"{w.name} viterbi")
            s0 = int(np.argmax(w.lengths))
            o = sym[w.offsets[s0]:w.offsets[s0] + w.lengths[s0]]
            o = np.where((o >= 0) & (o < w.M), o, 0)
            for a, b in zip(O.trace(w.pi[0], w.A[0], w.B[0], o, lib=san), O.trace(w.pi[0], w.A[0], w.B[0], o, lib=ref)):
                same(a, b, f"{w.name} trace")
            n += 1
    print(f"oracle under sanitizers: {n} cases identical to the ordinary build", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
