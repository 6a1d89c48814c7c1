"""Write exact_small.json: exact rational likelihoods and expected counts.

Every stored value is produced here by oracle/bruteforce.py (enumeration of all
state paths) in exact rational arithmetic, from small rational model banks
chosen below.  Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
from fractions import Fraction

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
from oracle import bruteforce  # noqa: E402


def rational_row(weights):
    s = sum(weights)
    return [Fraction(w, s) for w in weights]


CASES = [
    # name, pi weights, A weights, B weights, symbol strings
    ("two_state_sticky",
     [1, 3], [[7, 1], [2, 5]], [[9, 1], [1, 4]],
     [[0], [1, 1], [0, 1, 0], [1, 0, 0, 1, 1], [0, 0, 1, 1, 0, 1]]),
    ("three_state_asym",
     [2, 1, 5], [[1, 6, 1], [3, 1, 4], [2, 2, 7]], [[5, 1, 1, 2], [1, 7, 2, 1], [1, 1, 1, 9]],
     [[3], [0, 2], [1, 3, 0], [2, 2, 1, 0], [3, 0, 1, 2, 3, 1]]),
    ("three_state_zeros",
     [1, 0, 2], [[0, 3, 1], [1, 0, 1], [4, 1, 0]], [[1, 0, 3], [0, 2, 1], [5, 1, 0]],
     [[0], [2, 1], [0, 1, 2], [1, 1, 0, 2], [2, 0, 1, 1, 0, 2]]),
]


def fr(x):
    return f"{x.numerator}/{x.denominator}"


def main():
    out = []
    for name, pw, Aw, Bw, strings in CASES:
        pi = rational_row(pw)
        A = [rational_row(r) for r in Aw]
        B = [rational_row(r) for r in Bw]
        seqs = []
        for o in strings:
            P, n_pi, n_A, n_B = bruteforce.expected_counts(pi, A, B, o)
            seqs.append({"symbols": o, "P": fr(P),
                         "n_pi": [fr(x) for x in n_pi],
                         "n_A": [[fr(x) for x in r] for r in n_A],
                         "n_B": [[fr(x) for x in r] for r in n_B]})
        out.append({"name": name, "pi": [fr(x) for x in pi], "A": [[fr(x) for x in r] for r in A],
                    "B": [[fr(x) for x in r] for r in B], "sequences": seqs})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_small.json")
    with open(path, "w") as f:
        json.dump({"source": "oracle/bruteforce.py enumeration, exact rationals; textbook discrete-HMM "
                             "definition used for the forward / Baum-Welch functions of the paper's "
                             "activity-recognition stage (Sec. 2.7)",
                   "cases": out}, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
