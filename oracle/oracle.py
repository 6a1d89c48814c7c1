"""Python handle on the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this module.  It loads `hmm_oracle.c` (compiled with gcc on
first use, or by `build()`), upcasts the FP32 model bank exactly to FP64, and
adds the two small pieces of the gradient definition that live outside the C
file: the softmax parameterisation and the map from expected counts to
logit gradients.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no fast-math) and OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    lib.oracle_forward.restype = ctypes.c_int
    lib.oracle_forward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp,
                                   ctypes.c_int, _i32p, _i64p, _i32p, _i32p, _dp, ctypes.c_int]
    lib.oracle_classify.restype = None
    lib.oracle_classify.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _i32p]
    lib.oracle_classify_f32.restype = None
    lib.oracle_classify_f32.argtypes = [ctypes.c_int, ctypes.c_int, _fp, _i32p]
    lib.oracle_trace.restype = ctypes.c_double
    lib.oracle_trace.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _i32p, ctypes.c_int32,
                                 _dp, _dp, _dp]
    lib.oracle_counts.restype = ctypes.c_int
    lib.oracle_counts.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp,
                                  ctypes.c_int, _i32p, _i64p, _i32p, _i32p, _dp, _dp,
                                  _dp, _dp, _dp, ctypes.c_int]
    lib.oracle_viterbi.restype = ctypes.c_int
    lib.oracle_viterbi.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int,
                                   _i32p, _i64p, _i32p, _i32p, _dp, _i32p, _dp, ctypes.c_int]
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    return lib


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def load_library(path: str):
    """Bind another build of hmm_oracle.c (used by the tests that plant mistakes)."""
    return _bind(ctypes.CDLL(path))


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else ctypes.cast(None, t)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def forward(pi, A, B, symbols, offsets, lengths, model_of_seq=None, nthreads: int = 0, lib=None) -> np.ndarray:
    """log P(O_s | lambda_k) in FP64.

    model_of_seq None: [S][K] (every sequence against every model);
    otherwise [S] (each sequence against its own model).
    """
    pi, A, B = _f64(pi), _f64(A), _f64(B)
    K, N = pi.shape
    M = B.shape[2]
    assert A.shape == (K, N, N) and B.shape == (K, N, M)
    sym = np.ascontiguousarray(symbols, dtype=np.int32)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    lens = np.ascontiguousarray(lengths, dtype=np.int32)
    S = lens.shape[0]
    mos = None if model_of_seq is None else np.ascontiguousarray(model_of_seq, dtype=np.int32)
    out = np.empty((S,) if mos is not None else (S, K), dtype=np.float64)
    rc = (lib or _load()).oracle_forward(K, N, M, _ptr(pi, _dp), _ptr(A, _dp), _ptr(B, _dp), S,
                                _ptr(sym, _i32p), _ptr(off, _i64p), _ptr(lens, _i32p),
                                _ptr(mos, _i32p), _ptr(out, _dp), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_forward: bad arguments")
    return out


def classify(loglik: np.ndarray) -> np.ndarray:
    """Smallest index of the maximum per row; NaN skipped; all-NaN row -> -1."""
    ll = np.ascontiguousarray(loglik)
    S, K = ll.shape
    labels = np.empty(S, dtype=np.int32)
    if ll.dtype == np.float32:
        _load().oracle_classify_f32(S, K, _ptr(ll, _fp), _ptr(labels, _i32p))
    else:
        ll = _f64(ll)
        _load().oracle_classify(S, K, _ptr(ll, _dp), _ptr(labels, _i32p))
    return labels


def trace(pi, A, B, symbols, lib=None):
    """(loglik, alphahat[T][N], betahat[T][N], c[T]) of one sequence under one model."""
    pi, A, B = _f64(pi), _f64(A), _f64(B)
    N = pi.shape[0]
    M = B.shape[1]
    o = np.ascontiguousarray(symbols, dtype=np.int32)
    T = o.shape[0]
    ah = np.zeros((max(T, 1), N))
    bh = np.zeros((max(T, 1), N))
    c = np.zeros(max(T, 1))
    ll = (lib or _load()).oracle_trace(N, M, _ptr(pi, _dp), _ptr(A, _dp), _ptr(B, _dp), _ptr(o, _i32p), T,
                              _ptr(ah, _dp), _ptr(bh, _dp), _ptr(c, _dp))
    return ll, ah[:T], bh[:T], c[:T]


def counts(pi, A, B, symbols, offsets, lengths, model_of_seq, weights=None, nthreads: int = 0, lib=None):
    """(loglik[S], n_pi[K][N], n_A[K][N][N], n_B[K][N][M]) in FP64; each sequence with its own model."""
    pi, A, B = _f64(pi), _f64(A), _f64(B)
    K, N = pi.shape
    M = B.shape[2]
    sym = np.ascontiguousarray(symbols, dtype=np.int32)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    lens = np.ascontiguousarray(lengths, dtype=np.int32)
    mos = np.ascontiguousarray(model_of_seq, dtype=np.int32)
    S = lens.shape[0]
    w = None if weights is None else _f64(weights)
    ll = np.empty(S)
    npi = np.empty((K, N))
    nA = np.empty((K, N, N))
    nB = np.empty((K, N, M))
    rc = (lib or _load()).oracle_counts(K, N, M, _ptr(pi, _dp), _ptr(A, _dp), _ptr(B, _dp), S,
                               _ptr(sym, _i32p), _ptr(off, _i64p), _ptr(lens, _i32p), _ptr(mos, _i32p),
                               _ptr(w, _dp), _ptr(ll, _dp), _ptr(npi, _dp), _ptr(nA, _dp), _ptr(nB, _dp),
                               int(nthreads))
    if rc != 0:
        raise ValueError("oracle_counts: bad arguments")
    return ll, npi, nA, nB


def viterbi(pi, A, B, symbols, offsets, lengths, model_of_seq, nthreads: int = 0, lib=None):
    """(score[S], path[sum T] int32, margin[S]) in FP64; each sequence decoded with its own model.

    score = max over state paths of ln P(O, Q); path holds the decoded state of step t of
    sequence s at offsets[s] + t (smallest-index rule on ties); margin is the smallest gap
    between a choice on that path and its best alternative."""
    pi, A, B = _f64(pi), _f64(A), _f64(B)
    K, N = pi.shape
    M = B.shape[2]
    sym = np.ascontiguousarray(symbols, dtype=np.int32)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    lens = np.ascontiguousarray(lengths, dtype=np.int32)
    mos = np.ascontiguousarray(model_of_seq, dtype=np.int32)
    S = lens.shape[0]
    score = np.empty(S)
    margin = np.empty(S)
    path = np.full(sym.shape[0], -2, dtype=np.int32)
    rc = (lib or _load()).oracle_viterbi(K, N, M, _ptr(pi, _dp), _ptr(A, _dp), _ptr(B, _dp), S, _ptr(sym, _i32p),
                                         _ptr(off, _i64p), _ptr(lens, _i32p), _ptr(mos, _i32p), _ptr(score, _dp),
                                         _ptr(path, _i32p), _ptr(margin, _dp), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_viterbi: bad arguments")
    return score, path, margin


def softmax(logits) -> np.ndarray:
    """Row-wise softmax over the last axis, FP64, from the given (FP32) logits."""
    z = _f64(logits)
    z = z - z.max(axis=-1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=-1, keepdims=True)


def logit_grad(n: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Gradient w.r.t. softmax logits from the gradient n w.r.t. log-probabilities.

    With p = softmax(z) per row, d(ln p_j)/d z_l = [j = l] - p_l, so
    dL/dz_l = n_l - p_l * sum_j n_j.
    """
    n = _f64(n)
    p = _f64(p)
    return n - p * n.sum(axis=-1, keepdims=True)


def loglik_grad_from_logits(lpi, lA, lB, symbols, offsets, lengths, model_of_seq, weights=None,
                            nthreads: int = 0):
    """(loglik[S], g_pi, g_A, g_B): gradient of sum_s w_s log P w.r.t. the logits, FP64."""
    pi, A, B = softmax(lpi), softmax(lA), softmax(lB)
    ll, npi, nA, nB = counts(pi, A, B, symbols, offsets, lengths, model_of_seq, weights, nthreads)
    return ll, logit_grad(npi, pi), logit_grad(nA, A), logit_grad(nB, B)


def objective_from_logits(lpi, lA, lB, symbols, offsets, lengths, model_of_seq, weights=None,
                          nthreads: int = 0) -> float:
    """sum_s w_s log P(O_s | softmax-parameterised lambda_{m(s)}), FP64."""
    pi, A, B = softmax(lpi), softmax(lA), softmax(lB)
    ll = forward(pi, A, B, symbols, offsets, lengths, model_of_seq, nthreads)
    w = np.ones_like(ll) if weights is None else _f64(weights)
    return float(np.sum(w * ll))


def reestimate(n_rows, old_rows) -> np.ndarray:
    """Baum-Welch M-step for one parameter array: each row of expected counts divided by
    its sum (the maximum-likelihood row given the counts); a row whose counts sum to zero
    (a state never visited, a model without sequences) keeps its old values."""
    n = _f64(n_rows)
    old = _f64(old_rows)
    tot = n.sum(axis=-1, keepdims=True)
    with np.errstate(invalid="ignore", divide="ignore"):
        new = n / tot
    return np.where(tot > 0, new, old)


def baum_welch(pi, A, B, symbols, offsets, lengths, model_of_seq, iters: int, nthreads: int = 0):
    """EM for the bank (each sequence trains its own model): `iters` rounds of E-step
    (expected counts of the current parameters) and M-step (reestimate).  Returns the
    parameters after every round and the total log-likelihood before every round, FP64."""
    pi, A, B = _f64(pi), _f64(A), _f64(B)
    hist, lls = [], []
    for _ in range(iters):
        ll, npi, nA, nB = counts(pi, A, B, symbols, offsets, lengths, model_of_seq, nthreads=nthreads)
        lls.append(float(np.sum(ll)))
        pi, A, B = reestimate(npi, pi), reestimate(nA, A), reestimate(nB, B)
        hist.append((pi, A, B))
    return hist, lls
