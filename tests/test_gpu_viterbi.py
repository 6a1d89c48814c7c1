"""Viterbi decoding on the GPU vs the FP64 oracle, through the C ABI (MI355X only).

score  |s_gpu - s_oracle| / max(|s_oracle|, 1) <= 1e-5, infinities and NaNs equal.
path   The decoder takes its arg-max decisions on FP32 values, so the path is unique
       only up to that rounding.  rounding_bound() below bounds, per sequence, the
       error E of every FP32 delta value near the row maximum (ln A, ln B and ln pi
       from logf, one rounding per addition, a shift by the row maximum every 16
       steps).  Then:
         - where the oracle's margin (log-probability of its path minus that of the
           best other path) exceeds 2E, the GPU path must be the oracle's, index
           for index;
         - every other GPU path must be a valid state path whose FP64 log-probability
           is within 2E of the oracle's optimum (the decoder maximised an FP32
           evaluation of it that is within E of the exact value, and the optimum's
           FP32 evaluation is within E of the optimum);
         - each workload must have at least a stated share of index-exact paths, and
           the test prints how many paths were gated, exact, and near-ties.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1310_3322_amd import hmm, workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5
U32 = 2.0 ** -24          # unit roundoff of FP32
SHIFT_PERIOD = 16         # steps between the decoder's shifts by the row maximum


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


def rounding_bound(w, s, sym):
    """Bound E on the error of the decoder's FP32 delta values near the row maximum for
    sequence s (derivation: the Viterbi readings of the design notes).

    With M_t = max_j delta_t(j) (exact, FP64 max-plus here) and S_t the decoder's
    accumulated shift (M at the last shift step), a value within 1 of the row maximum
    has magnitude at most D_t = |M_t - S_{t-1}| + 1 in the frame it is computed in, and
    the logarithms on its best incoming edge satisfy |ln a| + |ln b| <= L_t =
    M_{t-1} - M_t + 1 (both are <= 0 and they bridge the two maxima).  Step t then adds
    at most u (D_{t-1} + L_t) for the candidate sum, u D_t for the emission sum, u D_t
    for a shift, and 2 ulp = 4 u L_t for the two FP32 logarithms; E is the sum over
    the steps.  A maximum of perturbed values moves by at most the largest perturbation,
    so the bound carries over from step to step."""
    k, T, off = int(w.owner[s]), int(w.lengths[s]), int(w.offsets[s])
    if T == 0:
        return 0.0
    o = sym[off:off + T]
    with np.errstate(divide="ignore"):
        la = np.log(w.A[k].astype(np.float64))
        lb = np.log(w.B[k].astype(np.float64))
        d = np.log(w.pi[k].astype(np.float64)) + lb[:, o[0]]
    Mprev = float(np.max(d))
    shift = 0.0
    E = U32 * (abs(Mprev) + 1.0) + 4 * U32 * (abs(Mprev) + 1.0)
    Dprev = abs(Mprev) + 1.0
    if SHIFT_PERIOD == 1:
        shift = Mprev
    for t in range(1, T):
        d = np.max(d[:, None] + la, axis=0) + lb[:, o[t]]
        Mt = float(np.max(d))
        if not math.isfinite(Mt):
            return math.inf
        Dt = abs(Mt - shift) + 1.0
        Lt = (Mprev - Mt) + 1.0
        E += U32 * (Dprev + Lt) + U32 * Dt + 4 * U32 * Lt
        if (t + 1) % SHIFT_PERIOD == 0:
            E += U32 * Dt
            shift = Mt
        Dprev = abs(Mt - shift) + 1.0
        Mprev = Mt
    return E


def check(w, symbols=None, min_exact_share=None, label=""):
    sym = w.symbols if symbols is None else symbols
    sc, path = hmm.viterbi(problem(w, sym))
    sc, path = sc.cpu().numpy().astype(np.float64), path.cpu().numpy()
    rs, rp, rm = O.viterbi(w.pi, w.A, w.B, sym, w.offsets, w.lengths, w.owner)
    return compare(w, np.arange(w.S), sc, path, w, sym, rs, rp, rm, min_exact_share, label)


def compare(w, seqs, sc, path, ref_w, ref_sym, rs, rp, rm, min_exact_share, label):
    """GPU scores and paths (sc, path, laid out as w) of the sequences `seqs` of w against
    the oracle's results rs / rp / rm for the same sequences laid out as ref_w with
    symbols ref_sym (w itself, or a subset of it)."""
    assert np.array_equal(np.isnan(sc[seqs]), np.isnan(rs))
    assert np.array_equal(sc[seqs][np.isinf(rs)], rs[np.isinf(rs)])
    fin = np.isfinite(rs)
    if fin.any():
        err = np.max(np.abs(sc[seqs][fin] - rs[fin]) / np.maximum(np.abs(rs[fin]), 1.0))
        assert err <= TOL, err
    gated = exact = ties = 0
    for i, s in enumerate(seqs):
        T, off, ro = int(w.lengths[s]), int(w.offsets[s]), int(ref_w.offsets[i])
        g, r = path[off:off + T], rp[ro:ro + T]
        if not np.isfinite(rs[i]):
            if np.isnan(rs[i]):
                assert np.all(g == -1), s
            continue
        if np.array_equal(g, r):
            exact += 1
        E = rounding_bound(ref_w, i, ref_sym)
        if rm[i] > 2 * E:
            gated += 1
            assert np.array_equal(g, r), (label, int(s), T, rm[i], E)
        else:
            ties += 1
            assert np.all((g >= 0) & (g < w.N)), s
            lp = path_logprob(ref_w, i, g, ref_sym)
            assert rs[i] - lp <= 2 * E + 1e-12 * max(1.0, abs(rs[i])), (label, int(s), lp, rs[i], E)
    n = int(np.sum(fin))
    print(f"  {label}: {n} finite paths, {gated} with margin > 2E (all index-exact), {ties} within 2E of a tie, "
          f"{exact} index-exact overall", flush=True)
    if min_exact_share is not None and n > 0:
        assert exact >= min_exact_share * n, (label, exact, n)
    return exact


# Smallest share of index-exact paths per workload (of the paths with a finite score).
# The decoder's FP32 rounding is about sqrt(T) u |delta| in practice, far below the
# worst-case bound 2E, so the paths differ from the oracle's only at near-ties.
EXACT_SHARE = 0.9


@pytest.mark.parametrize("cfg,scale", [("brute", 1.0), ("c1", 1.0), ("paper", 1.0), ("c2", 0.1), ("c3", 0.004)])
def test_viterbi_parity_workloads(cfg, scale):
    print(f"[case] viterbi {cfg} scale={scale}", flush=True)
    w = workloads.make_workload(cfg, scale=scale)
    if w.all_pairs:
        w.all_pairs = False
    check(w, min_exact_share=EXACT_SHARE, label=f"{cfg}x{scale}")


@pytest.mark.parametrize("N", [1, 2, 5, 16, 17, 31, 32, 33, 48, 64, 65, 100, 128, 129, 200, 256])
def test_viterbi_state_counts_and_ragged_lengths(N):
    """Every padding of the state axis (lane groups up to 64 states, workgroups of 4 threads
    per state above); lengths around the shift period (16) and the workgroup decoder's
    symbol chunk (64), T = 0 and 1."""
    print(f"[case] viterbi N={N}", flush=True)
    rng = np.random.default_rng([31, N])
    lengths = np.concatenate([[0, 1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 129, 300], rng.integers(1, 120, size=26)])
    w = workloads.random_lengths_workload(rng, K=3, N=N, M=11, lengths=lengths, all_pairs=False, conc=0.4)
    check(w, min_exact_share=EXACT_SHARE, label=f"N={N}")


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
    check(w, sym, label=f"special N={N}")


def _sampled(w, pick, label, min_exact_share):
    sc, path = hmm.viterbi(problem(w))
    sc, path = sc.cpu().numpy().astype(np.float64), path.cpu().numpy()
    assert np.all(np.isfinite(sc))
    sub = w.subset(pick)
    rs, rp, rm = O.viterbi(sub.pi, sub.A, sub.B, sub.symbols, sub.offsets, sub.lengths, sub.owner)
    compare(w, pick, sc, path, sub, sub.symbols, rs, rp, rm, min_exact_share, label)


def test_viterbi_full_c3_sampled():
    """The c3 bank and full batch, each sequence decoded with its owner; sampled sequences vs the oracle."""
    print("[case] viterbi c3 full", flush=True)
    w = workloads.make_workload("c3")
    w.all_pairs = False
    order = np.argsort(-w.lengths, kind="stable")
    rng = np.random.default_rng(9)
    pick = np.unique(np.concatenate([order[:8], order[-8:], rng.choice(w.S, 40, replace=False)]))
    _sampled(w, pick, "c3 full, sampled", EXACT_SHARE)


def test_viterbi_determinism():
    """Repeated calls give identical scores and paths, for the per-wave decoder (c2) and
    the workgroup decoder (65 states)."""
    rng = np.random.default_rng(3)
    big = workloads.random_lengths_workload(rng, K=2, N=65, M=4, lengths=np.array([5, 6, 70, 0, 1]), all_pairs=False)
    check(big, label="N=65 small")
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
    order = np.argsort(-w.lengths, kind="stable")
    rng = np.random.default_rng(5)
    pick = np.unique(np.concatenate([order[:2], order[-2:], rng.choice(w.S, 6, replace=False)]))
    _sampled(w, pick, "c5 5% batch, sampled", None)


def _decode(p, ws):
    sc, path = hmm.viterbi(p, ws=ws)
    return sc.cpu().numpy(), path.cpu().numpy(), hmm.workspace_error(ws)


@pytest.mark.parametrize("N", [5, 20, 33, 64, 100, 256])
def test_viterbi_rounds_match_one_round(N):
    """A workspace that keeps the delta rows of only a few sequences at once (decoding in
    many rounds) gives the scores, paths and error word of a workspace with room for every
    row (one round), bit for bit, for both decoders.  Invalid entries ride along: a bad
    symbol, a bad model index, lengths 0 and lengths beyond max_len (which store no rows)."""
    print(f"[case] viterbi rounds N={N}", flush=True)
    rng = np.random.default_rng(200 + N)
    lengths = rng.integers(1, 120, size=160).astype(np.int32)
    lengths[[3, 40]] = 0
    w = workloads.random_lengths_workload(rng, K=3, N=N, M=6, lengths=lengths, all_pairs=False)
    max_len = 110                                   # longer sequences are invalid
    sym = w.symbols.copy()
    s_sym = int(np.flatnonzero((w.lengths > 5) & (w.lengths <= max_len))[0])
    sym[w.offsets[s_sym] + 4] = 99                  # invalid symbol
    owner = w.owner.copy()
    owner[7] = 3                                    # invalid model index
    p = hmm.Problem(dev(w.pi), dev(w.A), dev(w.B), dev(sym), dev(w.offsets), dev(w.lengths), dev(owner),
                    max_len=max_len, total_symbols=w.total_symbols)
    one = _decode(p, p.viterbi_workspace(w.total_symbols))
    # sequences whose path range is written: a valid model and length (a bad symbol gives -1s)
    ok = (owner < w.K) & (w.lengths <= max_len)
    mask = np.zeros(w.total_symbols, bool)
    for s in np.flatnonzero(ok):
        mask[w.offsets[s]:w.offsets[s] + w.lengths[s]] = True
    bad = {7, s_sym} | set(np.flatnonzero(w.lengths > max_len).tolist())
    assert set(np.flatnonzero(np.isnan(one[0])).tolist()) == bad
    assert np.all(one[1][w.offsets[s_sym]:w.offsets[s_sym] + w.lengths[s_sym]] == -1)
    assert one[2] == min(bad)
    for rows in (2 * max_len, 2 * max_len + 7, 3 * max_len, w.total_symbols // 4):
        got = _decode(p, p.viterbi_workspace(rows))
        assert np.array_equal(got[0], one[0], equal_nan=True), rows
        assert np.array_equal(got[1][mask], one[1][mask]), rows
        assert got[2] == one[2], rows


def test_viterbi_c5_rounds_bounded_workspace():
    """A quarter of the c5 batch (4096 sequences of 256..4096 steps, 256 states): the default
    workspace (1.8 GiB of delta rows, several rounds), one of 1 GiB of rows and one with room
    for every row (9 GB, one round) give identical scores and paths; sampled sequences
    against the oracle."""
    print("[case] viterbi c5 rounds", flush=True)
    w = workloads.make_workload("c5", scale=0.25)
    w.all_pairs = False
    p = problem(w)
    dflt = p.workspace(hmm.OP_VITERBI)
    assert dflt.numel() <= 2_000_000_000
    assert p.viterbi_workspace_size(w.total_symbols) > 4 * dflt.numel()
    base = _decode(p, dflt)
    for rows in (1 << 20, w.total_symbols):
        got = _decode(p, p.viterbi_workspace(rows))
        assert np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1]), rows
        assert got[2] == base[2]
    order = np.argsort(-w.lengths, kind="stable")
    rng = np.random.default_rng(6)
    pick = np.unique(np.concatenate([order[:2], order[-2:], rng.choice(w.S, 4, replace=False)]))
    sub = w.subset(pick)
    rs, rp, rm = O.viterbi(sub.pi, sub.A, sub.B, sub.symbols, sub.offsets, sub.lengths, sub.owner)
    compare(w, pick, base[0].astype(np.float64), base[1], sub, sub.symbols, rs, rp, rm, None,
            "c5 quarter batch, default workspace, sampled")
