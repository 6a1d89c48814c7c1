"""Seeded synthetic workloads for the discrete-HMM bank.

This module only draws random numbers: model banks (Dirichlet rows or Gaussian
logits) and observation sequences sampled from the generative process of a
discrete HMM (first state from pi, each symbol from the row of B of the current
state, next state from the row of A of the current state).  It contains none of
the forward / backward arithmetic, so both the FP64 oracle and the GPU path can
take their inputs from it without sharing any of the method's code.

The paper (Sec. 5.7) evaluates a bank of six activity HMMs with five hidden
states over per-player symbol streams of the UCF teamwork dataset.  That data is
not available, so the configurations below are synthetic stand-ins of the same
structure (one HMM per activity class, ragged symbol streams), scaled up:

  c1     1 model,  N=8,   M=16,   one sequence, T=64
  brute  1 model,  N=3,   M=4,    one sequence, T=6 (small enough to enumerate)
  paper  6 models, N=5,   M=6,    147 sequences, T in [20, 200] (Sec. 5.7 shape)
  c2    12 models, N=16,  M=64,   4096 sequences, T ~ U{50..400}, 5 % noise
  c3    64 models, N=32,  M=256,  65536 sequences, log-uniform T in [16, 2048]
  c4     8 models, N=64,  M=512,  8192 sequences, T ~ U{100..1000}, logits
  c5    16 models, N=256, M=1024, 16384 sequences, T ~ U{256..4096}, banded A

Parameters are drawn in FP64 and cast to FP32 without renormalising; every
consumer receives the FP32 arrays (the oracle upcasts them exactly).
"""
from __future__ import annotations

import dataclasses
import zlib
from typing import Optional

import numpy as np

SEED_BASE = (1310, 3322)

CONFIG_NAMES = ("brute", "c1", "paper", "c2", "c3", "c4", "c5")


@dataclasses.dataclass
class Workload:
    name: str
    K: int
    N: int
    M: int
    pi: np.ndarray          # float32 [K][N]
    A: np.ndarray           # float32 [K][N][N], A[k][i][j] = P(q_{t+1}=j | q_t=i)
    B: np.ndarray           # float32 [K][N][M], B[k][i][o] = P(o_t=o | q_t=i)
    symbols: np.ndarray     # int32 [sum T]
    offsets: np.ndarray     # int64 [S]
    lengths: np.ndarray     # int32 [S]
    owner: np.ndarray       # int32 [S], model that generated each sequence
    all_pairs: bool         # True: every sequence is scored against all K models
    logits: Optional[tuple] = None   # (lpi, lA, lB) float32, softmax-parameterised banks
    seed: int = 0

    @property
    def S(self) -> int:
        return int(self.lengths.shape[0])

    @property
    def total_symbols(self) -> int:
        return int(self.symbols.shape[0])

    @property
    def max_len(self) -> int:
        return int(self.lengths.max()) if self.S else 0

    @property
    def model_of_seq(self) -> Optional[np.ndarray]:
        return None if self.all_pairs else self.owner

    def units(self) -> float:
        """State-steps: N^2 * sum(T) * models scored per sequence."""
        per_seq = self.K if self.all_pairs else 1
        return float(self.N) * self.N * float(self.lengths.astype(np.int64).sum()) * per_seq

    def subset(self, seq_ids: np.ndarray) -> "Workload":
        """Sequences `seq_ids` (in that order), re-packed contiguously."""
        seq_ids = np.asarray(seq_ids, dtype=np.int64)
        lens = self.lengths[seq_ids]
        offs = np.zeros(len(seq_ids), dtype=np.int64)
        if len(seq_ids):
            offs[1:] = np.cumsum(lens[:-1].astype(np.int64))
        syms = np.empty(int(lens.astype(np.int64).sum()), dtype=np.int32)
        for d, s in enumerate(seq_ids):
            o, t = int(self.offsets[s]), int(self.lengths[s])
            syms[offs[d]:offs[d] + t] = self.symbols[o:o + t]
        return dataclasses.replace(self, symbols=syms, offsets=offs, lengths=lens.astype(np.int32),
                                   owner=self.owner[seq_ids].astype(np.int32))


def rng_for(cfg: str, seed: int = 0) -> np.random.Generator:
    tag = CONFIG_NAMES.index(cfg) if cfg in CONFIG_NAMES else 1000 + zlib.crc32(cfg.encode()) % 100000
    return np.random.default_rng(np.random.SeedSequence([SEED_BASE[0], SEED_BASE[1], tag, seed]))


def dirichlet_rows(rng: np.random.Generator, shape_prefix: tuple, n: int, conc: float) -> np.ndarray:
    """FP64 rows drawn from a symmetric Dirichlet(conc) of dimension n."""
    g = rng.gamma(conc, 1.0, size=shape_prefix + (n,))
    s = g.sum(axis=-1, keepdims=True)
    # a row of all-zero gammas (possible for tiny conc in FP64) becomes uniform
    bad = s[..., 0] <= 0
    if np.any(bad):
        g[bad] = 1.0
        s = g.sum(axis=-1, keepdims=True)
    return g / s


def softmax_rows_for_sampling(logits: np.ndarray) -> np.ndarray:
    """FP64 row probabilities used only to draw sample sequences from a logit bank."""
    z = logits.astype(np.float64)
    z = z - z.max(axis=-1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=-1, keepdims=True)


class _RowSampler:
    """Inverse-CDF sampling from many categorical rows at once (guide-table search).

    rows: FP64 [R][n] non-negative weights.  Each row's cumulative sums are
    normalised to end at exactly 1.  guide[r][g] is the first column whose
    cumulative sum exceeds g/n, so a draw starts there and walks forward until
    the cumulative sum exceeds u (about one step on average).  Zero-weight
    entries are never drawn.
    """

    def __init__(self, rows: np.ndarray):
        R, n = rows.shape
        cdf = np.cumsum(rows, axis=1)
        cdf = cdf / cdf[:, -1:]
        cdf[:, -1] = 1.0
        self.n = n
        self.cdf = cdf.ravel()
        shifted = (cdf + np.arange(R, dtype=np.float64)[:, None]).ravel()
        q = (np.arange(R, dtype=np.float64)[:, None] + np.arange(n, dtype=np.float64)[None, :] / n).ravel()
        pos = np.searchsorted(shifted, q, side="right")
        col = pos - np.repeat(np.arange(R, dtype=np.int64), n) * n
        self.guide = np.minimum(col, n - 1).astype(np.int64)

    def draw(self, row_idx: np.ndarray, u: np.ndarray) -> np.ndarray:
        n = self.n
        base = row_idx.astype(np.int64) * n
        g = np.minimum((u * n).astype(np.int64), n - 1)
        col = self.guide[base + g]
        while True:
            adv = (self.cdf[base + col] <= u) & (col < n - 1)
            if not adv.any():
                break
            col = col + adv
        return col.astype(np.int32)


def sample_sequences(rng: np.random.Generator, pi: np.ndarray, A: np.ndarray, B: np.ndarray,
                     owner: np.ndarray, lengths: np.ndarray):
    """Draw one symbol stream per sequence from its owner's HMM.

    pi [K][N], A [K][N][N], B [K][N][M] are the FP32 banks (upcast here);
    returns (symbols int32 [sum T], offsets int64 [S]).
    """
    K, N = pi.shape
    M = B.shape[2]
    S = len(lengths)
    offsets = np.zeros(S, dtype=np.int64)
    if S:
        offsets[1:] = np.cumsum(lengths[:-1].astype(np.int64))
    total = int(lengths.astype(np.int64).sum())
    symbols = np.empty(total, dtype=np.int32)
    if S == 0 or total == 0:
        return symbols, offsets
    spi = _RowSampler(pi.astype(np.float64))
    sA = _RowSampler(A.astype(np.float64).reshape(K * N, N))
    sB = _RowSampler(B.astype(np.float64).reshape(K * N, M))
    order = np.argsort(-lengths.astype(np.int64), kind="stable")
    own = owner[order].astype(np.int64)
    lens = lengths[order].astype(np.int64)
    offs = offsets[order]
    q = spi.draw(own, rng.random(S))
    Tmax = int(lens[0])
    n_act = S
    for t in range(Tmax):
        while n_act > 0 and lens[n_act - 1] <= t:
            n_act -= 1
        if n_act == 0:
            break
        qa = q[:n_act].astype(np.int64)
        rows = own[:n_act] * N + qa
        o = sB.draw(rows, rng.random(n_act))
        symbols[offs[:n_act] + t] = o
        q[:n_act] = sA.draw(rows, rng.random(n_act))
    return symbols, offsets


def _bank_dirichlet(rng, K, N, M, conc_pi, conc_A, conc_B):
    pi = dirichlet_rows(rng, (K,), N, conc_pi)
    A = dirichlet_rows(rng, (K, N), N, conc_A)
    B = dirichlet_rows(rng, (K, N), M, conc_B)
    return pi.astype(np.float32), A.astype(np.float32), B.astype(np.float32)


def make_workload(cfg: str, seed: int = 0, scale: float = 1.0) -> Workload:
    """Build configuration `cfg` (see module docstring).

    `scale` < 1 keeps the model bank and the length distribution but draws
    only round(scale * S) sequences (at least one); it is meant for tests that
    need the real shapes at a size the oracle finishes quickly.
    """
    rng = rng_for(cfg, seed)

    def n_seq(S):
        return max(1, int(round(S * scale)))

    logits = None
    if cfg == "brute":
        K, N, M = 1, 3, 4
        pi, A, B = _bank_dirichlet(rng, K, N, M, 1.0, 1.0, 1.0)
        lengths = np.array([6], dtype=np.int32)
        owner = np.zeros(1, dtype=np.int32)
        all_pairs = False
    elif cfg == "c1":
        K, N, M = 1, 8, 16
        pi, A, B = _bank_dirichlet(rng, K, N, M, 1.0, 1.0, 1.0)
        lengths = np.array([64], dtype=np.int32)
        owner = np.zeros(1, dtype=np.int32)
        all_pairs = False
    elif cfg == "paper":
        K, N, M = 6, 5, 6
        pi, A, B = _bank_dirichlet(rng, K, N, M, 1.0, 1.0, 1.0)
        S = n_seq(147)
        lengths = rng.integers(20, 201, size=S).astype(np.int32)
        owner = rng.integers(0, K, size=S).astype(np.int32)
        all_pairs = True
    elif cfg == "c2":
        K, N, M = 12, 16, 64
        pi, A, B = _bank_dirichlet(rng, K, N, M, 1.0, 1.0, 1.0)
        S = n_seq(4096)
        lengths = rng.integers(50, 401, size=S).astype(np.int32)
        owner = rng.integers(0, K, size=S).astype(np.int32)
        all_pairs = True
    elif cfg == "c3":
        K, N, M = 64, 32, 256
        pi, A, B = _bank_dirichlet(rng, K, N, M, 0.5, 0.5, 0.5)
        S = n_seq(65536)
        u = rng.uniform(np.log(16.0), np.log(2049.0), size=S)
        lengths = np.clip(np.floor(np.exp(u)), 16, 2048).astype(np.int32)
        owner = (np.arange(S) % K).astype(np.int32)
        all_pairs = True
    elif cfg == "c4":
        K, N, M = 8, 64, 512
        lpi = rng.standard_normal((K, N)).astype(np.float32)
        lA = rng.standard_normal((K, N, N)).astype(np.float32)
        lB = rng.standard_normal((K, N, M)).astype(np.float32)
        logits = (lpi, lA, lB)
        pi = softmax_rows_for_sampling(lpi).astype(np.float32)
        A = softmax_rows_for_sampling(lA).astype(np.float32)
        B = softmax_rows_for_sampling(lB).astype(np.float32)
        S = n_seq(8192)
        lengths = rng.integers(100, 1001, size=S).astype(np.int32)
        owner = (np.arange(S) % K).astype(np.int32)
        all_pairs = False
    elif cfg == "c5":
        K, N, M = 16, 256, 1024
        pi = dirichlet_rows(rng, (K,), N, 1.0)
        rnd = dirichlet_rows(rng, (K, N), N, 0.1)
        band = np.zeros((N, N))
        for i in range(N):
            band[i, [(i + d) % N for d in range(8)]] = 1.0 / 8.0
        A = 0.5 * rnd + 0.5 * band[None, :, :]
        B = dirichlet_rows(rng, (K, N), M, 0.2)
        pi, A, B = pi.astype(np.float32), A.astype(np.float32), B.astype(np.float32)
        S = n_seq(16384)
        lengths = rng.integers(256, 4097, size=S).astype(np.int32)
        owner = (np.arange(S) % K).astype(np.int32)
        all_pairs = False
    else:
        raise ValueError(f"unknown workload {cfg!r}")

    symbols, offsets = sample_sequences(rng, pi, A, B, owner, lengths)
    if cfg == "c2":
        flip = rng.random(symbols.shape[0]) < 0.05
        symbols[flip] = rng.integers(0, M, size=int(flip.sum())).astype(np.int32)
    return Workload(name=cfg, K=K, N=N, M=M, pi=pi, A=A, B=B, symbols=symbols, offsets=offsets,
                    lengths=lengths, owner=owner, all_pairs=all_pairs, logits=logits, seed=seed)


def random_bank(rng: np.random.Generator, K: int, N: int, M: int, conc: float = 1.0):
    """A Dirichlet(conc) bank in FP32, for ad-hoc test shapes."""
    return _bank_dirichlet(rng, K, N, M, conc, conc, conc)


def random_lengths_workload(rng: np.random.Generator, K: int, N: int, M: int, lengths, all_pairs: bool,
                            conc: float = 1.0, name: str = "adhoc") -> Workload:
    """Ad-hoc workload with the given lengths; owners cycle over the K models."""
    pi, A, B = random_bank(rng, K, N, M, conc)
    lengths = np.asarray(lengths, dtype=np.int32)
    owner = (np.arange(len(lengths)) % K).astype(np.int32)
    symbols, offsets = sample_sequences(rng, pi, A, B, owner, lengths)
    return Workload(name=name, K=K, N=N, M=M, pi=pi, A=A, B=B, symbols=symbols, offsets=offsets,
                    lengths=lengths, owner=owner, all_pairs=all_pairs)
