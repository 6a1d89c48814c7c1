"""Python binding of libhmm_mi355x.so (argument marshalling only).

Every function here checks shapes and dtypes, fills the C structs of
include/hmm.h with device pointers of torch tensors, and calls the library on
the current HIP stream.  All arithmetic runs in the library's HIP kernels.
There is no CPU fallback: loading fails loudly if the library or the GPU is
missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhmm_mi355x.so")
LIB_DEBUG_PATH = os.path.join(_PKG, "libhmm_mi355x_debug.so")  # kernels with bounds checks (-DHMM_DEBUG)

HMM_OK = 0
STATUS = {0: "HMM_OK", -1: "HMM_ERR_NULL", -2: "HMM_ERR_SHAPE", -3: "HMM_ERR_WORKSPACE",
          -4: "HMM_ERR_UNSUPPORTED", -5: "HMM_ERR_HIP", -6: "HMM_ERR_ARG"}
OP_FORWARD, OP_CLASSIFY, OP_GRAD, OP_VITERBI = 0, 1, 2, 3
KERNEL_AUTO, KERNEL_PLAIN, KERNEL_BATCHED, KERNEL_TILE16, KERNEL_TILE32, KERNEL_COOP, KERNEL_SCAN = 0, 1, 2, 3, 4, 5, 6
EXPORTS = ("hmm_workspace_size", "hmm_viterbi_workspace_size", "hmm_grad_workspace_size", "hmm_forward_loglik", "hmm_classify", "hmm_classify_noalloc", "hmm_forward_backward_grad",
           "hmm_viterbi", "hmm_plan_order", "hmm_reestimate_rows", "hmm_softmax_rows", "hmm_logit_grad", "hmm_workspace_error", "hmm_debug_flags", "hmm_select_kernel",
           "hmm_tune_key_of", "hmm_tune_set", "hmm_tune_get", "hmm_tune_clear", "hmm_call_kernel",
           "hmm_profile_enable", "hmm_profile_read", "hmm_status_string")
TUNE_MAX, TUNE_MAX_WG = 256, 64
TUNE_XCD_OFF, TUNE_BT_GLOBAL, TUNE_BT_LDS = 1, 2, 4  # HMM_TUNE_* flags
STATIC_SCRATCH_BYTES = 32 << 20  # HMM_STATIC_SCRATCH_BYTES
PROF_FWD_BATCHED, PROF_ADJ_BATCHED, PROF_FWD_PLAIN, PROF_VITERBI = 0, 1, 2, 3


class HMMError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} returned {STATUS.get(status, status)}")
        self.status = status


class Bank(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("N", ctypes.c_int32), ("M", ctypes.c_int32),
                ("pi", ctypes.c_void_p), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p)]


class Batch(ctypes.Structure):
    _fields_ = [("S", ctypes.c_int32), ("symbols", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("lengths", ctypes.c_void_p), ("model_of_seq", ctypes.c_void_p),
                ("max_len", ctypes.c_int32), ("total_symbols", ctypes.c_int64)]


class TuneKey(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("all_pairs", ctypes.c_int32), ("K", ctypes.c_int32),
                ("N", ctypes.c_int32), ("M", ctypes.c_int32), ("s_bucket", ctypes.c_int32),
                ("len_bucket", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class TuneChoice(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("flags", ctypes.c_int32)]


_lib = None
_lib_path = None


def load_library(path: str = LIB_PATH, rebind: bool = False):
    """Loads and binds the library (no GPU needed for loading).  The first call binds
    `path` for the process; rebind=True binds `path` instead of the bound one (tests
    that run the debug build beside the normal one)."""
    global _lib, _lib_path
    if _lib is not None and not rebind:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() or python -m paper_1310_3322_amd.build")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    BP, QP = ctypes.POINTER(Bank), ctypes.POINTER(Batch)
    st = ctypes.c_int
    lib.hmm_workspace_size.restype = ctypes.c_size_t
    lib.hmm_workspace_size.argtypes = [BP, QP, ctypes.c_int]
    lib.hmm_viterbi_workspace_size.restype = ctypes.c_size_t
    lib.hmm_viterbi_workspace_size.argtypes = [BP, QP, ctypes.c_int64]
    lib.hmm_grad_workspace_size.restype = ctypes.c_size_t
    lib.hmm_grad_workspace_size.argtypes = [BP, QP, ctypes.c_int64]
    lib.hmm_forward_loglik.restype = st
    lib.hmm_forward_loglik.argtypes = [BP, QP, P, P, ctypes.c_size_t, P]
    lib.hmm_classify.restype = st
    lib.hmm_classify.argtypes = [BP, QP, P, P, P, ctypes.c_size_t, P]
    lib.hmm_classify_noalloc.restype = st
    lib.hmm_classify_noalloc.argtypes = [BP, QP, P, P, P]
    lib.hmm_forward_backward_grad.restype = st
    lib.hmm_forward_backward_grad.argtypes = [BP, QP, P, P, P, P, P, ctypes.c_int32, P, ctypes.c_size_t, P]
    lib.hmm_viterbi.restype = st
    lib.hmm_viterbi.argtypes = [BP, QP, P, P, P, ctypes.c_size_t, P]
    lib.hmm_plan_order.restype = st
    lib.hmm_plan_order.argtypes = [BP, QP, ctypes.c_int32, P, P, P, ctypes.c_size_t, P]
    lib.hmm_reestimate_rows.restype = st
    lib.hmm_reestimate_rows.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, P]
    lib.hmm_softmax_rows.restype = st
    lib.hmm_softmax_rows.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, P]
    lib.hmm_logit_grad.restype = st
    lib.hmm_logit_grad.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, P]
    lib.hmm_workspace_error.restype = st
    lib.hmm_workspace_error.argtypes = [P, P, ctypes.POINTER(ctypes.c_int32)]
    lib.hmm_debug_flags.restype = st
    lib.hmm_debug_flags.argtypes = [ctypes.POINTER(ctypes.c_uint32)]
    lib.hmm_select_kernel.restype = st
    lib.hmm_select_kernel.argtypes = [ctypes.c_int32]
    lib.hmm_tune_key_of.restype = st
    lib.hmm_tune_key_of.argtypes = [BP, QP, ctypes.c_int32, ctypes.POINTER(TuneKey)]
    lib.hmm_tune_set.restype = st
    lib.hmm_tune_set.argtypes = [ctypes.POINTER(TuneKey), ctypes.POINTER(TuneChoice)]
    lib.hmm_tune_get.restype = st
    lib.hmm_tune_get.argtypes = [ctypes.POINTER(TuneKey), ctypes.POINTER(TuneChoice), ctypes.POINTER(ctypes.c_int32)]
    lib.hmm_tune_clear.restype = st
    lib.hmm_tune_clear.argtypes = []
    lib.hmm_call_kernel.restype = st
    lib.hmm_call_kernel.argtypes = [BP, QP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.hmm_profile_enable.restype = st
    lib.hmm_profile_enable.argtypes = [ctypes.c_int32]
    lib.hmm_profile_read.restype = st
    lib.hmm_profile_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
    lib.hmm_status_string.restype = ctypes.c_char_p
    lib.hmm_status_string.argtypes = [ctypes.c_int]
    _lib, _lib_path = lib, path
    return lib


def _check(fn: str, rc: int):
    if rc != HMM_OK:
        raise HMMError(fn, rc)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("libhmm_mi355x needs a HIP GPU (gfx950); none is visible")


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Problem:
    """Device tensors of one bank and one batch, packed as the C structs."""

    def __init__(self, pi, A, B, symbols, offsets, lengths, model_of_seq=None,
                 max_len: Optional[int] = None, total_symbols: Optional[int] = None):
        _require_gpu()
        load_library()
        self.pi = _dev(pi, torch.float32, "pi")
        self.A = _dev(A, torch.float32, "A")
        self.B = _dev(B, torch.float32, "B")
        if self.pi.dim() != 2 or self.A.dim() != 3 or self.B.dim() != 3:
            raise ValueError("pi must be [K][N], A [K][N][N], B [K][N][M]")
        K, N = self.pi.shape
        M = self.B.shape[2]
        if tuple(self.A.shape) != (K, N, N) or tuple(self.B.shape[:2]) != (K, N):
            raise ValueError("inconsistent bank shapes")
        self.symbols = _dev(symbols, torch.int32, "symbols")
        self.offsets = _dev(offsets, torch.int64, "offsets")
        self.lengths = _dev(lengths, torch.int32, "lengths")
        S = self.lengths.shape[0]
        if self.offsets.shape[0] != S:
            raise ValueError("offsets and lengths differ in size")
        self.model_of_seq = None if model_of_seq is None else _dev(model_of_seq, torch.int32, "model_of_seq")
        if self.model_of_seq is not None and self.model_of_seq.shape[0] != S:
            raise ValueError("model_of_seq and lengths differ in size")
        if max_len is None:
            max_len = int(self.lengths.max().item()) if S else 0
        if total_symbols is None:
            total_symbols = int(self.symbols.numel())
        self.K, self.N, self.M, self.S = int(K), int(N), int(M), int(S)
        self.max_len, self.total_symbols = int(max_len), int(total_symbols)
        self.bank = Bank(self.K, self.N, self.M, _ptr(self.pi), _ptr(self.A), _ptr(self.B))
        self.batch = Batch(self.S, _ptr(self.symbols), _ptr(self.offsets), _ptr(self.lengths),
                           _ptr(self.model_of_seq), self.max_len, self.total_symbols)

    def batch_without_models(self) -> Batch:
        return Batch(self.S, _ptr(self.symbols), _ptr(self.offsets), _ptr(self.lengths), None,
                     self.max_len, self.total_symbols)

    def workspace_size(self, op: int, batch: Optional[Batch] = None) -> int:
        b = self.batch if batch is None else batch
        return int(load_library().hmm_workspace_size(ctypes.byref(self.bank), ctypes.byref(b), op))

    def workspace(self, op: int, batch: Optional[Batch] = None) -> torch.Tensor:
        n = self.workspace_size(op, batch)
        if n == 0:
            raise HMMError("hmm_workspace_size", -2)
        return torch.empty(n, dtype=torch.uint8, device=self.pi.device)

    def viterbi_workspace_size(self, rows: int) -> int:
        """Workspace bytes with which Viterbi decoding keeps `rows` delta rows per round."""
        return int(load_library().hmm_viterbi_workspace_size(ctypes.byref(self.bank), ctypes.byref(self.batch),
                                                             int(rows)))

    def grad_workspace_size(self, rows: int) -> int:
        """Workspace bytes with which the gradient stores the scaled alpha of `rows`
        steps (0: checkpoints only; every step of the batch needs rows >= the sum of
        its lengths)."""
        return int(load_library().hmm_grad_workspace_size(ctypes.byref(self.bank), ctypes.byref(self.batch),
                                                          int(rows)))

    def grad_workspace(self, rows: int) -> torch.Tensor:
        n = self.grad_workspace_size(rows)
        if n == 0:
            raise HMMError("hmm_grad_workspace_size", -2)
        return torch.empty(n, dtype=torch.uint8, device=self.pi.device)

    def viterbi_workspace(self, rows: int) -> torch.Tensor:
        n = self.viterbi_workspace_size(rows)
        if n == 0:
            raise HMMError("hmm_viterbi_workspace_size", -2)
        return torch.empty(n, dtype=torch.uint8, device=self.pi.device)


def select_kernel(kind: int):
    _check("hmm_select_kernel", load_library().hmm_select_kernel(int(kind)))


def tune_key(bank: Bank, batch: Batch, op: int) -> TuneKey:
    """Tuning-table key of a call (host only)."""
    k = TuneKey()
    _check("hmm_tune_key_of", load_library().hmm_tune_key_of(ctypes.byref(bank), ctypes.byref(batch), int(op),
                                                             ctypes.byref(k)))
    return k


def tune_set(key: TuneKey, kernel: Optional[int], wg_per_cu: int = 0, flags: int = 0):
    """Installs the choice (kernel family, workgroups per CU, TUNE_* flags) for `key`;
    kernel None removes the entry."""
    c = None if kernel is None else ctypes.byref(TuneChoice(int(kernel), int(wg_per_cu), int(flags)))
    _check("hmm_tune_set", load_library().hmm_tune_set(ctypes.byref(key), c))


def tune_get(key: TuneKey) -> Optional[tuple]:
    """(kernel, wg_per_cu, flags) installed for `key`, or None."""
    c = TuneChoice()
    found = ctypes.c_int32(0)
    _check("hmm_tune_get", load_library().hmm_tune_get(ctypes.byref(key), ctypes.byref(c), ctypes.byref(found)))
    return (int(c.kernel), int(c.wg_per_cu), int(c.flags)) if found.value else None


def tune_clear():
    _check("hmm_tune_clear", load_library().hmm_tune_clear())


def call_kernel(bank: Bank, batch: Batch, op: int) -> int:
    """Kernel family (KERNEL_*) a call of `op` on this shape would run now (host only)."""
    k = ctypes.c_int32(0)
    _check("hmm_call_kernel", load_library().hmm_call_kernel(ctypes.byref(bank), ctypes.byref(batch), int(op),
                                                             ctypes.byref(k)))
    return int(k.value)


def forward_loglik(p: Problem, out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
    """log P(O_s | lambda_k): [S][K] without model_of_seq, else [S]."""
    shape = (p.S,) if p.model_of_seq is not None else (p.S, p.K)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=p.pi.device)
    elif tuple(out.shape) != shape:
        raise ValueError(f"out must have shape {shape}")
    _dev(out, torch.float32, "out")
    if ws is None:
        ws = p.workspace(OP_FORWARD)
    rc = load_library().hmm_forward_loglik(ctypes.byref(p.bank), ctypes.byref(p.batch), _ptr(out), _ptr(ws),
                                           ws.numel(), _stream(stream))
    _check("hmm_forward_loglik", rc)
    return out


def classify(p: Problem, labels: Optional[torch.Tensor] = None, loglik: Optional[torch.Tensor] = None,
             ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Arg-max label over all K models per sequence (model_of_seq ignored)."""
    if labels is None:
        labels = torch.empty(p.S, dtype=torch.int32, device=p.pi.device)
    _dev(labels, torch.int32, "labels")
    if loglik is not None:
        _dev(loglik, torch.float32, "loglik")
        if tuple(loglik.shape) != (p.S, p.K):
            raise ValueError("loglik must be [S][K]")
    b = p.batch_without_models()
    if ws is None:
        ws = p.workspace(OP_CLASSIFY, b)
    rc = load_library().hmm_classify(ctypes.byref(p.bank), ctypes.byref(b), _ptr(labels), _ptr(loglik),
                                     _ptr(ws), ws.numel(), _stream(stream))
    _check("hmm_classify", rc)
    return labels


def classify_noalloc(p: Problem, labels: torch.Tensor, loglik: Optional[torch.Tensor] = None,
                     stream=None) -> torch.Tensor:
    """classify() on the library's static scratch array instead of a workspace; the caller
    passes the outputs, so nothing is allocated (the array is shared by every call on one
    GPU: calls must not overlap there)."""
    _dev(labels, torch.int32, "labels")
    if labels.shape[0] != p.S:
        raise ValueError("labels must be [S]")
    if loglik is not None:
        _dev(loglik, torch.float32, "loglik")
        if tuple(loglik.shape) != (p.S, p.K):
            raise ValueError("loglik must be [S][K]")
    b = p.batch_without_models()
    rc = load_library().hmm_classify_noalloc(ctypes.byref(p.bank), ctypes.byref(b), _ptr(labels), _ptr(loglik),
                                             _stream(stream))
    _check("hmm_classify_noalloc", rc)
    return labels


def forward_backward_grad(p: Problem, seq_weight: Optional[torch.Tensor] = None, phase: int = 0,
                          loglik: Optional[torch.Tensor] = None, counts=None, ws: Optional[torch.Tensor] = None,
                          stream=None):
    """Expected counts (gradient w.r.t. ln pi, ln A, ln B) and log-likelihoods.

    ws: the workspace, p.workspace(OP_GRAD) by default (the scaled alpha of every
    step stored between the passes when that takes at most 4 GiB, else
    checkpoints); p.grad_workspace(rows) sets the stored rows (0: checkpoints).
    Phases 1 and 2 of one gradient take the same ws.
    Returns (loglik [S], (n_pi [K][N], n_A [K][N][N], n_B [K][N][M]), ws).
    """
    if p.model_of_seq is None:
        raise ValueError("the gradient needs model_of_seq")
    dev = p.pi.device
    if loglik is None and phase != 2:
        loglik = torch.empty(p.S, dtype=torch.float32, device=dev)
    if counts is None and phase != 1:
        counts = (torch.empty((p.K, p.N), dtype=torch.float32, device=dev),
                  torch.empty((p.K, p.N, p.N), dtype=torch.float32, device=dev),
                  torch.empty((p.K, p.N, p.M), dtype=torch.float32, device=dev))
    if seq_weight is not None:
        _dev(seq_weight, torch.float32, "seq_weight")
        if seq_weight.shape[0] != p.S:
            raise ValueError("seq_weight must be [S]")
    if ws is None:
        ws = p.workspace(OP_GRAD)
    c = counts if counts is not None else (None, None, None)
    rc = load_library().hmm_forward_backward_grad(
        ctypes.byref(p.bank), ctypes.byref(p.batch), _ptr(seq_weight), _ptr(loglik), _ptr(c[0]), _ptr(c[1]),
        _ptr(c[2]), int(phase), _ptr(ws), ws.numel(), _stream(stream))
    _check("hmm_forward_backward_grad", rc)
    return loglik, counts, ws


def viterbi(p: Problem, score: Optional[torch.Tensor] = None, path: Optional[torch.Tensor] = None,
            ws: Optional[torch.Tensor] = None, stream=None):
    """Most likely state path of each sequence under its own model.

    Returns (score [S] = max_Q ln P(O, Q), path [total_symbols] int32 in the layout of the symbols).
    ws: any workspace from p.viterbi_workspace_size(min(max_len, total_symbols)) bytes up; its
    size sets how many delta rows a decoding round keeps (default p.workspace(OP_VITERBI))."""
    if p.model_of_seq is None:
        raise ValueError("Viterbi decoding needs model_of_seq")
    dev = p.pi.device
    if score is None:
        score = torch.empty(p.S, dtype=torch.float32, device=dev)
    if path is None:
        path = torch.empty(p.total_symbols, dtype=torch.int32, device=dev)
    _dev(score, torch.float32, "score")
    _dev(path, torch.int32, "path")
    if score.shape[0] != p.S or path.shape[0] != p.total_symbols:
        raise ValueError("score must be [S] and path [total_symbols]")
    if ws is None:
        ws = p.workspace(OP_VITERBI)
    rc = load_library().hmm_viterbi(ctypes.byref(p.bank), ctypes.byref(p.batch), _ptr(score), _ptr(path), _ptr(ws),
                                    ws.numel(), _stream(stream))
    _check("hmm_viterbi", rc)
    return score, path


def plan_order(p: Problem, op: int, all_pairs: Optional[bool] = None, ws: Optional[torch.Tensor] = None,
               stream=None):
    """The batched kernels' work list for `op`: (order [S], group_start [groups + 1]) int32.

    all_pairs (forward only): score every sequence against every model (one group);
    default: own model when the problem has model_of_seq."""
    own = p.model_of_seq is not None if all_pairs is None else not all_pairs
    if op == OP_CLASSIFY:
        own = False
    b = p.batch if own else p.batch_without_models()
    groups = p.K if own and op != OP_VITERBI else 1  # Viterbi: all models in one list
    dev = p.pi.device
    order = torch.empty(p.S, dtype=torch.int32, device=dev)
    gstart = torch.empty(groups + 1, dtype=torch.int32, device=dev)
    if ws is None:
        ws = p.workspace(op, b)
    rc = load_library().hmm_plan_order(ctypes.byref(p.bank), ctypes.byref(b), int(op), _ptr(order), _ptr(gstart),
                                       _ptr(ws), ws.numel(), _stream(stream))
    _check("hmm_plan_order", rc)
    return order, gstart


def reestimate_rows(n: torch.Tensor, old: torch.Tensor, out: Optional[torch.Tensor] = None,
                    stream=None) -> torch.Tensor:
    """Baum-Welch M-step for one parameter array (rows over the last axis)."""
    _dev(n, torch.float32, "n")
    _dev(old, torch.float32, "old")
    if tuple(n.shape) != tuple(old.shape):
        raise ValueError("n and old must have the same shape")
    if out is None:
        out = torch.empty_like(old)
    _dev(out, torch.float32, "out")
    cols = n.shape[-1]
    rows = n.numel() // cols if cols else 0
    rc = load_library().hmm_reestimate_rows(_ptr(n), _ptr(old), _ptr(out), rows, cols, _stream(stream))
    _check("hmm_reestimate_rows", rc)
    return out


def baum_welch(p: Problem, iters: int, stream=None):
    """EM on the bank (each sequence trains its own model): `iters` rounds of E-step
    (expected counts, hmm_forward_backward_grad with unit weights) and M-step
    (hmm_reestimate_rows), updating p.pi, p.A, p.B in place.  Returns the
    log-likelihoods of the sequences before each round, a device tensor [iters][S]."""
    if p.model_of_seq is None:
        raise ValueError("Baum-Welch needs model_of_seq")
    dev = p.pi.device
    ws = p.workspace(OP_GRAD)
    counts = (torch.empty((p.K, p.N), dtype=torch.float32, device=dev),
              torch.empty((p.K, p.N, p.N), dtype=torch.float32, device=dev),
              torch.empty((p.K, p.N, p.M), dtype=torch.float32, device=dev))
    lls = torch.empty((iters, p.S), dtype=torch.float32, device=dev)
    for it in range(iters):
        forward_backward_grad(p, phase=0, loglik=lls[it], counts=counts, ws=ws, stream=stream)
        for n, par in zip(counts, (p.pi, p.A, p.B)):
            reestimate_rows(n, par, out=par, stream=stream)
    return lls


def softmax_rows(logits: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    _dev(logits, torch.float32, "logits")
    if out is None:
        out = torch.empty_like(logits)
    cols = logits.shape[-1]
    rows = logits.numel() // cols if cols else 0
    rc = load_library().hmm_softmax_rows(_ptr(logits), _ptr(out), rows, cols, _stream(stream))
    _check("hmm_softmax_rows", rc)
    return out


def logit_grad(n: torch.Tensor, probs: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    _dev(n, torch.float32, "n")
    _dev(probs, torch.float32, "probs")
    if out is None:
        out = torch.empty_like(n)
    cols = n.shape[-1]
    rows = n.numel() // cols if cols else 0
    rc = load_library().hmm_logit_grad(_ptr(n), _ptr(probs), _ptr(out), rows, cols, _stream(stream))
    _check("hmm_logit_grad", rc)
    return out


def workspace_error(ws: torch.Tensor, stream=None) -> int:
    """Smallest sequence index the last call flagged (-1 if none); synchronises the stream."""
    v = ctypes.c_int32(0)
    rc = load_library().hmm_workspace_error(_ptr(ws), _stream(stream), ctypes.byref(v))
    _check("hmm_workspace_error", rc)
    return int(v.value)


def bound_library() -> Optional[str]:
    """Path of the library the wrappers call (None before the first load)."""
    return _lib_path


def debug_flags() -> int:
    """HMM_DEBUG_* bits of the bounds checks that failed since the last call (debug build
    only; synchronises the device).  Raises HMMError(HMM_ERR_UNSUPPORTED) in a normal build."""
    v = ctypes.c_uint32(0)
    _check("hmm_debug_flags", load_library().hmm_debug_flags(ctypes.byref(v)))
    return int(v.value)


def profile_enable(on: bool = True):
    """Bracket later main-kernel launches with HIP events (clears earlier records)."""
    _check("hmm_profile_enable", load_library().hmm_profile_enable(1 if on else 0))


def profile_read(kernel: int):
    """(total milliseconds, launches) of one kernel family since profile_enable; synchronises."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int32(0)
    _check("hmm_profile_read", load_library().hmm_profile_read(int(kernel), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


class HMMLogLik(torch.autograd.Function):
    """log P(O_s | softmax-parameterised lambda_{m(s)}) with the adjoint as backward.

    forward(logit_pi [K][N], logit_A [K][N][N], logit_B [K][N][M], symbols, offsets,
            lengths, model_of_seq, max_len) -> loglik [S]
    The forward keeps alpha checkpoints in the workspace; backward runs the
    backward kernel with the incoming gradient as sequence weights and maps the
    expected counts to logit gradients.
    """

    @staticmethod
    def forward(ctx, logit_pi, logit_A, logit_B, symbols, offsets, lengths, model_of_seq, max_len=None):
        pi = softmax_rows(logit_pi.contiguous())
        A = softmax_rows(logit_A.contiguous())
        B = softmax_rows(logit_B.contiguous())
        p = Problem(pi, A, B, symbols, offsets, lengths, model_of_seq, max_len=max_len)
        loglik, _, ws = forward_backward_grad(p, phase=1)
        ctx.problem = p
        ctx.ws = ws
        return loglik

    @staticmethod
    def backward(ctx, grad_out):
        p = ctx.problem
        w = grad_out.contiguous().to(torch.float32)
        _, (npi, nA, nB), _ = forward_backward_grad(p, seq_weight=w, phase=2, ws=ctx.ws)
        g_pi = logit_grad(npi, p.pi)
        g_A = logit_grad(nA, p.A)
        g_B = logit_grad(nB, p.B)
        return g_pi, g_A, g_B, None, None, None, None, None


def loglik_from_logits(logit_pi, logit_A, logit_B, symbols, offsets, lengths, model_of_seq, max_len=None):
    return HMMLogLik.apply(logit_pi, logit_A, logit_B, symbols, offsets, lengths, model_of_seq, max_len)
